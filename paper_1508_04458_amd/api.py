"""Python face of the C ABI: reconstruction contexts (a stack of scans of one geometry on
one GPU) and batches of contexts of different geometries.

Every method marshals torch tensors (device memory and the current stream) into the
matching `wamct_*` call; all arithmetic runs in the HIP kernels of libwamct.so."""
import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check, lib

_DT = {"f32": (_lib.F32, torch.float32), "f64": (_lib.F64, torch.float64)}


def _geometry(g) -> _lib.Geometry:
    if int(g.kind) == _lib.CONE:   # 3-D cone beam: detector columns are the "bins"
        return _lib.Geometry(int(g.kind), int(g.n), float(g.pixel), int(g.n_views), float(g.angle0),
                             float(g.angle_span), int(g.n_cols), float(g.col_pitch), float(g.sod), float(g.sdd),
                             int(g.nz), int(g.n_rows), float(g.row_pitch))
    return _lib.Geometry(int(g.kind), int(g.n), float(g.pixel), int(g.n_views), float(g.angle0),
                         float(g.angle_span), int(g.n_bins), float(g.bin_pitch), float(g.sod), float(g.sdd),
                         1, 1, 0.0)


_WAVELETS = {"haar": 0, "d4": 1}


def _options(levels, dtype, geometry, batch=1, wavelet_dims=0, wavelet="haar"):
    return _lib.Options(int(levels), _DT[dtype][0] if dtype in _DT else 99,
                        _DT[geometry][0] if geometry in _DT else 99, int(batch), int(wavelet_dims),
                        _WAVELETS.get(wavelet, 99))


def validate(g, levels: int, dtype: str = "f32", geometry: str = "f64", batch: int = 1,
             wavelet_dims: int = 0, wavelet: str = "haar") -> Optional[str]:
    """Host-only check of geometry and options; returns None when valid, else the message."""
    buf = ctypes.create_string_buffer(512)
    opt = _options(levels, dtype, geometry, batch, wavelet_dims, wavelet)
    st = lib.wamct_validate(ctypes.byref(_geometry(g)), ctypes.byref(opt), buf, 512)
    return None if st == _lib.OK else buf.value.decode()


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """A stack of `batch` scans of one geometry (counts, I0 each) and the state of
    Algorithm 1 (beta, tree) of every scan, solved in lockstep. With batch = 1 the
    per-scan leading dimension is left out of every returned tensor."""

    def __init__(self, geom, levels: int, dtype: str = "f32", device="cuda", geometry: str = "f64",
                 batch: int = 1, wavelet_dims: int = 0, wavelet: str = "haar"):
        if dtype not in _DT:
            raise ValueError("dtype must be 'f32' or 'f64'")
        self.geom = geom
        self.levels = int(levels)
        self.dtype_name = dtype
        self.dtype = _DT[dtype][1]
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the reconstruction runs on a HIP device only")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.n = int(geom.n)
        if int(geom.kind) == _lib.CONE:
            self.n_rays = int(geom.n_views) * int(geom.n_rows) * int(geom.n_cols)
            self.img_shape = (int(geom.nz), self.n, self.n)
        else:
            self.n_rays = int(geom.n_views) * int(geom.n_bins)
            self.img_shape = (self.n, self.n)
        self.npix = int(np.prod(self.img_shape))
        self.S = int(batch)
        self.wavelet_dims = int(wavelet_dims)
        self.wavelet = wavelet
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            opt = _options(self.levels, dtype, geometry, self.S, wavelet_dims, wavelet)
            check(lib.wamct_create(ctypes.byref(_geometry(geom)), ctypes.byref(opt),
                                   ctypes.c_void_p(stream), ctypes.byref(self._h)))

    # ------------------------------------------------------------------ plumbing
    def close(self):
        if self._h:
            lib.wamct_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fn, *args):
        check(fn(self._h, *args), self._h)

    def _arr(self, t: torch.Tensor, numel: int, name: str, dtype=None) -> torch.Tensor:
        dtype = dtype or self.dtype
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device or t.dtype != dtype or t.numel() != numel or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous {dtype} tensor of {numel} elements on {self.device}")
        return t

    def _shape(self, *dims):
        return dims if self.S == 1 else (self.S, *dims)

    def _new(self, numel: int, dtype=None, shape=None):
        t = torch.empty(numel, dtype=dtype or self.dtype, device=self.device)
        return t if shape is None else t.view(*shape)

    def _per_scan(self, values):
        return values[0] if self.S == 1 else list(values)

    # ------------------------------------------------------------------ data and state
    def set_data(self, d: torch.Tensor, i0) -> None:
        """d: [S, n_rays] counts; i0: a tensor of the same shape, one number for every scan,
        or a sequence of S numbers."""
        self._arr(d, self.S * self.n_rays, "d")
        if isinstance(i0, torch.Tensor):
            self._arr(i0, self.S * self.n_rays, "i0")
            self._call(lib.wamct_set_data, _ptr(d), _ptr(i0), None)
            return
        vals = [float(v) for v in i0] if isinstance(i0, (list, tuple)) else [float(i0)] * self.S
        if len(vals) != self.S:
            raise ValueError(f"expected {self.S} scalar I0 values")
        self._call(lib.wamct_set_data, _ptr(d), None, (ctypes.c_double * self.S)(*vals))

    def reset(self) -> None:
        self._call(lib.wamct_reset)

    def set_state(self, beta: torch.Tensor, mask: torch.Tensor) -> None:
        self._arr(beta, self.S * self.npix, "beta")
        self._arr(mask, self.S * self.npix, "mask", torch.uint8)
        self._call(lib.wamct_set_state, _ptr(beta), _ptr(mask))

    def get_state(self):
        nn = self.S * self.npix
        beta = self._new(nn, shape=self._shape(*self.img_shape))
        mask = self._new(nn, torch.uint8, self._shape(*self.img_shape))
        it = ctypes.c_int32()
        self._call(lib.wamct_get_state, _ptr(beta), _ptr(mask), ctypes.byref(it))
        return beta, mask, it.value

    # ------------------------------------------------------------------ Algorithm 1
    def iterate(self, n_iters: int, idiv: Optional[torch.Tensor] = None) -> Optional[torch.Tensor]:
        if idiv is not None:
            self._arr(idiv, self.S * n_iters, "idiv", torch.float64)
        self._call(lib.wamct_iterate, int(n_iters), _ptr(idiv))
        return idiv

    def expand(self, frac: float = 0.1):
        ns = (ctypes.c_int32 * self.S)()
        self._call(lib.wamct_expand, float(frac), ns)
        return self._per_scan(ns)

    def solve(self, n_iters: int, schedule: Sequence[int] = (), frac: float = 0.1,
              idiv: Optional[torch.Tensor] = None, trace: bool = True) -> Optional[torch.Tensor]:
        """Algorithm 1 with the tree schedule; returns the I-divergence trace [S, n_iters + 1]
        (None with trace=False, which also skips the extra full forward pass per iteration
        of ordered subsets)."""
        if idiv is None and trace:
            idiv = self._new(self.S * (n_iters + 1), torch.float64, self._shape(n_iters + 1))
        if idiv is not None:
            self._arr(idiv, self.S * (n_iters + 1), "idiv", torch.float64)
        sched = (ctypes.c_int32 * max(1, len(schedule)))(*[int(s) for s in schedule])
        self._call(lib.wamct_solve, int(n_iters), sched, len(schedule), float(frac), _ptr(idiv))
        return idiv

    def set_tree_schedule(self, at: Sequence[int], masks: Optional[torch.Tensor]) -> None:
        """Explicit tree sequence Z_s^(j): before update at[k] of a solve, masks[k] (uint8,
        [n_trees, S, *image] contiguous on the device) becomes the active set; solve() then
        takes no expansion list. An empty `at` clears the schedule."""
        n = len(at)
        if n:
            self._arr(masks, n * self.S * self.npix, "masks", torch.uint8)
        arr = (ctypes.c_int32 * max(1, n))(*[int(a) for a in at])
        self._call(lib.wamct_set_tree_schedule, n, arr, _ptr(masks) if n else None)

    def tree_schedule(self) -> List[int]:
        n = ctypes.c_int32()
        self._call(lib.wamct_get_tree_schedule, ctypes.byref(n), None, 0)
        arr = (ctypes.c_int32 * max(1, n.value))()
        self._call(lib.wamct_get_tree_schedule, ctypes.byref(n), arr, n.value)
        return [int(arr[k]) for k in range(n.value)]

    def set_walk_lanes(self, lanes: int) -> None:
        """Lanes per ray of the leaf walk: 1, 2 or 4 (0: by the launch's ray count)."""
        self._call(lib.wamct_set_walk_lanes, int(lanes))

    def walk_lanes(self) -> int:
        v = ctypes.c_int32()
        self._call(lib.wamct_get_walk_lanes, ctypes.byref(v))
        return v.value

    def set_tree_sharing(self, shared: bool) -> None:
        """Scans as z-slices of one volume sharing one tree grown on the slice-summed image."""
        self._call(lib.wamct_set_tree_sharing, 1 if shared else 0)

    def tree_sharing(self) -> bool:
        v = ctypes.c_int32()
        self._call(lib.wamct_get_tree_sharing, ctypes.byref(v))
        return bool(v.value)

    _RULES = {"value": _lib.RULE_VALUE, "gradient": _lib.RULE_GRADIENT}

    def set_tree_rule(self, rule: str) -> None:
        """"value" (the paper's rule: leaves holding a pixel above frac x max(mu) split) or
        "gradient" (leaves whose would-be details have the largest I-divergence gradient
        |Omega^T H^T (d - q-hat)| above frac x its maximum split)."""
        if rule not in self._RULES:
            raise ValueError("rule must be 'value' or 'gradient'")
        self._call(lib.wamct_set_tree_rule, self._RULES[rule])

    def tree_rule(self) -> str:
        v = ctypes.c_int32()
        self._call(lib.wamct_get_tree_rule, ctypes.byref(v))
        return {b: a for a, b in self._RULES.items()}[v.value]

    def set_penalty(self, lam: float) -> None:
        """Weight of the roughness penalty lambda R(mu) (0 = Algorithm 1 without penalty)."""
        self._call(lib.wamct_set_penalty, float(lam))

    def penalty(self) -> float:
        v = ctypes.c_double()
        self._call(lib.wamct_get_penalty, ctypes.byref(v))
        return v.value

    def set_subsets(self, n_subsets: int) -> None:
        """Ordered subsets of views: every iteration becomes a pass of n_subsets updates."""
        self._call(lib.wamct_set_subsets, int(n_subsets))

    def subsets(self) -> int:
        v = ctypes.c_int32()
        self._call(lib.wamct_get_subsets, ctypes.byref(v))
        return v.value

    def set_tiling(self, lanes: int) -> None:
        self._call(lib.wamct_set_tiling, int(lanes))

    def tiling(self) -> int:
        v = ctypes.c_int32()
        self._call(lib.wamct_get_tiling, ctypes.byref(v))
        return v.value

    # ------------------------------------------------------------------ operators
    def synthesize(self) -> torch.Tensor:
        mu = self._new(self.S * self.npix, shape=self._shape(*self.img_shape))
        self._call(lib.wamct_synthesize, _ptr(mu))
        return mu

    def project(self, mu: torch.Tensor) -> torch.Tensor:
        self._arr(mu, self.npix, "mu")
        p = self._new(self.n_rays)
        self._call(lib.wamct_project, _ptr(mu), _ptr(p))
        return p

    def backproject(self, y: torch.Tensor) -> torch.Tensor:
        self._arr(y, self.n_rays, "y")
        img = self._new(self.npix, shape=self.img_shape)
        self._call(lib.wamct_backproject, _ptr(y), _ptr(img))
        return img

    def backproject_split(self, y: torch.Tensor):
        self._arr(y, self.S * self.n_rays, "y")
        bp = self._new(self.S * self.npix, shape=self._shape(*self.img_shape))
        bm = self._new(self.S * self.npix, shape=self._shape(*self.img_shape))
        self._call(lib.wamct_backproject_split, _ptr(y), _ptr(bp), _ptr(bm))
        return bp, bm

    def forward(self):
        q = self._new(self.S * self.n_rays, shape=self._shape(self.n_rays))
        idiv = self._new(self.S, torch.float64)
        self._call(lib.wamct_forward, _ptr(q), _ptr(idiv))
        return q, idiv

    def idiv(self, q: torch.Tensor) -> torch.Tensor:
        self._arr(q, self.S * self.n_rays, "q")
        out = self._new(self.S, torch.float64)
        self._call(lib.wamct_idiv, _ptr(q), _ptr(out))
        return out

    def b(self) -> torch.Tensor:
        out = self._new(self.S * self.npix, shape=self._shape(*self.img_shape))
        self._call(lib.wamct_get_b, _ptr(out))
        return out

    def tree_stats(self) -> Dict[str, float]:
        """Per scan: Z0, W, active coefficients, held updates (lists when S > 1)."""
        z0, w = (ctypes.c_double * self.S)(), (ctypes.c_int64 * self.S)()
        na, nh = (ctypes.c_int64 * self.S)(), (ctypes.c_int64 * self.S)()
        self._call(lib.wamct_tree_stats, z0, w, na, nh)
        return dict(z0=self._per_scan(z0), w=self._per_scan(w), n_active=self._per_scan(na),
                    n_held=self._per_scan(nh))

    # ------------------------------------------------------------------ differentiable loss
    def loss(self, c: torch.Tensor, d: torch.Tensor, i0):
        """loss_b = I(d_b || I0 exp(-H Omega c_b)) for a batch c [B, n, n], d [B, n_rays].
        Returns (loss [B] float64, q [B, n_rays]) with q the checkpoint for loss_backward."""
        B = c.shape[0]
        self._arr(c, B * self.n * self.n, "c")
        self._arr(d, B * self.n_rays, "d")
        q = self._new(B * self.n_rays, shape=(B, self.n_rays))
        out = self._new(B, torch.float64)
        if isinstance(i0, torch.Tensor):
            self._arr(i0, B * self.n_rays, "i0")
            self._call(lib.wamct_loss, B, _ptr(c), _ptr(d), _ptr(i0), 0.0, _ptr(out), _ptr(q))
        else:
            self._call(lib.wamct_loss, B, _ptr(c), _ptr(d), None, float(i0), _ptr(out), _ptr(q))
        return out, q

    def loss_backward(self, q: torch.Tensor, d: torch.Tensor, gscale: Optional[torch.Tensor] = None) -> torch.Tensor:
        """grad_b = gscale_b Omega^T H^T (d_b - q_b), [B, n, n] (the adjoint of `loss`)."""
        B = q.shape[0]
        self._arr(q, B * self.n_rays, "q")
        self._arr(d, B * self.n_rays, "d")
        if gscale is not None:
            gscale = gscale.to(device=self.device, dtype=torch.float64).contiguous()
            self._arr(gscale, B, "gscale", torch.float64)
        grad = self._new(B * self.n * self.n, shape=(B, self.n, self.n))
        self._call(lib.wamct_loss_backward, B, _ptr(q), _ptr(d), _ptr(gscale), _ptr(grad))
        return grad

    # ------------------------------------------------------------------ timing
    def timing(self, enable: bool, classes: Optional[Sequence[str]] = None) -> None:
        """Record kernel durations with HIP events (all classes, or the named ones of
        "synth", "forward", "update", "tree", "other"); enable=False stops."""
        mask = 0
        if enable:
            names = _lib.KERNEL_CLASSES if classes is None else classes
            for c in names:
                mask |= 1 << _lib.KERNEL_CLASSES.index(c)
        self._call(lib.wamct_timing, mask)

    def get_timing(self) -> Dict[str, Dict[str, float]]:
        ms = (ctypes.c_double * _lib.NK)()
        cnt = (ctypes.c_int64 * _lib.NK)()
        self._call(lib.wamct_get_timing, ms, cnt)
        return {k: dict(ms=ms[i], launches=cnt[i]) for i, k in enumerate(_lib.KERNEL_CLASSES)}


class Batch:
    """Contexts of different geometries solved together: one iteration of all of them is
    captured into a HIP graph (graph=True) and replayed between tree expansions, the
    contexts spread over `n_streams` streams. The contexts must outlive the batch."""

    def __init__(self, contexts: Sequence[Context], n_streams: int = 4, graph: bool = True):
        self.contexts = list(contexts)
        if not self.contexts:
            raise ValueError("a batch needs at least one context")
        dev = self.contexts[0].device
        if any(c.device != dev for c in self.contexts):
            raise ValueError("all contexts of a batch must be on one device")
        self.device = dev
        self._h = ctypes.c_void_p()
        handles = (ctypes.c_void_p * len(self.contexts))(*[c._h.value for c in self.contexts])
        with torch.cuda.device(dev):
            stream = torch.cuda.current_stream(dev).cuda_stream
            _lib.check_batch(lib.wamct_batch_create(len(self.contexts), handles, int(n_streams),
                                                    1 if graph else 0, ctypes.c_void_p(stream),
                                                    ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib.wamct_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fn, *args):
        _lib.check_batch(fn(self._h, *args), self._h)

    def reset(self) -> None:
        self._call(lib.wamct_batch_reset)

    def solve(self, n_iters: int, schedule: Sequence[int] = (), frac: float = 0.1):
        """Returns the I-divergence traces, one tensor per context ([S, n_iters + 1], or
        [n_iters + 1] for a single-scan context)."""
        out = [c._new(c.S * (n_iters + 1), torch.float64, c._shape(n_iters + 1)) for c in self.contexts]
        ptrs = (ctypes.c_void_p * len(out))(*[t.data_ptr() for t in out])
        sched = (ctypes.c_int32 * max(1, len(schedule)))(*[int(s) for s in schedule])
        self._call(lib.wamct_batch_solve, int(n_iters), sched, len(schedule), float(frac), ptrs)
        return out

    def autotune(self, n_trial: int = 2, candidates: Optional[Sequence[int]] = None):
        """Backprojection tiling per context, chosen by timing; returns the choices."""
        chosen = (ctypes.c_int32 * len(self.contexts))()
        if candidates is None:
            self._call(lib.wamct_batch_autotune, int(n_trial), None, 0, chosen)
        else:
            cand = (ctypes.c_int32 * len(candidates))(*[int(c) for c in candidates])
            self._call(lib.wamct_batch_autotune, int(n_trial), cand, len(candidates), chosen)
        return list(chosen)

    def stats(self) -> Dict[str, object]:
        lanes = (ctypes.c_int32 * len(self.contexts))()
        gl, gn, cap = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._call(lib.wamct_batch_stats, lanes, ctypes.byref(gl), ctypes.byref(gn), ctypes.byref(cap))
        return dict(stream_of_context=list(lanes), graph_launches=gl.value, graph_nodes=gn.value,
                    captures=cap.value)


NOALLOC_MAX_PARTIALS = 1 << 20
NOALLOC_RAYS_PER_PARTIAL = 256


def idiv_noalloc(d: torch.Tensor, q: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """I(d_s || q_s) for every row s of d, q ([n_scans, n_rays] or [n_rays], float32 or
    float64, one dtype, on the current device) into `out` (float64 [n_scans]) through
    wamct_idiv_noalloc: no context and no device allocation by the library (its partial
    sums live in a static per-device buffer), enqueued on the current stream. `out` is the
    caller's, so nothing here allocates either."""
    if d.dtype != q.dtype or d.dtype not in (torch.float32, torch.float64):
        raise TypeError("d and q must share a dtype, float32 or float64")
    if d.shape != q.shape or d.dim() not in (1, 2):
        raise ValueError(f"d {tuple(d.shape)} and q {tuple(q.shape)} must have one shape [n_scans, n_rays]")
    if not (d.is_contiguous() and q.is_contiguous() and out.is_contiguous()):
        raise ValueError("d, q and out must be contiguous")
    scans = 1 if d.dim() == 1 else d.shape[0]
    if out.dtype != torch.float64 or out.numel() != scans:
        raise ValueError(f"out must be float64 with {scans} entries")
    dt = _lib.F32 if d.dtype == torch.float32 else _lib.F64
    stream = torch.cuda.current_stream(d.device).cuda_stream
    check(lib.wamct_idiv_noalloc(dt, int(d.shape[-1]), int(scans), _ptr(d), _ptr(q), _ptr(out),
                                 ctypes.c_void_p(stream)))
    return out
