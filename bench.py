"""Benchmark: tree-adaptive wavelet AM on one MI355X.

Default workload (what `python bench.py` runs): cone512, the 3-D circular cone beam
(512x512x256 volume, 720 views of a 256x1024 flat detector, 3-level 3-D Haar octree, FP32,
50 iterations with expansions at 11, 21 and 43). A step is one complete reconstruction of
Algorithm 1 with the tree rule from beta = 0 (Z0 and work lists rebuilt at every
expansion). Inputs (counts, I0) are resident in HBM before timing starts. The 2-D fan-beam
workload fan512 (512x512, 720 views x 1024 bins, 3-level Haar tree, 100 iterations with
expansions at 21/43/85) runs after it and is reported as the nested object "fan512".
Prints ONE JSON line.

Extra fields (for either workload):
  gray_voxel_per_s  sum_j 2 W_j / time, W_j = (ray, active coefficient) pairs with phi != 0
  full_am           image-domain AM (levels = 0) on the same GPU: it/s
  equal_idiv        iterations and time image-domain AM needs to reach the tree run's final
                    I-divergence (the Results section's "same objective function value level")
  gradient_rule     the same solve with the residual-gradient tree rule instead of the
                    paper's value rule (final I-divergence, time to the value rule's final)
  roofline          the dominant kernel class, timed with HIP events on the library's stream
                    over the timed steps, against stored-Phi-equivalent bytes (achieved, frac)
                    and, where the committed byte counters match the current sources, against
                    the measured bytes (measured_gbs, measured_frac)
  cpu_baseline      the FP64 CPU oracle on a bounded sample of the workload, with the host

Other workloads: --config fan512 alone, --config uneven (256 independent problems of uneven
size solved as one batch, graph-replayed) and --config loss16 (differentiable loss +
adjoint, 16 slices).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AM iter/s + GRay-voxel/s (fwd+back), tree vs full AM, same GPU, equal I-div"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cone512")
    ap.add_argument("--geometry", default="f64", choices=["f32", "f64"])
    ap.add_argument("--full-iters", type=int, default=300, help="cap for the equal-I-div full-AM run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-full-am", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=36)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-sized buffer 3 times (reference kernel for PMC byte counters)")
    ap.add_argument("--os-subsets", type=int, default=8, help="fan512: ordered-subsets comparison (0 = skip)")
    ap.add_argument("--no-gradient-rule", action="store_true", help="fan512: skip the residual-gradient rule leg")
    ap.add_argument("--no-d4", action="store_true", help="fan512: skip the Daubechies-4 leg")
    ap.add_argument("--d4-steps", type=int, default=3, help="fan512: timed solves of the Daubechies-4 leg")
    ap.add_argument("--problems", type=int, default=256, help="uneven: number of problems")
    ap.add_argument("--streams", type=int, default=4, help="uneven: streams of the batch")
    ap.add_argument("--no-graph", action="store_true", help="uneven: launch directly instead of graph replay")
    ap.add_argument("--autotune", action="store_true", help="uneven: tune the backprojection tiling first")
    ap.add_argument("--no-sequential", action="store_true", help="uneven: skip the one-context-at-a-time run")
    ap.add_argument("--cone-iters", type=int, default=0, help="cone: iterations per solve (0 = the config's)")
    ap.add_argument("--cone-full-iters", type=int, default=60,
                    help="cone: cap for the equal-I-div voxel-AM run")
    ap.add_argument("--no-fan512", action="store_true", help="cone512: skip the nested fan512 workload")
    ap.add_argument("--no-uneven", action="store_true", help="cone512: skip the nested uneven batch")
    ap.add_argument("--uneven-steps", type=int, default=2, help="cone512: timed steps of the nested uneven batch")
    ap.add_argument("--no-slices", action="store_true",
                    help="cone: skip the per-slice 2-D Haar representation (one shared tree)")
    ap.add_argument("--fan-steps", type=int, default=10, help="cone512: timed steps of the nested fan512 run")
    ap.add_argument("--fan-warmup", type=int, default=2, help="cone512: warm-up steps of the nested fan512 run")
    return ap.parse_args()


# sources whose change can change a kernel's traffic: kernels, the headers they include,
# and the host code that sets tilings and launch shapes
KERNEL_SOURCES_2D = ("wamct_kernels.hip", "wamct_geom.h", "wamct_internal.h", "wamct_worklist.h",
                     "wamct_api.hip", "wamct_ctx.h")
KERNEL_SOURCES_3D = ("wamct_kernels3.hip", "wamct_internal3.h", "wamct_internal.h", "wamct_worklist.h",
                     "wamct_api3.hip", "wamct_ctx.h")
KERNEL_SOURCES_D4 = ("wamct_d4.hip", "wamct_internal.h", "wamct_api.hip")


def kernel_source_hash(files=KERNEL_SOURCES_2D, tiling=None):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1508_04458_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if tiling is not None:
        h.update(f"tiling={int(tiling)}".encode())
    return h.hexdigest()[:16]


def host_info():
    """CPU model and logical CPU count of the host the CPU baseline ran on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def roofline(alg_bytes, ms, traffic, valu_issue=None, **kw):
    """Roofline object of one launch (or pass) of `ms` milliseconds: `achieved`/`frac` are the
    stored-Phi-equivalent (algorithmic) bytes over the time against the 8 TB/s HBM peak;
    `measured_gbs`/`measured_frac` are the measured memory-side bytes (`traffic`, from the
    committed byte counters, null when they were taken on other sources) over the same time."""
    a = alg_bytes / (ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": round(a, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(a / HBM_PEAK_GBS, 4), "traffic": traffic}
    if traffic:
        m = traffic / (ms * 1e-3) / 1e9
        r.update(measured_gbs=round(m, 1), measured_frac=round(m / HBM_PEAK_GBS, 4))
    else:
        r.update(measured_gbs=None, measured_frac=None)
    # measured VALU issue (wave64 VALU instructions per CU-cycle; a CU issues at most one):
    # the fraction of the VALU roof the same kernels reach, from the committed counters
    r["valu_issue_frac"] = valu_issue
    r.update(kw)
    return r


def measured_traffic(kernel_hash, config, phase, key="bytes_per_launch"):
    """A phase's measured figure from the committed rocprofv3 summary, only if taken on the
    current kernel source: HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated;
    key "bytes_per_launch") or the VALU issue rate (wave64 VALU instructions per CU-cycle,
    SQ_INSTS_VALU over 256 CUs x the active cycles; key "valu_issue")."""
    path = os.path.join(ROOT, "profiles", f"traffic_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash:
        return None
    return rec.get(key, {}).get(phase)


def measure_copy_peak(dev):
    """HBM bandwidth of a plain device copy on this GPU (1 GiB, read + write bytes over the
    HIP-event time of 10 copies after 2 warm-up copies), GB/s: the measured roof beside the
    8 TB/s published peak."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(gbs, 1)


GOLD_FAN512 = os.path.join(ROOT, "tests", "golden", "fan512_solve.npz")


def cpu_baseline(P, n_views_sample):
    """The FP64 oracle (never tuned) on a view subset of the same scan: Algorithm 1 over the
    rays of `n_views_sample` evenly spaced views, timed (trees, Phi builds and iterations; not
    H or b) and scaled by n_views / n_views_sample to AM iterations per second. For fan512 the
    solve follows the oracle's own tree sequence of the whole scan (tests/golden, written by
    the oracle alone), so every Phi_j holds the whole scan's active set on the sampled rays and
    the work per iteration is that of the whole scan's, in proportion; otherwise the tree rule
    runs on the subset."""
    import numpy as np
    g = P.geom
    step = max(1, g.n_views // n_views_sample)
    views = np.arange(0, g.n_views, step)[:n_views_sample]
    rows = (views[:, None] * g.n_bins + np.arange(g.n_bins)[None, :]).ravel()
    masks = None
    if P.name == "fan512" and os.path.exists(GOLD_FAN512):
        z = np.load(GOLD_FAN512, allow_pickle=False)
        nn = g.n * g.n
        mk = np.unpackbits(z["masks"], axis=1)[:, :nn].reshape(-1, g.n, g.n)
        masks = {int(a): mk[k] for k, a in enumerate(z["tree_at"]) if k > 0}
    job = ("fan", g, views, P.levels, P.d[rows], P.i0, P.n_iters, () if masks else tuple(P.schedule), masks)
    dt, final = _oracle_sample_job(job)
    scale = g.n_views / len(views)
    per_iter = dt * scale / P.n_iters
    trees = ("the whole scan's tree sequence of the oracle (trees at "
             f"{sorted(masks)})" if masks else f"its own tree rule (expansions {P.schedule})")
    out = {"value": 1.0 / per_iter, "unit": "AM iter/s", "cores": 1, "kind": "oracle",
           "sample": (f"FP64 NumPy/SciPy oracle, Algorithm 1, {P.n_iters} iterations on the rays of "
                      f"{len(views)} of {g.n_views} views following {trees}; solve time {dt:.1f} s "
                      f"scaled by {scale:.0f}; setup (H, b) excluded; single thread"),
           "host": host_info(), "final_idiv_sample": final}
    out["all_cores"] = _oracle_all_cores(job, scale, P.n_iters)
    return out


def _oracle_sample_job(job):
    """One oracle solve of a CPU-baseline sample (runs in the bench process or in a forked
    worker; NumPy/SciPy only): builds H (untimed), times Algorithm 1. -> (seconds, final I-div)."""
    if job[0] == "fan":
        _, g, views, levels, d, i0, n_iters, schedule, masks = job
        from oracle import siddon, wam
        H = siddon.system_matrix(g, views=views)
        t0 = time.perf_counter()
        r = wam.wam_solve(H, g.n, levels, d, i0, n_iters, g.pixel, schedule=schedule, masks=masks)
        return time.perf_counter() - t0, float(r["idiv"][-1])
    _, g, levels, d, i0, n_iters, schedule = job
    from oracle import vol3d
    H = vol3d.system_matrix3(g)
    t0 = time.perf_counter()
    r = vol3d.wam_solve3(H, g.n, g.nz, levels, d, i0, n_iters, g.pixel, schedule=schedule)
    return time.perf_counter() - t0, float(r["idiv"][-1])


def _oracle_all_cores(job, scale, n_iters):
    """The secondary CPU baseline: the same sample solved by W single-threaded worker processes
    at once (W = the host's logical CPUs, at most 16), each an independent problem; throughput =
    W samples per the slowest worker's solve time, scaled as the single-thread figure."""
    import concurrent.futures as cf
    import multiprocessing as mp
    w = max(1, min(16, os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(w, mp_context=mp.get_context("fork")) as ex:
        res = list(ex.map(_oracle_sample_job, [job] * w))
    slowest = max(dt for dt, _ in res)
    return {"value": w / (slowest * scale / n_iters), "unit": "AM iter/s", "cores": w,
            "sample": f"{w} concurrent single-threaded solves of the same sample (one per process; slowest "
                      f"{slowest:.1f} s, fastest {min(dt for dt, _ in res):.1f} s), scaled as the single-thread figure"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bench_uneven(args, steps=None, warmup=None, autotune=None):
    """Uneven batch: `problems` independent fan-beam scans (image side from {128, 256, 384,
    512}, views from {360, 540, 720}, 2n bins, I0 in [1e4, 1e5]), each solved with the
    3-level tree-adaptive AM (100 iterations, expansions 21/43/85). Scans of one geometry
    form one context (a stack); the contexts run together as one batch whose iterations
    are replayed from a captured HIP graph. A step solves every problem from beta = 0."""
    import numpy as np
    import torch
    from paper_1508_04458_amd import api, synth

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    autotune = args.autotune if autotune is None else autotune
    workers = max(1, min(16, os.cpu_count() or 1))
    specs = synth.uneven_specs(args.problems)
    log(f"drawing {len(specs)} problems with {workers} processes")
    t0 = time.perf_counter()
    probs = synth.make_uneven_batch(specs, workers=workers)
    log(f"problems ready in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    classes = {}
    for P in probs:
        classes.setdefault((P.geom.n, P.geom.n_views), []).append(P)
    keys = sorted(classes, key=lambda k: -k[0] * k[0] * k[1] * len(classes[k]))
    ctxs = []
    for k in keys:
        ps = classes[k]
        c = api.Context(ps[0].geom, ps[0].levels, "f32", device=dev, geometry=args.geometry, batch=len(ps))
        c.set_data(torch.as_tensor(np.concatenate([P.d for P in ps]), dtype=torch.float32, device=dev),
                   [P.i0 for P in ps])
        ctxs.append(c)
    del probs
    P0 = classes[keys[0]][0]
    J, sched = P0.n_iters, list(P0.schedule)
    batch = api.Batch(ctxs, n_streams=args.streams, graph=not args.no_graph)
    M = sum(c.S * c.n_rays for c in ctxs)
    NN = sum(c.S * c.n * c.n for c in ctxs)
    log(f"{len(ctxs)} contexts, {M / 1e6:.1f} M rays, {NN / 1e6:.1f} M pixels")

    # ---- W_j and |Z_s| per segment (untimed pass through the same schedule)
    batch.reset()
    marks = [0] + sched + [J]
    w_it = 0.0
    act_it = 0.0
    for k, (a, b) in enumerate(zip(marks[:-1], marks[1:])):
        for c in ctxs:
            if k > 0:
                c.expand(0.1)
            st = c.tree_stats()
            w = st["w"] if c.S > 1 else [st["w"]]
            na = st["n_active"] if c.S > 1 else [st["n_active"]]
            w_it += sum(w) * (b - a)
            act_it += sum(na) * (b - a)
            c.iterate(b - a)
    torch.cuda.synchronize()
    log("tree statistics done")

    def step():
        batch.reset()
        return batch.solve(J, sched, 0.1)

    tune = None
    for _ in range(warmup):
        step()
    if autotune:
        # one step with the default shapes, then the measured choice of tiling and leaf-walk
        # lanes per context (each candidate timed on the context's current, last tree)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        t_default = time.perf_counter() - t0
        defaults = [(c.tiling(), c.walk_lanes()) for c in ctxs]
        chosen = batch.autotune(1)
        lanes = [c.walk_lanes() for c in ctxs]
        log(f"autotune: tiling {chosen}, walk lanes {lanes}")
        step()
        tune = {"ms_per_step_default_shapes": round(t_default * 1e3, 3),
                "default_tiling_lanes": defaults,
                "chosen_tiling": chosen, "chosen_walk_lanes": lanes,
                "classes": [[c.n, c.geom.n_views, c.S] for c in ctxs]}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt * 1e3 / steps
    n_prob = sum(c.S for c in ctxs)
    it_s = n_prob * J * steps / dt
    if tune is not None:
        tune["ms_per_step_tuned"] = round(ms_step, 3)
        tune["speedup"] = round(tune["ms_per_step_default_shapes"] / ms_step, 3)
    final = [float(t.reshape(-1, J + 1)[:, -1].sum().item()) for t in tr]
    stats = batch.stats()
    log(f"batch: {ms_step:.1f} ms per step")

    seq = None
    if not args.no_sequential:
        # the same contexts one after another on one stream, no batch (same kernels)
        for c in ctxs:
            c.reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for c in ctxs:
            c.reset()
            c.solve(J, sched, 0.1)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t1
        seq = {"ms_per_step": round(t_seq * 1e3, 3), "iter_per_s": round(n_prob * J / t_seq, 2),
               "batch_speedup": round(t_seq * 1e3 / ms_step, 3)}
        log(f"sequential: {t_seq * 1e3:.1f} ms")

    # whole iteration against the HBM-equivalent roofline: Phi stored would move 8 B per
    # (ray, active coefficient) pair in each of the two passes, 8 B per ray (d, q-hat) and
    # 16 B per active coefficient (beta, b, b-hat+-)
    alg = 16.0 * w_it + 8.0 * M * J + 16.0 * act_it
    per_step_s = ms_step * 1e-3
    roof = {"bound": "hbm", "achieved": round(alg / per_step_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(alg / per_step_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "whole batch iteration (graph replay)", "alg_bytes_per_step": int(alg)}
    out = {"metric": METRIC, "value": round(it_s, 2), "unit": "AM iter/s (problem-iterations)", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if args.geometry == "f32" else "f32 data, f64 ray geometry", "data": "synthetic",
           "config": {"workload": f"uneven batch: {n_prob} fan-beam problems (n in {{128,256,384,512}}, views in "
                                  f"{{360,540,720}}, 2n bins, I0 in [1e4,1e5]), {len(ctxs)} geometry classes, "
                                  f"3-level tree AM, {J} iterations, expansions at {sched}",
                      "problems": n_prob, "classes": len(ctxs), "rays": M, "pixels": NN,
                      "streams": args.streams, "graph": not args.no_graph},
           "gray_voxel_per_s": round(2 * w_it * steps / dt / 1e9, 3),
           "final_idiv_sum": sum(final), "batch_stats": stats, "autotune": tune, "sequential": seq,
           "roofline": roof}
    for c in ctxs:
        c.close()
    torch.cuda.empty_cache()
    return out


def bench_loss(args):
    """Differentiable path: loss_b = I(d_b || I0 exp(-H Omega c_b)) and its hand-written
    adjoint for a batch of 16 slices of the 256x256 fan-beam scan (360 views, 512 bins,
    2-level Haar, every coefficient free, I0 = 5e4). A step is one loss + gradient
    evaluation of the whole batch through the autograd function."""
    import numpy as np
    import torch
    from paper_1508_04458_amd import api, synth
    from paper_1508_04458_amd.autograd import wam_loss

    B = 16
    probs = [synth.make_problem("fan256", problem_idx=k) for k in range(B)]
    g = probs[0].geom
    L = probs[0].levels
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctx = api.Context(g, L, "f32", device=dev, geometry=args.geometry)
    d = torch.as_tensor(np.stack([P.d for P in probs]), dtype=torch.float32, device=dev)
    # coefficients: random small values (the work does not depend on them)
    c0 = np.stack([synth.random_image(g.n, 100 + k, 0.0, 0.004) for k in range(B)])
    c = torch.as_tensor(c0, dtype=torch.float32, device=dev).requires_grad_(True)
    i0 = probs[0].i0

    def step():
        c.grad = None
        loss = wam_loss(c, d, i0, ctx)
        loss.sum().backward()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing(True, ("forward", "update"))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = ctx.get_timing()
    ctx.timing(False)
    full = api.Context(g, 0, "f32", device=dev, geometry=args.geometry)
    nnz = full.tree_stats()["w"]                       # nonzeros of H (every pixel active)
    full.close()
    M = g.n_rays
    ms_step = dt * 1e3 / args.steps
    # forward pixel walk: 8 B per nonzero of H (stored-matrix equivalent) + d, q per ray
    fw = tim["forward"]
    fw_ms = fw["ms"] / max(1, fw["launches"])
    alg_fw = 8.0 * nnz + 12.0 * M
    roof = {"bound": "hbm", "achieved": round(alg_fw / (fw_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(alg_fw / (fw_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_forward<float,double,8>", "avg_launch_ms": round(fw_ms, 5), "launches": fw["launches"],
            "alg_bytes_per_launch": int(alg_fw)}
    out = {"metric": METRIC, "value": round(args.steps / dt, 3), "unit": "loss+grad evals/s (16-slice batch)",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 data, f64 ray geometry, f64 loss", "data": "synthetic",
           "config": {"workload": f"differentiable loss: {B} fan-beam slices {g.n}x{g.n}, {g.n_views} views x "
                                  f"{g.n_bins} bins, {L}-level Haar (all coefficients), I0 = {i0:g}",
                      "batch": B, "rays": M, "pixels": g.n * g.n},
           "slice_evals_per_s": round(B * args.steps / dt, 2),
           "gray_voxel_per_s": round(2 * nnz * B * args.steps / dt / 1e9, 3),
           "time_ms_per_step_by_kernel": {k: round(v["ms"] / args.steps, 4) for k, v in tim.items()
                                          if k in ("forward", "update")},
           "roofline": roof}
    print(json.dumps(out), flush=True)


def cone_cpu_baseline(name, n_full_rays, n_full_side):
    """The FP64 3-D oracle (never tuned) on the downscaled cone-beam case in full (its
    synthesis matrix at full size would not fit a CPU run): Algorithm 1 with the octree rule
    and its schedule; solve time (trees, Phi builds, iterations; not H or b) scaled to the
    full workload by the ratio of rays x volume side (the number of ray-voxel crossings)."""
    from paper_1508_04458_amd import synth
    P = synth.make_cone_problem(name)
    g = P.geom
    job = ("cone", g, P.levels, P.d, P.i0, P.n_iters, tuple(P.schedule))
    dt, _ = _oracle_sample_job(job)
    scale = (n_full_rays * n_full_side) / (g.n_rays * g.n)
    per_iter = dt * scale / P.n_iters
    return {"value": 1.0 / per_iter, "unit": "AM iter/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 NumPy/SciPy 3-D oracle, octree AM, {P.n_iters} iterations (expansions "
                       f"{P.schedule}) on the downscaled case {name} ({g.n}^2 x {g.nz}, {g.n_views} views of "
                       f"{g.n_rows} x {g.n_cols}); solve time {dt:.1f} s scaled by rays x side = {scale:.0f}; "
                       f"setup (H, b) excluded; single thread"),
            "host": host_info(), "all_cores": _oracle_all_cores(job, scale, P.n_iters)}


def bench_cone(args):
    """3-D circular cone beam: 512x512x256 volume (1 mm voxels), 720 views of a 256x1024
    flat detector, 200 random ellipsoids + 10 metal cylinders, I0 = 1e5, 3-level 3-D Haar
    octree AM in FP32, 50 iterations with expansions at 11, 21 and 43. A step is one
    complete reconstruction from beta = 0."""
    if not args.no_cpu_baseline:
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
    import numpy as np
    import torch
    from paper_1508_04458_amd import api, synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    log(f"{args.config}: drawing the phantom (line integrals on the GPU) and the counts")
    P = synth.make_cone_problem(args.config, device=dev)
    g = P.geom
    log(f"phantom and counts ready in {time.perf_counter() - t_gen:.1f} s; {g.n_rays} rays")
    J = args.cone_iters or P.n_iters
    sched = [int(s) for s in synth.scaled_schedule(J, P.levels)]
    d = torch.as_tensor(P.d, dtype=torch.float32, device=dev)
    P = dataclasses_replace(P, d=None, line_integrals=None)
    ctx = api.Context(g, P.levels, "f32", device=dev)
    t1 = time.perf_counter()
    ctx.set_data(d, P.i0)
    torch.cuda.synchronize()
    log(f"context and b = Omega^T H^T d ready in {time.perf_counter() - t1:.1f} s")
    idiv = torch.empty(J + 1, dtype=torch.float64, device=dev)

    # ---- warmup 1 doubles as the per-tree statistics run (W_j, |Z_s|, Z0)
    ctx.reset()
    marks = [0] + sched + [J]
    seg = []
    for k, (a, b) in enumerate(zip(marks[:-1], marks[1:])):
        if k > 0:
            ctx.expand(0.1)
        st = ctx.tree_stats()
        seg.append(dict(start=a, iters=b - a, w=st["w"], n_active=st["n_active"], z0=st["z0"]))
        ctx.iterate(b - a)
        torch.cuda.synchronize()
        log(f"tree {k}: {st['n_active']} active, W = {st['w']:.3e}, iterations {a}..{b}")
    pairs = sum(2 * s["w"] * s["iters"] for s in seg)
    w_avg = sum(s["w"] * s["iters"] for s in seg) / J
    active_avg = sum(s["n_active"] * s["iters"] for s in seg) / J

    def step():
        ctx.reset()
        ctx.solve(J, sched, 0.1, idiv)

    for _ in range(max(0, args.warmup - 1)):
        step()
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"step {k + 1}/{args.steps} done")
    dt = time.perf_counter() - t0
    tim = ctx.get_timing()
    ctx.timing(False)
    tr = idiv.cpu().numpy()
    it_s = J * args.steps / dt
    M, N = g.n_rays, g.n_voxels

    khash = kernel_source_hash(KERNEL_SOURCES_3D, ctx.tiling())

    # algorithmic bytes of the same passes with Phi stored: 8 B per (ray, active coefficient)
    # pair, 4 B per active coefficient read (forward) or 12 B (b, beta read, beta written),
    # 8 B per ray (d read and q-hat written; q-hat read by the update: 4 B)
    fw, up = tim["forward"], tim["update"]
    fw_ms = fw["ms"] / max(1, fw["launches"])
    up_ms = up["ms"] / max(1, J * args.steps)
    alg_fw = 8.0 * w_avg + 4.0 * active_avg + 8.0 * M
    alg_up = 8.0 * w_avg + 4.0 * M + 12.0 * active_avg
    r_fw = roofline(alg_fw, fw_ms, measured_traffic(khash, args.config, "forward"),
                    measured_traffic(khash, args.config, "forward", "valu_issue"), kernel="k3_forward<float>",
                    avg_launch_ms=round(fw_ms, 4), launches=fw["launches"], alg_bytes_per_launch=int(alg_fw),
                    kernel_hash=khash)
    r_up = roofline(alg_up, up_ms, measured_traffic(khash, args.config, "update"),
                    measured_traffic(khash, args.config, "update", "valu_issue"),
                    kernels="k3_gather_part + k3_gather_finish per octree level", avg_pass_ms=round(up_ms, 4),
                    passes=J * args.steps, alg_bytes_per_pass=int(alg_up), kernel_hash=khash)
    dominant = "update" if up["ms"] >= fw["ms"] else "forward"
    out = {"metric": METRIC, "value": round(it_s, 3), "unit": "AM iter/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 data, f64 ray geometry", "data": "synthetic",
           "config": {"workload": f"{args.config}: 3-D cone beam {g.n}x{g.n}x{g.nz}, {g.n_views} views x "
                                  f"{g.n_rows}x{g.n_cols} detector, {P.levels}-level 3-D Haar octree AM, {J} "
                                  f"iterations, expansions at {sched}",
                      "levels": P.levels, "iterations": J, "schedule": sched, "rays": M, "voxels": N},
           "gray_voxel_per_s": round(pairs * args.steps / dt / 1e9, 3),
           "final_idiv": float(tr[-1]), "idiv_decreasing": bool(np.all(np.diff(tr) <= 1e-6 * np.abs(tr[:-1]))),
           "trees": seg,
           "time_ms_per_step_by_kernel": {k: round(v["ms"] / args.steps, 2) for k, v in tim.items()},
           "roofline": r_up if dominant == "update" else r_fw,
           "roofline_other": r_fw if dominant == "update" else r_up}
    ctx.close()
    if not args.no_gradient_rule:
        # the same solve with the residual-gradient tree rule
        grc = api.Context(g, P.levels, "f32", device=dev)
        grc.set_tree_rule("gradient")
        grc.set_data(d, P.i0)
        grc.reset()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        gtr = grc.solve(J, sched, 0.1).cpu().numpy()
        t_gr = time.perf_counter() - t3
        hit = np.nonzero(gtr <= tr[-1])[0]
        k_gr = int(hit[0]) if hit.size else None
        out["gradient_rule"] = {
            "iter_per_s": round(J / t_gr, 3), "ms_per_solve": round(t_gr * 1e3, 1),
            "final_idiv": float(gtr[-1]), "final_active": int(grc.tree_stats()["n_active"]),
            "iters_to_value_rule_final_idiv": k_gr,
            "time_to_value_rule_final_idiv_ms": None if k_gr is None else round(k_gr * t_gr / J * 1e3, 1)}
        grc.close()
        log(f"gradient rule: {J / t_gr:.3f} it/s, final I-div {gtr[-1]:.4e} (value rule {tr[-1]:.4e})")
    if not args.no_slices:
        # the Results section's own representation of a volume: a 2-D Haar transform per
        # z-slice, one tree grown on the slice-summed image (same schedule and fraction)
        slc = api.Context(g, P.levels, "f32", device=dev, wavelet_dims=2)
        slc.set_data(d, P.i0)
        slc.reset()
        s_tr = slc.solve(J, sched, 0.1).cpu().numpy()          # traced run (untimed)
        s_st = slc.tree_stats()
        torch.cuda.synchronize()
        slc.timing(True)
        t4 = time.perf_counter()
        slc.reset()
        slc.solve(J, sched, 0.1, trace=False)
        torch.cuda.synchronize()
        t_sl = time.perf_counter() - t4
        s_tim = slc.get_timing()
        slc.timing(False)
        hit = np.nonzero(s_tr <= tr[-1])[0]
        k_sl = int(hit[0]) if hit.size else None
        out["slices"] = {
            "representation": "2-D Haar per z-slice, one tree grown on the slice-summed image",
            "iter_per_s": round(J / t_sl, 3), "ms_per_solve": round(t_sl * 1e3, 1),
            "final_idiv": float(s_tr[-1]), "final_active": int(s_st["n_active"]), "final_w": int(s_st["w"]),
            "idiv_decreasing": bool(np.all(np.diff(s_tr) <= 1e-6 * np.abs(s_tr[:-1]))),
            "iters_to_octree_final_idiv": k_sl,
            "time_to_octree_final_idiv_ms": None if k_sl is None else round(k_sl * t_sl / J * 1e3, 1),
            "time_ms_per_solve_by_kernel": {k: round(v["ms"], 2) for k, v in s_tim.items()}}
        slc.close()
        log(f"per-slice 2-D Haar: {J / t_sl:.3f} it/s, final I-div {s_tr[-1]:.4e} (octree {tr[-1]:.4e})")
    if not args.no_full_am:
        # voxel AM (levels = 0) from mu = 0 until it reaches the tree run's final I-divergence
        # (or the cap): the Results section compares the two at the same objective value
        full = api.Context(g, 0, "f32", device=dev)
        full.set_data(d, P.i0)
        full.reset()
        torch.cuda.synchronize()
        target = float(tr[-1])
        # run until the lower of the value-rule and gradient-rule final I-divergences
        stop_at = min(target, out.get("gradient_rule", {}).get("final_idiv", target),
                      out.get("slices", {}).get("final_idiv", target))
        cap, chunk = args.cone_full_iters, 5
        buf = torch.empty(chunk, dtype=torch.float64, device=dev)
        trace, done, t_run = [], 0, 0.0
        while done < cap:
            n = min(chunk, cap - done)
            t2 = time.perf_counter()
            full.iterate(n, buf[:n])
            torch.cuda.synchronize()
            t_run += time.perf_counter() - t2
            trace += buf[:n].cpu().tolist()      # I-div before each of these updates
            done += n
            if min(trace[1:] or [math.inf]) <= stop_at:
                break
        last = full.forward()[1]                 # I-div after the last update
        trace.append(float(last.item() if hasattr(last, "item") else last))
        f_it_s = done / t_run
        w_pix = full.tree_stats()["w"]
        hit = [k for k, v in enumerate(trace) if v <= target]
        k_star = hit[0] if hit else None
        out["full_am"] = {"iter_per_s": round(f_it_s, 3), "iterations_run": done, "w_per_pass": int(w_pix),
                          "gray_voxel_per_s": round(2 * w_pix * f_it_s / 1e9, 3)}
        eq = {"tree_final_idiv": target, "full_iters_to_reach": k_star, "full_idiv_at_end": trace[-1],
              "cap": cap}
        if k_star is not None:
            t_eq = k_star / f_it_s
            eq.update(full_time_ms=round(t_eq * 1e3, 1), tree_time_ms=round(dt * 1e3 / args.steps, 1),
                      tree_speedup=round(t_eq / (dt / args.steps), 3))
        out["equal_idiv"] = eq
        for key in ("gradient_rule", "slices"):
            if key not in out:
                continue
            gr = out[key]
            hit = [k for k, v in enumerate(trace) if v <= gr["final_idiv"]]
            k_f = hit[0] if hit else None
            gr.update(full_am_iters_to_its_final_idiv=k_f,
                      full_am_time_to_its_final_idiv_ms=None if k_f is None else round(k_f / f_it_s * 1e3, 1),
                      speedup_vs_full_am=None if k_f is None else round(k_f / f_it_s / (gr["ms_per_solve"] * 1e-3), 3))
        out["pixel_equiv_gray_voxel_per_s"] = round(2 * w_pix * it_s / 1e9, 3)
        full.close()
        log(f"voxel AM: {f_it_s:.3f} it/s, {done} iterations, reaches the tree run's I-div after {k_star}")
    if not args.no_cpu_baseline:
        log("CPU oracle on the downscaled case")
        out["cpu_baseline"] = cone_cpu_baseline("cone64", M, g.n)
    del d
    torch.cuda.empty_cache()
    return out


def copy_calibration(args, dev, out):
    """Three device copies of a buffer of known size at the end of the run: the reference
    that scales the byte counters of a profiling run (FETCH_SIZE, WRITE_SIZE per copy)."""
    if args.copy_calibration <= 0:
        return
    import torch
    src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_calibration_bytes"] = int(src.numel() * 4)


def dataclasses_replace(obj, **kw):
    import dataclasses
    return dataclasses.replace(obj, **kw)


def bench_fan(args, config, steps, warmup):
    """2-D fan beam (fan512: 512x512 image, 720 views x 1024 bins, 40 ellipses + 4 metal disks,
    I0 = 1e5, 3-level Haar tree AM in FP32, 100 iterations with expansions at 21, 43 and 85).
    A step is one complete reconstruction from beta = 0. Returns the result object."""
    import numpy as np
    import torch
    from paper_1508_04458_amd import api, synth

    P = synth.make_problem(config)
    g = P.geom
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    d = torch.as_tensor(P.d, dtype=torch.float32, device=dev)
    ctx = api.Context(g, P.levels, "f32", device=dev, geometry=args.geometry)
    ctx.set_data(d, P.i0)
    J, sched = P.n_iters, list(P.schedule)
    idiv = torch.empty(J + 1, dtype=torch.float64, device=dev)

    # ---- tree statistics per segment (untimed): W_j and |Z_s| of each tree
    ctx.reset()
    marks = [0] + sched + [J]
    seg = []
    for k, (a, b) in enumerate(zip(marks[:-1], marks[1:])):
        if k > 0:
            ctx.expand(0.1)
        st = ctx.tree_stats()
        seg.append(dict(start=a, iters=b - a, w=st["w"], n_active=st["n_active"], z0=st["z0"]))
        ctx.iterate(b - a)
    pairs = sum(2 * s["w"] * s["iters"] for s in seg)
    w_update_avg = sum(s["w"] * s["iters"] for s in seg) / J
    active_avg = sum(s["n_active"] * s["iters"] for s in seg) / J

    def step():
        ctx.reset()
        ctx.solve(J, sched, 0.1, idiv)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # HIP events around the two kernel classes whose rooflines are reported
    ctx.timing(True, ("forward", "update"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = ctx.get_timing()
    ctx.timing(False)
    tr = idiv.cpu().numpy()
    ms_step = dt * 1e3 / steps
    it_s = J * steps / dt

    # ---- roofline of the dominant kernel: the tree walk (forward projection over the leaves
    # of Z_s, Beer's law, I-divergence term). Algorithmic bytes are those of the same pass
    # with Phi stored (the paper lists Phi as an input of Algorithm 1): 8 B per (ray, active
    # coefficient) pair (FP32 value + int32 index), 4 B per active coefficient (beta), 8 B
    # per ray (d read, q-hat written). The kernel itself recomputes Phi on the fly.
    M = g.n_rays
    fw = tim["forward"]
    fw_ms = fw["ms"] / max(1, fw["launches"])
    alg_fw = 8.0 * w_update_avg + 4.0 * active_avg + 8.0 * M
    khash = kernel_source_hash(KERNEL_SOURCES_2D, ctx.tiling())
    roof = roofline(alg_fw, fw_ms, measured_traffic(khash, config, "forward"),
                    measured_traffic(khash, config, "forward", "valu_issue"), kernel="k_forward_rec<float,double>",
                    avg_launch_ms=round(fw_ms, 5), launches=fw["launches"], alg_bytes_per_launch=int(alg_fw),
                    kernel_hash=khash)
    # the update pass (sign-split backprojection + eq. 1.9 zero; one or two kernels per level)
    up = tim["update"]
    upd_ms = up["ms"] / max(1, up["launches"])
    alg_up = 8.0 * w_update_avg + 4.0 * M + 12.0 * active_avg
    roof_up = roofline(alg_up, upd_ms, measured_traffic(khash, config, "update"),
                       measured_traffic(khash, config, "update", "valu_issue"),
                       kernels="k_gather_part + k_gather_finish over the chunked tree levels (+ k_gather per "
                               "level that fills the GPU alone)",
                       avg_pass_ms=round(upd_ms, 5), passes=up["launches"], alg_bytes_per_pass=int(alg_up))
    timing_ms = {k: round(v["ms"] / steps, 4) for k, v in tim.items() if k in ("forward", "update")}

    out = {"metric": METRIC, "value": round(it_s, 2), "unit": "AM iter/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if args.geometry == "f32" else "f32 data, f64 ray geometry",
           "data": "synthetic",
           "config": {"workload": f"{config}: 2-D fan beam {g.n}x{g.n}, {g.n_views} views x {g.n_bins} bins, "
                                  f"{P.levels}-level tree-adaptive wavelet AM, {J} iterations, expansions at {sched}",
                      "levels": P.levels, "iterations": J, "schedule": sched, "rays": M, "pixels": g.n * g.n},
           "gray_voxel_per_s": round(pairs * steps / dt / 1e9, 3),
           "pixel_equiv_gray_voxel_per_s": None,
           "final_idiv": float(tr[-1]),
           "trees": seg,
           "time_ms_per_step_by_kernel": timing_ms,
           "roofline": roof,
           "roofline_update": roof_up}

    # ---- full-image AM (levels = 0) on the same GPU: equal-I-div comparison
    full_trace = None
    if not args.no_full_am:
        full = api.Context(g, 0, "f32", device=dev, geometry=args.geometry)
        full.set_data(d, P.i0)
        cap = args.full_iters
        fidiv = torch.empty(cap + 1, dtype=torch.float64, device=dev)
        full.reset()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        full.solve(cap, [], 0.1, fidiv)
        torch.cuda.synchronize()
        t_full = time.perf_counter() - t1
        ft = fidiv.cpu().numpy()
        full_trace = (ft, cap / t_full)
        w_pix = full.tree_stats()["w"]
        target = tr[-1]
        hit = np.nonzero(ft <= target)[0]
        k_star = int(hit[0]) if hit.size else None
        full_it_s = cap / t_full
        eq = {"tree_final_idiv": float(target), "full_iters_to_reach": k_star,
              "full_idiv_at_cap": float(ft[-1]), "cap": cap}
        if k_star is not None:
            t_eq = k_star / full_it_s
            eq.update(full_time_ms=round(t_eq * 1e3, 3), tree_time_ms=round(ms_step, 3),
                      tree_speedup=round(t_eq * 1e3 / ms_step, 3))
        out["full_am"] = {"iter_per_s": round(full_it_s, 2), "w_per_pass": int(w_pix),
                          "gray_voxel_per_s": round(2 * w_pix * full_it_s / 1e9, 3)}
        out["pixel_equiv_gray_voxel_per_s"] = round(2 * w_pix * it_s / 1e9, 3)
        out["equal_idiv"] = eq
        full.close()
        log(f"{config}: image-domain AM reaches the tree run's I-div after {k_star} iterations")

    # ---- the same solve with the residual-gradient tree rule (same schedule and fraction)
    if not args.no_gradient_rule:
        grc = api.Context(g, P.levels, "f32", device=dev, geometry=args.geometry)
        grc.set_tree_rule("gradient")
        grc.set_data(d, P.i0)
        grc.reset()
        gtr = grc.solve(J, sched, 0.1).cpu().numpy()          # traced run (untimed)
        g_active = grc.tree_stats()["n_active"]
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(2):
            grc.reset()
            grc.solve(J, sched, 0.1, trace=False)
        torch.cuda.synchronize()
        t_gr = (time.perf_counter() - t3) / 2
        target = tr[-1]
        hit = np.nonzero(gtr <= target)[0]
        k_gr = int(hit[0]) if hit.size else None
        out["gradient_rule"] = {
            "iter_per_s": round(J / t_gr, 2), "ms_per_solve": round(t_gr * 1e3, 3), "final_idiv": float(gtr[-1]),
            "final_active": int(g_active), "iters_to_value_rule_final_idiv": k_gr,
            "time_to_value_rule_final_idiv_ms": None if k_gr is None else round(k_gr * t_gr / J * 1e3, 3)}
        if full_trace is not None:
            # image-domain AM to the gradient-rule run's final I-divergence
            ft, f_it_s = full_trace
            hit = np.nonzero(ft <= gtr[-1])[0]
            k_f = int(hit[0]) if hit.size else None
            out["gradient_rule"].update(
                full_am_iters_to_its_final_idiv=k_f,
                full_am_time_to_its_final_idiv_ms=None if k_f is None else round(k_f / f_it_s * 1e3, 3),
                speedup_vs_full_am=None if k_f is None else round(k_f / f_it_s / t_gr, 3))
        grc.close()

    # ---- wavelet AM with ordered subsets of views (same tree schedule, passes of S updates)
    if args.os_subsets > 1:
        S = args.os_subsets
        osc = api.Context(g, P.levels, "f32", device=dev, geometry=args.geometry)
        osc.set_subsets(S)
        osc.set_data(d, P.i0)
        osc.reset()
        otr = osc.solve(J, sched, 0.1).cpu().numpy()          # traced run (untimed)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(2):
            osc.reset()
            osc.solve(J, sched, 0.1, trace=False)
        torch.cuda.synchronize()
        t_os = (time.perf_counter() - t2) / 2
        target = tr[-1]
        hit = np.nonzero(otr <= target)[0]
        k_os = int(hit[0]) if hit.size else None
        out["ordered_subsets"] = {
            "subsets": S, "passes": J, "ms_per_solve": round(t_os * 1e3, 3), "pass_per_s": round(J / t_os, 2),
            "final_idiv": float(otr[-1]), "passes_to_tree_final_idiv": k_os,
            "time_to_tree_final_idiv_ms": None if k_os is None else round(k_os * t_os / J * 1e3, 3),
            "idiv_at_pass": {str(k): float(otr[k]) for k in (1, 2, 5, 10, 21, 43, 85) if k <= J}}
        osc.close()

    # ---- the same solve with the Daubechies-4 basis (same tree rule, schedule and fraction):
    # per-pixel synthesis, pixel-walk forward, support-walking sign-split gather
    if not args.no_d4:
        dc = api.Context(g, P.levels, "f32", device=dev, geometry=args.geometry, wavelet="d4")
        dc.set_data(d, P.i0)
        dc.reset()
        dseg = []
        for k, (a, b) in enumerate(zip(marks[:-1], marks[1:])):     # traced run (untimed)
            if k > 0:
                dc.expand(0.1)
            st = dc.tree_stats()
            dseg.append(dict(start=a, iters=b - a, w=st["w"], n_active=st["n_active"], z0=st["z0"]))
            dc.iterate(b - a)
        dc.reset()
        didiv = torch.empty(J + 1, dtype=torch.float64, device=dev)
        dc.solve(J, sched, 0.1, didiv)
        dtr = didiv.cpu().numpy()
        n_d4 = max(1, args.d4_steps)
        torch.cuda.synchronize()
        dc.timing(True, ("update",))
        t4 = time.perf_counter()
        for _ in range(n_d4):
            dc.reset()
            dc.solve(J, sched, 0.1, didiv)
        torch.cuda.synchronize()
        t_d4 = (time.perf_counter() - t4) / n_d4
        dtim = dc.get_timing()["update"]
        dc.timing(False)
        d_upd_ms = dtim["ms"] / max(1, dtim["launches"])
        d_w = sum(x["w"] * x["iters"] for x in dseg) / J
        d_act = sum(x["n_active"] * x["iters"] for x in dseg) / J
        d_alg = 8.0 * d_w + 4.0 * M + 12.0 * d_act
        d4hash = kernel_source_hash(KERNEL_SOURCES_D4, None)
        hit = np.nonzero(tr <= dtr[-1])[0]
        k_h = int(hit[0]) if hit.size else None
        out["wavelet_d4"] = {
            "iter_per_s": round(J / t_d4, 2), "ms_per_solve": round(t_d4 * 1e3, 3), "steps": n_d4,
            "final_idiv": float(dtr[-1]), "trees": dseg,
            "haar_iters_to_d4_final_idiv": k_h,
            "haar_time_to_d4_final_idiv_ms": None if k_h is None else round(k_h * ms_step / J, 3),
            "roofline_update": roofline(d_alg, d_upd_ms, measured_traffic(d4hash, "d4_fan512", "update"),
                                        measured_traffic(d4hash, "d4_fan512", "update", "valu_issue"),
                                        kernels="k_d4_gather (one wave per work item, support walk)",
                                        avg_pass_ms=round(d_upd_ms, 5), passes=dtim["launches"],
                                        alg_bytes_per_pass=int(d_alg),
                                        note="phi recomputed by walking every ray through each active "
                                             "support; bound by VALU issue, not by memory")}
        dc.close()
        log(f"{config}: Daubechies-4 {J / t_d4:.1f} it/s, final I-div {dtr[-1]:.4e}")

    if not args.no_cpu_baseline:
        log(f"{config}: CPU oracle on {args.cpu_views} views")
        out["cpu_baseline"] = cpu_baseline(P, args.cpu_views)
    ctx.close()
    del d
    torch.cuda.empty_cache()
    return out



def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the view-sharded "
              "multi-GPU design is not built.", file=sys.stderr)
        sys.exit(2)
    if args.config == "uneven":
        print(json.dumps(bench_uneven(args)), flush=True)
        return
    if args.config == "loss16":
        bench_loss(args)
        return
    if not args.no_cpu_baseline:
        # the CPU baseline is a single-threaded oracle
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
    import torch
    dev = torch.device("cuda", 0)
    copy_gbs = measure_copy_peak(dev)
    if args.config.startswith("cone"):
        out = bench_cone(args)
        if args.config == "cone512" and not args.no_fan512:
            log("fan512 (nested)")
            fan = bench_fan(args, "fan512", args.fan_steps, args.fan_warmup)
            for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
                fan.pop(k, None)
            out["fan512"] = fan
        if args.config == "cone512" and not args.no_uneven:
            log("uneven batch (nested)")
            un = bench_uneven(args, steps=args.uneven_steps, warmup=1, autotune=True)
            for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data"):
                un.pop(k, None)
            out["uneven"] = un
    else:
        out = bench_fan(args, args.config, args.steps, args.warmup)
    out["hbm_copy_peak_gbs"] = copy_gbs
    copy_calibration(args, dev, out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
