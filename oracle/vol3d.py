"""3-D cone-beam scan, 3-D Haar basis and the octree tree rule, FP64 (test infrastructure;
see oracle/__init__.py).

Geometry (the paper gives none; this project's reading, stated for every implementation):
  * volume n x n x nz voxels of edge `pixel`, centred on the origin, layout [z][y][x];
    voxel (s, r, c) covers x in [(c - n/2) pixel, (c + 1 - n/2) pixel), y likewise with r,
    z in [(s - nz/2) pixel, (s + 1 - nz/2) pixel) (half-open boxes);
  * circular orbit: view v at angle a = angle0 + v * angle_span / n_views; source at
    sod (cos a, sin a, 0); flat detector centred at -(sdd - sod)(cos a, sin a, 0) with
    column axis (-sin a, cos a, 0) and row axis (0, 0, 1); detector element (row rr, col cc)
    at offsets u = (cc - (n_cols - 1)/2) col_pitch, w = (rr - (n_rows - 1)/2) row_pitch;
  * one ray per element, source to element centre; ray index y = (v n_rows + rr) n_cols + cc;
  * voxels are half-open boxes and a line lying on a voxel boundary belongs to the voxel on
    the + side, placed as exact arithmetic places it (as for the 2-D fan beam): a view cosine
    or sine within 1e-12 of zero is exactly zero, a direction component within 1e-12 of zero
    is zero and the line moves to the centre of the voxel slab holding the source (an origin
    within 1e-9 voxel of a slab boundary lies on it).

3-D Haar (config 5 names a "3-level 3D Haar" transform): orthonormal and separable, in a
3-D Mallat layout. At level l (1..L), with m = n >> l and mz = nz >> l, node (l, k, i, j)
covers the voxel block z in [k 2^l, (k+1) 2^l), y in [i 2^l, ...), x in [j 2^l, ...). Its
seven details t = (tz, ty, tx) in {0,1}^3 minus (0,0,0) sit at [k + tz mz][i + ty m][j + tx m]
and have the basis function 2^(-3l/2) prod over the axes with t_a = 1 of (+1 on the lower
half of the block, -1 on the upper half). The approximation of root (k, i, j) sits at
[k][i][j] (k < nz >> L, i, j < n >> L), basis 2^(-3L/2) on the root block. A node is split
when its seven details are active (tree masks use the same layout).
"""
import numpy as np
import scipy.sparse as sp

from . import haar, wam
from .geometry import axis_cos_sin, snap_axis_parallel

DETAILS = [(tz, ty, tx) for tz in (0, 1) for ty in (0, 1) for tx in (0, 1) if (tz, ty, tx) != (0, 0, 0)]


# ------------------------------------------------------------------ geometry

def rays3(g, views=None, ids=None):
    """(origin [M,3], unit direction [M,3]) of the cone-beam rays of the selected views, or
    of the rays with the given indices y = (v n_rows + rr) n_cols + cc."""
    if ids is not None:
        ids = np.asarray(ids, np.int64)
        v, rr, cc = ids // (g.n_rows * g.n_cols), (ids // g.n_cols) % g.n_rows, ids % g.n_cols
        A = g.angle0 + v * (g.angle_span / g.n_views)
        W = (rr - (g.n_rows - 1) / 2.0) * g.row_pitch
        U = (cc - (g.n_cols - 1) / 2.0) * g.col_pitch
    else:
        ang = g.angle0 + np.arange(g.n_views, dtype=np.float64) * (g.angle_span / g.n_views)
        if views is not None:
            ang = ang[np.asarray(views)]
        u = (np.arange(g.n_cols) - (g.n_cols - 1) / 2.0) * g.col_pitch
        w = (np.arange(g.n_rows) - (g.n_rows - 1) / 2.0) * g.row_pitch
        A, W, U = np.meshgrid(ang, w, u, indexing="ij")
        A, W, U = A.ravel(), W.ravel(), U.ravel()
    ca, sa = axis_cos_sin(A)
    src = np.stack([g.sod * ca, g.sod * sa, np.zeros_like(A)], axis=1)
    det = np.stack([-(g.sdd - g.sod) * ca - U * sa, -(g.sdd - g.sod) * sa + U * ca, W], axis=1)
    d = det - src
    return snap_axis_parallel(src, d / np.linalg.norm(d, axis=1, keepdims=True), [g.n, g.n, g.nz], g.pixel)


def edges3(g):
    """Boundary coordinates along x (= y) and z."""
    exy = (np.arange(g.n + 1, dtype=np.float64) - g.n / 2.0) * g.pixel
    ez = (np.arange(g.nz + 1, dtype=np.float64) - g.nz / 2.0) * g.pixel
    return exy, ez


def _slab(o, e, lo, hi):
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (lo - o) / e
        t1 = (hi - o) / e
    tmin, tmax = np.minimum(t0, t1), np.maximum(t0, t1)
    par = e == 0.0
    inside = (o >= lo) & (o < hi)
    tmin = np.where(par, np.where(inside, -np.inf, np.inf), tmin)
    tmax = np.where(par, np.where(inside, np.inf, -np.inf), tmax)
    return tmin, tmax


def box_chord3(o, e, lo, hi):
    """Length of each line o + t e inside the box [lo, hi) (3-vectors; broadcasting)."""
    a0, b0 = _slab(o[..., 0], e[..., 0], lo[..., 0], hi[..., 0])
    a1, b1 = _slab(o[..., 1], e[..., 1], lo[..., 1], hi[..., 1])
    a2, b2 = _slab(o[..., 2], e[..., 2], lo[..., 2], hi[..., 2])
    t0 = np.maximum(np.maximum(a0, a1), a2)
    t1 = np.minimum(np.minimum(b0, b1), b2)
    return np.where(t1 > t0, t1 - t0, 0.0)


def trace3(g, o, e):
    """Siddon in 3-D for a batch of rays: every crossing with a voxel boundary plane inside
    the volume, sorted; each gap goes to the voxel holding its midpoint.
    Returns (ray index, voxel index s n^2 + r n + c, length)."""
    exy, ez = edges3(g)
    lo = np.array([exy[0], exy[0], ez[0]])
    hi = np.array([exy[-1], exy[-1], ez[-1]])
    tin = np.full(o.shape[0], -np.inf)
    tout = np.full(o.shape[0], np.inf)
    for a in range(3):
        a0, b0 = _slab(o[:, a], e[:, a], lo[a], hi[a])
        tin, tout = np.maximum(tin, a0), np.minimum(tout, b0)
    hit = tout > tin
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = (exy[None, :] - o[:, 0:1]) / e[:, 0:1]
        ty = (exy[None, :] - o[:, 1:2]) / e[:, 1:2]
        tz = (ez[None, :] - o[:, 2:3]) / e[:, 2:3]
    t = np.concatenate([tx, ty, tz, tin[:, None], tout[:, None]], axis=1)
    t = np.where(np.isfinite(t), t, tout[:, None])
    t = np.clip(t, tin[:, None], tout[:, None])
    t[~hit] = 0.0
    t.sort(axis=1)
    seg = np.diff(t, axis=1)
    mid = 0.5 * (t[:, 1:] + t[:, :-1])
    with np.errstate(invalid="ignore"):
        pts = [o[:, a:a + 1] + mid * e[:, a:a + 1] for a in range(3)]
    c = np.searchsorted(exy, np.nan_to_num(pts[0], nan=-np.inf), side="right") - 1
    r = np.searchsorted(exy, np.nan_to_num(pts[1], nan=-np.inf), side="right") - 1
    s = np.searchsorted(ez, np.nan_to_num(pts[2], nan=-np.inf), side="right") - 1
    n, nz = g.n, g.nz
    keep = (seg > 0) & hit[:, None] & (c >= 0) & (c < n) & (r >= 0) & (r < n) & (s >= 0) & (s < nz)
    ray_idx = np.broadcast_to(np.arange(o.shape[0])[:, None], seg.shape)[keep]
    return ray_idx, ((s * n + r) * n + c)[keep], seg[keep]


def project_rays3(g, vol, ids, rays_per_batch=256):
    """Line integrals of the volume `vol` [nz, n, n] along the rays with the given indices
    (one row of H each, traced as in `trace3`)."""
    o, e = rays3(g, ids=ids)
    flat = np.asarray(vol, np.float64).ravel()
    out = np.zeros(o.shape[0])
    for s0 in range(0, o.shape[0], rays_per_batch):
        ri, vi, li = trace3(g, o[s0:s0 + rays_per_batch], e[s0:s0 + rays_per_batch])
        out[s0:s0 + rays_per_batch] = np.bincount(ri, weights=flat[vi] * li, minlength=min(rays_per_batch, o.shape[0] - s0))
    return out


def project_coef_rays3(g, coef, levels, ids, rays_per_batch=256):
    """Line integrals of the volume Omega coef along the rays with the given indices, with the
    volume synthesised only at the voxels those rays cross (rows of Omega)."""
    o, e = rays3(g, ids=ids)
    flat = np.asarray(coef, np.float64).ravel()
    out = np.zeros(o.shape[0])
    for s0 in range(0, o.shape[0], rays_per_batch):
        ri, vi, li = trace3(g, o[s0:s0 + rays_per_batch], e[s0:s0 + rays_per_batch])
        uv, inv = np.unique(vi, return_inverse=True)
        mu = synthesis_matrix3(g.n, g.nz, levels, voxels=uv) @ flat
        out[s0:s0 + rays_per_batch] = np.bincount(ri, weights=mu[inv] * li, minlength=min(rays_per_batch, o.shape[0] - s0))
    return out


def box_shadow3(g, lo, hi, margin=1):
    """Indices of the rays that can meet the box [lo, hi): in each view, the detector
    elements inside the bounding rectangle of the central projections of the box's eight
    corners, widened by `margin` elements (a superset: a ray through the box meets the
    detector inside the convex hull of those projections). The box must lie on the
    detector's side of the source plane."""
    ang = g.angle0 + np.arange(g.n_views, dtype=np.float64) * (g.angle_span / g.n_views)
    ca, sa = np.cos(ang)[:, None], np.sin(ang)[:, None]
    cx = np.array([lo[0], hi[0]])[[0, 1, 0, 1, 0, 1, 0, 1]][None, :]
    cy = np.array([lo[1], hi[1]])[[0, 0, 1, 1, 0, 0, 1, 1]][None, :]
    cz = np.array([lo[2], hi[2]])[[0, 0, 0, 0, 1, 1, 1, 1]][None, :]
    depth = g.sod - (cx * ca + cy * sa)             # distance from the source plane
    if np.any(depth <= 0):
        raise ValueError("box reaches behind the source")
    t = g.sdd / depth
    u = t * (-cx * sa + cy * ca)
    w = t * cz
    c0 = np.floor(u.min(1) / g.col_pitch + (g.n_cols - 1) / 2.0).astype(np.int64) - margin
    c1 = np.ceil(u.max(1) / g.col_pitch + (g.n_cols - 1) / 2.0).astype(np.int64) + margin
    r0 = np.floor(w.min(1) / g.row_pitch + (g.n_rows - 1) / 2.0).astype(np.int64) - margin
    r1 = np.ceil(w.max(1) / g.row_pitch + (g.n_rows - 1) / 2.0).astype(np.int64) + margin
    out = []
    for v in range(g.n_views):
        cols = np.arange(max(c0[v], 0), min(c1[v], g.n_cols - 1) + 1)
        rows = np.arange(max(r0[v], 0), min(r1[v], g.n_rows - 1) + 1)
        if cols.size and rows.size:
            out.append(((v * g.n_rows + rows[:, None]) * g.n_cols + cols[None, :]).ravel())
    return np.concatenate(out) if out else np.zeros(0, np.int64)


def node_phi3(g, o, e, lev, k, i, j):
    """Projections along the rays (o, e) of the basis functions of node (lev, k, i, j), from
    the chords of the node's eight octant boxes by direct clipping: a dict from each detail's
    position (z, y, x) in the Mallat layout to its phi, plus the key 'approx' for the
    2^(-3 lev / 2)-scaled block sum (a coefficient of the basis when lev is the coarsest level)."""
    exy, ez = edges3(g)
    s, h = 1 << lev, 1 << (lev - 1)
    ch = {}
    for bz in (0, 1):
        for by in (0, 1):
            for bx in (0, 1):
                lo = np.array([exy[j * s + bx * h], exy[i * s + by * h], ez[k * s + bz * h]])
                hi = np.array([exy[j * s + (bx + 1) * h], exy[i * s + (by + 1) * h], ez[k * s + (bz + 1) * h]])
                ch[bz, by, bx] = box_chord3(o, e, lo, hi)
    sc = 2.0 ** (-1.5 * lev)
    m, mz = g.n >> lev, g.nz >> lev
    out = {"approx": sum(ch.values()) * sc}
    for tz, ty, tx in DETAILS:
        acc = 0.0
        for (bz, by, bx), c in ch.items():
            sgn = (-1.0 if (tz and bz) else 1.0) * (-1.0 if (ty and by) else 1.0) * (-1.0 if (tx and bx) else 1.0)
            acc = acc + sgn * c
        out[k + tz * mz, i + ty * m, j + tx * m] = acc * sc
    return out


def system_matrix3(g, views=None, rays_per_batch=2048):
    """H (rays x voxels, CSR) of the cone-beam scan."""
    o, e = rays3(g, views)
    rows, cols, vals = [], [], []
    for s0 in range(0, o.shape[0], rays_per_batch):
        ri, vi, li = trace3(g, o[s0:s0 + rays_per_batch], e[s0:s0 + rays_per_batch])
        rows.append(ri + s0)
        cols.append(vi)
        vals.append(li)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(o.shape[0], g.n * g.n * g.nz))
    H.sum_duplicates()
    return H


# ------------------------------------------------------------------ 3-D Haar

def synthesis_matrix3(n, nz, levels, voxels=None):
    """Omega (voxels x coefficients, CSR), built voxel by voxel: voxel (s, r, c) receives
    2^(-3L/2) from its root's approximation and 2^(-3l/2) sign_t from detail t of the level-l
    node containing it. With `voxels` (flat indices (s n + r) n + c), only those rows, in
    that order."""
    if n % (1 << levels) or nz % (1 << levels):
        raise ValueError("volume sides must be divisible by 2^levels")
    if voxels is None:
        s, r, c = np.meshgrid(np.arange(nz), np.arange(n), np.arange(n), indexing="ij")
        s, r, c = s.ravel(), r.ravel(), c.ravel()
    else:
        flat = np.asarray(voxels, np.int64)
        s, r, c = flat // (n * n), (flat // n) % n, flat % n
    vox = np.arange(s.size)
    L = levels

    def at(z, y, x):
        return (z * n + y) * n + x

    rows = [vox]
    cols = [at(s >> L, r >> L, c >> L)]
    vals = [np.full(vox.size, 2.0 ** (-1.5 * L))]
    for lev in range(1, L + 1):
        m, mz = n >> lev, nz >> lev
        k, i, j = s >> lev, r >> lev, c >> lev
        upper = [(s >> (lev - 1)) & 1, (r >> (lev - 1)) & 1, (c >> (lev - 1)) & 1]
        for tz, ty, tx in DETAILS:
            sign = np.ones(vox.size)
            for t, up in zip((tz, ty, tx), upper):
                if t:
                    sign = sign * np.where(up, -1.0, 1.0)
            rows.append(vox)
            cols.append(at(k + tz * mz, i + ty * m, j + tx * m))
            vals.append(sign * 2.0 ** (-1.5 * lev))
    N = n * n * nz
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(s.size, N))


def cascade_analysis3(vol, levels):
    """Textbook recursive 2x2x2 Haar analysis (independent of `synthesis_matrix3`)."""
    a = np.array(vol, np.float64)
    nz, n = a.shape[0], a.shape[1]
    out = np.zeros_like(a)
    for lev in range(1, levels + 1):
        m, mz = n >> lev, nz >> lev
        sub = {(bz, by, bx): a[bz::2, by::2, bx::2] for bz in (0, 1) for by in (0, 1) for bx in (0, 1)}
        for tz, ty, tx in DETAILS:
            acc = np.zeros((mz, m, m))
            for (bz, by, bx), v in sub.items():
                sgn = (-1.0 if (tz and bz) else 1.0) * (-1.0 if (ty and by) else 1.0) * (-1.0 if (tx and bx) else 1.0)
                acc += sgn * v
            out[tz * mz:tz * mz + mz, ty * m:ty * m + m, tx * m:tx * m + m] = acc / (2.0 * np.sqrt(2.0))
        a = sum(sub.values()) / (2.0 * np.sqrt(2.0))
    out[:a.shape[0], :a.shape[1], :a.shape[2]] = a
    return out


def cascade_synthesis3(coef, levels):
    """Textbook recursive 2x2x2 Haar synthesis, the inverse of `cascade_analysis3`: from the
    coarsest level down, each approximation and its seven details give the eight children
    v(bz, by, bx) = sum over t of sign_t(b) c_t / (2 sqrt 2)."""
    c = np.array(coef, np.float64)
    nz, n = c.shape[0], c.shape[1]
    a = c[:nz >> levels, :n >> levels, :n >> levels].copy()
    for lev in range(levels, 0, -1):
        m, mz = n >> lev, nz >> lev
        det = {t: c[t[0] * mz:t[0] * mz + mz, t[1] * m:t[1] * m + m, t[2] * m:t[2] * m + m] for t in DETAILS}
        out = np.empty((2 * mz, 2 * m, 2 * m))
        for bz in (0, 1):
            for by in (0, 1):
                for bx in (0, 1):
                    acc = a.copy()
                    for (tz, ty, tx), dv in det.items():
                        sgn = (-1.0 if (tz and bz) else 1.0) * (-1.0 if (ty and by) else 1.0) * (-1.0 if (tx and bx) else 1.0)
                        acc += sgn * dv
                    out[bz::2, by::2, bx::2] = acc / (2.0 * np.sqrt(2.0))
        a = out
    return a


# ------------------------------------------------------------------ octree masks

def approx_mask3(n, nz, levels):
    m = np.zeros((nz, n, n), np.uint8)
    m[:nz >> levels, :n >> levels, :n >> levels] = 1
    return m


def split_flags3(mask, lev):
    nz, n = mask.shape[0], mask.shape[1]
    m, mz = n >> lev, nz >> lev
    return mask[:mz, :m, m:2 * m].astype(bool)


def set_split3(mask, lev, flags):
    nz, n = mask.shape[0], mask.shape[1]
    m, mz = n >> lev, nz >> lev
    f = flags.astype(np.uint8)
    for tz, ty, tx in DETAILS:
        mask[tz * mz:tz * mz + mz, ty * m:ty * m + m, tx * m:tx * m + m] = f


def valid_mask3(mask, levels):
    nz, n = mask.shape[0], mask.shape[1]
    if not mask[:nz >> levels, :n >> levels, :n >> levels].all():
        return False
    for lev in range(1, levels + 1):
        m, mz = n >> lev, nz >> lev
        f = split_flags3(mask, lev)
        for tz, ty, tx in DETAILS:
            if not np.array_equal(mask[tz * mz:tz * mz + mz, ty * m:ty * m + m, tx * m:tx * m + m].astype(bool), f):
                return False
        if lev < levels:
            p = split_flags3(mask, lev + 1)
            parent = p.repeat(2, 0).repeat(2, 1).repeat(2, 2)
            if (f & ~parent).any():
                return False
    return True


def expand_tree3(beta, mask, levels, frac, Omega):
    """Tree rule of the Results section on the 3-D image: mu = Omega beta, thr = frac *
    max(mu) (nothing if max <= 0); every leaf (a node at level >= 1 not split whose parent
    is split, or a root) with a voxel above thr (strict) splits once. Decisions on the old
    tree. Returns (new mask, number of split nodes)."""
    nz, n = mask.shape[0], mask.shape[1]
    mu = (Omega @ np.asarray(beta, np.float64).ravel()).reshape(nz, n, n)
    top = mu.max()
    new = mask.copy()
    if top <= 0:
        return new, 0
    thr = frac * top
    count = 0
    for lev in range(1, levels + 1):
        m, mz, s = n >> lev, nz >> lev, 1 << lev
        split = split_flags3(mask, lev)
        if lev == levels:
            parent = np.ones((mz, m, m), bool)
        else:
            parent = split_flags3(mask, lev + 1).repeat(2, 0).repeat(2, 1).repeat(2, 2)
        leaf = ~split & parent
        bmax = mu.reshape(mz, s, m, s, m, s).max(axis=(1, 3, 5))
        grow = leaf & (bmax > thr)
        count += int(grow.sum())
        set_split3(new, lev, split | grow)
    return new, count


def expand_tree3_gradient(beta, mask, levels, frac, Omega, H, d, i0):
    """Residual-gradient rule on the octree (oracle.wam.expand_tree_gradient in 3-D): c =
    Omega^T H^T (d - q-hat) at the current beta; a leaf scores max |c| over its node's seven
    details; leaves scoring above frac x the largest score split once (nothing if all are 0).
    Returns (new mask, number of nodes split)."""
    nz, n = mask.shape[0], mask.shape[1]
    q = wam.beer_mean(i0, H @ (Omega @ np.asarray(beta, np.float64).ravel()))
    c = (Omega.T @ (H.T @ (np.asarray(d, np.float64) - q))).reshape(nz, n, n)
    scores, leaves = {}, {}
    for lev in range(1, levels + 1):
        m, mz = n >> lev, nz >> lev
        split = split_flags3(mask, lev)
        if lev == levels:
            parent = np.ones((mz, m, m), bool)
        else:
            parent = split_flags3(mask, lev + 1).repeat(2, 0).repeat(2, 1).repeat(2, 2)
        leaves[lev] = ~split & parent
        det = np.stack([np.abs(c[tz * mz:tz * mz + mz, ty * m:ty * m + m, tx * m:tx * m + m])
                        for tz, ty, tx in DETAILS])
        scores[lev] = np.where(leaves[lev], det.max(axis=0), 0.0)
    top = max((s_.max() for s_ in scores.values()), default=0.0)
    new = mask.copy()
    if not top > 0:
        return new, 0
    thr = frac * top
    count = 0
    for lev in range(1, levels + 1):
        grow = leaves[lev] & (scores[lev] > thr)
        count += int(grow.sum())
        set_split3(new, lev, split_flags3(mask, lev) | grow)
    return new, count


# ------------------------------------------------------------------ Algorithm 1 in 3-D

def wam_solve3(H, n, nz, levels, d, i0, n_iters, pixel, schedule=(), frac=0.1, Omega=None, beta0=None,
               mask0=None, rule="value"):
    """Algorithm 1 with the octree rule on a 3-D volume (same steps as wam.wam_solve: eq. 1.6
    b for every coefficient, eq. 1.61 Z0 per tree, eq. 1.10 sign split, eq. 1.9 zero)."""
    if Omega is None:
        Omega = synthesis_matrix3(n, nz, levels)
    d = np.asarray(d, np.float64)
    N = n * n * nz
    beta = np.zeros(N) if beta0 is None else np.array(beta0, np.float64).ravel()
    mask = approx_mask3(n, nz, levels) if mask0 is None else np.array(mask0, np.uint8)
    b_all = Omega.T @ (H.T @ d)
    trace, trees, z0s, held_total = [], [], [], 0
    Phi = None
    for j in range(n_iters):
        changed = False
        if j in schedule:
            if rule == "gradient":
                mask, _ = expand_tree3_gradient(beta, mask, levels, frac, Omega, H, d, i0)
            else:
                mask, _ = expand_tree3(beta, mask, levels, frac, Omega)
            changed = True
        if Phi is None or changed:
            Phi, act = wam.phi_matrix(H, Omega, mask, pixel)
            Php, Phm = wam.split_phi(Phi)
            z0 = wam.z0_of(Phi)
            trees.append((j, mask.copy()))
            z0s.append(z0)
        q_hat = wam.beer_mean(i0, Phi @ beta[act])
        trace.append(wam.idiv(d, q_hat))
        delta, held = wam.closed_form_update(b_all[act], Php.T @ q_hat, Phm.T @ q_hat, z0)
        held_total += int(held.sum())
        beta[act] += delta
    trace.append(wam.idiv(d, wam.beer_mean(i0, H @ (Omega @ beta))))
    return dict(beta=beta.reshape(nz, n, n), mu=(Omega @ beta).reshape(nz, n, n), idiv=np.array(trace),
                trees=trees, z0=z0s, held=held_total, mask=mask, b=b_all.reshape(nz, n, n))


# ------------------------------------------------------------------ 2-D Haar per z-slice

# The Results section represents its volumes slice by slice: "each z-slice" carries a
# Level-3 2-D Haar transform, and one tree serves the whole volume, grown where the image
# summed over the slices exceeds 0.1 of its maximum. Coefficients of slice s sit in the 2-D
# Mallat layout of haar.py at [s][y][x]; node (l, s, i, j) covers the voxels [i 2^l,
# (i+1) 2^l) x [j 2^l, (j+1) 2^l) of slice s (one voxel deep).

def slice_synthesis_matrix3(n, nz, levels):
    """Omega of the per-slice representation: block diagonal, the 2-D synthesis matrix of
    haar.py once per slice (voxel (s, r, c) and coefficient (s, y, x) both at (s n + .) n + .)."""
    return sp.kron(sp.identity(nz, format="csr"), haar.synthesis_matrix(n, levels), format="csr")


def slice_mask3(mask2d, nz):
    """The volume's mask: the one 2-D tree in every slice."""
    return np.repeat(np.asarray(mask2d, np.uint8)[None], nz, axis=0)


def expand_tree_slices3(beta, mask2d, levels, frac, Omega2d):
    """Tree rule of the Results section for slices sharing one tree: the synthesized images of
    the slices summed over z (= Omega2d applied to the summed coefficients), thr = frac x the
    summed image's maximum, and every leaf of the shared tree with a pixel of the summed
    image above thr (strict) splits once (nothing when the maximum is <= 0). beta: [nz, n, n].
    Returns (new 2-D mask, nodes split)."""
    summed = np.asarray(beta, np.float64).sum(axis=0)
    return wam.expand_tree(summed, mask2d, levels, frac, Omega2d)


def slice_wam_solve3(H, n, nz, levels, d, i0, n_iters, pixel, schedule=(), frac=0.1, beta0=None, mask0=None,
                     masks=None):
    """Algorithm 1 on a cone-beam volume whose slices carry 2-D Haar transforms sharing one
    tree (same steps as wam_solve3: b for every coefficient (eq. 1.6), Z0 (eq. 1.61) per tree,
    the sign split of eq. 1.10 and the zero of eq. 1.9 for every active coefficient; the tree
    rule of expand_tree_slices3 before each scheduled update). masks: optional {j: 2-D mask}
    giving the shared tree before update j (overrides the rule there). mask0 is a 2-D mask.
    Returns beta [nz, n, n], mu, the I-divergence trace (n_iters + 1), the trees (j, 2-D mask),
    Z0 and W = nnz(Phi) per tree, the held count and the final 2-D mask."""
    O2 = haar.synthesis_matrix(n, levels)
    Omega = slice_synthesis_matrix3(n, nz, levels)
    d = np.asarray(d, np.float64)
    N = n * n * nz
    beta = np.zeros(N) if beta0 is None else np.array(beta0, np.float64).ravel()
    mask2 = haar.approx_mask(n, levels) if mask0 is None else np.array(mask0, np.uint8)
    masks = masks or {}
    b_all = Omega.T @ (H.T @ d)
    trace, trees, z0s, ws, held_total = [], [], [], [], 0
    Phi = None
    for j in range(n_iters):
        changed = False
        if j in masks:
            mask2 = np.array(masks[j], np.uint8)
            changed = True
        elif j in schedule:
            mask2, _ = expand_tree_slices3(beta.reshape(nz, n, n), mask2, levels, frac, O2)
            changed = True
        if Phi is None or changed:
            Phi, act = wam.phi_matrix(H, Omega, slice_mask3(mask2, nz), pixel)
            Php, Phm = wam.split_phi(Phi)
            z0 = wam.z0_of(Phi)
            trees.append((j, mask2.copy()))
            z0s.append(z0)
            ws.append(int(Phi.nnz))
        q_hat = wam.beer_mean(i0, Phi @ beta[act])
        trace.append(wam.idiv(d, q_hat))
        delta, held = wam.closed_form_update(b_all[act], Php.T @ q_hat, Phm.T @ q_hat, z0)
        held_total += int(held.sum())
        beta[act] += delta
    trace.append(wam.idiv(d, wam.beer_mean(i0, H @ (Omega @ beta))))
    return dict(beta=beta.reshape(nz, n, n), mu=(Omega @ beta).reshape(nz, n, n), idiv=np.array(trace),
                trees=trees, z0=z0s, w=ws, held=held_total, mask=mask2, b=b_all.reshape(nz, n, n))


def slice_node_phi3(g, o, e, lev, s, i, j):
    """Projections along the rays (o, e) of the three detail basis functions of the per-slice
    node (lev, s, i, j), from box clipping of its four quadrants (one voxel deep in slice s):
    [D1, D2, D3] with D1 = 2^-lev (TL - TR + BL - BR), D2 = 2^-lev (TL + TR - BL - BR),
    D3 = 2^-lev (TL - TR - BL + BR) over the quadrant chords (T = smaller y index, L = smaller x)."""
    exy, ez = edges3(g)
    h = 1 << (lev - 1)
    q = {}
    for by in (0, 1):
        for bx in (0, 1):
            x0, y0 = (2 * j + bx) * h, (2 * i + by) * h
            lo = np.array([exy[x0], exy[y0], ez[s]])
            hi = np.array([exy[x0 + h], exy[y0 + h], ez[s + 1]])
            q[(by, bx)] = box_chord3(o, e, lo, hi)
    tl, tr, bl, br = q[(0, 0)], q[(0, 1)], q[(1, 0)], q[(1, 1)]
    sc = 2.0 ** -lev
    return [sc * (tl - tr + bl - br), sc * (tl + tr - bl - br), sc * (tl - tr - bl + br)]
