"""System matrix H of the Beer's-law model, FP64 (test infrastructure; see oracle/__init__.py).

h(y|x) is the length of the intersection of ray y with pixel x (Introduction: the
definition of q(mu)(y) = I0(y) exp(-sum_x h(y|x) mu(x))). Two independent routes:

  * `system_matrix`: plane-crossing ray tracing (Siddon, 1985). For each ray take the
    parameters t of every crossing with a pixel boundary line inside the image square,
    sort them, and assign each gap [t_k, t_k+1] (length t_k+1 - t_k, since directions are
    unit vectors) to the pixel that contains its midpoint.
  * `box_chord` / `dense_matrix`: the chord of the ray through one axis-aligned box by
    slab clipping, evaluated for every (ray, pixel) pair; only for tiny grids, as a check.

A ray lying exactly on a pixel boundary line belongs to the pixel on the + side of that
line in both routes (half-open boxes [x0, x1) x [y0, y1)).
"""
import numpy as np
import scipy.sparse as sp

from .geometry import rays, pixel_edges


def _slab(o, e, lo, hi):
    """Parameter interval of the line o + t e inside lo <= coordinate < hi (one axis)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (lo - o) / e
        t1 = (hi - o) / e
    tmin = np.minimum(t0, t1)
    tmax = np.maximum(t0, t1)
    par = e == 0.0
    inside = (o >= lo) & (o < hi)
    tmin = np.where(par, np.where(inside, -np.inf, np.inf), tmin)
    tmax = np.where(par, np.where(inside, np.inf, -np.inf), tmax)
    return tmin, tmax


def box_chord(origin, direction, x0, x1, y0, y1):
    """Length of each ray inside the box [x0,x1) x [y0,y1) (broadcasting over inputs)."""
    ox, oy = origin[..., 0], origin[..., 1]
    ex, ey = direction[..., 0], direction[..., 1]
    ax, bx = _slab(ox, ex, x0, x1)
    ay, by = _slab(oy, ey, y0, y1)
    lo = np.maximum(ax, ay)
    hi = np.minimum(bx, by)
    return np.where(hi > lo, hi - lo, 0.0)


def dense_matrix(g, origin=None, direction=None):
    """Brute-force H (M x n*n) by clipping every ray against every pixel box."""
    if origin is None:
        origin, direction = rays(g)
    edges = pixel_edges(g)
    n = g.n
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x0 = edges[c.ravel()]
    x1 = edges[c.ravel() + 1]
    y0 = edges[r.ravel()]
    y1 = edges[r.ravel() + 1]
    return box_chord(origin[:, None, :], direction[:, None, :], x0[None], x1[None], y0[None], y1[None])


def trace(g, origin, direction):
    """Siddon ray tracing for a batch of rays -> (ray_index, pixel_index, length) arrays."""
    n = g.n
    edges = pixel_edges(g)
    ox, oy = origin[:, 0], origin[:, 1]
    ex, ey = direction[:, 0], direction[:, 1]
    # interval of each ray inside the image square
    ax, bx = _slab(ox, ex, edges[0], edges[-1])
    ay, by = _slab(oy, ey, edges[0], edges[-1])
    t_in = np.maximum(ax, ay)
    t_out = np.minimum(bx, by)
    hit = t_out > t_in
    # crossings with every vertical and horizontal boundary line
    with np.errstate(divide="ignore", invalid="ignore"):
        tx = (edges[None, :] - ox[:, None]) / ex[:, None]
        ty = (edges[None, :] - oy[:, None]) / ey[:, None]
    t = np.concatenate([tx, ty, t_in[:, None], t_out[:, None]], axis=1)
    t = np.where(np.isfinite(t), t, t_out[:, None])
    t = np.clip(t, t_in[:, None], t_out[:, None])
    t[~hit] = 0.0
    t.sort(axis=1)
    seg = np.diff(t, axis=1)
    mid = 0.5 * (t[:, 1:] + t[:, :-1])
    with np.errstate(invalid="ignore"):
        xm = ox[:, None] + mid * ex[:, None]
        ym = oy[:, None] + mid * ey[:, None]
    # half-open pixels [edge_k, edge_k+1): locate midpoints by comparison with the edges
    col = np.searchsorted(edges, np.nan_to_num(xm, nan=-np.inf), side="right") - 1
    row = np.searchsorted(edges, np.nan_to_num(ym, nan=-np.inf), side="right") - 1
    keep = (seg > 0) & hit[:, None] & (col >= 0) & (col < n) & (row >= 0) & (row < n)
    ray_idx = np.broadcast_to(np.arange(origin.shape[0])[:, None], seg.shape)[keep]
    return ray_idx, (row * n + col)[keep], seg[keep]


def system_matrix(g, views=None, rays_per_batch=4096):
    """H as CSR (rows: rays of the selected views in order, columns: pixels r*n + c)."""
    origin, direction = rays(g, views)
    m = origin.shape[0]
    rows, cols, vals = [], [], []
    for s in range(0, m, rays_per_batch):
        ri, pi, li = trace(g, origin[s:s + rays_per_batch], direction[s:s + rays_per_batch])
        rows.append(ri + s)
        cols.append(pi)
        vals.append(li)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, g.n * g.n))
    H.sum_duplicates()
    return H


def project_rays(g, image, ray_ids):
    """p(y) = sum_x h(y|x) mu(x) for a few selected rays (global ray indices)."""
    origin, direction = rays(g)
    ri, pi, li = trace(g, origin[ray_ids], direction[ray_ids])
    out = np.zeros(len(ray_ids))
    np.add.at(out, ri, li * image.ravel()[pi])
    return out
