"""Rays of a 2-D scan, FP64 (test infrastructure; see oracle/__init__.py).

The paper states no scan geometry (its data come from a baggage scanner whose geometry
is not given), so the conventions below are this project's reading:
  * view v at angle a = angle0 + v * angle_span / n_views;
  * bin b at detector coordinate u = (b - (n_bins - 1) / 2) * bin_pitch;
  * parallel beam: the line x cos a + y sin a = u, direction (-sin a, cos a);
  * fan beam with a flat detector: source at sod * (cos a, sin a), detector centre at
    -(sdd - sod) * (cos a, sin a), detector axis (-sin a, cos a); the ray joins the
    source to the bin centre;
  * pixels are half-open boxes, and a line lying on a pixel boundary belongs to the pixel
    on the + side. Positions are placed as exact arithmetic places them, not as the
    rounding of cos, sin and their products would: a view cosine or sine within 1e-12 of
    zero is exactly zero (angle0 + v * angle_span / n_views is then a multiple of pi/2,
    whose source or foot point lies on an axis), a direction component within 1e-12 of
    zero is exactly zero (the line is axis-parallel), and the origin coordinate of an
    axis-parallel line within 1e-9 pixel of a pixel boundary lies on that boundary. Such a
    line is moved, parallel to the axis, to the centre of the pixel row (column) holding
    the ray's origin (the source of a fan-beam ray, the foot point u (cos a, sin a) of a
    parallel-beam ray), which keeps every chord and never splits one by a 1e-16 tilt.
Ray index y = v * n_bins + b. Every geometry attribute is read by name from `g`.
"""
import numpy as np


def view_angles(g):
    return g.angle0 + np.arange(g.n_views, dtype=np.float64) * (g.angle_span / g.n_views)


def bin_offsets(g):
    return (np.arange(g.n_bins, dtype=np.float64) - (g.n_bins - 1) / 2.0) * g.bin_pitch


def axis_cos_sin(ang):
    """(cos a, sin a) with values within 1e-12 of zero set to exactly zero (their partner is
    then exactly +-1): an angle that is a multiple of pi/2 in exact arithmetic puts the
    source on an axis, which the rounding of cos and sin (about 1e-16) would not."""
    c, s = np.cos(ang), np.sin(ang)
    cz, sz = np.abs(c) < 1e-12, np.abs(s) < 1e-12
    c = np.where(cz, 0.0, np.where(sz, np.sign(c), c))
    s = np.where(sz, 0.0, np.where(cz, np.sign(s), s))
    return c, s


def rays(g, views=None):
    """(origin [M,2], unit direction [M,2]) for the selected views (default: all)."""
    ang = view_angles(g)
    if views is not None:
        ang = ang[np.asarray(views)]
    u = bin_offsets(g)
    nv, nb = ang.size, u.size
    ca, sa = axis_cos_sin(ang)
    cos_a = np.repeat(ca, nb)
    sin_a = np.repeat(sa, nb)
    uu = np.tile(u, nv)
    if g.kind == 0:      # parallel
        origin = np.stack([uu * cos_a, uu * sin_a], axis=1)
        direction = np.stack([-sin_a, cos_a], axis=1)
    elif g.kind == 1:    # fan, flat detector
        src = g.sod * np.stack([cos_a, sin_a], axis=1)
        det = (-(g.sdd - g.sod)) * np.stack([cos_a, sin_a], axis=1) \
            + uu[:, None] * np.stack([-sin_a, cos_a], axis=1)
        v = det - src
        direction = v / np.linalg.norm(v, axis=1, keepdims=True)
        origin = src
    else:
        raise ValueError("geometry kind must be 0 (parallel) or 1 (fan)")
    return snap_axis_parallel(origin, direction, [g.n, g.n], g.pixel)


def snap_axis_parallel(origin, direction, sizes, pixel, tol=1e-12, edge_tol=1e-9):
    """Rays with a direction component below `tol` in magnitude: that component set to 0 and
    the origin moved along that axis to the centre of the pixel slab that holds it (grid of
    `sizes` pixels per axis, centred at 0); an origin within `edge_tol` pixel of a slab
    boundary is on it, so the slab is the one on the + side."""
    o = np.array(origin, dtype=np.float64)
    e = np.array(direction, dtype=np.float64)
    for a, n in enumerate(sizes):
        m = np.abs(e[:, a]) < tol
        if m.any():
            f = o[m, a] / pixel + 0.5 * n
            r = np.round(f)
            f = np.where(np.abs(f - r) <= edge_tol, r, f)
            o[m, a] = (np.floor(f) + 0.5 - 0.5 * n) * pixel
            e[m, a] = 0.0
    return o, e


def pixel_edges(g):
    """x (equally y) coordinates of the n+1 pixel boundaries, image centred at 0."""
    return (np.arange(g.n + 1, dtype=np.float64) - g.n / 2.0) * g.pixel
