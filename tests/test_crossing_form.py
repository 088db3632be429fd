"""The gathers form a node's Haar detail projections without the chords of its quadrants or
octants: from the ray's parameter interval [lo, hi] inside the node box and its crossings c of
the box's mid-lines (mid-planes) clamped into that interval. With s the sign of the ray's
direction along an axis and the details + on the lower half of each axis they use,
  one axis:    s (2 c - lo - hi)
  two axes:    s s' (hi - lo - 2 |c - c'|)
  three axes:  s s' s'' (2 (c1 - c2 + c3) - lo - hi), c1 <= c2 <= c3 the sorted crossings,
the signed lengths of a product of half indicators along the ray. This pins that identity
(written out here, independently of the kernels) against the oracle's own phi: H Omega in 2-D
(rays clipped against every pixel, the Haar synthesis matrix) and the octant box clipping of
a 3-D node (vol3d.node_phi3), on random rays, axis-parallel ones among them (a zero direction
component gets the reciprocal +-1e300, as the kernels' ray factors do).
"""
import numpy as np

from oracle import haar, siddon, vol3d
from paper_1508_04458_amd import synth


def _inv(e):
    return np.where(e == 0.0, 1e300, 1.0 / np.where(e == 0.0, 1.0, e))


def _interval_and_crossings(o, e, lo_c, hi_c):
    """Per ray: [lo, hi] inside the box [lo_c, hi_c] (per axis) and the mid-plane crossings
    clamped into it; axes along the last dimension."""
    inv = _inv(e)
    t0 = (lo_c - o) * inv
    t2 = (hi_c - o) * inv
    t1 = (0.5 * (lo_c + hi_c) - o) * inv
    lo = np.max(np.minimum(t0, t2), axis=-1)
    hi = np.min(np.maximum(t0, t2), axis=-1)
    c = np.clip(t1, lo[..., None], np.maximum(hi, lo)[..., None])
    return lo, hi, c, np.where(inv < 0, -1.0, 1.0)


def _rays(dim, m, rng, radius):
    """Rays from a sphere (circle) of the given radius towards random points of the central
    region; every fourth ray has one direction component exactly zero."""
    o = rng.normal(size=(m, dim))
    o *= radius / np.linalg.norm(o, axis=1, keepdims=True)
    target = rng.uniform(-0.4, 0.4, size=(m, dim)) * radius
    e = target - o
    zero = rng.integers(0, dim, m)
    pick = np.arange(m) % 4 == 0
    e[pick, zero[pick]] = 0.0
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    return o, e


def test_crossing_form_2d_matches_h_omega():
    n, L = 16, 2
    g = synth.parallel_geometry(n, 4, 8)      # only n and the pixel size are used
    rng = np.random.default_rng(0)
    o, e = _rays(2, 3000, rng, 0.75 * n * g.pixel)
    H = siddon.dense_matrix(g, o, e)                                   # rays x pixels
    Omega = haar.synthesis_matrix(n, L).toarray()
    edges = (np.arange(n + 1) - 0.5 * n) * g.pixel
    checked = 0
    for lev in (1, 2):
        s, m = 1 << lev, n >> lev
        for i in range(m):
            for j in range(m):
                lo_c = np.array([edges[j * s], edges[i * s]])
                hi_c = np.array([edges[(j + 1) * s], edges[(i + 1) * s]])
                lo, hi, c, sg = _interval_and_crossings(o, e, lo_c, hi_c)
                box = np.maximum(hi - lo, 0.0)
                hit = box > 0
                cx, cy = c[:, 0], c[:, 1]
                det = {(i, m + j): sg[:, 0] * (2 * cx - lo - hi),
                       (m + i, j): sg[:, 1] * (2 * cy - lo - hi),
                       (m + i, m + j): sg[:, 0] * sg[:, 1] * (hi - lo - 2 * np.abs(cx - cy))}
                for (r, col), v in det.items():
                    ref = H @ Omega[:, r * n + col]
                    got = np.where(hit, v, 0.0) * 2.0 ** -lev
                    assert np.abs(got - ref).max() <= 1e-12 * n * g.pixel, (lev, i, j, r, col)
                    checked += int(np.count_nonzero(ref))
    assert checked > 1000


def test_crossing_form_3d_matches_octant_clipping():
    g = synth.cone_geometry(16, 8, 4, 4, 8)   # only n, nz and the voxel size are used
    rng = np.random.default_rng(1)
    o, e = _rays(3, 4000, rng, 0.75 * g.n * g.pixel)
    exy, ez = vol3d.edges3(g)
    checked = 0
    for lev, k, i, j in [(1, 1, 3, 4), (1, 2, 4, 3), (2, 0, 1, 2), (2, 1, 2, 1), (1, 3, 0, 7), (2, 1, 3, 3)]:
        s = 1 << lev
        m, mz = g.n >> lev, g.nz >> lev
        ref = vol3d.node_phi3(g, o, e, lev, k, i, j)
        lo_c = np.array([exy[j * s], exy[i * s], ez[k * s]])
        hi_c = np.array([exy[(j + 1) * s], exy[(i + 1) * s], ez[(k + 1) * s]])
        lo, hi, c, sg = _interval_and_crossings(o, e, lo_c, hi_c)
        box = np.maximum(hi - lo, 0.0)
        hit = box > 0
        cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
        sx, sy, sz = sg[:, 0], sg[:, 1], sg[:, 2]
        med = np.maximum(np.minimum(cx, cy), np.minimum(np.maximum(cx, cy), cz))
        lh = lo + hi
        one = {0: sx * (2 * cx - lh), 1: sy * (2 * cy - lh), 2: sz * (2 * cz - lh)}
        cc = (cx, cy, cz)
        sgn = (sx, sy, sz)
        sc = 2.0 ** (-1.5 * lev)
        assert np.abs(np.where(hit, box, 0.0) * sc - ref["approx"]).max() <= 1e-12 * g.n
        for tz, ty, tx in vol3d.DETAILS:
            axes = [a for a, t in ((0, tx), (1, ty), (2, tz)) if t]
            if len(axes) == 1:
                v = one[axes[0]]
            elif len(axes) == 2:
                a, b = axes
                v = sgn[a] * sgn[b] * (hi - lo - 2 * np.abs(cc[a] - cc[b]))
            else:
                v = sx * sy * sz * (2 * (cx + cy + cz - 2 * med) - lh)
            got = np.where(hit, v, 0.0) * sc
            r = ref[k + tz * mz, i + ty * m, j + tx * m]
            assert np.abs(got - r).max() <= 1e-12 * g.n, (lev, k, i, j, tz, ty, tx)
            checked += int(np.count_nonzero(r))
    assert checked > 1000
