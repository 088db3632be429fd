"""The 3-D phantom generator (paper_1508_04458_amd/synth.py), CPU only: exact line integrals
of painted ellipsoids and cylinders against closed forms and brute-force sampling, and
the cone-beam ray layout."""
import math

import numpy as np
import pytest

from paper_1508_04458_amd import synth


def sphere(c, r, mu):
    return dict(kind="ellipsoid", c=np.asarray(c, float), rot=np.eye(3), semi=np.array([r, r, r], float), mu=mu)


def cylinder(c, r, h, mu):
    return dict(kind="cylinder", c=np.asarray(c, float), r=r, h=h, mu=mu)


def lines_along_x(offsets):
    o = np.array([[-100.0, y, z] for y, z in offsets])
    e = np.tile([1.0, 0.0, 0.0], (len(offsets), 1))
    return o, e


def test_sphere_chord_closed_form():
    offs = [(0.0, 0.0), (3.0, 1.0), (4.0, -2.9), (6.0, 0.0)]
    o, e = lines_along_x(offs)
    p = synth.line_integrals3([sphere([0, 0, 0], 5.0, 0.1)], o, e)
    ref = [0.1 * 2 * math.sqrt(max(25.0 - y * y - z * z, 0.0)) for y, z in offs]
    np.testing.assert_allclose(p, ref, atol=1e-12)


def test_painting_order():
    o, e = lines_along_x([(0.0, 0.0), (1.0, 1.0)])
    outer, inner = sphere([0, 0, 0], 6.0, 0.05), sphere([0, 0, 0], 2.0, 0.2)
    Lo = 2 * np.sqrt(36.0 - np.array([0.0, 2.0]))
    Li = 2 * np.sqrt(4.0 - np.array([0.0, 2.0]))
    np.testing.assert_allclose(synth.line_integrals3([outer, inner], o, e), 0.05 * (Lo - Li) + 0.2 * Li, atol=1e-12)
    np.testing.assert_allclose(synth.line_integrals3([inner, outer], o, e), 0.05 * Lo, atol=1e-12)


def test_cylinder_chords():
    cyl = cylinder([1.0, 0.0, 2.0], 3.0, 10.0, 0.2)
    o, e = lines_along_x([(0.0, 2.0), (2.0, 6.9), (2.0, 7.1)])       # across the axis
    p = synth.line_integrals3([cyl], o, e)
    np.testing.assert_allclose(p, [0.2 * 6.0, 0.2 * 2 * math.sqrt(5.0), 0.0], atol=1e-12)
    o = np.array([[1.5, 0.5, -50.0], [1.0, 0.0, 100.0]])            # along the axis, both ways
    e = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    np.testing.assert_allclose(synth.line_integrals3([cyl], o, e), [2.0, 2.0], atol=1e-12)


def test_many_shapes_match_sampling():
    """70 random shapes (more than one 32-bit word of the covering set) against a midpoint
    sum along each line (error <= 2 boundaries per shape x step x max mu)."""
    g = synth.cone_geometry(32, 16, 2, 3, 8, sod=100.0, sdd=200.0)
    shapes = synth.make_ellipsoids(np.random.default_rng(5), 32, 16, 1.0, 64, 0.06, 6)
    o, e = synth.cone_rays(g)
    p = synth.line_integrals3(shapes, o, e)
    ts = np.arange(0.0, 200.0, 0.01) + 0.005
    for r in range(o.shape[0]):
        x = o[r] + ts[:, None] * e[r]
        v = np.zeros(ts.size)
        for sh in shapes:
            if sh["kind"] == "ellipsoid":
                ins = ((((x - sh["c"]) @ sh["rot"].T) / sh["semi"]) ** 2).sum(1) < 1
            else:
                ins = (((x[:, 0] - sh["c"][0]) ** 2 + (x[:, 1] - sh["c"][1]) ** 2 < sh["r"] ** 2)
                       & (np.abs(x[:, 2] - sh["c"][2]) < 0.5 * sh["h"]))
            v = np.where(ins, sh["mu"], v)
        assert abs(v.sum() * 0.01 - p[r]) <= 2 * len(shapes) * 0.01 * 0.2 + 1e-9


def test_cone_rays_layout():
    g = synth.cone_geometry(16, 8, 4, 3, 5, sod=50.0, sdd=90.0)
    o, e = synth.cone_rays(g)
    assert o.shape == (g.n_rays, 3)
    np.testing.assert_allclose(np.linalg.norm(e, axis=1), 1.0, atol=1e-15)
    # ray (view 2, row 1, col 4): from the source through the detector element centre
    a = 2 * 2 * math.pi / 4
    r = (2 * g.n_rows + 1) * g.n_cols + 4
    src = g.sod * np.array([math.cos(a), math.sin(a), 0.0])
    u, w = 2 * g.col_pitch, 0.0
    det = -(g.sdd - g.sod) * np.array([math.cos(a), math.sin(a), 0.0]) + u * np.array([-math.sin(a), math.cos(a), 0.0])
    det[2] = w
    np.testing.assert_allclose(o[r], src, atol=1e-12)
    np.testing.assert_allclose(e[r], (det - src) / np.linalg.norm(det - src), atol=1e-14)
    # a sub-range equals the same rows of the whole table
    o2, e2 = synth.cone_rays(g, 7, 23)
    np.testing.assert_array_equal(o2, o[7:23])
    np.testing.assert_array_equal(e2, e[7:23])
