"""The seeded input generator: determinism, shapes, and the schedule reading."""
import math

import numpy as np

from oracle import haar
from paper_1508_04458_amd import synth


def test_problem_is_deterministic_and_integer():
    a = synth.make_problem("fan96", seed=3)
    b = synth.make_problem("fan96", seed=3)
    c = synth.make_problem("fan96", seed=4)
    np.testing.assert_array_equal(a.d, b.d)
    assert not np.array_equal(a.d, c.d)
    assert a.d.shape == (a.geom.n_views * a.geom.n_bins,)
    assert np.all(a.d == np.round(a.d)) and a.d.min() >= 0


def test_schedule_reading():
    # 64/128/256 of 300 iterations with three levels, scaled to the run length
    assert synth.scaled_schedule(300, 3) == [64, 128, 256]
    assert synth.scaled_schedule(100, 3) == [21, 43, 85]
    assert synth.scaled_schedule(20, 1) == [4]


def test_fan_pitch_rule():
    g = synth.fan_geometry(512, 720, 1024)
    rc = 256 * math.sqrt(2)
    # the outermost bins see the circumscribed circle tangentially
    half = 0.5 * g.n_bins * g.bin_pitch
    assert abs(math.atan(half / g.sdd) - math.asin(rc / g.sod)) < 1e-12


def test_random_tree_masks_are_trees():
    for s in range(5):
        assert haar.valid_mask(synth.random_tree_mask(64, 3, s), 3)


def test_rasterize_mean_value():
    ell = np.array([[0.0, 0.0, 10.0, 10.0, 0.0, 0.02]])
    img = synth.rasterize(ell, 64, 1.0, supersample=8)
    assert abs(img.sum() - 0.02 * math.pi * 100) < 0.02 * 2.0


def test_line_integrals_match_quadrature_of_painted_phantom():
    """Exact painted-phantom line integrals vs brute-force quadrature along the ray."""
    P = synth.make_problem("fan96")
    o, e = synth.ray_lines(P.geom)
    tc = -(o * e).sum(1)
    ts = np.linspace(-80, 80, 400001)
    dt = ts[1] - ts[0]
    for r in np.random.default_rng(0).choice(len(o), 8, replace=False):
        x = o[r, 0] + (tc[r] + ts) * e[r, 0]
        y = o[r, 1] + (tc[r] + ts) * e[r, 1]
        v = np.zeros_like(ts)
        for cx, cy, a, b, th, mu in P.ellipses:
            c, s = math.cos(th), math.sin(th)
            u = ((x - cx) * c + (y - cy) * s) / a
            w = (-(x - cx) * s + (y - cy) * c) / b
            v = np.where(u * u + w * w <= 1, mu, v)
        assert abs(P.line_integrals[r] - v.sum() * dt) <= 1e-4 * max(1.0, P.line_integrals[r])


def test_painted_values_stay_in_range():
    P = synth.make_problem("fan128")
    img = synth.rasterize(P.ellipses, 128, 1.0, 2)
    assert img.max() <= 0.2 + 1e-12 and img.min() >= 0.0
