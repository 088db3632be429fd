"""Pins of the roughness-penalized update of the oracle (oracle.wam: roughness,
roughness_grad, penalized_update, wam_solve(penalty=...)), CPU only:

  * R and its gradient: a hand-computed 2x3 image; central differences of R;
  * the Hessian bound 8: R(mu + e) - R(mu) - grad.e <= 4 |e|^2 for random e (and the bound is
    nearly reached by the checkerboard);
  * penalized_update returns the root of G (residual ~ 0), and with lambda -> 0 it tends to
    the eq. 1.9 root;
  * the penalized objective I + lambda R falls at every iteration (the combined surrogate
    majorizes it) and across expansions; lambda = 0 is Algorithm 1; a larger lambda gives a
    smoother image.
"""
import numpy as np

from oracle import haar, siddon, wam
from paper_1508_04458_amd import synth


def test_roughness_hand_example_and_gradient():
    mu = np.array([[1.0, 2.0, 4.0], [0.0, 3.0, 3.0]])
    # horizontal pairs: (1,2),(2,4),(0,3),(3,3); vertical: (1,0),(2,3),(4,3)
    assert wam.roughness(mu) == 0.5 * (1 + 4 + 9 + 0 + 1 + 1 + 1)
    g = wam.roughness_grad(mu)
    np.testing.assert_array_equal(g, [[(1 - 2) + (1 - 0), (2 - 1) + (2 - 4) + (2 - 3), (4 - 2) + (4 - 3)],
                                      [(0 - 3) + (0 - 1), (3 - 0) + (3 - 3) + (3 - 2), (3 - 3) + (3 - 4)]])
    rng = np.random.default_rng(1)
    x = rng.normal(size=(5, 7))
    h = 1e-6
    for _ in range(8):
        e = np.zeros_like(x)
        e[rng.integers(5), rng.integers(7)] = h
        fd = (wam.roughness(x + e) - wam.roughness(x - e)) / (2 * h)
        assert abs(fd - float((wam.roughness_grad(x) * e).sum() / h)) <= 1e-7


def test_hessian_bound_eight():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(16, 16))
    for _ in range(20):
        e = rng.normal(size=x.shape)
        gap = wam.roughness(x + e) - wam.roughness(x) - float((wam.roughness_grad(x) * e).sum())
        assert gap <= 0.5 * wam.PENALTY_CURVATURE * float((e * e).sum()) + 1e-9
    cb = np.fromfunction(lambda i, j: (-1.0) ** (i + j), (16, 16))
    assert wam.roughness(cb) >= 0.9 * 0.5 * 7.0 * float((cb * cb).sum())   # close to the bound


def test_penalized_update_is_the_root():
    rng = np.random.default_rng(3)
    k = 200
    b = rng.uniform(-50, 200, k)
    bp = rng.uniform(0, 100, k)
    bm = -rng.uniform(0, 30, k)
    bp[:10] = 0.0
    bm[10:20] = 0.0
    g = rng.normal(0, 5, k)
    z0, lam = 3.0, 0.7
    dl = wam.penalized_update(b, bp, bm, z0, lam, g)
    G = b - bp * np.exp(-z0 * dl) - bm * np.exp(z0 * dl) + lam * (g + 8 * dl)
    assert np.max(np.abs(G)) <= 1e-9 * np.max(np.abs(b) + bp - bm)
    ok = bp > 0
    d0, held = wam.closed_form_update(b[ok], bp[ok], bm[ok], z0)
    dsmall = wam.penalized_update(b[ok], bp[ok], bm[ok], z0, 1e-9, g[ok])
    fine = ~held
    assert np.max(np.abs(dsmall[fine] - d0[fine])) <= 1e-6 * max(1.0, np.max(np.abs(d0[fine])))


def _problem():
    g = synth.fan_geometry(32, 40, 64)
    H = siddon.system_matrix(g)
    ell = synth.make_ellipses(np.random.default_rng(4), g.n, g.pixel, 6, 0.06, 1)
    o, e = synth.ray_lines(g)
    d = np.random.default_rng(5).poisson(5e3 * np.exp(-synth.line_integrals(ell, o, e))).astype(float)
    return g, H, d, 5e3


def test_penalized_objective_is_monotone_and_smoother():
    g, H, d, i0 = _problem()
    L = 2
    r0 = wam.wam_solve(H, g.n, L, d, i0, 12, g.pixel, schedule=[3, 7])
    rz = wam.wam_solve(H, g.n, L, d, i0, 12, g.pixel, schedule=[3, 7], penalty=1e-12)
    np.testing.assert_allclose(rz["beta"], r0["beta"], rtol=0, atol=1e-9 * np.abs(r0["beta"]).max())
    lam = 50.0
    r = wam.wam_solve(H, g.n, L, d, i0, 12, g.pixel, schedule=[3, 7], penalty=lam)
    obj = r["objective"]
    assert np.all(np.diff(obj) <= 1e-12 * np.abs(obj[:-1])), np.diff(obj)
    assert wam.roughness(r["mu"]) < wam.roughness(r0["mu"])
