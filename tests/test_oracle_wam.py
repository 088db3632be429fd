"""Pins of the CPU reference's Algorithm 1 and tree rule against closed forms, brute
force, invariants the paper states (monotone decrease of the cost), special cases that
reduce to the image-domain AM of O'Sullivan-Benac, and the hand example."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import geometry, haar, siddon, wam
from paper_1508_04458_amd import synth
from golden_io import load
from test_oracle_siddon import square_chord_closed_form


@pytest.fixture(scope="module")
def p64():
    P = synth.make_problem("parallel64")
    return P, siddon.system_matrix(P.geom)


@pytest.fixture(scope="module")
def f96():
    P = synth.make_problem("fan96")
    return P, siddon.system_matrix(P.geom)


# ------------------------------------------------------------------ golden example

def test_golden_phi_z0_and_steps():
    gold = load("tiny2x2_parallel.txt")
    g = synth.parallel_geometry(2, 4, 2, 1.0)
    H = siddon.system_matrix(g)
    O = haar.synthesis_matrix(2, 1)
    Phi, act = wam.phi_matrix(H, O, haar.full_mask(2), 1.0)
    for r in range(8):
        np.testing.assert_allclose(Phi.toarray()[r], gold[f"Phi_row {r}"], atol=1e-14)
    assert abs(wam.z0_of(Phi) - gold["Z0_full"][0]) < 1e-14
    Pa, _ = wam.phi_matrix(H, O, haar.approx_mask(2, 1), 1.0)
    assert abs(wam.z0_of(Pa) - gold["Z0_approx"][0]) < 1e-14
    assert abs(wam.z0_of(H) - gold["Z0_pixel"][0]) < 1e-14
    r = wam.wam_solve(H, 2, 1, np.full(8, 50.0), 100.0, 1, 1.0)
    np.testing.assert_allclose(r["mu"].ravel(), gold["step_approx_mu"][0], rtol=1e-14)
    r = wam.am_solve(H, 2, gold["step_pixel_d"], 100.0, 1, 1.0)
    np.testing.assert_allclose(r["mu"].ravel(), gold["step_pixel_mu"], rtol=1e-13)


# ------------------------------------------------------------------ I-divergence

def test_idiv_definition_cases():
    d = np.array([0.0, 3.0, 5.0])
    q = np.array([2.0, 3.0, 1.0])
    # 0 log 0 = 0 gives q for d = 0; 0 when d = q; 5 log 5 - 5 + 1 otherwise
    assert abs(wam.idiv(d, q) - (2.0 + 0.0 + 5 * math.log(5) - 4.0)) < 1e-14
    rng = np.random.default_rng(0)
    d = rng.poisson(50, 100).astype(float)
    q = rng.uniform(10, 90, 100)
    assert wam.idiv(d, q) >= 0 and abs(wam.idiv(d, d)) < 1e-12


# ------------------------------------------------------------------ Z0 closed forms (P7)

@pytest.mark.parametrize("fix", ["p64", "f96"])
def test_z0_closed_forms(fix, request):
    P, H = request.getfixturevalue(fix)
    g = P.geom
    o, e = geometry.rays(g)
    chord = square_chord_closed_form(o, e, 0.5 * g.n * g.pixel)
    assert abs(wam.z0_of(H) - chord.max()) < 1e-10
    for L in range(1, P.levels + 1):
        O = haar.synthesis_matrix(g.n, L)
        Phi, _ = wam.phi_matrix(H, O, haar.approx_mask(g.n, L), g.pixel)
        assert abs(wam.z0_of(Phi) - 2.0 ** -L * chord.max()) < 1e-10


# ------------------------------------------------------------------ closed-form root (P8)

def _bisect_minimizer(b, bp, bm, z0):
    """Minimize f(x) = b x + (bp e^{-z0 x} - bm e^{z0 x}) / z0 (eq. 1.8 along one
    coefficient, up to constants) by bisection on its derivative (eq. 1.9)."""
    g = lambda x: b - bp * math.exp(-z0 * x) - bm * math.exp(z0 * x)
    lo, hi = -50.0 / z0, 50.0 / z0
    assert g(lo) < 0 < g(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) < 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_root_matches_bisection_and_residual():
    rng = np.random.default_rng(1)
    k = 400
    bp = rng.uniform(0.1, 10, k)
    bm = -rng.uniform(0, 10, k)
    bm[:50] = 0.0
    b = rng.uniform(-5, 10, k)
    b[:50] = np.abs(b[:50]) + 0.1
    z0 = 3.7
    delta, held = wam.closed_form_update(b, bp, bm, z0)
    assert not held.any()
    t = np.exp(-z0 * delta)
    res = b - bp * t - bm / t
    assert np.all(np.abs(res) <= 1e-12 * (np.abs(b) + bp + np.abs(bm)))
    for i in range(0, k, 7):
        assert abs(delta[i] - _bisect_minimizer(b[i], bp[i], bm[i], z0)) < 1e-9
    # b-hat- = 0: the AM log-ratio update
    np.testing.assert_allclose(delta[:50], np.log(bp[:50] / b[:50]) / z0, rtol=1e-13)


def test_root_degenerate_cases():
    b = np.array([0.0, 1.0, -1.0, 2.0, -2.0, -3.0])
    bp = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 0.0])
    bm = np.array([0.0, 0.0, 0.0, 0.0, 0.0, -2.0])
    delta, held = wam.closed_form_update(b, bp, bm, 2.0)
    # no data -> 0; bp = bm = 0 with b != 0 -> no data either (delta 0, not held)
    assert delta[0] == 0 and not held[0] and delta[1] == 0 and delta[2] == 0
    # bm = 0, b > 0: log ratio
    assert abs(delta[3] - math.log(1 / 2.0) / 2.0) < 1e-15
    # bm = 0, b < 0: no finite minimizer -> held
    assert held[4] and delta[4] == 0
    # bp = 0, bm < 0, b < 0: linear, t = bm / b
    assert abs(delta[5] - (-math.log(2.0 / 3.0) / 2.0)) < 1e-15 and not held[5]


# ------------------------------------------------------------------ surrogate (P9)

def test_surrogate_majorizes_and_touches(f96):
    P, H = f96
    g = P.geom
    O = haar.synthesis_matrix(g.n, 2)
    mask = synth.random_tree_mask(g.n, 2, 4)
    Phi, act = wam.phi_matrix(H, O, mask, g.pixel)
    z0 = wam.z0_of(Phi)
    rng = np.random.default_rng(2)
    beta = rng.normal(0, 0.02, act.size)
    b = (O.T @ (H.T @ P.d))[act]
    q = wam.beer_mean(P.i0, Phi @ beta)
    I_hat = wam.idiv(P.d, q)
    assert abs(wam.surrogate_increment(b, q, Phi, z0, np.zeros(act.size))) == 0.0
    for scale in (1e-3, 1e-2, 5e-2):
        for _ in range(3):
            dlt = rng.normal(0, scale, act.size)
            lhs = wam.idiv(P.d, wam.beer_mean(P.i0, Phi @ (beta + dlt))) - I_hat
            rhs = wam.surrogate_increment(b, q, Phi, z0, dlt)
            assert lhs <= rhs + 1e-9 * abs(I_hat)
    # gradient of the surrogate at delta = 0 is Phi^T (d - q) = b - b-hat+ - b-hat- (eq. 1.9)
    Pp, Pm = wam.split_phi(Phi)
    grad = b - Pp.T @ q - Pm.T @ q
    np.testing.assert_allclose(grad, Phi.T @ (P.d - q), rtol=1e-9, atol=1e-6 * np.abs(grad).max())
    h = 1e-6
    for z in rng.integers(0, act.size, 5):
        ez = np.zeros(act.size)
        ez[z] = h
        fd = (wam.surrogate_increment(b, q, Phi, z0, ez) - wam.surrogate_increment(b, q, Phi, z0, -ez)) / (2 * h)
        assert abs(fd - grad[z]) <= 1e-5 * (abs(grad[z]) + np.abs(b[z]))


def test_split_signs_and_adjoint(f96):
    P, H = f96
    O = haar.synthesis_matrix(P.geom.n, 3)
    Phi, act = wam.phi_matrix(H, O, haar.full_mask(P.geom.n), 1.0)
    Pp, Pm = wam.split_phi(Phi)
    rng = np.random.default_rng(3)
    y = rng.uniform(0, 1, Phi.shape[0])
    x = rng.normal(size=Phi.shape[1])
    bp, bm = Pp.T @ y, Pm.T @ y
    assert bp.min() >= 0 and bm.max() <= 0
    np.testing.assert_allclose(bp + bm, Phi.T @ y, rtol=1e-12, atol=1e-10)
    assert abs((Phi @ x) @ y - x @ (bp + bm)) < 1e-9 * abs((Phi @ x) @ y)
    # Phi = H Omega as operators
    np.testing.assert_allclose(Phi @ x, H @ (O @ x), rtol=1e-10, atol=1e-10)


def test_detail_sign_convention_does_not_change_iterates(f96):
    """Flipping the sign convention of one detail band swaps b-hat+ and b-hat- for it;
    the image iterates are unchanged."""
    P, H = f96
    n = P.geom.n
    O = haar.synthesis_matrix(n, 2)
    flip = np.ones(n * n)
    m = n >> 1
    idx = (np.arange(m)[:, None] * n + (m + np.arange(m))[None, :]).ravel()   # level-1 D1
    flip[idx] = -1
    O2 = (O @ sp.diags(flip)).tocsr()
    kw = dict(schedule=[2, 5], frac=0.1)
    r1 = wam.wam_solve(H, n, 2, P.d, P.i0, 9, 1.0, Omega=O, **kw)
    r2 = wam.wam_solve(H, n, 2, P.d, P.i0, 9, 1.0, Omega=O2, **kw)
    np.testing.assert_allclose(r1["mu"], r2["mu"], atol=1e-12)
    np.testing.assert_allclose(r1["idiv"], r2["idiv"], rtol=1e-13)


# ------------------------------------------------------------------ monotone decrease (P10)

@pytest.mark.parametrize("fix,iters", [("p64", 20), ("f96", 12)])
def test_monotone_decrease_across_expansions(fix, iters, request):
    P, H = request.getfixturevalue(fix)
    r = wam.wam_solve(H, P.geom.n, P.levels, P.d, P.i0, iters, P.geom.pixel, schedule=P.schedule)
    tr = r["idiv"]
    assert len(r["trees"]) == 1 + len(P.schedule)
    assert np.all(tr[1:] <= tr[:-1] * (1 + 1e-13)), np.diff(tr).max()
    assert r["held"] == 0


def test_monotone_fan128_adaptive():
    P = synth.make_problem("fan128")
    H = siddon.system_matrix(P.geom)
    r = wam.wam_solve(H, 128, 3, P.d, P.i0, P.n_iters, 1.0, schedule=P.schedule)
    assert np.all(np.diff(r["idiv"]) <= 1e-13 * r["idiv"][:-1])
    sizes = [int(m.sum()) for _, m in r["trees"]]
    assert sizes == sorted(sizes) and sizes[-1] > sizes[0]


# ------------------------------------------------------------------ reduction to pixel AM (P11)

def test_approximation_tree_equals_coarse_pixel_am():
    """With only approximation coefficients active, wavelet AM with L levels is pixel AM
    on the 2^L-coarser grid: beta_LL = 2^L mu_coarse and Z0 scales by 2^-L."""
    n, L = 64, 2
    g = synth.parallel_geometry(n, 40, 96, 1.0)
    gc = synth.Geometry(0, n >> L, 1.0 * (1 << L), 40, 0.0, math.pi, 96, 1.0)
    P = synth.make_problem("parallel64")
    o, e = geometry.rays(g)
    p = synth.line_integrals(P.ellipses, o, e)
    d = np.random.default_rng(9).poisson(1e4 * np.exp(-p)).astype(float)
    H = siddon.system_matrix(g)
    Hc = siddon.system_matrix(gc)
    rw = wam.wam_solve(H, n, L, d, 1e4, 8, 1.0)
    ra = wam.am_solve(Hc, n >> L, d, 1e4, 8, 1.0 * (1 << L))
    mu_c = np.repeat(np.repeat(ra["mu"], 1 << L, 0), 1 << L, 1)
    np.testing.assert_allclose(rw["mu"], mu_c, atol=1e-12)
    np.testing.assert_allclose(rw["idiv"], ra["idiv"], rtol=1e-12)
    assert abs(rw["z0"][0] - ra["z0"][0] / (1 << L)) < 1e-12


# ------------------------------------------------------------------ fixed point (P12)

def test_consistent_data_is_a_fixed_point(f96):
    P, H = f96
    n = P.geom.n
    O = haar.synthesis_matrix(n, 2)
    mask = synth.random_tree_mask(n, 2, 8)
    beta = np.random.default_rng(4).uniform(0.0, 0.02, (n, n)) * mask
    beta[: n >> 2, : n >> 2] += 0.05 * (1 << 2)
    d = wam.beer_mean(1e4, H @ (O @ beta.ravel()))
    r = wam.wam_solve(H, n, 2, d, 1e4, 2, 1.0, beta0=beta, mask0=mask)
    np.testing.assert_allclose(r["beta"], beta, atol=1e-12)


# ------------------------------------------------------------------ expansion rule (P13)

def test_expansion_hand_built():
    n, L = 8, 2
    O = haar.synthesis_matrix(n, L)
    mu = np.zeros((n, n))
    mu[0:4, 0:4] = 1.0      # root (0,0): value 1 = the maximum
    mu[0:4, 4:8] = 0.05     # root (0,1): below 0.1 * max
    mu[4:8, 0:4] = 0.1      # root (1,0): equal to the threshold -> not split (strict >)
    mu[4:8, 4:8] = 0.2      # root (1,1): above
    beta = haar.cascade_analysis(mu, L)
    mask = haar.approx_mask(n, L)
    new, cnt = wam.expand_tree(beta, mask, L, 0.1, O)
    assert cnt == 2
    np.testing.assert_array_equal(haar.split_flags(new, 2), [[True, False], [False, True]])
    assert not haar.split_flags(new, 1).any()          # one level per event
    # second event: the children of the split roots are leaves now; values 1 and 0.2 > 0.1
    beta2 = beta.copy()
    new2, cnt2 = wam.expand_tree(beta2, new, L, 0.1, O)
    assert cnt2 == 8
    f1 = haar.split_flags(new2, 1)
    assert f1[:2, :2].all() and f1[2:, 2:].all() and not f1[:2, 2:].any() and not f1[2:, :2].any()
    assert haar.valid_mask(new2, L)
    # nothing expands when the image maximum is not positive
    _, c0 = wam.expand_tree(-np.abs(beta), mask, L, 0.1, O)
    assert c0 == 0


def test_expansion_keeps_image_and_idiv_continuous(f96):
    P, H = f96
    n = P.geom.n
    r = wam.wam_solve(H, n, 2, P.d, P.i0, 6, 1.0, record_beta=True)
    O = haar.synthesis_matrix(n, 2)
    new, cnt = wam.expand_tree(r["beta"], r["mask"], 2, 0.1, O)
    assert cnt > 0 and haar.valid_mask(new, 2)
    # newly active coefficients start at zero: the image does not change
    assert np.all(r["beta"].ravel()[np.flatnonzero(new.ravel() & ~r["mask"].ravel())] == 0)
    r2 = wam.wam_solve(H, n, 2, P.d, P.i0, 1, 1.0, beta0=r["beta"], mask0=new)
    assert abs(r2["idiv"][0] - r["idiv"][-1]) <= 1e-12 * r["idiv"][-1]


# ------------------------------------------------------------------ gradient (P14)

def test_loss_gradient_matches_central_differences():
    g = synth.fan_geometry(32, 40, 64)
    H = siddon.system_matrix(g)
    O = haar.synthesis_matrix(32, 2)
    o, e = geometry.rays(g)
    ell = np.array([[2.0, -1.0, 9.0, 6.0, 0.4, 0.04]])
    d = np.random.default_rng(3).poisson(5e4 * np.exp(-synth.line_integrals(ell, o, e))).astype(float)
    c = haar.cascade_analysis(synth.rasterize(ell, 32, 1.0), 2).ravel()
    c += np.random.default_rng(4).normal(0, 1e-3, c.size)
    loss, grad, q = wam.loss_and_grad(H, O, d, 5e4, c)
    rng = np.random.default_rng(5)
    h = 1e-3
    for z in rng.choice(c.size, 64, replace=False):
        cp, cm = c.copy(), c.copy()
        cp[z] += h
        cm[z] -= h
        fd = (wam.loss_and_grad(H, O, d, 5e4, cp)[0] - wam.loss_and_grad(H, O, d, 5e4, cm)[0]) / (2 * h)
        # central-difference truncation bound h^2/6 |f'''| with f''' = -sum_y q phi^3
        # (q evaluated within e^{h |phi|} of the centre), plus rounding of the loss
        phi = H @ O[:, [z]].toarray().ravel()
        bound = h * h / 6 * np.sum(q * np.abs(phi) ** 3) * math.exp(h * np.abs(phi).max())
        assert abs(fd - grad[z]) <= bound + 1e-13 * abs(loss) / h + 1e-12, (z, fd, grad[z], bound)
