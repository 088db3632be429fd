"""Pins of the CPU reference's Haar synthesis Omega (eq. 1.2): orthonormality, agreement
with an independent textbook cascade, leaf constancy on trees, and the hand example."""
import numpy as np
import pytest

from oracle import haar, siddon, geometry, wam
from paper_1508_04458_amd import synth
from golden_io import load


@pytest.mark.parametrize("n,L", [(2, 1), (8, 1), (8, 3), (16, 2), (32, 4)])
def test_orthonormal_and_matches_cascade(n, L):
    O = haar.synthesis_matrix(n, L)
    np.testing.assert_allclose((O.T @ O).toarray(), np.eye(n * n), atol=1e-14)
    rng = np.random.default_rng(n + L)
    beta = rng.normal(size=(n, n))
    mu = (O @ beta.ravel()).reshape(n, n)
    np.testing.assert_allclose(mu, haar.cascade_synthesis(beta, L), atol=1e-13)
    np.testing.assert_allclose(haar.cascade_analysis(mu, L), beta, atol=1e-13)
    assert abs(np.linalg.norm(mu) - np.linalg.norm(beta)) < 1e-12


def test_golden_2x2_columns():
    O = haar.synthesis_matrix(2, 1).toarray()
    np.testing.assert_allclose(O[:, 0], [0.5, 0.5, 0.5, 0.5])
    np.testing.assert_allclose(O[:, 1], [0.5, -0.5, 0.5, -0.5])
    np.testing.assert_allclose(O[:, 2], [0.5, 0.5, -0.5, -0.5])
    np.testing.assert_allclose(O[:, 3], [0.5, -0.5, -0.5, 0.5])


def test_cascade_hand_example():
    # a = 4, b = 2, c = 6, d = 0  ->  LL = 6, D1 = (4-2+6-0)/2 = 4, D2 = (4+2-6-0)/2 = 0, D3 = (4-2-6+0)/2 = -2
    out = haar.cascade_analysis(np.array([[4.0, 2.0], [6.0, 0.0]]), 1)
    np.testing.assert_allclose(out, [[6.0, 4.0], [0.0, -2.0]])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_leaf_constant_on_random_tree(seed):
    n, L = 32, 3
    mask = synth.random_tree_mask(n, L, seed)
    assert haar.valid_mask(mask, L)
    O = haar.synthesis_matrix(n, L)
    beta = np.random.default_rng(seed).normal(size=(n, n)) * mask
    mu = (O @ beta.ravel()).reshape(n, n)
    lev = haar.leaf_level_map(mask, L)
    for r in range(n):
        for c in range(n):
            s = 1 << lev[r, c]
            r0, c0 = (r // s) * s, (c // s) * s
            assert abs(mu[r, c] - mu[r0, c0]) < 1e-13


def test_valid_mask_rejects_orphans():
    n, L = 16, 2
    m = haar.approx_mask(n, L)
    assert haar.valid_mask(m, L)
    bad = m.copy()
    f = np.zeros((8, 8), bool)
    f[3, 3] = True           # a level-1 node split while its parent is not
    haar.set_split(bad, 1, f)
    assert not haar.valid_mask(bad, L)


@pytest.mark.parametrize("name,L", [("parallel64", 2), ("fan96", 3)])
def test_phi_columns_equal_quadrant_chords(name, L):
    """phi(y|z) from H Omega (sparse product) equals 2^-l sum_q s_k(q) chord(y, quadrant q)
    computed by brute-force box clipping (and 2^-L chord(y, block) for approximations)."""
    g = synth.CONFIGS[name]["geom"]()
    H = siddon.system_matrix(g)
    O = haar.synthesis_matrix(g.n, L)
    Phi, act = wam.phi_matrix(H, O, haar.full_mask(g.n), g.pixel)
    Phi = Phi.tocsc()
    o, e = geometry.rays(g)
    edges = geometry.pixel_edges(g)
    rng = np.random.default_rng(5)
    n = g.n
    for _ in range(12):
        lev = int(rng.integers(1, L + 1))
        m = n >> lev
        i, j = rng.integers(0, m, 2)
        s = 1 << lev
        h = s >> 1
        q = {}
        for qy in (0, 1):
            for qx in (0, 1):
                x0 = edges[j * s + qx * h]
                x1 = edges[j * s + (qx + 1) * h]
                y0 = edges[i * s + qy * h]
                y1 = edges[i * s + (qy + 1) * h]
                q[qy, qx] = siddon.box_chord(o, e, x0, x1, y0, y1)
        d1 = (q[0, 0] - q[0, 1] + q[1, 0] - q[1, 1]) * 2.0 ** -lev
        d2 = (q[0, 0] + q[0, 1] - q[1, 0] - q[1, 1]) * 2.0 ** -lev
        d3 = (q[0, 0] - q[0, 1] - q[1, 0] + q[1, 1]) * 2.0 ** -lev
        for zr, zc, ref in ((i, m + j, d1), (m + i, j, d2), (m + i, m + j, d3)):
            col = np.asarray(Phi[:, zr * n + zc].todense()).ravel()
            ref = np.where(np.abs(ref) <= 1e-12 * g.pixel, 0.0, ref)
            assert np.abs(col - ref).max() < 1e-12
        if lev == L:
            llc = np.asarray(Phi[:, i * n + j].todense()).ravel()
            ref = sum(q.values()) * 2.0 ** -L
            assert np.abs(llc - ref).max() < 1e-12


# ------------------------------------------------------------------ Daubechies-4 (periodic)

def test_d4_filters_and_orthonormal_basis():
    """The D4 filters satisfy the orthonormality and two-vanishing-moment conditions in closed
    form, and the 2-D synthesis matrix is orthonormal."""
    from oracle import daub
    h, g = daub.H4, daub.G4
    np.testing.assert_allclose(h.sum(), np.sqrt(2.0), atol=1e-15)
    np.testing.assert_allclose((h * h).sum(), 1.0, atol=1e-15)
    np.testing.assert_allclose(h[0] * h[2] + h[1] * h[3], 0.0, atol=1e-15)   # double shifts orthogonal
    np.testing.assert_allclose(g.sum(), 0.0, atol=1e-15)
    np.testing.assert_allclose((np.arange(4) * g).sum(), 0.0, atol=1e-14)    # second vanishing moment
    for n, L in ((8, 1), (16, 2), (32, 3)):
        O = daub.synthesis_matrix(n, L).toarray()
        np.testing.assert_allclose(O.T @ O, np.eye(n * n), atol=1e-13)


def test_d4_perfect_reconstruction_against_filter_bank():
    """Analysis by the textbook periodic filter bank equals Omega^T (so Omega inverts it)."""
    from oracle import daub
    n, L = 32, 3
    O = daub.synthesis_matrix(n, L)
    img = np.random.default_rng(4).normal(size=(n, n))
    coef = daub.cascade_analysis(img, L)
    np.testing.assert_allclose(coef.ravel(), O.T @ img.ravel(), atol=1e-12)
    np.testing.assert_allclose((O @ coef.ravel()).reshape(n, n), img, atol=1e-12)


def test_d4_vanishing_moments_and_supports():
    """A constant image has only approximation coefficients; a periodic ramp's interior
    wavelet coefficients along x vanish (two vanishing moments); every basis function of level
    l lives on a 3 * 2^l - 2 pixel square starting at its node's block (mod n)."""
    from oracle import daub
    n, L = 32, 2
    O = daub.synthesis_matrix(n, L).toarray()
    c = O.T @ np.ones(n * n)
    coef = c.reshape(n, n)
    assert np.abs(coef[n >> L:, :]).max() < 1e-12 and np.abs(coef[:, n >> L:]).max() < 1e-12
    x = np.tile(np.arange(n, dtype=float), (n, 1))          # ramp along x: linear in the interior
    cr = (O.T @ x.ravel()).reshape(n, n)
    m = n >> 1
    d1 = cr[:m, m:2 * m]                                     # level-1 D1: psi in x
    np.testing.assert_allclose(d1[:, :m - 2], 0.0, atol=1e-11)   # supports not wrapping past x = n
    for l in range(1, L + 1):
        m = n >> l
        s = 3 * (1 << l) - 2
        for (i, j) in ((0, 0), (m - 1, m - 1), (1, m - 2)):
            col = O[:, (m + i) * n + (m + j)].reshape(n, n)
            rows = {(r - (i << l)) % n for r in np.nonzero(np.abs(col).sum(1) > 0)[0]}
            cs = {(cc - (j << l)) % n for cc in np.nonzero(np.abs(col).sum(0) > 0)[0]}
            assert max(rows) < s and max(cs) < s


def test_d4_phi_equals_dense_h_times_basis():
    """phi(y|z) for D4 coefficients from the dense brute-force H (box clipping) times the
    basis image, against H Omega of the solver's sparse path; and Algorithm 1 with the D4
    Omega stays monotone across expansions (Summary: the I-divergence never increases)."""
    from oracle import daub, siddon, wam
    from paper_1508_04458_amd import synth
    g = synth.fan_geometry(16, 12, 23, sod=40.0, sdd=70.0)
    L = 2
    O = daub.synthesis_matrix(g.n, L)
    Hd = siddon.dense_matrix(g)
    mask = np.ones((g.n, g.n), np.uint8)
    Phi, act = wam.phi_matrix(siddon.system_matrix(g), O, mask, g.pixel)
    np.testing.assert_allclose(Phi.toarray(), np.where(np.abs(Hd @ O.toarray()) <= 1e-12 * g.pixel, 0.0,
                                                       Hd @ O.toarray())[:, act], atol=1e-12)
    P = synth.make_problem("parallel64")
    H = siddon.system_matrix(P.geom)
    r = wam.wam_solve(H, P.geom.n, 3, P.d, P.i0, 12, P.geom.pixel, schedule=[3, 6, 9],
                      Omega=daub.synthesis_matrix(P.geom.n, 3))
    assert np.all(r["idiv"][1:] <= r["idiv"][:-1] * (1 + 1e-13))
    assert len(r["trees"]) == 4 and r["trees"][-1][1].sum() > r["trees"][0][1].sum()
