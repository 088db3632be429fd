"""Pins of the residual-gradient tree rule of the oracle (oracle.wam.expand_tree_gradient),
CPU only:

  * the leaf scores are derivatives of the I-divergence: central differences of
    I(d || I0 exp(-H Omega beta)) along single detail coefficients (active and inactive)
    equal c = Omega^T H^T (d - q-hat) within the truncation bound;
  * consistent data (d = q-hat of the current beta) give c = 0 and no split;
  * frac = 0 splits exactly the leaves with a nonzero score, one level, into a valid tree;
  * Algorithm 1 with this rule keeps the I-divergence decreasing across expansions.
"""
import numpy as np

from oracle import haar, siddon, wam
from paper_1508_04458_amd import synth


def small_problem():
    g = synth.parallel_geometry(16, 24, 30, 1.0)
    H = siddon.system_matrix(g)
    ell = synth.make_ellipses(np.random.default_rng(4), g.n, g.pixel, 5, 0.08, 1)
    o, e = synth.ray_lines(g)
    d = np.random.default_rng(5).poisson(3e3 * np.exp(-synth.line_integrals(ell, o, e))).astype(float)
    return g, H, d, 3e3


def idiv_of(H, O, d, i0, beta):
    return wam.idiv(d, wam.beer_mean(i0, H @ (O @ beta)))


def test_scores_are_idiv_derivatives():
    g, H, d, i0 = small_problem()
    L = 2
    O = haar.synthesis_matrix(g.n, L)
    mask = synth.random_tree_mask(g.n, L, 3, p_split=0.5)
    rng = np.random.default_rng(6)
    beta = (rng.normal(0, 0.01, g.n * g.n) * mask.ravel())
    beta.reshape(g.n, g.n)[:g.n >> L, :g.n >> L] = 0.05 * (1 << L)
    q = wam.beer_mean(i0, H @ (O @ beta))
    c = O.T @ (H.T @ (d - q))
    h = 1e-5
    for z in rng.choice(np.arange(g.n * g.n), 12, replace=False):
        e = np.zeros_like(beta)
        e[z] = h
        fd = (idiv_of(H, O, d, i0, beta + e) - idiv_of(H, O, d, i0, beta - e)) / (2 * h)
        assert abs(fd - c[z]) <= 1e-6 * max(1.0, abs(c[z])), (z, fd, c[z])


def test_consistent_data_split_nothing():
    g, H, _, i0 = small_problem()
    L = 2
    O = haar.synthesis_matrix(g.n, L)
    mask = haar.approx_mask(g.n, L)
    beta = np.zeros(g.n * g.n)
    beta.reshape(g.n, g.n)[:g.n >> L, :g.n >> L] = np.random.default_rng(7).uniform(0.05, 0.3, (g.n >> L,) * 2)
    d = wam.beer_mean(i0, H @ (O @ beta))
    new, count = wam.expand_tree_gradient(beta, mask, L, 0.1, O, H, d, i0)
    assert count == 0 and np.array_equal(new, mask)


def test_frac_zero_splits_every_leaf_with_a_gradient():
    g, H, d, i0 = small_problem()
    L = 2
    O = haar.synthesis_matrix(g.n, L)
    mask = synth.random_tree_mask(g.n, L, 8, p_split=0.4)
    beta = np.zeros(g.n * g.n)
    new, count = wam.expand_tree_gradient(beta, mask, L, 0.0, O, H, d, i0)
    q = wam.beer_mean(i0, H @ (O @ beta))
    c = (O.T @ (H.T @ (d - q))).reshape(g.n, g.n)
    expect = 0
    for lev in range(1, L + 1):
        m = g.n >> lev
        split = haar.split_flags(mask, lev)
        parent = np.ones((m, m), bool) if lev == L else \
            np.repeat(np.repeat(haar.split_flags(mask, lev + 1), 2, 0), 2, 1)
        leaf = ~split & parent
        nz = (np.abs(c[:m, m:2 * m]) + np.abs(c[m:2 * m, :m]) + np.abs(c[m:2 * m, m:2 * m])) > 0
        grown = haar.split_flags(new, lev) & ~split
        np.testing.assert_array_equal(grown, leaf & nz)
        expect += int((leaf & nz).sum())
    assert count == expect > 0
    assert haar.valid_mask(new, L)


def test_gradient_rule_solve_is_monotone():
    g, H, d, i0 = small_problem()
    L = 2
    r = wam.wam_solve(H, g.n, L, d, i0, 12, g.pixel, schedule=[3, 6, 9], rule="gradient")
    tr = r["idiv"]
    assert np.all(np.diff(tr) <= 1e-12 * np.abs(tr[:-1]))
    assert len(r["trees"]) == 4 and haar.valid_mask(r["mask"], L)
