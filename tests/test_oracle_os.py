"""Pins of the ordered-subsets wavelet AM oracle (oracle.wam.os_wam_solve), CPU only.

  * one subset is Algorithm 1 itself (equal to wam_solve to rounding);
  * the subsets partition the rays, and the per-subset b_s add up to b (eq. 1.6);
  * Z0_s of the approximation-only tree is 2^-L times the largest chord through the image
    over the subset's rays (closed form of a square);
  * every sub-iteration is an exact AM step for its subset, so I(d_s || q_s) never rises
    (the AM guarantee of the Summary, applied to the subset objective);
  * consistent (noise-free) data of a coefficient image on the tree are a fixed point of
    every sub-iteration.
"""
import numpy as np
import pytest

from oracle import geometry, haar, siddon, wam
from paper_1508_04458_amd import synth
from test_oracle_siddon import square_chord_closed_form


@pytest.fixture(scope="module")
def fan64():
    g = synth.fan_geometry(64, 45, 92)
    ell = synth.make_ellipses(np.random.default_rng(5), g.n, g.pixel, 8, 0.06, 1)
    o, e = synth.ray_lines(g)
    d = np.random.default_rng(6).poisson(3e4 * np.exp(-synth.line_integrals(ell, o, e))).astype(float)
    return g, siddon.system_matrix(g), d


def test_one_subset_is_algorithm_1(fan64):
    g, H, d = fan64
    ref = wam.wam_solve(H, g.n, 2, d, 3e4, 8, g.pixel, schedule=[3, 6])
    os1 = wam.os_wam_solve(H, g.n, 2, d, 3e4, 8, g.pixel, g.n_views, 1, schedule=[3, 6])
    np.testing.assert_allclose(os1["beta"], ref["beta"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(os1["idiv"], ref["idiv"], rtol=1e-13)
    np.testing.assert_array_equal(os1["mask"], ref["mask"])
    assert os1["held"] == ref["held"]


def test_subsets_partition_rays_and_b():
    rows = wam.subset_rows(10, 7, 3)
    allr = np.sort(np.concatenate(rows))
    np.testing.assert_array_equal(allr, np.arange(70))
    assert [len(r) for r in rows] == [28, 21, 21]
    assert set(rows[1] // 7) == {1, 4, 7}
    g = synth.fan_geometry(32, 20, 48)
    H = siddon.system_matrix(g)
    d = synth.random_vector(g.n_rays, 3, 0, 50)
    r = wam.os_wam_solve(H, g.n, 1, d, 100.0, 1, g.pixel, g.n_views, 4)
    b = haar.synthesis_matrix(g.n, 1).T @ (H.T @ d)
    np.testing.assert_allclose(sum(r["b_sub"]).ravel(), b, rtol=1e-12, atol=1e-9)
    with pytest.raises(ValueError):
        wam.subset_rows(5, 3, 6)


@pytest.mark.parametrize("S", [3, 5])
def test_subset_z0_closed_form(fan64, S):
    g, H, d = fan64
    L = 2
    r = wam.os_wam_solve(H, g.n, L, d, 3e4, 1, g.pixel, g.n_views, S)
    o, e = geometry.rays(g)
    chord = square_chord_closed_form(o, e, 0.5 * g.n * g.pixel)
    for s, rows in enumerate(wam.subset_rows(g.n_views, g.n_bins, S)):
        ref = 2.0 ** -L * chord[rows].max()
        assert abs(r["z0"][0][s] - ref) <= 1e-11 * ref


@pytest.mark.parametrize("S", [2, 5])
def test_every_subiteration_decreases_its_subset_idiv(fan64, S):
    g, H, d = fan64
    r = wam.os_wam_solve(H, g.n, 2, d, 3e4, 6, g.pixel, g.n_views, S, schedule=[2, 4], record_sub=True)
    assert len(r["sub"]) == 6 * S
    for before, after in r["sub"]:
        assert after <= before * (1 + 1e-12), (before, after)
    # and the passes do reduce the full objective on this problem
    assert r["idiv"][-1] < r["idiv"][0]


def test_consistent_data_is_a_fixed_point():
    g = synth.fan_geometry(32, 24, 48)
    H = siddon.system_matrix(g)
    L = 2
    mask = synth.random_tree_mask(g.n, L, 4, p_split=0.6)
    O = haar.synthesis_matrix(g.n, L)
    rng = np.random.default_rng(4)
    beta = rng.normal(0, 0.002, g.n * g.n) * mask.ravel()
    nL = g.n >> L
    beta.reshape(g.n, g.n)[:nL, :nL] = 0.03 * (1 << L)
    d = 1e4 * np.exp(-(H @ (O @ beta)))          # noise-free, non-integer counts
    r = wam.os_wam_solve(H, g.n, L, d, 1e4, 2, g.pixel, g.n_views, 4, beta0=beta, mask0=mask)
    assert np.max(np.abs(r["beta"].ravel() - beta)) <= 1e-10
    assert r["held"] == 0
    assert abs(r["idiv"][-1]) <= 1e-8


# ------------------------------------------------------------------ slices sharing one tree

def test_single_slice_volume_is_algorithm_1(fan64):
    g, H, d = fan64
    ref = wam.wam_solve(H, g.n, 2, d, 3e4, 8, g.pixel, schedule=[3, 6])
    vol = wam.volume_wam_solve(H, g.n, 2, [d], [3e4], 8, g.pixel, schedule=[3, 6])
    np.testing.assert_allclose(vol["betas"][0], ref["beta"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(vol["idiv"][0], ref["idiv"], rtol=1e-13)
    np.testing.assert_array_equal(vol["mask"], ref["mask"])


def test_identical_slices_reproduce_one_slice(fan64):
    """Two identical slices: the summed image is twice each slice (exact), so the tree and
    every slice's iterates equal those of one slice alone."""
    g, H, d = fan64
    ref = wam.wam_solve(H, g.n, 2, d, 3e4, 8, g.pixel, schedule=[3, 6])
    vol = wam.volume_wam_solve(H, g.n, 2, [d, d], [3e4, 3e4], 8, g.pixel, schedule=[3, 6])
    np.testing.assert_array_equal(vol["mask"], ref["mask"])
    for p in range(2):
        np.testing.assert_array_equal(vol["betas"][p], ref["beta"])


def test_tree_follows_the_slice_sum():
    """Hand-made coefficients (approximation only, 2 levels, 16x16): slice 0 bright in root
    (0, 0), slice 1 in root (3, 3) at the same value -> the summed image splits both roots;
    with slice 1 at 5 % of that value only root (0, 0) splits (5 % < 10 % of the maximum)."""
    g = synth.parallel_geometry(16, 12, 24, 1.0)
    H = siddon.system_matrix(g)
    L = 2
    d = [np.zeros(g.n_rays)] * 2
    for v1, split_33 in ((1.0, True), (0.05, False)):
        betas = np.zeros((2, 16, 16))
        betas[0, 0, 0] = 4.0            # approximation of root (0, 0): mu = 1 on its block
        betas[1, 3, 3] = 4.0 * v1
        vol = wam.volume_wam_solve(H, 16, L, d, [1.0, 1.0], 1, g.pixel, schedule=[0], betas0=betas)
        split = haar.split_flags(vol["mask"], L)
        expect = np.zeros((4, 4), bool)
        expect[0, 0] = True
        expect[3, 3] = split_33
        np.testing.assert_array_equal(split, expect)
