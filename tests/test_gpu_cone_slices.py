"""Cone beam with the Results section's per-slice representation (a 2-D Haar transform of
every z-slice, one tree shared by the slices, grown on the slice-summed image) on the GPU
against the FP64 oracle (oracle.vol3d.slice_wam_solve3), element by element.

Tolerances as for the octree (tests/test_gpu_cone.py): projections |dp| <= 1e-5 max(|p|,
1e-3 max p) (FP32) / 1e-11 (FP64); backprojections and b 2e-5 / 1e-11 of the largest value;
Z0 1e-11, W 1e-4; FP64 solve with the GPU's own expansions: masks exact, beta relative L2
1e-9, I-divergence rtol 1e-10, held counts equal; FP32 with the oracle's tree sequence fed
in: beta relative L2 1e-4, I-divergence rtol 2e-5.
"""
import numpy as np
import pytest
import torch

from oracle import haar, vol3d, wam
from paper_1508_04458_amd import synth
from test_gpu_cone import dev, host, problem, proj_tol, rel_l2

pytestmark = pytest.mark.gpu


def make_ctx(g, levels, dtype, d=None, i0=None):
    from paper_1508_04458_amd import api
    print(f"\n[case] cone slices n={g.n} nz={g.nz} views={g.n_views} det={g.n_rows}x{g.n_cols} L={levels} {dtype}",
          flush=True)
    c = api.Context(g, levels, dtype, wavelet_dims=2)
    if d is not None:
        c.set_data(dev(d, dtype), i0)
    return c


def slice_tree(n, nz, L, seed, p=0.5):
    return vol3d.slice_mask3(synth.random_tree_mask(n, L, seed, p_split=p), nz)


@pytest.mark.parametrize("levels,dtype,seed,p", [(1, "f64", 0, 0.5), (2, "f64", 1, 0.6), (2, "f32", 2, 0.5),
                                                 (3, "f64", 3, 1.0), (3, "f32", 4, 0.7)])
def test_slice_split_backprojection_z0_w_match_oracle(levels, dtype, seed, p):
    P, H = problem("cone32")
    g = P.geom
    mask = slice_tree(g.n, g.nz, levels, seed, p)
    c = make_ctx(g, levels, dtype)
    c.set_state(dev(np.zeros(g.n_voxels), dtype), dev(mask.ravel(), torch.uint8))
    O = vol3d.slice_synthesis_matrix3(g.n, g.nz, levels)
    Phi, act = wam.phi_matrix(H, O, mask, g.pixel)
    if dtype == "f64":
        st = c.tree_stats()
        assert abs(st["z0"] - wam.z0_of(Phi)) <= 1e-11 * st["z0"]
        assert abs(st["w"] - Phi.nnz) <= 1e-4 * Phi.nnz
        assert st["n_active"] == act.size
    y = synth.random_vector(g.n_rays, 20 + seed)
    bp, bm = (host(t).ravel() for t in c.backproject_split(dev(y, dtype)))
    Pp, Pm = wam.split_phi(Phi)
    rp = np.zeros(g.n_voxels)
    rm = np.zeros(g.n_voxels)
    rp[act] = Pp.T @ y
    rm[act] = Pm.T @ y
    tol = (2e-5 if dtype == "f32" else 1e-11) * max(np.abs(rp).max(), np.abs(rm).max())
    assert np.abs(bp - rp).max() <= tol
    assert np.abs(bm - rm).max() <= tol
    assert bp.min() >= 0 and bm.max() <= 0
    assert np.all(bp[mask.ravel() == 0] == 0) and np.all(bm[mask.ravel() == 0] == 0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_slice_forward_synthesis_and_b_match_oracle(dtype):
    P, H = problem("cone32")
    g, L = P.geom, 2
    mask = slice_tree(g.n, g.nz, L, 7, 0.6)
    rng = np.random.default_rng(8)
    beta = rng.normal(0, 0.002, (g.nz, g.n, g.n)) * mask
    beta[:, :g.n >> L, :g.n >> L] = 0.02 * (1 << L) + rng.uniform(0, 0.01, (g.nz, g.n >> L, g.n >> L))
    c = make_ctx(g, L, dtype, P.d, P.i0)
    c.set_state(dev(beta.ravel(), dtype), dev(mask.ravel(), torch.uint8))
    O = vol3d.slice_synthesis_matrix3(g.n, g.nz, L)
    mu_ref = O @ beta.ravel()
    mu = host(c.synthesize()).ravel()
    assert np.abs(mu - mu_ref).max() <= (1e-6 if dtype == "f32" else 1e-13) * np.abs(mu_ref).max()
    p_ref = H @ mu_ref
    q_ref = wam.beer_mean(P.i0, p_ref)
    q, idv = c.forward()
    q = host(q).ravel()
    assert np.all(np.abs(q - q_ref) <= q_ref * proj_tol(p_ref, dtype) * 1.01 +
                  (1e-7 if dtype == "f32" else 1e-13) * q_ref)
    want = wam.idiv(P.d, q_ref)
    assert abs(host(idv)[0] - want) <= (1e-5 if dtype == "f32" else 1e-11) * want
    b = host(c.b()).ravel()
    ref = O.T @ (H.T @ P.d)
    assert np.abs(b - ref).max() <= (2e-5 if dtype == "f32" else 1e-11) * np.abs(ref).max()


def test_slice_solve_fp64_own_tree_matches_oracle():
    """FP64 end to end with the GPU's own slice-summed expansions."""
    P, H = problem("cone32")
    g, L = P.geom, P.levels
    ref = vol3d.slice_wam_solve3(H, g.n, g.nz, L, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule)
    c = make_ctx(g, L, "f64", P.d, P.i0)
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    beta, mask, it = c.get_state()
    assert it == P.n_iters
    m = host(mask).reshape(g.nz, g.n, g.n)
    np.testing.assert_array_equal(m, vol3d.slice_mask3(ref["mask"], g.nz))
    assert rel_l2(host(beta).reshape(g.nz, g.n, g.n), ref["beta"]) <= 1e-9
    assert rel_l2(host(c.synthesize()).reshape(g.nz, g.n, g.n), ref["mu"]) <= 1e-9
    np.testing.assert_allclose(idv, ref["idiv"], rtol=1e-10)
    st = c.tree_stats()
    assert st["n_held"] == ref["held"]
    assert abs(st["z0"] - ref["z0"][-1]) <= 1e-11 * ref["z0"][-1]
    assert len(ref["trees"]) == len(P.schedule) + 1 and ref["trees"][-1][1].sum() > ref["trees"][0][1].sum()


def test_slice_solve_fp32_with_oracle_tree_sequence():
    """FP32 solve fed the oracle's tree sequence through the device tree schedule."""
    P, H = problem("cone32")
    g, L = P.geom, P.levels
    ref = vol3d.slice_wam_solve3(H, g.n, g.nz, L, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule)
    c = make_ctx(g, L, "f32", P.d, P.i0)
    at = [j for j, _ in ref["trees"]][1:]
    masks = np.stack([vol3d.slice_mask3(m, g.nz) for _, m in ref["trees"]][1:]).reshape(len(at), -1)
    c.set_tree_schedule(at, dev(masks, torch.uint8))
    idv = host(c.solve(P.n_iters, (), 0.1))
    np.testing.assert_allclose(idv, ref["idiv"], rtol=2e-5)
    assert np.all(idv[1:] <= idv[:-1] * (1 + 1e-6))
    assert rel_l2(host(c.get_state()[0]).reshape(g.nz, g.n, g.n), ref["beta"]) <= 1e-4


def test_slice_expansion_decision_matches_oracle():
    """Given the oracle's coefficients, the GPU's slice-summed rule splits the oracle's leaves
    (exactly in FP64)."""
    P, H = problem("cone32")
    g, L = P.geom, P.levels
    ref = vol3d.slice_wam_solve3(H, g.n, g.nz, L, P.d, P.i0, P.schedule[0], g.pixel)
    c = make_ctx(g, L, "f64", P.d, P.i0)
    m0 = vol3d.slice_mask3(haar.approx_mask(g.n, L), g.nz)
    c.set_state(dev(ref["beta"].ravel(), "f64"), dev(m0.ravel(), torch.uint8))
    n_split = c.expand(0.1)
    want, cnt = vol3d.expand_tree_slices3(ref["beta"], haar.approx_mask(g.n, L), L, 0.1,
                                          haar.synthesis_matrix(g.n, L))
    np.testing.assert_array_equal(host(c.get_state()[1]).reshape(g.nz, g.n, g.n), vol3d.slice_mask3(want, g.nz))
    assert n_split == cnt and cnt > 0


def test_slice_errors():
    from paper_1508_04458_amd import api, _lib
    P, H = problem("cone32")
    g = P.geom
    c = make_ctx(g, 2, "f64", P.d, P.i0)
    with pytest.raises(_lib.WamctError) as e:
        c.set_tree_rule("gradient")
    assert e.value.status == _lib.E_UNSUPPORTED
    bad = slice_tree(g.n, g.nz, 2, 30, 0.8)
    bad[3] = vol3d.slice_mask3(haar.approx_mask(g.n, 2), 1)[0]    # one slice with another tree
    with pytest.raises(_lib.WamctError) as e:
        c.set_state(dev(np.zeros(g.n_voxels), "f64"), dev(bad.ravel(), torch.uint8))
    assert e.value.status == _lib.E_INVALID
    # nz need not be divisible by 2^levels with per-slice wavelets (it must for the octree)
    g2 = synth.cone_geometry(16, 6, 5, 6, 30, sod=60.0, sdd=100.0)
    assert api.validate(g2, 2, "f64", wavelet_dims=2) is None
    assert api.validate(g2, 2, "f64") is not None
    assert api.validate(g2, 2, "f64", wavelet_dims=5) is not None


# ------------------------------------------------------------------ benchmark size

def _cone512():
    return synth.CONE_CONFIGS["cone512"]["geom"]()


def test_cone512_slices_forward_sampled_rays():
    """The cone512 geometry (188.7 M rays, 512 x 512 x 256, 3 levels per slice), FP32, on 400
    sampled rays through Omega beta of a random shared tree (oracle: every slice synthesized by
    the textbook 2-D cascade, 3-D Siddon of the sampled rays)."""
    from test_gpu_cone512 import I0, at, sample_rays
    g, L = _cone512(), 3
    mask2 = synth.random_tree_mask(g.n, L, 61, p_split=0.55)
    rng = np.random.default_rng(61)
    beta = rng.standard_normal((g.nz, g.n, g.n), dtype=np.float32) * np.float32(0.002) * mask2[None]
    r = g.n >> L
    beta[:, :r, :r] = (0.02 * (1 << L) + rng.uniform(0, 0.01, (g.nz, r, r))).astype(np.float32)
    c = make_ctx(g, L, "f32")
    c.set_data(torch.full((g.n_rays,), 0.5 * I0, dtype=torch.float32, device="cuda"), I0)
    c.set_state(torch.from_numpy(beta.ravel()).cuda(), torch.from_numpy(vol3d.slice_mask3(mask2, g.nz).ravel()).cuda())
    q, _ = c.forward()
    ids = sample_rays(g, 400, 62)
    print(f"[cone512 slices] oracle: {ids.size} sampled rays", flush=True)
    vol = np.stack([haar.cascade_synthesis(beta[s].astype(np.float64), L) for s in range(g.nz)])
    p_ref = vol3d.project_rays3(g, vol, ids)
    q_ref = I0 * np.exp(-p_ref)
    got = at(q, ids)
    tol = q_ref * (1e-5 * np.maximum(np.abs(p_ref), 1e-3 * p_ref.max()) + 2e-7)
    assert np.all(np.abs(got - q_ref) <= tol), np.max(np.abs(got - q_ref) / q_ref)


def test_cone512_slices_split_backprojection_sampled_nodes():
    """Sign-split backprojection at sampled per-slice nodes of every level (each node's phi
    over every ray of its detector shadow, by quadrant clipping), 1e-5 of the larger sum."""
    g, L = _cone512(), 3
    n, nz = g.n, g.nz
    mask2 = synth.random_tree_mask(n, L, 63, p_split=0.6)
    c = make_ctx(g, L, "f32")
    c.set_state(torch.zeros(g.n_voxels, dtype=torch.float32, device="cuda"),
                torch.from_numpy(vol3d.slice_mask3(mask2, nz).ravel()).cuda())
    y = np.random.default_rng(63).random(g.n_rays, dtype=np.float32)
    bp, bm = (host(t).reshape(nz, n, n) for t in c.backproject_split(torch.from_numpy(y).cuda()))
    exy, ez = vol3d.edges3(g)
    rng = np.random.default_rng(64)
    checked = 0
    for lev in range(L, 0, -1):
        m, s_ = n >> lev, 1 << lev
        split = haar.split_flags(mask2, lev)
        cand = np.argwhere(split)
        for i, j in cand[rng.choice(len(cand), min(3, len(cand)), replace=False)]:
            s = int(rng.integers(0, nz))
            lo = np.array([exy[j * s_], exy[i * s_], ez[s]])
            hi = np.array([exy[(j + 1) * s_], exy[(i + 1) * s_], ez[s + 1]])
            ids = vol3d.box_shadow3(g, lo, hi)
            o, e = vol3d.rays3(g, ids=ids)
            phis = vol3d.slice_node_phi3(g, o, e, lev, s, i, j)
            print(f"[cone512 slices] node ({lev}, {s}, {i}, {j}): {ids.size} rays", flush=True)
            yy = y[ids].astype(np.float64)
            for (zr, zc), ph in zip(((i, m + j), (m + i, j), (m + i, m + j)), phis):
                ph = np.where(np.abs(ph) <= 1e-12 * g.pixel, 0.0, ph)
                rp, rm = float(yy @ np.maximum(ph, 0.0)), float(yy @ np.minimum(ph, 0.0))
                scale = max(abs(rp), abs(rm), 1e-30)
                assert abs(bp[s, zr, zc] - rp) <= 1e-5 * scale, (lev, s, i, j, bp[s, zr, zc], rp)
                assert abs(bm[s, zr, zc] - rm) <= 1e-5 * scale, (lev, s, i, j, bm[s, zr, zc], rm)
                checked += 1
    assert checked >= 27
