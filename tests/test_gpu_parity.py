"""HIP path vs the FP64 CPU oracle, element by element on seeded inputs.

Tolerances (floating point; stated with their reasons in the design notes):
  * projections: |dp| <= 1e-5 max(|p|, 1e-3 max p) per ray in FP32, 1e-11 in FP64;
  * images after K iterations: relative L2 <= 1e-4 (FP32), 1e-9 (FP64);
  * backprojections (sums of ~10^3-10^4 FP32 terms): |d| <= 2e-5 max|x| per element;
  * tree masks: bit-exact, except leaves within 1e-6 (relative) of the threshold.
"""
import math

import numpy as np
import pytest
import torch

from oracle import geometry, haar, siddon, wam
from paper_1508_04458_amd import synth

pytestmark = pytest.mark.gpu

TORCH_DT = {"f32": torch.float32, "f64": torch.float64}


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=TORCH_DT[dtype] if isinstance(dtype, str) else dtype,
                           device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy() if t.is_floating_point() else t.detach().cpu().numpy()


def make_ctx(geom, levels, dtype, d=None, i0=None):
    from paper_1508_04458_amd import api
    print(f"\n[case] n={geom.n} views={geom.n_views} bins={geom.n_bins} kind={geom.kind} L={levels} {dtype}", flush=True)
    c = api.Context(geom, levels, dtype)
    if d is not None:
        c.set_data(dev(d, dtype), i0)
    return c


_CACHE = {}


def problem(name):
    if name not in _CACHE:
        P = synth.make_problem(name)
        _CACHE[name] = (P, siddon.system_matrix(P.geom))
    return _CACHE[name]


def proj_tol(p_ref, dtype):
    rel = 1e-5 if dtype == "f32" else 1e-11
    return rel * np.maximum(np.abs(p_ref), 1e-3 * np.abs(p_ref).max())


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------------ operators

@pytest.mark.parametrize("name,dtype", [("parallel64", "f64"), ("parallel64", "f32"), ("fan96", "f32"),
                                        ("fan128", "f32"), ("fan96", "f64")])
def test_project_matches_oracle(name, dtype):
    P, H = problem(name)
    g = P.geom
    c = make_ctx(g, 0, dtype)
    for img in (synth.random_image(g.n, 1), synth.rasterize(P.ellipses, g.n, g.pixel)):
        p = host(c.project(dev(img.ravel(), dtype)))
        ref = H @ img.ravel()
        assert np.all(np.abs(p - ref) <= proj_tol(ref, dtype)), np.abs(p - ref).max()


def test_project_rays_missing_the_image():
    g = synth.parallel_geometry(32, 7, 90, 1.0)          # detector much wider than the image
    c = make_ctx(g, 0, "f64")
    img = synth.random_image(32, 2)
    p = host(c.project(dev(img.ravel(), "f64")))
    ref = siddon.system_matrix(g) @ img.ravel()
    assert np.all(p[ref == 0] == 0) and (ref == 0).sum() > 100
    assert np.abs(p - ref).max() <= 1e-11 * ref.max()


@pytest.mark.parametrize("name,dtype", [("parallel64", "f64"), ("fan96", "f32"), ("fan128", "f32")])
def test_backproject_matches_oracle(name, dtype):
    P, H = problem(name)
    g = P.geom
    c = make_ctx(g, 0, dtype)
    y = synth.random_vector(g.n_rays, 3)
    img = host(c.backproject(dev(y, dtype))).ravel()
    ref = H.T @ y
    tol = (2e-5 if dtype == "f32" else 1e-11) * np.abs(ref).max()
    assert np.abs(img - ref).max() <= tol
    # adjoint identity between the GPU's own forward (leaf walk) and backward (box clipping)
    x = synth.random_image(g.n, 4).ravel()
    hx = host(c.project(dev(x, dtype)))
    lhs, rhs = float(hx @ y), float(x @ img)
    assert abs(lhs - rhs) <= (1e-5 if dtype == "f32" else 1e-11) * abs(lhs)


@pytest.mark.parametrize("name,levels,dtype,seed", [("parallel64", 1, "f64", 0), ("parallel64", 3, "f64", 1),
                                                    ("fan96", 2, "f32", 2), ("fan128", 3, "f32", 3),
                                                    ("fan128", 3, "f64", 4), ("parallel64", 6, "f64", 20),
                                                    ("fan128", 7, "f64", 15), ("fan128", 5, "f32", 15)])
def test_split_backprojection_matches_oracle(name, levels, dtype, seed):
    """Random trees of 1 to 7 levels: up to 7 level segments, gathered in one launch."""
    P, H = problem(name)
    g = P.geom
    mask = synth.random_tree_mask(g.n, levels, seed, p_split=0.6)
    c = make_ctx(g, levels, dtype)
    beta = np.zeros((g.n, g.n))
    c.set_state(dev(beta.ravel(), dtype), dev(mask.ravel(), torch.uint8))
    y = synth.random_vector(g.n_rays, seed)
    bp, bm = (host(t) for t in c.backproject_split(dev(y, dtype)))
    O = haar.synthesis_matrix(g.n, levels)
    Phi, act = wam.phi_matrix(H, O, mask, g.pixel)
    Pp, Pm = wam.split_phi(Phi)
    rp = np.zeros(g.n * g.n)
    rm = np.zeros(g.n * g.n)
    rp[act] = Pp.T @ y
    rm[act] = Pm.T @ y
    scale = max(np.abs(rp).max(), np.abs(rm).max())
    tol = (2e-5 if dtype == "f32" else 1e-11) * scale
    assert np.abs(bp.ravel() - rp).max() <= tol
    assert np.abs(bm.ravel() - rm).max() <= tol
    assert bp.min() >= 0 and bm.max() <= 0
    inactive = mask.ravel() == 0
    assert np.all(bp.ravel()[inactive] == 0) and np.all(bm.ravel()[inactive] == 0)


@pytest.mark.parametrize("name,dtype", [("parallel64", "f64"), ("fan96", "f32")])
def test_b_precompute_matches_oracle(name, dtype):
    P, H = problem(name)
    g = P.geom
    c = make_ctx(g, P.levels, dtype, P.d, P.i0)
    b = host(c.b()).ravel()
    ref = haar.synthesis_matrix(g.n, P.levels).T @ (H.T @ P.d)
    tol = (2e-5 if dtype == "f32" else 1e-11) * np.abs(ref).max()
    assert np.abs(b - ref).max() <= tol


@pytest.mark.parametrize("name,levels,dtype,seed", [("parallel64", 1, "f64", 5), ("fan96", 2, "f32", 6),
                                                    ("fan128", 3, "f32", 7), ("parallel64", 6, "f64", 20),
                                                    ("fan128", 7, "f64", 24)])
def test_z0_and_w_match_oracle(name, levels, dtype, seed):
    P, H = problem(name)
    g = P.geom
    O = haar.synthesis_matrix(g.n, levels)
    c = make_ctx(g, levels, dtype)
    for mask in (haar.approx_mask(g.n, levels), synth.random_tree_mask(g.n, levels, seed),
                 haar.full_mask(g.n)):
        c.set_state(dev(np.zeros(g.n * g.n), dtype), dev(mask.ravel(), torch.uint8))
        st = c.tree_stats()
        Phi, act = wam.phi_matrix(H, O, mask, g.pixel)
        assert abs(st["z0"] - wam.z0_of(Phi)) <= 1e-11 * st["z0"]
        assert abs(st["w"] - Phi.nnz) <= 1e-4 * Phi.nnz
        assert st["n_active"] == act.size


# ------------------------------------------------------------------ one step of Algorithm 1

def _random_state(g, levels, seed):
    mask = synth.random_tree_mask(g.n, levels, seed, p_split=0.5)
    rng = np.random.default_rng(seed)
    beta = rng.normal(0, 0.002, (g.n, g.n)) * mask
    nL = g.n >> levels
    beta[:nL, :nL] = 0.02 * (1 << levels) + rng.uniform(0, 0.01, (nL, nL))
    return beta, mask


@pytest.mark.parametrize("name,dtype,seed", [("parallel64", "f64", 8), ("fan96", "f32", 9), ("fan128", "f32", 10),
                                             ("fan128", "f64", 11)])
def test_forward_and_one_update_match_oracle(name, dtype, seed):
    P, H = problem(name)
    g = P.geom
    L = P.levels
    beta, mask = _random_state(g, L, seed)
    c = make_ctx(g, L, dtype, P.d, P.i0)
    c.set_state(dev(beta.ravel(), dtype), dev(mask.ravel(), torch.uint8))
    q, idv = c.forward()
    O = haar.synthesis_matrix(g.n, L)
    p_ref = H @ (O @ beta.ravel())
    q_ref = wam.beer_mean(P.i0, p_ref)
    q = host(q)
    # q = I0 exp(-p): relative error of q is the absolute error of p
    assert np.all(np.abs(q - q_ref) <= q_ref * proj_tol(p_ref, dtype) * 1.01 + (1e-7 if dtype == "f32" else 1e-13) * q_ref)
    assert abs(host(idv)[0] - wam.idiv(P.d, q_ref)) <= (1e-5 if dtype == "f32" else 1e-11) * wam.idiv(P.d, q_ref)
    c.iterate(1)
    b1, m1, it = c.get_state()
    ref = wam.wam_solve(H, g.n, L, P.d, P.i0, 1, g.pixel, beta0=beta, mask0=mask, Omega=O)
    assert it == 1 and np.array_equal(host(m1), mask)
    err = rel_l2(host(b1), ref["beta"])
    assert err <= (1e-4 if dtype == "f32" else 1e-10), err


# ------------------------------------------------------------------ full runs

def test_solve_parity_parallel64_fp64_own_tree():
    """FP64 end to end with the GPU taking its own expansion decisions (config: 64x64
    parallel, 1-level tree, 20 iterations, expansion at iteration 4)."""
    P, H = problem("parallel64")
    g = P.geom
    ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule)
    c = make_ctx(g, P.levels, "f64", P.d, P.i0)
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    beta, mask, it = c.get_state()
    assert it == P.n_iters
    np.testing.assert_array_equal(host(mask), ref["mask"])
    assert rel_l2(host(beta), ref["beta"]) <= 1e-9
    assert rel_l2(host(c.synthesize()), ref["mu"]) <= 1e-9
    np.testing.assert_allclose(idv, ref["idiv"], rtol=1e-10)
    assert c.tree_stats()["n_held"] == 0


def test_solve_parity_fan128_fp32_oracle_tree_sequence():
    """FP32 end to end on a 128x128 fan-beam case with the tree sequence Z_s^(j) fed in
    from the oracle (Algorithm 1 takes it as an input), 30 iterations, 3 levels."""
    P, H = problem("fan128")
    g = P.geom
    ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule)
    c = make_ctx(g, P.levels, "f32", P.d, P.i0)
    trees = dict(ref["trees"])
    idv = torch.empty(P.n_iters + 1, dtype=torch.float64, device="cuda")
    j = 0
    marks = sorted(trees) + [P.n_iters]
    for a, b in zip(marks[:-1], marks[1:]):
        beta, _, _ = c.get_state()
        c.set_state(beta.reshape(-1).contiguous(), dev(trees[a].ravel(), torch.uint8))
        c.iterate(b - a, idv[a:b])
    q, last = c.forward()
    idv[P.n_iters:] = last
    beta, mask, _ = c.get_state()
    assert rel_l2(host(c.synthesize()), ref["mu"]) <= 1e-4
    assert rel_l2(host(beta), ref["beta"]) <= 1e-4
    np.testing.assert_allclose(host(idv), ref["idiv"], rtol=2e-5)


def test_gpu_expansion_decisions_match_oracle():
    """Given the same coefficients, the GPU's tree rule splits the same leaves, except
    leaves whose value is within 1e-6 (relative) of the threshold."""
    P, H = problem("fan128")
    g = P.geom
    L = P.levels
    ref = wam.wam_solve(H, g.n, L, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule, record_beta=True)
    O = haar.synthesis_matrix(g.n, L)
    for dtype in ("f64", "f32"):
        c = make_ctx(g, L, dtype, P.d, P.i0)
        for (j, m_prev), (j2, m_next) in zip(ref["trees"][:-1], ref["trees"][1:]):
            beta = ref["betas"][j2 - 1]
            c.set_state(dev(beta, dtype), dev(m_prev.ravel(), torch.uint8))
            c.expand(0.1)
            _, mg, _ = c.get_state()
            mg = host(mg)
            if dtype == "f32":
                beta = beta.astype(np.float32).astype(np.float64)
            mu = (O @ beta).reshape(g.n, g.n)
            thr = 0.1 * mu.max()
            diff = np.argwhere(mg != m_next)
            for r, cc in diff:
                # locate the node of this Mallat position and check it is a tie
                k = max(r, cc)
                lev = next(t for t in range(1, L + 1) if k >= (g.n >> t))
                m = g.n >> lev
                i, jj = r % m, cc % m
                s = 1 << lev
                val = mu[i * s:(i + 1) * s, jj * s:(jj + 1) * s].max()
                assert abs(val - thr) <= 1e-6 * max(1.0, abs(thr)), (dtype, lev, i, jj, val, thr)
            if dtype == "f64":
                assert len(diff) == 0


def test_monotone_idiv_fan128_own_tree():
    P, _ = problem("fan128")
    c = make_ctx(P.geom, P.levels, "f32", P.d, P.i0)
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    assert np.all(idv[1:] <= idv[:-1] * (1 + 1e-6)), np.max(idv[1:] / idv[:-1])
    assert c.tree_stats()["n_held"] == 0


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_pixel_am_levels0_matches_oracle(dtype):
    P, H = problem("fan96")
    g = P.geom
    ref = wam.am_solve(H, g.n, P.d, P.i0, 15, g.pixel)
    c = make_ctx(g, 0, dtype, P.d, P.i0)
    idv = host(c.solve(15))
    assert rel_l2(host(c.synthesize()), ref["mu"]) <= (1e-4 if dtype == "f32" else 1e-9)
    np.testing.assert_allclose(idv, ref["idiv"], rtol=2e-5 if dtype == "f32" else 1e-10)


def test_per_ray_i0_equals_scalar():
    P, _ = problem("fan96")
    g = P.geom
    a = make_ctx(g, 2, "f32", P.d, P.i0)
    b = make_ctx(g, 2, "f32")
    b.set_data(dev(P.d, "f32"), dev(np.full(g.n_rays, P.i0), "f32"))
    ia = host(a.solve(6, [2], 0.1))
    ib = host(b.solve(6, [2], 0.1))
    np.testing.assert_array_equal(ia, ib)
    np.testing.assert_array_equal(host(a.get_state()[0]), host(b.get_state()[0]))


def test_runs_are_bitwise_deterministic():
    P, _ = problem("fan128")
    out = []
    for _ in range(2):
        c = make_ctx(P.geom, P.levels, "f32", P.d, P.i0)
        idv = host(c.solve(12, [3, 6, 9], 0.1))
        out.append((idv, host(c.get_state()[0])))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_zero_counts_hold_every_coefficient():
    """d = 0: b = 0 and the surrogate has no finite minimizer for the approximations
    (t = b / b-hat+ = 0); every update is held and counted, nothing becomes NaN."""
    g = synth.fan_geometry(32, 20, 48)
    c = make_ctx(g, 1, "f32", np.zeros(g.n_rays), 100.0)
    c.iterate(2)
    beta, _, _ = c.get_state()
    assert np.all(host(beta) == 0)
    st = c.tree_stats()
    assert st["n_held"] == 2 * (32 >> 1) ** 2


def test_state_and_data_validation_errors():
    from paper_1508_04458_amd import _lib
    g = synth.fan_geometry(32, 20, 48)
    c = make_ctx(g, 2, "f32")
    with pytest.raises(_lib.WamctError) as e:
        c.iterate(1)
    assert e.value.status == _lib.E_STATE
    bad = synth.random_tree_mask(32, 2, 1)
    bad[0, 31] = 1 - bad[0, 31]                      # one detail of a node without its siblings
    with pytest.raises(_lib.WamctError) as e:
        c.set_state(dev(np.zeros(32 * 32), "f32"), dev(bad.ravel(), torch.uint8))
    assert e.value.status == _lib.E_INVALID
    d = np.ones(g.n_rays)
    d[5] = -1
    with pytest.raises(_lib.WamctError) as e:
        c.set_data(dev(d, "f32"), 100.0)
    assert e.value.status == _lib.E_INVALID
    d[5] = np.nan
    with pytest.raises(_lib.WamctError):
        c.set_data(dev(d, "f32"), 100.0)
    with pytest.raises(_lib.WamctError):
        c.set_data(dev(np.ones(g.n_rays), "f32"), -3.0)


def test_forward_tree_large_non_power_of_two_image():
    """Leaf walk on a 1200x1200 image with a random 4-level tree (75x75 roots)."""
    g = synth.parallel_geometry(1200, 5, 1700, 1.0)
    L = 4
    mask = synth.random_tree_mask(g.n, L, 21, p_split=0.5)
    rng = np.random.default_rng(21)
    beta = rng.normal(0, 0.002, (g.n, g.n)) * mask
    nL = g.n >> L
    beta[:nL, :nL] = 0.02 * (1 << L)
    c = make_ctx(g, L, "f32", np.ones(g.n_rays), 100.0)
    c.set_state(dev(beta.ravel(), "f32"), dev(mask.ravel(), torch.uint8))
    q, _ = c.forward()
    H = siddon.system_matrix(g)
    p_ref = H @ (haar.synthesis_matrix(g.n, L) @ beta.astype(np.float32).astype(np.float64).ravel())
    p = -np.log(host(q) / 100.0)
    # q is stored in FP32: compare p through q with the FP32 storage error of q added
    assert np.all(np.abs(p - p_ref) <= proj_tol(p_ref, "f32") + 2e-7), np.abs(p - p_ref).max()


def test_fp32_ray_geometry_matches_oracle():
    """The FP32 ray-geometry build (wamct_options.geometry = F32). Ray parameters reach the
    image half-diagonal (~90 mm for fan128), so FP32 rounding puts ~5e-6 mm on every plane
    parameter: an absolute error per chord, at most ~2n crossings x 5e-6 mm x max mu (0.2)
    ~ 2.6e-4 per ray, so projections are held to 5e-5 x max p (~3e-4) in absolute terms;
    after 8 iterations beta and the I-divergence meet the FP32-data bars (relative L2 1e-4,
    rtol 2e-5): the chord errors are far below the FP32 storage of q-hat and beta."""
    from paper_1508_04458_amd import api
    P, H = problem("fan128")
    g = P.geom
    print(f"\n[case] fan128 FP32 ray geometry", flush=True)
    c = api.Context(g, 0, "f32", geometry="f32")
    img = synth.rasterize(P.ellipses, g.n, g.pixel)
    p = host(c.project(dev(img.ravel(), "f32")))
    ref = H @ img.ravel()
    assert np.abs(p - ref).max() <= 5e-5 * np.abs(ref).max()
    c2 = api.Context(g, P.levels, "f32", geometry="f32")
    c2.set_data(dev(P.d, "f32"), P.i0)
    J = 8
    idv = host(c2.solve(J))
    ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, J, g.pixel)
    err = rel_l2(host(c2.get_state()[0]), ref["beta"])
    print(f"beta rel L2 {err:.2e}, idiv max rel {np.max(np.abs(idv / ref['idiv'] - 1)):.2e}", flush=True)
    assert err <= 1e-4
    np.testing.assert_allclose(idv, ref["idiv"], rtol=2e-5)


def test_golden_hand_example_on_the_gpu():
    """The smallest problem (2x2 image, 4 views x 2 bins, one Haar level), against the values
    derived by hand in tests/golden/tiny2x2_parallel.txt: H column by column, Phi row by row
    (split backprojection of unit ray vectors on the full tree), Z0 of the approximation-only
    tree, the full tree and pixel AM, and one update of each kind. FP64 at 1e-12."""
    from golden_io import load
    gold = load("tiny2x2_parallel.txt")
    g = synth.parallel_geometry(2, 4, 2, 1.0)
    c0 = make_ctx(g, 0, "f64")
    for x in range(4):
        e = np.zeros(4)
        e[x] = 1.0
        col = host(c0.project(dev(e, "f64")))
        np.testing.assert_allclose(col, [gold[f"H_row {r}"][x] for r in range(8)], atol=1e-12)
    c = make_ctx(g, 1, "f64", np.full(8, 50.0), 100.0)
    assert abs(c.tree_stats()["z0"] - gold["Z0_approx"][0]) <= 1e-12
    c.set_state(dev(np.zeros(4), "f64"), dev(haar.full_mask(2).ravel(), torch.uint8))
    assert abs(c.tree_stats()["z0"] - gold["Z0_full"][0]) <= 1e-12
    for r in range(8):
        y = np.zeros(8)
        y[r] = 1.0
        bp, bm = (host(t).ravel() for t in c.backproject_split(dev(y, "f64")))
        np.testing.assert_allclose(bp + bm, gold[f"Phi_row {r}"], atol=1e-12)
        np.testing.assert_allclose(bp, np.maximum(gold[f"Phi_row {r}"], 0), atol=1e-12)
    c1 = make_ctx(g, 1, "f64", np.full(8, 50.0), 100.0)
    c1.iterate(1)
    np.testing.assert_allclose(host(c1.synthesize()).ravel(), gold["step_approx_mu"][0], rtol=1e-12)
    cp = make_ctx(g, 0, "f64", np.asarray(gold["step_pixel_d"]), 100.0)
    assert abs(cp.tree_stats()["z0"] - gold["Z0_pixel"][0]) <= 1e-12
    cp.iterate(1)
    np.testing.assert_allclose(host(cp.synthesize()).ravel(), gold["step_pixel_mu"], rtol=1e-12)


def test_scan_that_misses_the_image_is_rejected():
    """No ray crosses the image (every bin outside it): Z0 = 0, the update is undefined, and
    creating the context fails with WAMCT_E_INVALID (tree and pixel AM alike)."""
    from paper_1508_04458_amd import _lib
    g = synth.parallel_geometry(8, 3, 2, 100.0)        # bins at u = -50 and +50 mm
    for levels in (0, 1):
        with pytest.raises(_lib.WamctError) as e:
            make_ctx(g, levels, "f64")
        assert e.value.status == _lib.E_INVALID and "Z0 = 0" in str(e.value)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_walk_lanes_all_match_oracle(dtype):
    """The leaf walk cut into 1, 2 or 4 pieces per ray (the autotuner's second knob) gives
    the oracle's projections each time; invalid lane counts are rejected."""
    from paper_1508_04458_amd import _lib
    P, H = problem("fan128")
    g = P.geom
    L = P.levels
    beta, mask = _random_state(g, L, 21)
    O = haar.synthesis_matrix(g.n, L)
    p_ref = H @ (O @ beta.ravel())
    q_ref = wam.beer_mean(P.i0, p_ref)
    c = make_ctx(g, L, dtype, P.d, P.i0)
    c.set_state(dev(beta.ravel(), dtype), dev(mask.ravel(), torch.uint8))
    assert c.walk_lanes() == 4          # 46,080 rays (< 2^17): four lanes per ray by default
    for k in (1, 2, 4):
        c.set_walk_lanes(k)
        assert c.walk_lanes() == k
        q = host(c.forward()[0])
        assert np.all(np.abs(q - q_ref) <= q_ref * proj_tol(p_ref, dtype) * 1.01 +
                      (1e-7 if dtype == "f32" else 1e-13) * q_ref), k
    for bad in (3, 8, -1):
        with pytest.raises(_lib.WamctError):
            c.set_walk_lanes(bad)
    full = make_ctx(g, 0, dtype)
    with pytest.raises(_lib.WamctError) as e:
        full.set_walk_lanes(2)
    assert e.value.status == _lib.E_UNSUPPORTED
