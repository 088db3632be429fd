"""Daubechies-4 (periodic) wavelets on the GPU vs the FP64 oracle (oracle.daub's Omega in
oracle.wam), element by element on seeded inputs.

Tolerances: FP64 operators 1e-11 of the largest value, FP32 2e-5 (sums of ~10^3-10^4
terms); iterates after K updates: relative L2 1e-9 (FP64), 1e-4 (FP32); FP64 trees of the
GPU's own expansions bit-exact; expansion decisions exact except leaves whose block maximum is
within 1e-6 (relative) of the threshold.
"""
import numpy as np
import pytest
import torch

from oracle import daub, haar, siddon, wam
from paper_1508_04458_amd import synth

pytestmark = pytest.mark.gpu

TORCH_DT = {"f32": torch.float32, "f64": torch.float64}


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=TORCH_DT[dtype] if isinstance(dtype, str) else dtype,
                           device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy() if t.is_floating_point() else t.detach().cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


_CACHE = {}


def problem(name):
    if name not in _CACHE:
        P = synth.make_problem(name)
        _CACHE[name] = (P, siddon.system_matrix(P.geom))
    return _CACHE[name]


_OMEGA = {}


def omega(n, levels):
    if (n, levels) not in _OMEGA:
        _OMEGA[(n, levels)] = daub.synthesis_matrix(n, levels)
    return _OMEGA[(n, levels)]


def make_ctx(geom, levels, dtype, d=None, i0=None):
    from paper_1508_04458_amd import api
    print(f"\n[case] d4 n={geom.n} views={geom.n_views} bins={geom.n_bins} kind={geom.kind} L={levels} {dtype}",
          flush=True)
    c = api.Context(geom, levels, dtype, wavelet="d4")
    if d is not None:
        c.set_data(dev(d, dtype), i0)
    return c


def tol(dtype):
    return 2e-5 if dtype == "f32" else 1e-11


CASES = [("parallel64", 3, "f64", 1), ("parallel64", 2, "f32", 2), ("fan96", 2, "f32", 3), ("fan96", 3, "f64", 4),
         ("fan96", 1, "f64", 5)]


@pytest.mark.parametrize("name,levels,dtype,seed", CASES)
def test_synthesis_matches_oracle(name, levels, dtype, seed):
    P, _ = problem(name)
    n = P.geom.n
    c = make_ctx(P.geom, levels, dtype)
    beta = np.random.default_rng(seed).normal(0.0, 1.0, (n, n))
    c.set_state(dev(beta.ravel(), dtype), dev(haar.full_mask(n).ravel(), torch.uint8))
    mu = host(c.synthesize()).ravel()
    if dtype == "f32":
        beta = beta.astype(np.float32).astype(np.float64)
    ref = omega(n, levels) @ beta.ravel()
    assert np.abs(mu - ref).max() <= (1e-6 if dtype == "f32" else 1e-12) * np.abs(ref).max()


@pytest.mark.parametrize("name,levels,dtype", [("parallel64", 3, "f64"), ("fan96", 2, "f32"), ("fan96", 3, "f64")])
def test_b_precompute_matches_oracle(name, levels, dtype):
    P, H = problem(name)
    c = make_ctx(P.geom, levels, dtype, P.d, P.i0)
    b = host(c.b()).ravel()
    ref = omega(P.geom.n, levels).T @ (H.T @ P.d)
    assert np.abs(b - ref).max() <= tol(dtype) * np.abs(ref).max()


@pytest.mark.parametrize("name,levels,dtype,seed", CASES)
def test_split_backprojection_matches_oracle(name, levels, dtype, seed):
    P, H = problem(name)
    g = P.geom
    mask = synth.random_tree_mask(g.n, levels, seed, p_split=0.6)
    c = make_ctx(g, levels, dtype)
    c.set_state(dev(np.zeros(g.n * g.n), dtype), dev(mask.ravel(), torch.uint8))
    y = synth.random_vector(g.n_rays, seed)
    bp, bm = (host(t).ravel() for t in c.backproject_split(dev(y, dtype)))
    Phi, act = wam.phi_matrix(H, omega(g.n, levels), mask, g.pixel)
    Pp, Pm = wam.split_phi(Phi)
    rp = np.zeros(g.n * g.n)
    rm = np.zeros(g.n * g.n)
    rp[act] = Pp.T @ y
    rm[act] = Pm.T @ y
    scale = max(np.abs(rp).max(), np.abs(rm).max())
    assert np.abs(bp - rp).max() <= tol(dtype) * scale
    assert np.abs(bm - rm).max() <= tol(dtype) * scale
    assert bp.min() >= 0 and bm.max() <= 0
    inactive = mask.ravel() == 0
    assert np.all(bp[inactive] == 0) and np.all(bm[inactive] == 0)


@pytest.mark.parametrize("name,levels,dtype,seed", [("parallel64", 3, "f64", 6), ("fan96", 2, "f32", 7),
                                                    ("fan96", 3, "f64", 8)])
def test_z0_and_w_match_oracle(name, levels, dtype, seed):
    P, H = problem(name)
    g = P.geom
    O = omega(g.n, levels)
    c = make_ctx(g, levels, dtype)
    for mask in (haar.approx_mask(g.n, levels), synth.random_tree_mask(g.n, levels, seed),
                 haar.full_mask(g.n)):
        c.set_state(dev(np.zeros(g.n * g.n), dtype), dev(mask.ravel(), torch.uint8))
        st = c.tree_stats()
        Phi, act = wam.phi_matrix(H, O, mask, g.pixel)
        assert abs(st["z0"] - wam.z0_of(Phi)) <= 1e-11 * st["z0"]
        assert abs(st["w"] - Phi.nnz) <= 1e-4 * Phi.nnz
        assert st["n_active"] == act.size


def _random_state(g, levels, seed):
    mask = synth.random_tree_mask(g.n, levels, seed, p_split=0.5)
    rng = np.random.default_rng(seed)
    beta = rng.normal(0, 0.002, (g.n, g.n)) * mask
    nL = g.n >> levels
    beta[:nL, :nL] = 0.02 * (1 << levels) + rng.uniform(0, 0.01, (nL, nL))
    return beta, mask


@pytest.mark.parametrize("name,levels,dtype,seed", [("parallel64", 3, "f64", 9), ("fan96", 2, "f32", 10),
                                                    ("fan96", 3, "f64", 11)])
def test_forward_and_one_update_match_oracle(name, levels, dtype, seed):
    P, H = problem(name)
    g = P.geom
    O = omega(g.n, levels)
    beta, mask = _random_state(g, levels, seed)
    c = make_ctx(g, levels, dtype, P.d, P.i0)
    c.set_state(dev(beta.ravel(), dtype), dev(mask.ravel(), torch.uint8))
    q, idv = c.forward()
    bref = beta.astype(np.float32).astype(np.float64) if dtype == "f32" else beta
    p_ref = H @ (O @ bref.ravel())
    q_ref = wam.beer_mean(P.i0, p_ref)
    q = host(q)
    rel = 2e-6 if dtype == "f32" else 1e-12
    assert np.all(np.abs(q - q_ref) <= rel * q_ref * np.maximum(1.0, p_ref))
    assert abs(host(idv)[0] - wam.idiv(P.d, q_ref)) <= (1e-5 if dtype == "f32" else 1e-11) * wam.idiv(P.d, q_ref)
    c.iterate(1)
    b1, m1, it = c.get_state()
    ref = wam.wam_solve(H, g.n, levels, P.d, P.i0, 1, g.pixel, beta0=bref, mask0=mask, Omega=O)
    assert it == 1 and np.array_equal(host(m1), mask)
    err = rel_l2(host(b1), ref["beta"])
    assert err <= (1e-4 if dtype == "f32" else 1e-10), err
    assert c.tree_stats()["n_held"] == ref["held"]


@pytest.mark.parametrize("name,levels", [("parallel64", 3), ("fan96", 2), ("fan96", 3)])
def test_solve_parity_fp64_own_tree(name, levels):
    """FP64 end to end with the GPU taking its own expansion decisions (block-maximum rule)."""
    P, H = problem(name)
    g = P.geom
    O = omega(g.n, levels)
    ref = wam.wam_solve(H, g.n, levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule, Omega=O)
    c = make_ctx(g, levels, "f64", P.d, P.i0)
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    beta, mask, it = c.get_state()
    assert it == P.n_iters
    np.testing.assert_array_equal(host(mask), ref["mask"])
    assert rel_l2(host(beta), ref["beta"]) <= 1e-9
    assert rel_l2(host(c.synthesize()), ref["mu"]) <= 1e-9
    np.testing.assert_allclose(idv, ref["idiv"], rtol=1e-10)
    st = c.tree_stats()
    assert st["n_held"] == ref["held"]
    assert abs(st["z0"] - ref["z0"][-1]) <= 1e-11 * ref["z0"][-1]
    assert st["w"] == ref["w"][-1]


def test_solve_parity_fan96_fp32_oracle_tree_sequence():
    """FP32 end to end with the oracle's tree sequence Z_s^(j) fed in (Algorithm 1 takes it
    as an input)."""
    P, H = problem("fan96")
    g = P.geom
    L = 3
    ref = wam.wam_solve(H, g.n, L, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule, Omega=omega(g.n, L))
    c = make_ctx(g, L, "f32", P.d, P.i0)
    trees = dict(ref["trees"])
    idv = torch.empty(P.n_iters + 1, dtype=torch.float64, device="cuda")
    marks = sorted(trees) + [P.n_iters]
    for a, b in zip(marks[:-1], marks[1:]):
        beta, _, _ = c.get_state()
        c.set_state(beta.reshape(-1).contiguous(), dev(trees[a].ravel(), torch.uint8))
        c.iterate(b - a, idv[a:b])
    _, last = c.forward()
    idv[P.n_iters:] = last
    beta, _, _ = c.get_state()
    assert rel_l2(host(beta), ref["beta"]) <= 1e-4
    assert rel_l2(host(c.synthesize()), ref["mu"]) <= 1e-4
    np.testing.assert_allclose(host(idv), ref["idiv"], rtol=2e-5)


def test_expansion_decisions_match_oracle():
    """Given the same coefficients, the GPU's block-maximum rule splits the oracle's leaves
    (except ties within 1e-6 of the threshold)."""
    P, H = problem("fan96")
    g = P.geom
    L = 3
    O = omega(g.n, L)
    ref = wam.wam_solve(H, g.n, L, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule, Omega=O, record_beta=True)
    assert len(ref["trees"]) >= 2
    for dtype in ("f64", "f32"):
        c = make_ctx(g, L, dtype, P.d, P.i0)
        for (j, m_prev), (j2, m_next) in zip(ref["trees"][:-1], ref["trees"][1:]):
            beta = ref["betas"][j2 - 1]
            c.set_state(dev(beta, dtype), dev(m_prev.ravel(), torch.uint8))
            c.expand(0.1)
            mg = host(c.get_state()[1])
            if dtype == "f32":
                beta = beta.astype(np.float32).astype(np.float64)
            exp_mask, _ = wam.expand_tree(beta, m_prev, L, 0.1, O)
            mu = (O @ beta.ravel()).reshape(g.n, g.n)
            thr = 0.1 * mu.max()
            for r, cc in np.argwhere(mg != exp_mask):
                k = max(r, cc)
                lev = next(t for t in range(1, L + 1) if k >= (g.n >> t))
                m, s = g.n >> lev, 1 << lev
                i, jj = r % m, cc % m
                val = mu[i * s:(i + 1) * s, jj * s:(jj + 1) * s].max()
                assert abs(val - thr) <= 1e-6 * max(1.0, abs(thr)), (dtype, lev, i, jj, val, thr)
            if dtype == "f64":
                np.testing.assert_array_equal(mg, m_next)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_loss_and_gradient_match_oracle(dtype):
    P, H = problem("parallel64")
    g = P.geom
    L = 3
    O = omega(g.n, L)
    c = make_ctx(g, L, dtype)
    rng = np.random.default_rng(12)
    coef = rng.normal(0, 0.002, (2, g.n, g.n))
    coef[:, :g.n >> L, :g.n >> L] += 0.15
    if dtype == "f32":
        coef = coef.astype(np.float32).astype(np.float64)
    d = np.stack([P.d, P.d[::-1].copy()])
    loss, q = c.loss(dev(coef.reshape(2, g.n, g.n), dtype), dev(d, dtype), P.i0)
    grad = host(c.loss_backward(q, dev(d, dtype)))
    for k in range(2):
        lref, gref, _ = wam.loss_and_grad(H, O, d[k], P.i0, coef[k].ravel())
        assert abs(host(loss)[k] - lref) <= (1e-5 if dtype == "f32" else 1e-10) * lref
        assert np.abs(grad[k].ravel() - gref).max() <= (1e-4 if dtype == "f32" else 1e-9) * np.abs(gref).max()


def test_monotone_idiv_and_deterministic_fp32():
    P, _ = problem("fan96")
    out = []
    for _ in range(2):
        c = make_ctx(P.geom, 3, "f32", P.d, P.i0)
        idv = host(c.solve(P.n_iters, P.schedule, 0.1))
        assert np.all(idv[1:] <= idv[:-1] * (1 + 1e-6)), np.max(idv[1:] / idv[:-1])
        out.append((idv, host(c.get_state()[0])))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_unsupported_combinations_fail_cleanly():
    from paper_1508_04458_amd import _lib
    P, _ = problem("parallel64")
    c = make_ctx(P.geom, 3, "f32", P.d, P.i0)
    for call in (lambda: c.set_subsets(3), lambda: c.set_penalty(0.1), lambda: c.set_tree_rule("gradient"),
                 lambda: c.set_tree_sharing(True), lambda: c.set_walk_lanes(2)):
        with pytest.raises(_lib.WamctError) as e:
            call()
        assert e.value.status == _lib.E_UNSUPPORTED, str(e.value)
    assert c.walk_lanes() == 0 and c.subsets() == 1
    # the context still works after the rejected calls
    idv = host(c.solve(3, [1], 0.1))
    assert np.all(np.isfinite(idv))


def draw_d4(seed):
    """A random 2-D configuration for the Daubechies-4 basis: levels 1-3 with n >> L in
    4..10 (n up to 80), parallel or fan beam, odd and even view and bin counts, phantom and
    Poisson counts as for the named workloads, a random expansion schedule."""
    rng = np.random.default_rng([seed, 4044])
    L = int(rng.integers(1, 4))
    n = int(rng.integers(4, 11)) * (1 << L)
    if n > 80:
        n = 80 // (1 << L) * (1 << L)
    views = int(rng.integers(7, 61))
    i0 = float(rng.choice([2e3, 1e4, 5e4]))
    if rng.uniform() < 0.5:
        bins = int(rng.integers(int(1.45 * n), int(1.45 * n) + 9))
        g = synth.parallel_geometry(n, views, bins, 1.0)
    else:
        bins = int(rng.integers(n, 2 * n + 1))
        g = synth.fan_geometry(n, views, bins, sod=4.0 * n, sdd=7.0 * n)
    ell = synth.make_ellipses(rng, n, g.pixel, int(rng.integers(2, 7)), 0.06, int(rng.integers(0, 2)))
    o, e = synth.ray_lines(g)
    d = rng.poisson(i0 * np.exp(-synth.line_integrals(ell, o, e))).astype(np.float64)
    n_it = int(rng.integers(6, 13))
    sched = sorted(set(int(x) for x in rng.integers(1, n_it, size=min(L, 3))))
    return g, L, d, i0, n_it, sched


@pytest.mark.parametrize("seed", range(6))
def test_random_d4_solve_fp64(seed):
    """Whole FP64 solves on random configurations with the GPU's own expansions: masks exact,
    beta relative L2 1e-9, I-divergence rtol 1e-10, held counts equal."""
    from paper_1508_04458_amd import api
    g, L, d, i0, n_it, sched = draw_d4(seed)
    print(f"\n[case] d4 seed {seed}: kind {g.kind} n={g.n} L={L} views={g.n_views} bins={g.n_bins} "
          f"iters {n_it} schedule {sched}", flush=True)
    H = siddon.system_matrix(g)
    ref = wam.wam_solve(H, g.n, L, d, i0, n_it, g.pixel, schedule=sched, Omega=omega(g.n, L))
    c = api.Context(g, L, "f64", wavelet="d4")
    c.set_data(dev(d, "f64"), i0)
    idv = host(c.solve(n_it, sched, 0.1))
    beta, mask, _ = c.get_state()
    np.testing.assert_array_equal(host(mask), ref["mask"])
    assert rel_l2(host(beta), ref["beta"]) <= 1e-9
    np.testing.assert_allclose(idv, ref["idiv"], rtol=1e-10)
    assert c.tree_stats()["n_held"] == ref["held"]


def test_tree_schedule_fp64_matches_oracle():
    """The oracle's tree sequence Z_s^(j) given as Algorithm 1's input through the device-side
    schedule (no host round trip of the state): beta 1e-9, I-divergence rtol 1e-10."""
    P, H = problem("fan96")
    g = P.geom
    L = 3
    O = omega(g.n, L)
    ref = wam.wam_solve(H, g.n, L, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule, Omega=O)
    trees = ref["trees"][1:]
    c = make_ctx(g, L, "f64", P.d, P.i0)
    masks = torch.stack([dev(m.ravel(), torch.uint8) for _, m in trees])
    c.set_tree_schedule([j for j, _ in trees], masks)
    idv = host(c.solve(P.n_iters, [], 0.1))
    beta, mask, _ = c.get_state()
    np.testing.assert_array_equal(host(mask), ref["mask"])
    assert rel_l2(host(beta), ref["beta"]) <= 1e-9
    np.testing.assert_allclose(idv, ref["idiv"], rtol=1e-10)


def test_batch_with_haar_and_d4_contexts_equals_each_alone():
    """A Daubechies-4 context and a Haar context in one batch (graph replay on two streams):
    each reproduces its own solve bit for bit (FP32)."""
    from paper_1508_04458_amd import api
    P, _ = problem("fan96")
    g = P.geom
    ctxs = [api.Context(g, 3, "f32", wavelet="d4"), api.Context(g, 3, "f32")]
    alone = []
    for c in ctxs:
        c.set_data(dev(P.d, "f32"), P.i0)
        idv = host(c.solve(P.n_iters, P.schedule, 0.1))
        alone.append((idv, host(c.get_state()[0]), host(c.get_state()[1])))
        c.reset()
    batch = api.Batch(ctxs, n_streams=2, graph=True)
    out = batch.solve(P.n_iters, P.schedule, 0.1)
    for c, (idv, beta, mask), got in zip(ctxs, alone, out):
        b2, m2, it = c.get_state()
        assert it == P.n_iters
        np.testing.assert_array_equal(host(got), idv)
        np.testing.assert_array_equal(host(b2), beta)
        np.testing.assert_array_equal(host(m2), mask)
    assert batch.stats()["graph_launches"] == P.n_iters
