"""Parity at the cone-beam benchmark's full size (cone512: 512 x 512 x 256 volume, 720 views
of a 256 x 1024 detector, 3-level 3-D Haar octree, FP32 data), in the configuration bench.py
times, on outputs the oracle can compute one by one:

  * projection of a random volume and the tree forward pass (Omega beta, Beer's law) on
    sampled rays (oracle: 3-D Siddon of those rays, the volume synthesised at the voxels
    they cross);
  * the sign-split backprojection at sampled octree nodes: each node's phi over every ray
    that can meet it (detector shadow of its box), by octant clipping;
  * the first update of the approximation-only octree: Z0 = 2^(-3L/2) x the longest chord
    through the volume, b and the closed-form root update (1/Z0) ln(b-hat+ / b) at sampled
    roots;
  * the benchmark's own 50-iteration solve: I-divergence non-increasing, octree grows.

Tolerances: projections 1e-5 max(|p|, 1e-3 max p) per ray (FP32 storage of the volume is
applied to the oracle's input, so only summation order differs); q additionally 2e-7
relative (FP32 storage); backprojections 1e-5 of the larger of |b-hat+|, |b-hat-| per
coefficient (FP32 sums of about 1e5 terms each, b-hat+ formed as (A + S) / 2 from
magnitude and signed sums); b 1e-5 relative; root updates 1e-5 relative plus 2e-5 / Z0
(the error of ln(b-hat+ / b) for 1e-5-relative b-hat+ and b, divided by Z0).
"""
import math

import numpy as np
import pytest
import torch

from oracle import vol3d
from paper_1508_04458_amd import synth
from test_gpu_cone import host, random_octree_mask
from test_oracle_3d import longest_chord

pytestmark = pytest.mark.gpu

LEVELS = 3
I0 = 1e5


@pytest.fixture(scope="module")
def geom():
    return synth.CONE_CONFIGS["cone512"]["geom"]()


def make_ctx(g, levels):
    from paper_1508_04458_amd import api
    print(f"\n[cone512] context L={levels} f32, {g.n_rays} rays", flush=True)
    return api.Context(g, levels, "f32")


def sample_rays(g, k, seed):
    """k random rays plus the first and last ray of the scan and of one mid view."""
    rng = np.random.default_rng([seed, 512])
    per_view = g.n_rows * g.n_cols
    fixed = [0, g.n_rays - 1, 360 * per_view, 361 * per_view - 1, 360 * per_view + per_view // 2 + g.n_cols // 2]
    return np.unique(np.concatenate([rng.choice(g.n_rays, k, replace=False), fixed]))


def at(t, ids):
    return host(t[torch.as_tensor(ids, device=t.device)])


def test_cone512_projection_sampled_rays(geom):
    g = geom
    c = make_ctx(g, 0)
    vol = np.random.default_rng(51).random((g.nz, g.n, g.n), dtype=np.float32) * np.float32(0.05)
    p = c.project(torch.from_numpy(vol.ravel()).cuda())
    full_max = float(p.max())
    ids = sample_rays(g, 500, 1)
    print(f"[cone512] oracle: {ids.size} sampled rays", flush=True)
    ref = vol3d.project_rays3(g, vol.astype(np.float64), ids)
    got = at(p, ids)
    tol = 1e-5 * np.maximum(np.abs(ref), 1e-3 * full_max)
    assert np.all(np.abs(got - ref) <= tol), np.abs(got - ref).max()
    assert np.any(ref == 0) and np.all(got[ref == 0] == 0)       # rays that miss the volume


def test_cone512_tree_forward_sampled_rays(geom):
    g = geom
    L = LEVELS
    mask = random_octree_mask(g.n, g.nz, L, 52, 0.55)
    rng = np.random.default_rng(52)
    beta = rng.standard_normal((g.nz, g.n, g.n), dtype=np.float32) * np.float32(0.002) * mask
    r = (g.nz >> L, g.n >> L, g.n >> L)
    beta[:r[0], :r[1], :r[2]] = (0.02 * 2 ** (1.5 * L) + rng.uniform(0, 0.01, r)).astype(np.float32)
    c = make_ctx(g, L)
    c.set_data(torch.full((g.n_rays,), 0.5 * I0, dtype=torch.float32, device="cuda"), I0)
    c.set_state(torch.from_numpy(beta.ravel()).cuda(), torch.from_numpy(mask.ravel()).cuda())
    q, _ = c.forward()
    ids = sample_rays(g, 400, 2)
    print(f"[cone512] oracle: {ids.size} sampled rays through Omega beta", flush=True)
    p_ref = vol3d.project_coef_rays3(g, beta.astype(np.float64), L, ids)
    q_ref = I0 * np.exp(-p_ref)
    got = at(q, ids)
    tol = q_ref * (1e-5 * np.maximum(np.abs(p_ref), 1e-3 * p_ref.max()) + 2e-7)
    assert np.all(np.abs(got - q_ref) <= tol), np.max(np.abs(got - q_ref) / q_ref)


def test_cone512_split_backprojection_sampled_nodes(geom):
    g = geom
    L = LEVELS
    n, nz = g.n, g.nz
    mask = random_octree_mask(n, nz, L, 53, 0.6)
    c = make_ctx(g, L)
    c.set_state(torch.zeros(g.n_voxels, dtype=torch.float32, device="cuda"), torch.from_numpy(mask.ravel()).cuda())
    y = np.random.default_rng(53).random(g.n_rays, dtype=np.float32)
    bp, bm = (host(t).reshape(nz, n, n) for t in c.backproject_split(torch.from_numpy(y).cuda()))
    exy, ez = vol3d.edges3(g)
    rng = np.random.default_rng(54)
    checked, worst = 0, 0.0
    for lev in range(L, 0, -1):
        m, mz = n >> lev, nz >> lev
        split = vol3d.split_flags3(mask, lev)
        cand = np.argwhere(np.ones((mz, m, m), bool)) if lev == L else np.argwhere(split)
        for k, i, j in cand[rng.choice(len(cand), min(4, len(cand)), replace=False)]:
            s = 1 << lev
            lo = np.array([exy[j * s], exy[i * s], ez[k * s]])
            hi = np.array([exy[(j + 1) * s], exy[(i + 1) * s], ez[(k + 1) * s]])
            ids = vol3d.box_shadow3(g, lo, hi)
            o, e = vol3d.rays3(g, ids=ids)
            phis = vol3d.node_phi3(g, o, e, lev, k, i, j)
            approx = phis.pop("approx")
            coefs = list(phis.items()) if split[k, i, j] else []
            if lev == L:
                coefs.append(((k, i, j), approx))
            print(f"[cone512] node ({lev}, {k}, {i}, {j}): {ids.size} rays, {len(coefs)} coefficients", flush=True)
            yy = y[ids].astype(np.float64)
            for (zz, zy, zx), ph in coefs:
                ph = np.where(np.abs(ph) <= 1e-12 * g.pixel, 0.0, ph)
                rp = float(yy @ np.maximum(ph, 0.0))
                rm = float(yy @ np.minimum(ph, 0.0))
                scale = max(abs(rp), abs(rm), 1e-30)
                ep, em = abs(bp[zz, zy, zx] - rp), abs(bm[zz, zy, zx] - rm)
                worst = max(worst, ep / scale, em / scale)
                assert ep <= 1e-5 * scale, (lev, k, i, j, zz, zy, zx, bp[zz, zy, zx], rp)
                assert em <= 1e-5 * scale, (lev, k, i, j, zz, zy, zx, bm[zz, zy, zx], rm)
                checked += 1
    print(f"[cone512] {checked} coefficients, worst relative error {worst:.2e}", flush=True)
    assert checked >= 40
    inactive = mask == 0
    assert np.all(bp[inactive] == 0) and np.all(bm[inactive] == 0)


def test_cone512_first_update_and_z0(geom):
    """First iteration from beta = 0 on the approximation-only octree: q-hat = I0 on every
    ray, so each root's update is (1/Z0) ln(b-hat+ / b) with b-hat+ = I0 sum_y phi and
    b = sum_y d phi, phi = 2^(-3L/2) x the chord through the root's 8 x 8 x 8 block; roots
    no ray meets have b = b-hat+ = 0 and are held at zero."""
    g = geom
    L = LEVELS
    n, nz = g.n, g.nz
    d = np.random.default_rng(55).integers(1, int(I0), g.n_rays, dtype=np.int32).astype(np.float32)
    c = make_ctx(g, L)
    c.set_data(torch.from_numpy(d).cuda(), I0)
    st = c.tree_stats()
    print("[cone512] oracle: longest chord over the scan", flush=True)
    z0_ref = 2.0 ** (-1.5 * L) * longest_chord(g)
    assert abs(st["z0"] - z0_ref) <= 1e-11 * z0_ref, (st["z0"], z0_ref)
    r = (nz >> L, n >> L, n >> L)
    assert st["n_active"] == r[0] * r[1] * r[2]
    b_all = host(c.b()).reshape(nz, n, n)
    c.iterate(1)
    beta = host(c.get_state()[0]).reshape(nz, n, n)
    exy, ez = vol3d.edges3(g)
    s = 1 << L
    rng = np.random.default_rng(56)
    roots = [(0, 0, 0), (r[0] - 1, r[1] - 1, r[2] - 1), (r[0] // 2, r[1] // 2, r[2] // 2), (0, r[1] // 2, 0),
             (r[0] - 1, 0, r[2] // 3)] + [tuple(int(x) for x in rng.integers(0, r)) for _ in range(10)]
    sc = 2.0 ** (-1.5 * L)
    for k, i, j in roots:
        lo = np.array([exy[j * s], exy[i * s], ez[k * s]])
        hi = np.array([exy[(j + 1) * s], exy[(i + 1) * s], ez[(k + 1) * s]])
        ids = vol3d.box_shadow3(g, lo, hi)
        o, e = vol3d.rays3(g, ids=ids)
        ch = vol3d.box_chord3(o, e, lo, hi)
        b = sc * float(d[ids].astype(np.float64) @ ch)
        bplus = sc * I0 * float(ch.sum())
        print(f"[cone512] root ({k}, {i}, {j}): {ids.size} rays, b {b:.6e}", flush=True)
        assert abs(b_all[k, i, j] - b) <= 1e-5 * b, (k, i, j, b_all[k, i, j], b)
        ref = 0.0 if b == 0 else math.log(bplus / b) / z0_ref
        assert abs(beta[k, i, j] - ref) <= 1e-5 * abs(ref) + 2e-5 / z0_ref, (k, i, j, beta[k, i, j], ref)
    held = int(np.sum(b_all[:r[0], :r[1], :r[2]] == 0))
    assert c.tree_stats()["n_held"] == held


def test_cone512_bench_solve_is_monotone(geom):
    """The benchmark's own solve (phantom of 200 ellipsoids and 10 metal cylinders, 50
    iterations, expansions at the scaled schedule): I-divergence non-increasing (FP64 sums
    of FP32 iterates, factor 1 + 1e-6), the octree grows at the expansions."""
    print("\n[cone512] drawing the phantom on the GPU (about 40 s)", flush=True)
    P = synth.make_cone_problem("cone512", device="cuda")
    print("[cone512] phantom ready", flush=True)
    c = make_ctx(P.geom, P.levels)
    c.set_data(torch.from_numpy(P.d.astype(np.float32)).cuda(), P.i0)
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    print(f"[cone512] I-divergence {idv[0]:.4e} -> {idv[-1]:.4e}", flush=True)
    assert np.all(idv[1:] <= idv[:-1] * (1 + 1e-6)), np.max(idv[1:] / idv[:-1])
    g = P.geom
    assert c.tree_stats()["n_active"] > (g.n >> P.levels) ** 2 * (g.nz >> P.levels)
