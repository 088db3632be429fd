"""Parity at the benchmark's full size (fan512: 512x512 fan beam, 720 views x 1024 bins,
3-level tree, FP32 data), in the configuration bench.py times, on outputs the oracle can
compute one by one: sampled rays, sampled tree nodes (their phi over all 737280 rays by box
clipping), and the first update, whose Z0 has a closed form."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry, haar, siddon, wam
from paper_1508_04458_amd import synth
from test_gpu_parity import dev, host, make_ctx, proj_tol
from test_oracle_siddon import square_chord_closed_form

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fan512():
    print("\n[fan512] generating the scan (about 20 s)", flush=True)
    P = synth.make_problem("fan512")
    o, e = geometry.rays(P.geom)
    print("[fan512] scan ready", flush=True)
    return P, o, e


def _node_phi(g, o, e, lev, i, j):
    """(phi_LL or None, phi_D1, phi_D2, phi_D3) of node (lev, i, j) over all rays, from
    quadrant chords by brute-force box clipping (pinned against H Omega in the oracle tests)."""
    edges = geometry.pixel_edges(g)
    s, h = 1 << lev, 1 << (lev - 1)
    q = {}
    for qy in (0, 1):
        for qx in (0, 1):
            q[qy, qx] = siddon.box_chord(o, e, edges[j * s + qx * h], edges[j * s + (qx + 1) * h],
                                         edges[i * s + qy * h], edges[i * s + (qy + 1) * h])
    sc = 2.0 ** -lev
    d1 = (q[0, 0] - q[0, 1] + q[1, 0] - q[1, 1]) * sc
    d2 = (q[0, 0] + q[0, 1] - q[1, 0] - q[1, 1]) * sc
    d3 = (q[0, 0] - q[0, 1] - q[1, 0] + q[1, 1]) * sc
    ll = sum(q.values()) * sc
    return ll, d1, d2, d3


def test_fan512_projection_sampled_rays(fan512):
    P, o, e = fan512
    g = P.geom
    c = make_ctx(g, P.levels, "f32")
    rng = np.random.default_rng(0)
    ids = np.sort(rng.choice(g.n_rays, 600, replace=False))
    for img in (synth.rasterize(P.ellipses, g.n, g.pixel), synth.random_image(g.n, 5)):
        p = host(c.project(dev(img.ravel(), "f32")))
        img32 = img.astype(np.float32).astype(np.float64)
        ref = siddon.project_rays(g, img32, ids)
        full_max = float(p.max())
        tol = 1e-5 * np.maximum(np.abs(ref), 1e-3 * full_max)
        assert np.all(np.abs(p[ids] - ref) <= tol), np.abs(p[ids] - ref).max()


def test_fan512_tree_forward_sampled_rays(fan512):
    P, o, e = fan512
    g = P.geom
    L = P.levels
    mask = synth.random_tree_mask(g.n, L, 31, p_split=0.55)
    rng = np.random.default_rng(31)
    beta = (rng.normal(0, 0.002, (g.n, g.n)) * mask).astype(np.float32)
    nL = g.n >> L
    beta[:nL, :nL] = (0.02 * (1 << L) + rng.uniform(0, 0.01, (nL, nL))).astype(np.float32)
    c = make_ctx(g, L, "f32", P.d, P.i0)
    c.set_state(dev(beta.ravel(), "f32"), dev(mask.ravel(), torch.uint8))
    q, _ = c.forward()
    q = host(q)
    mu = haar.cascade_synthesis(beta.astype(np.float64), L)
    ids = np.sort(rng.choice(g.n_rays, 600, replace=False))
    p_ref = siddon.project_rays(g, mu, ids)
    q_ref = P.i0 * np.exp(-p_ref)
    # q has the relative error of p's absolute error, plus FP32 storage of q
    tol = q_ref * (1e-5 * np.maximum(np.abs(p_ref), 1e-3 * p_ref.max()) + 2e-7)
    assert np.all(np.abs(q[ids] - q_ref) <= tol), np.max(np.abs(q[ids] - q_ref) / q_ref)


def test_fan512_split_backprojection_sampled_nodes(fan512):
    P, o, e = fan512
    g = P.geom
    L = P.levels
    n = g.n
    mask = synth.random_tree_mask(n, L, 32, p_split=0.6)
    c = make_ctx(g, L, "f32")
    c.set_state(dev(np.zeros(n * n), "f32"), dev(mask.ravel(), torch.uint8))
    y = synth.random_vector(g.n_rays, 32).astype(np.float32).astype(np.float64)
    bp, bm = (host(t) for t in c.backproject_split(dev(y, "f32")))
    rng = np.random.default_rng(32)
    checked = 0
    for lev in range(L, 0, -1):
        m = n >> lev
        split = haar.split_flags(mask, lev)
        cand = np.argwhere(split) if lev < L else np.argwhere(np.ones((m, m), bool))
        for i, j in cand[rng.choice(len(cand), min(6, len(cand)), replace=False)]:
            print(f"[fan512] node ({lev}, {i}, {j})", flush=True)
            ll, d1, d2, d3 = _node_phi(g, o, e, lev, i, j)
            phis = [(i, m + j, d1), (m + i, j, d2), (m + i, m + j, d3)] if split[i, j] else []
            if lev == L:
                phis.append((i, j, ll))
            for zr, zc, ph in phis:
                ph = np.where(np.abs(ph) <= 1e-12 * g.pixel, 0.0, ph)
                rp = float(np.sum(y * np.maximum(ph, 0)))
                rm = float(np.sum(y * np.minimum(ph, 0)))
                scale = max(abs(rp), abs(rm), 1e-30)
                assert abs(bp[zr, zc] - rp) <= 2e-6 * scale + 1e-6, (lev, i, j, bp[zr, zc], rp)
                assert abs(bm[zr, zc] - rm) <= 2e-6 * scale + 1e-6, (lev, i, j, bm[zr, zc], rm)
                checked += 1
    assert checked >= 20


def test_fan512_first_update_and_z0(fan512):
    """First iteration of the benchmark solve (beta = 0, approximation-only tree), for all
    4096 roots: q-hat = I0; Z0 = 2^-L max_y chord(y, image) (closed form); b-hat+ and b of a
    root are 2^-L times the backprojections of I0 and d through its 8x8-pixel block, taken from
    the oracle's Siddon matrix of the same rays on the 64x64 grid of 8 mm blocks; the update is
    (1/Z0) ln(b-hat+ / b); roots crossed only by zero-count rays (b = 0) have no finite
    minimizer and are held (counted, beta stays 0)."""
    P, o, e = fan512
    g = P.geom
    L = P.levels
    n = g.n
    c = make_ctx(g, L, "f32", P.d, P.i0)
    st = c.tree_stats()
    z0_ref = 2.0 ** -L * square_chord_closed_form(o, e, 0.5 * n * g.pixel).max()
    assert abs(st["z0"] - z0_ref) <= 1e-11 * z0_ref
    assert st["n_active"] == (n >> L) ** 2
    c.iterate(1)
    beta, _, _ = c.get_state()
    beta = host(beta)[: n >> L, : n >> L]
    gc = synth.Geometry(g.kind, n >> L, g.pixel * (1 << L), g.n_views, g.angle0, g.angle_span, g.n_bins,
                        g.bin_pitch, g.sod, g.sdd)
    print("[fan512] oracle coarse-grid matrix", flush=True)
    Hc = siddon.system_matrix(gc)
    d32 = P.d.astype(np.float32).astype(np.float64)
    b = 2.0 ** -L * (Hc.T @ d32)
    bplus = 2.0 ** -L * P.i0 * np.asarray(Hc.sum(axis=0)).ravel()
    dark = b == 0
    ref = np.where(dark, 0.0, np.log(bplus / np.where(dark, 1.0, b)) / z0_ref).reshape(n >> L, n >> L)
    err = np.abs(beta - ref)
    assert np.all(err <= 2e-6 * np.abs(ref) + 1e-7), err.max()
    assert c.tree_stats()["n_held"] == int(dark.sum())


def test_fan512_bench_solve_is_monotone(fan512):
    """The benchmark's own 100-iteration tree-adaptive solve: I-divergence non-increasing
    (FP64 sums of FP32 iterates, factor 1 + 1e-6) and the tree grows at the expansions."""
    P, o, e = fan512
    c = make_ctx(P.geom, P.levels, "f32", P.d, P.i0)
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    assert np.all(idv[1:] <= idv[:-1] * (1 + 1e-6)), np.max(idv[1:] / idv[:-1])
    st = c.tree_stats()
    assert st["n_active"] > (P.geom.n >> P.levels) ** 2
