"""The largest problems the library accepts, on a few views (sizes at the limits that
wamct_validate enforces; the coefficient and work-list encodings are sized for them):

  * 2-D: an 8192 x 8192 image (the maximum side: pixel coordinates fill the 13-bit fields of
    a work item), parallel beam of 4 views x 11600 bins, 4-level tree;
  * 3-D: a 512 x 512 x 512 volume (maximum side and depth: voxel coordinates fill the 9-bit
    fields), cone beam of 8 views x 96 x 160 with rows spanning the whole depth, 3-level
    octree.

Each case: the tree forward pass on sampled rays against the oracle (the image synthesised
by the textbook cascade, or at the crossed voxels), Z0 of the approximation-only tree
against 2^-L (2-D) / 2^(-3L/2) (3-D) x the longest chord through the image, the sign-split
backprojection at sampled nodes, and a few iterations with the I-divergence non-increasing.
FP32 data, tolerances as at the benchmark sizes.
"""
import math

import numpy as np
import pytest
import torch

from oracle import geometry, haar, siddon, vol3d
from paper_1508_04458_amd import synth
from test_gpu_cone import random_octree_mask
from test_oracle_3d import longest_chord
from test_oracle_siddon import square_chord_closed_form

pytestmark = pytest.mark.gpu


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy() if t.is_floating_point() else t.detach().cpu().numpy()


def at(t, ids):
    return host(t[torch.as_tensor(ids, device=t.device)])


def test_image_8192_parallel():
    from paper_1508_04458_amd import api
    g = synth.parallel_geometry(8192, 4, 11600, 1.0)
    L = 4
    print(f"\n[limits] 2-D n={g.n} L={L}, {g.n_rays} rays", flush=True)
    c = api.Context(g, L, "f32")
    c.set_data(torch.full((g.n_rays,), 5e3, dtype=torch.float32, device="cuda"), 1e4)
    o, e = geometry.rays(g)
    st = c.tree_stats()
    z0_ref = 2.0 ** -L * square_chord_closed_form(o, e, 0.5 * g.n * g.pixel).max()
    assert abs(st["z0"] - z0_ref) <= 1e-11 * z0_ref
    mask = synth.random_tree_mask(g.n, L, 81, p_split=0.5)
    rng = np.random.default_rng(81)
    beta = (rng.standard_normal((g.n, g.n), dtype=np.float32) * np.float32(0.0005)) * mask
    nL = g.n >> L
    beta[:nL, :nL] = (0.002 * (1 << L) + rng.uniform(0, 0.001, (nL, nL))).astype(np.float32)
    c.set_state(torch.from_numpy(beta.ravel()).cuda(), torch.from_numpy(mask.ravel()).cuda())
    q, _ = c.forward()
    ids = np.unique(np.concatenate([rng.choice(g.n_rays, 150, replace=False), [0, g.n_rays - 1]]))
    print("[limits] oracle synthesis and sampled rays", flush=True)
    mu = haar.cascade_synthesis(beta.astype(np.float64), L)
    p_ref = siddon.project_rays(g, mu, ids)
    q_ref = 1e4 * np.exp(-p_ref)
    got = at(q, ids)
    tol = q_ref * (1e-5 * np.maximum(np.abs(p_ref), 1e-3 * p_ref.max()) + 2e-7)
    assert np.all(np.abs(got - q_ref) <= tol), np.max(np.abs(got - q_ref) / q_ref)
    # split backprojection at the node farthest from the origin and at a middle one
    y = np.random.default_rng(82).random(g.n_rays, dtype=np.float32)
    bp, bm = (host(t) for t in c.backproject_split(torch.from_numpy(y).cuda()))
    edges = geometry.pixel_edges(g)
    checked = 0
    for lev in (1, 2):
        m = g.n >> lev
        split = haar.split_flags(mask, lev)
        cand = np.argwhere(split)
        picks = [cand[np.argmax(cand[:, 0] + cand[:, 1])], cand[len(cand) // 2]]
        for i, j in picks:
            s, h = 1 << lev, 1 << (lev - 1)
            qd = {}
            for qy in (0, 1):
                for qx in (0, 1):
                    qd[qy, qx] = siddon.box_chord(o, e, edges[j * s + qx * h], edges[j * s + (qx + 1) * h],
                                                  edges[i * s + qy * h], edges[i * s + (qy + 1) * h])
            sc = 2.0 ** -lev
            phis = [(i, m + j, (qd[0, 0] - qd[0, 1] + qd[1, 0] - qd[1, 1]) * sc),
                    (m + i, j, (qd[0, 0] + qd[0, 1] - qd[1, 0] - qd[1, 1]) * sc),
                    (m + i, m + j, (qd[0, 0] - qd[0, 1] - qd[1, 0] + qd[1, 1]) * sc)]
            for zr, zc, ph in phis:
                ph = np.where(np.abs(ph) <= 1e-12 * g.pixel, 0.0, ph)
                rp = float(y.astype(np.float64) @ np.maximum(ph, 0.0))
                rm = float(y.astype(np.float64) @ np.minimum(ph, 0.0))
                scale = max(abs(rp), abs(rm), 1e-30)
                assert abs(bp[zr, zc] - rp) <= 1e-5 * scale + 1e-6, (lev, i, j, bp[zr, zc], rp)
                assert abs(bm[zr, zc] - rm) <= 1e-5 * scale + 1e-6, (lev, i, j, bm[zr, zc], rm)
                checked += 1
    assert checked == 12
    idv = host(c.solve(3, [], 0.1))
    assert np.all(idv[1:] <= idv[:-1] * (1 + 1e-6))


def test_volume_512_cubed_cone():
    from paper_1508_04458_amd import api
    base = synth.cone_geometry(512, 512, 8, 96, 160)
    # rows spanning the whole depth at the isocentre (the default pitch covers 96 slices)
    g = synth.Geometry3(**{**base.__dict__, "row_pitch": 1.1 * 512 * base.sdd / base.sod / 96})
    L = 3
    print(f"\n[limits] cone n={g.n} nz={g.nz} L={L}, {g.n_rays} rays", flush=True)
    c = api.Context(g, L, "f32")
    c.set_data(torch.full((g.n_rays,), 5e3, dtype=torch.float32, device="cuda"), 1e4)
    st = c.tree_stats()
    z0_ref = 2.0 ** (-1.5 * L) * longest_chord(g)
    assert abs(st["z0"] - z0_ref) <= 1e-11 * z0_ref
    mask = random_octree_mask(g.n, g.nz, L, 83, 0.5)
    rng = np.random.default_rng(83)
    beta = (rng.standard_normal((g.nz, g.n, g.n), dtype=np.float32) * np.float32(0.0005)) * mask
    r = (g.nz >> L, g.n >> L, g.n >> L)
    beta[:r[0], :r[1], :r[2]] = (0.002 * 2 ** (1.5 * L) + rng.uniform(0, 0.001, r)).astype(np.float32)
    c.set_state(torch.from_numpy(beta.ravel()).cuda(), torch.from_numpy(mask.ravel()).cuda())
    q, _ = c.forward()
    ids = np.unique(np.concatenate([rng.choice(g.n_rays, 150, replace=False), [0, g.n_rays - 1]]))
    print("[limits] oracle: sampled rays through Omega beta", flush=True)
    p_ref = vol3d.project_coef_rays3(g, beta.astype(np.float64), L, ids)
    q_ref = 1e4 * np.exp(-p_ref)
    got = at(q, ids)
    tol = q_ref * (1e-5 * np.maximum(np.abs(p_ref), 1e-3 * p_ref.max()) + 2e-7)
    assert np.all(np.abs(got - q_ref) <= tol), np.max(np.abs(got - q_ref) / q_ref)
    # split backprojection at the node farthest from the origin and at a middle one, per level
    y = np.random.default_rng(84).random(g.n_rays, dtype=np.float32)
    bp, bm = (host(t).reshape(g.nz, g.n, g.n) for t in c.backproject_split(torch.from_numpy(y).cuda()))
    exy, ez = vol3d.edges3(g)
    checked = 0
    for lev in (1, 2, 3):
        split = vol3d.split_flags3(mask, lev)
        cand = np.argwhere(split)
        picks = [cand[np.argmax(cand.sum(axis=1))], cand[len(cand) // 2]]
        for k, i, j in picks:
            s = 1 << lev
            lo = np.array([exy[j * s], exy[i * s], ez[k * s]])
            hi = np.array([exy[(j + 1) * s], exy[(i + 1) * s], ez[(k + 1) * s]])
            sh = vol3d.box_shadow3(g, lo, hi)
            if sh.size == 0:
                continue
            o, e = vol3d.rays3(g, ids=sh)
            phis = vol3d.node_phi3(g, o, e, lev, k, i, j)
            phis.pop("approx")
            yy = y[sh].astype(np.float64)
            for (zz, zy, zx), ph in phis.items():
                ph = np.where(np.abs(ph) <= 1e-12 * g.pixel, 0.0, ph)
                rp = float(yy @ np.maximum(ph, 0.0))
                rm = float(yy @ np.minimum(ph, 0.0))
                scale = max(abs(rp), abs(rm), 1e-30)
                assert abs(bp[zz, zy, zx] - rp) <= 1e-5 * scale + 1e-6, (lev, k, i, j, bp[zz, zy, zx], rp)
                assert abs(bm[zz, zy, zx] - rm) <= 1e-5 * scale + 1e-6, (lev, k, i, j, bm[zz, zy, zx], rm)
                checked += 1
    assert checked >= 28
    idv = host(c.solve(3, [], 0.1))
    assert np.all(idv[1:] <= idv[:-1] * (1 + 1e-6))
