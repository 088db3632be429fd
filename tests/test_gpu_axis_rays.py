"""Rays on the symmetry lines of the grid. Four views at 0, 90, 180 and 270 degrees and odd
detectors put central rays along the grid axes (a direction component of 0, placed by the
reading of axis-parallel lines) and through node mid-lines and mid-planes, where detail values
of phi vanish exactly in real arithmetic and only rounding residue is left. The sign-split
backprojection (eq. 1.10) has to match the FP64 oracle there, and its exact zeros (a
coefficient that no ray sees with phi > 0 has b-hat+ = 0, with phi < 0 b-hat- = 0) have to sit
where the oracle's are: a residue counted as a value would move such a coefficient to the
other branch of the eq. 1.9 root. Z0 and W (eq. 1.61) are checked on the same trees.
"""
import math

import numpy as np
import pytest
import torch

from oracle import daub, haar, siddon, vol3d, wam
from paper_1508_04458_amd import synth
from test_gpu_cone import random_octree_mask

pytestmark = pytest.mark.gpu


def dev(x, dtype):
    tdt = {"f32": torch.float32, "f64": torch.float64}.get(dtype, dtype)
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=tdt)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _context(g, levels, **kw):
    from paper_1508_04458_amd import api
    print(f"\n[case] axis rays kind={getattr(g, 'kind', 'cone')} n={g.n} views={g.n_views} L={levels} {kw}",
          flush=True)
    return api.Context(g, levels, "f64", **kw)


def _check(c, H, O, mask, g, n_coef, seed, exact_zeros=True):
    c.set_state(dev(np.zeros(n_coef), "f64"), dev(mask.ravel(), torch.uint8))
    Phi, act = wam.phi_matrix(H, O, mask, g.pixel)
    st = c.tree_stats()
    assert abs(st["z0"] - wam.z0_of(Phi)) <= 1e-11 * st["z0"]
    assert abs(st["w"] - Phi.nnz) <= 1e-4 * Phi.nnz
    y = np.random.default_rng(seed).uniform(0.5, 1.5, g.n_rays)
    bp, bm = (host(t).ravel() for t in c.backproject_split(dev(y, "f64")))
    Pp, Pm = wam.split_phi(Phi)
    rp = np.zeros(n_coef)
    rm = np.zeros(n_coef)
    rp[act] = Pp.T @ y
    rm[act] = Pm.T @ y
    tol = 1e-11 * max(np.abs(rp).max(), np.abs(rm).max())
    assert np.abs(bp - rp).max() <= tol
    assert np.abs(bm - rm).max() <= tol
    assert bp.min() >= 0 and bm.max() <= 0
    if not exact_zeros:
        return None
    # exact zeros where no ray sees the coefficient with that sign (y > 0 everywhere)
    pos = np.zeros(n_coef, bool)
    neg = np.zeros(n_coef, bool)
    pos[act] = np.asarray((Pp != 0).sum(axis=0)).ravel() > 0
    neg[act] = np.asarray((Pm != 0).sum(axis=0)).ravel() > 0
    assert np.all(bp[~pos] == 0) and np.all(bm[~neg] == 0)
    assert np.all(bp[pos] > 0) and np.all(bm[neg] < 0)
    # the symmetric views do produce vanishing details: some active details (never a root,
    # whose phi is a positive chord) see no ray with phi > 0
    return int(np.sum(~pos[act])), int(np.sum(~neg[act]))


@pytest.mark.parametrize("kind", ["fan", "parallel"])
def test_axis_rays_2d_split_backprojection(kind):
    if kind == "fan":
        g = synth.fan_geometry(16, 4, 33, sod=40.0, sdd=70.0)
    else:
        g = synth.parallel_geometry(16, 4, 33, bin_pitch=0.5, angle_span=2.0 * math.pi)
    H = siddon.system_matrix(g)
    L = 2
    O = haar.synthesis_matrix(g.n, L)
    c = _context(g, L)
    for seed in (0, 1):
        mask = synth.random_tree_mask(g.n, L, 70 + seed, p_split=0.8)
        no_pos, no_neg = _check(c, H, O, mask, g, g.n * g.n, seed)
        assert no_pos > 0


@pytest.mark.parametrize("dims", [3, 2])
def test_axis_rays_cone_split_backprojection(dims):
    g = synth.cone_geometry(16, 8, 4, 9, 33, sod=40.0, sdd=70.0)
    H = vol3d.system_matrix3(g)
    L = 2
    if dims == 3:
        O = vol3d.synthesis_matrix3(g.n, g.nz, L)
        c = _context(g, L)
    else:
        O = vol3d.slice_synthesis_matrix3(g.n, g.nz, L)
        c = _context(g, L, wavelet_dims=2)
    for seed in (0, 1):
        if dims == 3:
            mask = random_octree_mask(g.n, g.nz, L, 90 + seed, p=0.8)
        else:
            mask = vol3d.slice_mask3(synth.random_tree_mask(g.n, L, 80 + seed, p_split=0.8), g.nz)
        no_pos, no_neg = _check(c, H, O, mask, g, g.n_voxels, seed)
        assert no_pos > 0


def test_axis_rays_daubechies4_split_backprojection():
    """The same symmetric fan scan with the Daubechies-4 basis (values, Z0 and W; its phi are
    sums of chords times irrational basis samples, so vanishing entries are not structural)."""
    g = synth.fan_geometry(16, 4, 33, sod=40.0, sdd=70.0)
    H = siddon.system_matrix(g)
    L = 2
    O = daub.synthesis_matrix(g.n, L)
    c = _context(g, L, wavelet="d4")
    for seed in (0, 1):
        mask = synth.random_tree_mask(g.n, L, 75 + seed, p_split=0.8)
        _check(c, H, O, mask, g, g.n * g.n, seed, exact_zeros=False)
