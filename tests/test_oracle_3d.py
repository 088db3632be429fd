"""Pins of the 3-D cone-beam oracle (oracle/vol3d.py), CPU only.

  * 3-D Siddon H equals brute-force box clipping of every (ray, voxel) pair, and for rays
    in the mid-plane z = 0 each row sum equals the closed-form chord of the square;
  * 3-D Haar: orthonormal; Omega^T equals an independent recursive 2x2x2 analysis; a
    hand-computed 2x2x2 example;
  * Z0 of the approximation-only octree = 2^(-3L/2) max chord through the volume;
  * approximation-only 3-D wavelet AM equals voxel AM on the 2^L-coarser grid (exact);
  * the I-divergence decreases at every iteration, across octree expansions;
  * noise-free data are a fixed point; the octree rule splits exactly the leaves holding
    a voxel above the threshold (hand-made case).
"""
import math

import numpy as np
import pytest

from oracle import vol3d, wam
from paper_1508_04458_amd import synth
from test_oracle_siddon import square_chord_closed_form


def tiny_geom(n=8, nz=4, views=5, rows=6, cols=12):
    return synth.cone_geometry(n, nz, views, rows, cols, sod=40.0, sdd=70.0)


def test_siddon3_equals_box_clipping():
    for g in (tiny_geom(), tiny_geom(8, 8, 3, 7, 9)):
        o, e = vol3d.rays3(g)
        H = vol3d.system_matrix3(g).toarray()
        exy, ez = vol3d.edges3(g)
        s, r, c = np.meshgrid(np.arange(g.nz), np.arange(g.n), np.arange(g.n), indexing="ij")
        lo = np.stack([exy[c.ravel()], exy[r.ravel()], ez[s.ravel()]], axis=1)
        hi = np.stack([exy[c.ravel() + 1], exy[r.ravel() + 1], ez[s.ravel() + 1]], axis=1)
        dense = vol3d.box_chord3(o[:, None, :], e[:, None, :], lo[None], hi[None])
        np.testing.assert_allclose(H, dense, atol=1e-12)


def test_mid_plane_rays_match_square_closed_form():
    g = synth.cone_geometry(16, 4, 7, 1, 40, sod=60.0, sdd=100.0)   # one row: the z = 0 plane
    o, e = vol3d.rays3(g)
    assert np.all(e[:, 2] == 0)
    H = vol3d.system_matrix3(g)
    ref = square_chord_closed_form(o[:, :2], e[:, :2] / np.linalg.norm(e[:, :2], axis=1, keepdims=True),
                                   0.5 * g.n * g.pixel)
    np.testing.assert_allclose(np.asarray(H.sum(axis=1)).ravel(), ref, rtol=1e-12, atol=1e-12)


def test_haar3_orthonormal_and_cascade():
    n, nz, L = 8, 4, 2
    O = vol3d.synthesis_matrix3(n, nz, L)
    I = (O.T @ O).toarray()
    np.testing.assert_allclose(I, np.eye(n * n * nz), atol=1e-13)
    vol = np.random.default_rng(1).normal(size=(nz, n, n))
    np.testing.assert_allclose((O.T @ vol.ravel()).reshape(nz, n, n), vol3d.cascade_analysis3(vol, L), atol=1e-12)


def test_haar3_hand_example():
    # one level on a 2x2x2 volume: approximation = sum / (2 sqrt 2); detail (tz, ty, tx) =
    # sum of +-v / (2 sqrt 2) with - on the upper half of each flagged axis
    v = np.arange(1.0, 9.0).reshape(2, 2, 2)          # v[z][y][x] = 1..8
    c = (vol3d.synthesis_matrix3(2, 2, 1).T @ v.ravel()).reshape(2, 2, 2)
    k = 2 * np.sqrt(2)
    assert abs(c[0, 0, 0] - 36 / k) < 1e-12
    assert abs(c[0, 0, 1] - (1 - 2 + 3 - 4 + 5 - 6 + 7 - 8) / k) < 1e-12      # tx
    assert abs(c[0, 1, 0] - (1 + 2 - 3 - 4 + 5 + 6 - 7 - 8) / k) < 1e-12      # ty
    assert abs(c[1, 0, 0] - (1 + 2 + 3 + 4 - 5 - 6 - 7 - 8) / k) < 1e-12      # tz
    assert abs(c[1, 1, 1] - (1 - 2 - 3 + 4 - 5 + 6 + 7 - 8) / k) < 1e-12      # tz ty tx


def test_z0_closed_form_and_coarse_grid_reduction():
    """Approximation-only octree: Z0 = 2^(-3L/2) max chord through the volume, and the
    whole solve equals voxel AM on the grid of root blocks."""
    g = synth.cone_geometry(16, 8, 9, 8, 30, sod=60.0, sdd=100.0)
    L = 1
    H = vol3d.system_matrix3(g)
    shapes = synth.make_ellipsoids(np.random.default_rng(3), g.n, g.nz, g.pixel, 4, 0.06, 0)
    o, e = vol3d.rays3(g)
    d = np.random.default_rng(4).poisson(2e4 * np.exp(-synth.line_integrals3(shapes, o, e))).astype(float)
    r = vol3d.wam_solve3(H, g.n, g.nz, L, d, 2e4, 5, g.pixel)
    lo = np.array([-8.0, -8.0, -4.0])
    chord = vol3d.box_chord3(o, e, lo, -lo)
    assert abs(r["z0"][0] - 2 ** (-1.5 * L) * chord.max()) <= 1e-12 * r["z0"][0]
    gc = synth.cone_geometry(8, 4, 9, 8, 30, sod=60.0, sdd=100.0, pixel=2.0)
    gc = synth.Geometry3(**{**gc.__dict__, "col_pitch": g.col_pitch, "row_pitch": g.row_pitch})
    Hc = vol3d.system_matrix3(gc)
    # pixel AM on the coarse grid (Omega = I), written with the generic 3-D solver (levels 0)
    rc = vol3d.wam_solve3(Hc, gc.n, gc.nz, 0, d, 2e4, 5, gc.pixel)
    mu = r["mu"][::2, ::2, ::2]
    np.testing.assert_allclose(mu, rc["mu"], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(r["idiv"], rc["idiv"], rtol=1e-11)


@pytest.fixture(scope="module")
def cone32():
    P = synth.make_cone_problem("cone32")
    return P, vol3d.system_matrix3(P.geom)


def test_monotone_across_expansions(cone32):
    P, H = cone32
    g = P.geom
    r = vol3d.wam_solve3(H, g.n, g.nz, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule)
    tr = r["idiv"]
    assert np.all(np.diff(tr) <= 1e-12 * np.abs(tr[:-1])), np.diff(tr)
    assert len(r["trees"]) == len(P.schedule) + 1
    assert vol3d.valid_mask3(r["mask"], P.levels)
    assert r["mask"].sum() > (g.n >> P.levels) ** 2 * (g.nz >> P.levels)


def test_fixed_point_and_tree_rule():
    g = synth.cone_geometry(8, 8, 6, 6, 14, sod=40.0, sdd=70.0)
    L = 2
    H = vol3d.system_matrix3(g)
    O = vol3d.synthesis_matrix3(g.n, g.nz, L)
    mask = vol3d.approx_mask3(g.n, g.nz, L)
    beta = np.zeros((g.nz, g.n, g.n))
    beta[:2, :2, :2] = np.random.default_rng(5).uniform(0.05, 0.2, (2, 2, 2)) * 2 ** (1.5 * L)
    # octree rule: only root (1, 0, 1) holds a value above 0.1 of the maximum
    beta2 = np.zeros_like(beta)
    beta2[1, 0, 1] = 1.0
    beta2[0, 1, 1] = 0.05
    new, count = vol3d.expand_tree3(beta2.ravel(), mask, L, 0.1, O)
    split = vol3d.split_flags3(new, L)
    expect = np.zeros((2, 2, 2), bool)
    expect[1, 0, 1] = True
    np.testing.assert_array_equal(split, expect)
    assert count == 1 and vol3d.valid_mask3(new, L)
    # noise-free data of beta on the tree: a fixed point
    d = 3e4 * np.exp(-(H @ (O @ beta.ravel())))
    r = vol3d.wam_solve3(H, g.n, g.nz, L, d, 3e4, 2, g.pixel, beta0=beta, mask0=mask)
    assert np.max(np.abs(r["beta"] - beta)) <= 1e-10
    assert abs(r["idiv"][-1]) <= 1e-8


def test_gradient_rule_scores_are_derivatives_and_solve_is_monotone():
    """Residual-gradient rule in 3-D: c = Omega^T H^T (d - q-hat) equals central differences of
    the I-divergence along single coefficients; consistent data split nothing; the solve with
    the rule stays monotone across expansions."""
    g = synth.cone_geometry(8, 8, 6, 6, 14, sod=40.0, sdd=70.0)
    L = 2
    H = vol3d.system_matrix3(g)
    O = vol3d.synthesis_matrix3(g.n, g.nz, L)
    shapes = synth.make_ellipsoids(np.random.default_rng(9), g.n, g.nz, g.pixel, 3, 0.08, 0)
    o, e = vol3d.rays3(g)
    i0 = 2e3
    d = np.random.default_rng(10).poisson(i0 * np.exp(-synth.line_integrals3(shapes, o, e))).astype(float)
    rng = np.random.default_rng(11)
    beta = rng.normal(0, 0.01, g.n_voxels)
    q = wam.beer_mean(i0, H @ (O @ beta))
    c = O.T @ (H.T @ (d - q))
    h = 1e-5
    f = lambda b: wam.idiv(d, wam.beer_mean(i0, H @ (O @ b)))
    for z in rng.choice(np.arange(g.n_voxels), 10, replace=False):
        ez = np.zeros_like(beta)
        ez[z] = h
        fd = (f(beta + ez) - f(beta - ez)) / (2 * h)
        assert abs(fd - c[z]) <= 1e-6 * max(1.0, abs(c[z])), (z, fd, c[z])
    mask = vol3d.approx_mask3(g.n, g.nz, L)
    b0 = np.zeros(g.n_voxels)
    b0.reshape(g.nz, g.n, g.n)[:g.nz >> L, :g.n >> L, :g.n >> L] = 0.1
    dq = wam.beer_mean(i0, H @ (O @ b0))
    new, count = vol3d.expand_tree3_gradient(b0, mask, L, 0.1, O, H, dq, i0)
    assert count == 0 and np.array_equal(new, mask)
    r = vol3d.wam_solve3(H, g.n, g.nz, L, d, i0, 8, g.pixel, schedule=[2, 5], rule="gradient")
    assert np.all(np.diff(r["idiv"]) <= 1e-12 * np.abs(r["idiv"][:-1]))
    assert vol3d.valid_mask3(r["mask"], L) and len(r["trees"]) == 3


# ------------------------------------------------------------------ sampled-ray helpers

def test_rays_by_index_and_sampled_projection():
    g = tiny_geom(8, 4, 5, 6, 12)
    o, e = vol3d.rays3(g)
    ids = np.array([0, 5, 71, 72, 200, g.n_rays - 1])
    o2, e2 = vol3d.rays3(g, ids=ids)
    np.testing.assert_allclose(o2, o[ids], atol=1e-13)
    np.testing.assert_allclose(e2, e[ids], atol=1e-15)
    vol = np.random.default_rng(2).uniform(0, 1, (g.nz, g.n, g.n))
    H = vol3d.system_matrix3(g)
    np.testing.assert_allclose(vol3d.project_rays3(g, vol, ids, rays_per_batch=4), (H @ vol.ravel())[ids],
                               rtol=1e-12, atol=1e-12)


def test_cascade_synthesis3_inverts_analysis_and_equals_omega():
    n, nz, L = 8, 8, 3
    coef = np.random.default_rng(3).normal(size=(nz, n, n))
    O = vol3d.synthesis_matrix3(n, nz, L)
    np.testing.assert_allclose(vol3d.cascade_synthesis3(coef, L).ravel(), O @ coef.ravel(), atol=1e-12)
    vol = np.random.default_rng(4).normal(size=(4, 8, 8))
    np.testing.assert_allclose(vol3d.cascade_synthesis3(vol3d.cascade_analysis3(vol, 2), 2), vol, atol=1e-12)
    rows = np.array([7, 0, 300, 511, 7])
    np.testing.assert_allclose(vol3d.synthesis_matrix3(n, nz, L, voxels=rows).toarray(), O[rows].toarray(), atol=0)


def test_sampled_projection_of_coefficients():
    g = tiny_geom(8, 8, 5, 6, 12)
    L = 2
    coef = np.random.default_rng(7).normal(size=(g.nz, g.n, g.n))
    ids = np.array([3, 40, 41, 170, 359])
    ref = (vol3d.system_matrix3(g) @ (vol3d.synthesis_matrix3(g.n, g.nz, L) @ coef.ravel()))[ids]
    np.testing.assert_allclose(vol3d.project_coef_rays3(g, coef, L, ids, rays_per_batch=2), ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(vol3d.project_rays3(g, vol3d.cascade_synthesis3(coef, L), ids), ref,
                               rtol=1e-12, atol=1e-12)


def test_box_shadow_holds_every_ray_through_the_box():
    g = tiny_geom(8, 4, 7, 9, 15)
    o, e = vol3d.rays3(g)
    exy, ez = vol3d.edges3(g)
    rng = np.random.default_rng(5)
    for _ in range(20):
        x0, x1 = np.sort(rng.choice(g.n + 1, 2, replace=False))
        y0, y1 = np.sort(rng.choice(g.n + 1, 2, replace=False))
        z0, z1 = np.sort(rng.choice(g.nz + 1, 2, replace=False))
        lo, hi = np.array([exy[x0], exy[y0], ez[z0]]), np.array([exy[x1], exy[y1], ez[z1]])
        hit = np.flatnonzero(vol3d.box_chord3(o, e, lo, hi) > 0)
        sh = vol3d.box_shadow3(g, lo, hi)
        assert np.isin(hit, sh).all()
        assert np.unique(sh).size == sh.size
    one = vol3d.box_shadow3(g, np.array([exy[3], exy[3], ez[1]]), np.array([exy[4], exy[4], ez[2]]))
    assert one.size < g.n_rays // 4


def test_node_phi_from_octant_clipping_equals_h_omega():
    g = tiny_geom(8, 8, 4, 7, 11)
    L = 2
    o, e = vol3d.rays3(g)
    Phi = (vol3d.system_matrix3(g) @ vol3d.synthesis_matrix3(g.n, g.nz, L)).tocsc()
    n = g.n
    rng = np.random.default_rng(6)
    for _ in range(8):
        lev = int(rng.integers(1, L + 1))
        k, i, j = (int(x) for x in rng.integers(0, n >> lev, 3))
        phis = vol3d.node_phi3(g, o, e, lev, k, i, j)
        keys = [key for key in phis if key != "approx"] + ([(k, i, j)] if lev == L else [])
        assert len(keys) == 7 + (lev == L)
        for key in keys:
            ref = phis["approx"] if key == (k, i, j) and lev == L else phis[key]
            col = Phi[:, (key[0] * n + key[1]) * n + key[2]].toarray().ravel()
            assert np.abs(col - ref).max() < 1e-12


def longest_chord(g):
    """Longest chord through the volume over every ray of the scan. The volume is invariant
    under 90-degree rotations about z and under the mirrors y -> -y and z -> -z; with the
    orbit starting at angle 0 in 720 equal steps and a detector centred on the central ray,
    these map the rays of view v onto those of views v + 180 and 720 - v, and row rr onto
    row n_rows - 1 - rr. Views 0..90 and the lower half of the rows therefore hold every
    chord length of the scan."""
    assert g.n_views % 4 == 0 and g.angle0 == 0.0 and abs(g.angle_span - 2 * math.pi) < 1e-15
    exy, ez = vol3d.edges3(g)
    lo, hi = np.array([exy[0], exy[0], ez[0]]), np.array([exy[-1], exy[-1], ez[-1]])
    rows = np.arange((g.n_rows + 1) // 2)
    cols = np.arange(g.n_cols)
    best = 0.0
    for v in range(g.n_views // 8 + 1):
        ids = ((v * g.n_rows + rows[:, None]) * g.n_cols + cols[None, :]).ravel()
        o, e = vol3d.rays3(g, ids=ids)
        best = max(best, float(vol3d.box_chord3(o, e, lo, hi).max()))
    return best


def test_longest_chord_symmetry_reduction():
    """The reduced scan of `longest_chord` finds the maximum of a full scan."""
    for g in (synth.cone_geometry(16, 8, 24, 10, 40, sod=40.0, sdd=80.0),
              synth.cone_geometry(16, 16, 16, 9, 33, sod=30.0, sdd=60.0)):
        o, e = vol3d.rays3(g)
        lo = np.array([-g.n / 2, -g.n / 2, -g.nz / 2]) * g.pixel
        assert abs(longest_chord(g) - vol3d.box_chord3(o, e, lo, -lo).max()) <= 1e-12 * g.n


def test_cone_central_column_at_quarter_turns_takes_the_plus_side():
    """Hand-derived: a 4x4x4 volume of 1 mm voxels, views at 0, 90, 180 and 270 degrees, 3
    detector columns (the central column's rays lie in the plane x = 0 at 90 and 270 degrees
    and y = 0 at 0 and 180, a voxel boundary) and 4 rows (no ray in the plane z = 0). Every
    voxel such a ray crosses is in voxel column (row) 2, the + side, and the chords of one ray
    add up to its path length through the volume."""
    g = synth.cone_geometry(4, 4, 4, 4, 3, sod=10.0, sdd=20.0)
    H = vol3d.system_matrix3(g).toarray().reshape(4, 4, 3, 4, 4, 4)   # [v][row][col][z][y][x]
    o, e = vol3d.rays3(g)
    for v in range(4):
        for rr in range(4):
            h = H[v, rr, 1]
            z, y, x = np.nonzero(h)
            assert z.size > 0
            if v % 2:
                assert np.all(x == 2), (v, rr, x)
            else:
                assert np.all(y == 2), (v, rr, y)
            ray = (v * 4 + rr) * 3 + 1
            exy, ez = vol3d.edges3(g)
            want = vol3d.box_chord3(o[ray:ray + 1], e[ray:ray + 1], np.array([[exy[2], -2.0, ez[0]]]) if v % 2
                                    else np.array([[-2.0, exy[2], ez[0]]]),
                                    np.array([[exy[3], 2.0, ez[-1]]]) if v % 2 else np.array([[2.0, exy[3], ez[-1]]]))
            np.testing.assert_allclose(h.sum(), want[0], atol=1e-12)


# ------------------------------------------------------------------ 2-D Haar per z-slice

def test_slice_haar_is_orthonormal_and_the_2d_cascade_per_slice():
    """The per-slice synthesis applies the textbook 2-D cascade to every slice on its own."""
    from oracle import haar
    n, nz, L = 8, 3, 2
    O = vol3d.slice_synthesis_matrix3(n, nz, L).toarray()
    np.testing.assert_allclose(O.T @ O, np.eye(n * n * nz), atol=1e-13)
    beta = np.random.default_rng(0).normal(size=(nz, n, n))
    mu = (O @ beta.ravel()).reshape(nz, n, n)
    for s in range(nz):
        np.testing.assert_allclose(mu[s], haar.cascade_synthesis(beta[s], L), atol=1e-13)


def _box_matrix(g, o, e, boxes_lo, boxes_hi):
    return vol3d.box_chord3(o[:, None, :], e[:, None, :], boxes_lo[None], boxes_hi[None])


def test_slice_node_phi_from_quadrant_clipping_equals_h_omega():
    """phi(y|z) of a per-slice detail = 2^-l (signed sum of its quadrants' chords) along cone
    rays, against the columns of H Omega; every level, nodes in several slices."""
    g = tiny_geom(8, 5, 4, 6, 12)
    L = 3
    o, e = vol3d.rays3(g)
    Phi = (vol3d.system_matrix3(g) @ vol3d.slice_synthesis_matrix3(g.n, g.nz, L)).toarray()
    for lev in range(1, L + 1):
        m = g.n >> lev
        for s in (0, 2, 4):
            for i, j in ((0, 0), (m - 1, 0), (m - 1, m - 1)):
                phis = vol3d.slice_node_phi3(g, o, e, lev, s, i, j)
                for (zr, zc), ph in zip(((i, m + j), (m + i, j), (m + i, m + j)), phis):
                    col = (s * g.n + zr) * g.n + zc
                    np.testing.assert_allclose(Phi[:, col], ph, atol=1e-12)


def test_slice_z0_closed_form_and_coarse_box_reduction():
    """Approximation-only per-slice tree: Z0 = 2^-L max chord through the volume, and the
    whole solve equals voxel AM over the 2^L x 2^L x 1 root boxes (system matrix of the boxes
    by direct box clipping), with mu constant on each box."""
    g = tiny_geom(8, 4, 5, 6, 12)
    L = 1
    o, e = vol3d.rays3(g)
    H = vol3d.system_matrix3(g)
    shapes = synth.make_ellipsoids(np.random.default_rng(7), g.n, g.nz, g.pixel, 3, 0.06, 0)
    d = np.random.default_rng(8).poisson(2e4 * np.exp(-synth.line_integrals3(shapes, o, e))).astype(float)
    r = vol3d.slice_wam_solve3(H, g.n, g.nz, L, d, 2e4, 6, g.pixel)
    lo = np.array([-g.n / 2, -g.n / 2, -g.nz / 2]) * g.pixel
    assert abs(r["z0"][0] - 2.0 ** -L * vol3d.box_chord3(o, e, lo, -lo).max()) <= 1e-12 * r["z0"][0]
    exy, ez = vol3d.edges3(g)
    nb, s_ = g.n >> L, 1 << L
    bs, bi, bj = np.meshgrid(np.arange(g.nz), np.arange(nb), np.arange(nb), indexing="ij")
    blo = np.stack([exy[bj.ravel() * s_], exy[bi.ravel() * s_], ez[bs.ravel()]], axis=1)
    bhi = np.stack([exy[(bj.ravel() + 1) * s_], exy[(bi.ravel() + 1) * s_], ez[bs.ravel() + 1]], axis=1)
    import scipy.sparse as sp
    Hc = sp.csr_matrix(_box_matrix(g, o, e, blo, bhi))
    rc = vol3d.wam_solve3(Hc, nb, g.nz, 0, d, 2e4, 6, g.pixel)
    np.testing.assert_allclose(r["mu"][:, ::s_, ::s_], rc["mu"], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(r["idiv"], rc["idiv"], rtol=1e-11)
    # and mu is constant on every root box
    np.testing.assert_allclose(r["mu"], np.repeat(np.repeat(rc["mu"], s_, 1), s_, 2), rtol=1e-10, atol=1e-13)


def test_slice_solve_is_monotone_across_expansions_and_noise_free_data_are_fixed():
    g = tiny_geom(16, 6, 8, 8, 24)
    L = 2
    o, e = vol3d.rays3(g)
    H = vol3d.system_matrix3(g)
    shapes = synth.make_ellipsoids(np.random.default_rng(9), g.n, g.nz, g.pixel, 5, 0.06, 1)
    d = np.random.default_rng(10).poisson(5e4 * np.exp(-synth.line_integrals3(shapes, o, e))).astype(float)
    r = vol3d.slice_wam_solve3(H, g.n, g.nz, L, d, 5e4, 12, g.pixel, schedule=[3, 7])
    tr = r["idiv"]
    assert np.all(tr[1:] <= tr[:-1] * (1 + 1e-13))
    assert len(r["trees"]) == 3 and r["trees"][2][1].sum() > r["trees"][0][1].sum()
    # consistent data from a slice-leaf-constant volume on the final tree: a fixed point
    from oracle import haar
    O = vol3d.slice_synthesis_matrix3(g.n, g.nz, L)
    beta = np.where(vol3d.slice_mask3(r["mask"], g.nz) > 0, r["beta"], 0.0)
    q = 3e4 * np.exp(-(H @ (O @ beta.ravel())))
    again = vol3d.slice_wam_solve3(H, g.n, g.nz, L, q, 3e4, 2, g.pixel, beta0=beta, mask0=r["mask"])
    np.testing.assert_allclose(again["beta"], beta, atol=1e-12)
    assert haar.valid_mask(r["mask"], L)


def test_slice_rule_splits_where_the_summed_image_exceeds_the_threshold():
    """Hand-made: two slices of 4x4 with 1-level nodes (2x2 blocks). Slice 0 holds 1.0 on the
    top-left block, both slices hold 0.06 on the bottom-right block: each 0.06 is below 0.1 x
    max, their sum 0.12 is above it, so the top-left and bottom-right roots split (shared by
    both slices) and the other two do not."""
    from oracle import haar
    n, nz, L = 4, 2, 1
    mu = np.zeros((nz, n, n))
    mu[0, :2, :2] = 1.0
    mu[:, 2:, 2:] = 0.06
    mu[1, 2:, :2] = 0.05                          # 0.05 in one slice only: stays
    beta = np.stack([haar.cascade_analysis(mu[s], L) for s in range(nz)])
    new, cnt = vol3d.expand_tree_slices3(beta, haar.approx_mask(n, L), L, 0.1, haar.synthesis_matrix(n, L))
    assert cnt == 2
    np.testing.assert_array_equal(haar.split_flags(new, 1), [[True, False], [False, True]])
