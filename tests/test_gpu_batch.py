"""Stacks of scans in one context and uneven batches of contexts, against the FP64 oracle
and against the same contexts solved one at a time.

  * a stack (several scans of one geometry, each with its own data, I0 and tree) gives,
    per scan, the oracle's solve (FP64: masks exact, beta relative L2 <= 1e-9, I-div
    rtol 1e-10);
  * a batch (contexts of different image sizes and view counts, replayed from a captured
    HIP graph or launched directly on several streams) gives bitwise the results of each
    context solved alone, and the oracle's per scan;
  * the tiling autotuner only changes summation order.
"""
import collections

import numpy as np
import pytest
import torch

from oracle import siddon, wam
from paper_1508_04458_amd import synth
from test_gpu_parity import dev, host, rel_l2

pytestmark = pytest.mark.gpu

SMALL = dict(sizes=(32, 48, 64), views=(40, 60))
N_IT = 20


def _api():
    from paper_1508_04458_amd import api
    return api


def _stack_ctx(problems, dtype):
    P0 = problems[0]
    g = P0.geom
    print(f"\n[stack] n={g.n} views={g.n_views} bins={g.n_bins} scans={len(problems)} {dtype}", flush=True)
    c = _api().Context(g, P0.levels, dtype, batch=len(problems))
    d = np.concatenate([P.d for P in problems])
    c.set_data(dev(d, dtype), [P.i0 for P in problems])
    return c


def _uneven_contexts(n_problems, seed, dtype):
    specs = synth.uneven_specs(n_problems, seed, **SMALL)
    probs = synth.make_uneven_batch(specs, seed, n_iters=N_IT)
    classes = collections.defaultdict(list)
    for P in probs:
        classes[(P.geom.n, P.geom.n_views)].append(P)
    keys = sorted(classes)
    return [(_stack_ctx(classes[k], dtype), classes[k]) for k in keys]


def test_stack_matches_oracle_per_scan_fp64():
    """Three fan96 scans with their own phantoms and I0, plus a scan with zero counts
    whose coefficients are all held and whose tree never grows."""
    probs = [synth.make_problem("fan96", problem_idx=k, i0=i0) for k, i0 in enumerate((5e4, 2e4, 8e4))]
    g = probs[0].geom
    zero = synth.Problem(g, np.zeros(g.n_rays), 3e4, probs[0].ellipses, probs[0].line_integrals,
                         probs[0].levels, probs[0].n_iters, probs[0].schedule, "f64")
    stack = probs + [zero]
    c = _stack_ctx(stack, "f64")
    P0 = probs[0]
    idv = host(c.solve(P0.n_iters, P0.schedule, 0.1))
    beta, mask, it = c.get_state()
    beta, mask = host(beta), host(mask)
    assert it == P0.n_iters and idv.shape == (4, P0.n_iters + 1)
    H = siddon.system_matrix(g)
    st = c.tree_stats()
    for k, P in enumerate(probs):
        ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule)
        np.testing.assert_array_equal(mask[k], ref["mask"])
        assert rel_l2(beta[k].ravel(), ref["beta"].ravel()) <= 1e-9, k
        np.testing.assert_allclose(idv[k], ref["idiv"], rtol=1e-10)
        assert st["n_held"][k] == ref["held"], k
    roots = (g.n >> P0.levels) ** 2
    assert np.all(beta[3] == 0)
    assert st["n_active"][3] == roots
    assert st["n_held"][3] == roots * P0.n_iters


def test_stack_rejects_bad_scalar_i0():
    from paper_1508_04458_amd import _lib
    g = synth.fan_geometry(32, 20, 48)
    c = _api().Context(g, 1, "f32", batch=2)
    d = dev(np.ones(2 * g.n_rays), "f32")
    with pytest.raises(_lib.WamctError) as e:
        c.set_data(d, [100.0, -1.0])
    assert e.value.status == _lib.E_INVALID
    with pytest.raises(ValueError):
        c.set_data(d, [100.0])
    c.set_data(d, [100.0, 50.0])


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_each_context_alone(graph):
    """FP32, uneven sizes: the batch reproduces every context's own solve bit for bit."""
    ctxs = _uneven_contexts(7, 3, "f32")
    P0 = ctxs[0][1][0]
    alone = []
    for c, _ in ctxs:
        idv = host(c.solve(N_IT, P0.schedule, 0.1))
        beta, mask, _ = c.get_state()
        alone.append((idv, host(beta), host(mask)))
        c.reset()
    batch = _api().Batch([c for c, _ in ctxs], n_streams=3, graph=graph)
    out = batch.solve(N_IT, P0.schedule, 0.1)
    for (c, _), (idv, beta, mask), got in zip(ctxs, alone, out):
        b2, m2, it = c.get_state()
        assert it == N_IT
        np.testing.assert_array_equal(host(got), idv)
        np.testing.assert_array_equal(host(b2), beta)
        np.testing.assert_array_equal(host(m2), mask)
    st = batch.stats()
    if graph:
        assert st["graph_launches"] == N_IT
        assert st["captures"] == len(P0.schedule) + 1
    else:
        assert st["graph_launches"] == 0
    # a second solve after a batch reset gives the same again
    batch.reset()
    again = batch.solve(N_IT, P0.schedule, 0.1)
    for a, b in zip(out, again):
        np.testing.assert_array_equal(host(a), host(b))


def test_batch_matches_oracle_and_autotune_keeps_results_fp64():
    """FP64 uneven batch after autotuning (tiling and leaf-walk lanes per ray): every scan
    matches the oracle's solve."""
    ctxs = _uneven_contexts(5, 4, "f64")
    batch = _api().Batch([c for c, _ in ctxs], n_streams=2, graph=True)
    cand = [1 << 12, 1 << 16, 1 << 20]
    chosen = batch.autotune(1, cand)
    assert len(chosen) == len(ctxs) and all(v in cand for v in chosen)
    assert [c.tiling() for c, _ in ctxs] == chosen
    assert all(c.walk_lanes() in (1, 2, 4) for c, _ in ctxs)     # the second, measured knob
    P0 = ctxs[0][1][0]
    out = batch.solve(N_IT, P0.schedule, 0.1)
    for (c, probs), idv in zip(ctxs, out):
        g = probs[0].geom
        H = siddon.system_matrix(g)
        beta, mask, _ = c.get_state()
        beta, mask, idv = host(beta), host(mask), host(idv)
        if len(probs) == 1:
            beta, mask, idv = beta[None], mask[None], idv[None]
        for k, P in enumerate(probs):
            ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, N_IT, g.pixel, schedule=P.schedule)
            np.testing.assert_array_equal(mask[k], ref["mask"])
            assert rel_l2(beta[k].ravel(), ref["beta"].ravel()) <= 1e-9, (g.n, g.n_views, k)
            np.testing.assert_allclose(idv[k], ref["idiv"], rtol=1e-10)


def test_tiling_changes_only_summation_order():
    P = synth.make_problem("fan128")
    out = []
    for lanes in (1 << 12, 1 << 20, 1 << 24):
        c = _api().Context(P.geom, P.levels, "f64")
        c.set_tiling(lanes)
        assert c.tiling() == lanes
        c.set_data(dev(P.d, "f64"), P.i0)
        out.append((host(c.solve(12, [3, 6, 9], 0.1)), host(c.get_state()[0])))
    for idv, beta in out[1:]:
        np.testing.assert_allclose(idv, out[0][0], rtol=1e-12)
        assert rel_l2(beta, out[0][1]) <= 1e-11


# ------------------------------------------------------------------ slices sharing one tree

def test_shared_tree_slices_match_oracle_fp64():
    """Three z-slices (own phantoms and I0) sharing one tree grown on the slice-summed image:
    every slice's solve equals the oracle's (shared mask exact, beta 1e-9, I-div 1e-10)."""
    probs = [synth.make_problem("fan96", problem_idx=k, i0=i0) for k, i0 in enumerate((5e4, 2e4, 8e4))]
    g = probs[0].geom
    P0 = probs[0]
    c = _stack_ctx(probs, "f64")
    c.set_tree_sharing(True)
    assert c.tree_sharing()
    idv = host(c.solve(P0.n_iters, P0.schedule, 0.1))
    beta, mask, _ = c.get_state()
    beta, mask = host(beta), host(mask)
    ref = wam.volume_wam_solve(siddon.system_matrix(g), g.n, P0.levels, [P.d for P in probs],
                               [P.i0 for P in probs], P0.n_iters, g.pixel, schedule=P0.schedule)
    for k in range(len(probs)):
        np.testing.assert_array_equal(mask[k], ref["mask"])
        assert rel_l2(beta[k].ravel(), ref["betas"][k].ravel()) <= 1e-9, k
        np.testing.assert_allclose(idv[k], ref["idiv"][k], rtol=1e-10)
    assert sum(c.tree_stats()["n_held"]) == ref["held"]


def test_shared_tree_of_identical_slices_is_the_single_tree():
    P = synth.make_problem("fan96")
    g = P.geom
    one = _api().Context(g, P.levels, "f64")
    one.set_data(dev(P.d, "f64"), P.i0)
    i1 = host(one.solve(P.n_iters, P.schedule, 0.1))
    two = _stack_ctx([P, P], "f64")
    two.set_tree_sharing(True)
    i2 = host(two.solve(P.n_iters, P.schedule, 0.1))
    b2, m2, _ = two.get_state()
    b1, m1, _ = one.get_state()
    for k in range(2):
        np.testing.assert_array_equal(host(m2)[k], host(m1))
        np.testing.assert_allclose(i2[k], i1, rtol=1e-12)
        assert rel_l2(host(b2)[k], host(b1)) <= 1e-12
