"""The residual-gradient tree rule on the GPU against the FP64 oracle
(oracle.wam.expand_tree_gradient inside oracle.wam.wam_solve).

  * FP64 with the GPU's own expansions: masks exact, beta relative L2 <= 1e-9, I-divergence
    rtol 1e-10, held counts equal (one scan; a stack of scans with their own data and I0);
  * FP32: the I-divergence falls at every iteration (factor 1 + 1e-6) and ends within 1e-3
    of the oracle's (leaf decisions near the threshold may differ in FP32);
  * a batch holding a gradient-rule context gives bitwise that context's own solve;
  * cone beam (3-D octree, seven details per node): FP64 against the 3-D oracle as above;
  * errors: unknown rule, the rule with tree sharing.
"""
import numpy as np
import pytest
import torch

from oracle import siddon, wam
from paper_1508_04458_amd import synth
from test_gpu_parity import dev, host, make_ctx, problem, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["parallel64", "fan96"])
def test_gradient_rule_matches_oracle_fp64(name):
    P, H = problem(name)
    g = P.geom
    ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule, rule="gradient")
    c = make_ctx(g, P.levels, "f64")
    c.set_tree_rule("gradient")
    assert c.tree_rule() == "gradient"
    c.set_data(dev(P.d, "f64"), P.i0)
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    beta, mask, _ = c.get_state()
    np.testing.assert_array_equal(host(mask), ref["mask"])
    assert rel_l2(host(beta), ref["beta"]) <= 1e-9
    np.testing.assert_allclose(idv, ref["idiv"], rtol=1e-10)
    assert c.tree_stats()["n_held"] == ref["held"]
    # the rule grows a different tree than the value rule on this phantom
    ref_v = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule)
    assert not np.array_equal(ref_v["mask"], ref["mask"])


def test_gradient_rule_stack_fp64():
    from paper_1508_04458_amd import api
    probs = [synth.make_problem("fan96", problem_idx=k, i0=i0) for k, i0 in enumerate((5e4, 2e4))]
    g = probs[0].geom
    H = siddon.system_matrix(g)
    print(f"\n[stack] fan96 x2 gradient rule f64", flush=True)
    c = api.Context(g, probs[0].levels, "f64", batch=2)
    c.set_tree_rule("gradient")
    c.set_data(dev(np.concatenate([P.d for P in probs]), "f64"), [P.i0 for P in probs])
    J, sched = 10, [2, 5, 8]
    idv = host(c.solve(J, sched, 0.1))
    beta, mask, _ = c.get_state()
    for p, P in enumerate(probs):
        ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, J, g.pixel, schedule=sched, rule="gradient")
        np.testing.assert_array_equal(host(mask[p]), ref["mask"])
        assert rel_l2(host(beta[p]), ref["beta"]) <= 1e-9
        np.testing.assert_allclose(idv[p], ref["idiv"], rtol=1e-10)


def test_gradient_rule_fp32_monotone():
    P, H = problem("fan128")
    g = P.geom
    c = make_ctx(g, P.levels, "f32", P.d, P.i0)
    c.set_tree_rule("gradient")
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    assert np.all(idv[1:] <= idv[:-1] * (1 + 1e-6)), np.max(idv[1:] / idv[:-1])
    ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule, rule="gradient")
    assert abs(idv[-1] - ref["idiv"][-1]) <= 1e-3 * ref["idiv"][-1]


def test_gradient_rule_context_in_a_batch():
    from paper_1508_04458_amd import api
    P1, _ = problem("fan96")
    P2, _ = problem("fan128")
    J, sched = 12, [3, 6, 9]
    solo = make_ctx(P1.geom, P1.levels, "f32", P1.d, P1.i0)
    solo.set_tree_rule("gradient")
    i_solo = host(solo.solve(J, sched, 0.1))
    c1 = make_ctx(P1.geom, P1.levels, "f32", P1.d, P1.i0)
    c1.set_tree_rule("gradient")
    c2 = make_ctx(P2.geom, P2.levels, "f32", P2.d, P2.i0)
    b = api.Batch([c1, c2], n_streams=2)
    tr = b.solve(J, sched, 0.1)
    np.testing.assert_array_equal(host(tr[0]), i_solo)
    np.testing.assert_array_equal(host(c1.get_state()[0]), host(solo.get_state()[0]))


def test_tree_rule_errors():
    from paper_1508_04458_amd import _lib
    P, _ = problem("fan96")
    c = make_ctx(P.geom, P.levels, "f32")
    with pytest.raises(ValueError):
        c.set_tree_rule("edges")
    with pytest.raises(_lib.WamctError) as e:
        _lib.check(_lib.lib.wamct_set_tree_rule(c._h, 7), c._h)
    assert e.value.status == _lib.E_INVALID
    c.set_tree_rule("gradient")
    with pytest.raises(_lib.WamctError) as e:
        c.set_tree_sharing(True)
    assert e.value.status == _lib.E_UNSUPPORTED
    c.set_tree_rule("value")
    c.set_tree_sharing(True)
    with pytest.raises(_lib.WamctError) as e:
        c.set_tree_rule("gradient")
    assert e.value.status == _lib.E_UNSUPPORTED


def test_gradient_rule_cone_fp64():
    """Cone beam, 3-D octree: the rule with the seven details of each node."""
    from oracle import vol3d
    from paper_1508_04458_amd import api
    P = synth.make_cone_problem("cone32")
    g = P.geom
    H = vol3d.system_matrix3(g)
    ref = vol3d.wam_solve3(H, g.n, g.nz, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule,
                           rule="gradient")
    print("\n[case] cone32 gradient rule f64", flush=True)
    c = api.Context(g, P.levels, "f64")
    c.set_tree_rule("gradient")
    c.set_data(dev(P.d, "f64"), P.i0)
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    beta, mask, _ = c.get_state()
    np.testing.assert_array_equal(host(mask), ref["mask"])
    assert rel_l2(host(beta), ref["beta"]) <= 1e-9
    np.testing.assert_allclose(idv, ref["idiv"], rtol=1e-10)
    assert c.tree_stats()["n_held"] == ref["held"]
