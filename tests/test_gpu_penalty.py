"""Roughness-penalized updates on the GPU against the FP64 oracle (oracle.wam.wam_solve with
penalty = lambda): the GPU solves each coefficient's root by safeguarded Newton, the oracle by
bisection on the same bracket.

  * FP64 with the GPU's own expansions (value rule): masks exact, beta relative L2 <= 1e-9,
    I-divergence rtol 1e-10; a two-scan stack likewise;
  * FP32: beta relative L2 <= 1e-4 and I-divergence rtol 2e-5 on a fixed tree; the final
    penalized objective I + lambda R (R from the GPU's synthesized image) within 1e-5 of the
    oracle's, and rougher images without the penalty;
  * lambda = 0 after a positive lambda gives back Algorithm 1 bit for bit;
  * errors: lambda < 0, the penalty with ordered subsets, a cone-beam context.
"""
import numpy as np
import pytest
import torch

from oracle import siddon, wam
from paper_1508_04458_amd import synth
from test_gpu_parity import dev, host, make_ctx, problem, rel_l2

pytestmark = pytest.mark.gpu

LAM = 1e6


@pytest.mark.parametrize("name", ["parallel64", "fan96"])
def test_penalty_matches_oracle_fp64(name):
    P, H = problem(name)
    g = P.geom
    ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule, penalty=LAM)
    c = make_ctx(g, P.levels, "f64")
    c.set_penalty(LAM)
    assert c.penalty() == LAM
    c.set_data(dev(P.d, "f64"), P.i0)
    idv = host(c.solve(P.n_iters, P.schedule, 0.1))
    beta, mask, _ = c.get_state()
    np.testing.assert_array_equal(host(mask), ref["mask"])
    assert rel_l2(host(beta), ref["beta"]) <= 1e-9
    np.testing.assert_allclose(idv, ref["idiv"], rtol=1e-10)
    assert np.all(np.diff(ref["objective"]) <= 1e-12 * np.abs(ref["objective"][:-1]))


def test_penalty_stack_fp64():
    from paper_1508_04458_amd import api
    probs = [synth.make_problem("fan96", problem_idx=k, i0=i0) for k, i0 in enumerate((5e4, 2e4))]
    g = probs[0].geom
    H = siddon.system_matrix(g)
    print(f"\n[stack] fan96 x2 penalty f64", flush=True)
    c = api.Context(g, probs[0].levels, "f64", batch=2)
    c.set_penalty(LAM)
    c.set_data(dev(np.concatenate([P.d for P in probs]), "f64"), [P.i0 for P in probs])
    J, sched = 10, [3, 6]
    idv = host(c.solve(J, sched, 0.1))
    beta = host(c.get_state()[0])
    for p, P in enumerate(probs):
        ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, J, g.pixel, schedule=sched, penalty=LAM)
        assert rel_l2(beta[p], ref["beta"]) <= 1e-9
        np.testing.assert_allclose(idv[p], ref["idiv"], rtol=1e-10)


def test_penalty_fp32_fixed_tree():
    P, H = problem("fan128")
    g = P.geom
    J = 10
    ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, J, g.pixel, penalty=LAM)
    c = make_ctx(g, P.levels, "f32", P.d, P.i0)
    c.set_penalty(LAM)
    idv = host(c.solve(J))
    assert rel_l2(host(c.get_state()[0]), ref["beta"]) <= 1e-4
    np.testing.assert_allclose(idv, ref["idiv"], rtol=2e-5)
    mu = host(c.synthesize())
    obj = idv[-1] + LAM * wam.roughness(mu)
    assert abs(obj - ref["objective"][-1]) <= 1e-5 * ref["objective"][-1]
    plain = make_ctx(g, P.levels, "f32", P.d, P.i0)
    plain.solve(J)
    assert wam.roughness(host(plain.synthesize())) > wam.roughness(mu)


def test_penalty_zero_is_algorithm_1():
    P, _ = problem("fan96")
    a = make_ctx(P.geom, P.levels, "f32", P.d, P.i0)
    b = make_ctx(P.geom, P.levels, "f32", P.d, P.i0)
    b.set_penalty(LAM)
    b.set_penalty(0.0)
    ia, ib = host(a.solve(8, [3], 0.1)), host(b.solve(8, [3], 0.1))
    np.testing.assert_array_equal(ia, ib)
    np.testing.assert_array_equal(host(a.get_state()[0]), host(b.get_state()[0]))


def test_penalty_errors():
    from paper_1508_04458_amd import _lib, api
    P, _ = problem("fan96")
    c = make_ctx(P.geom, P.levels, "f32")
    with pytest.raises(_lib.WamctError) as e:
        c.set_penalty(-1.0)
    assert e.value.status == _lib.E_INVALID
    c.set_subsets(3)
    with pytest.raises(_lib.WamctError) as e:
        c.set_penalty(1.0)
    assert e.value.status == _lib.E_UNSUPPORTED
    c.set_subsets(1)
    c.set_penalty(1.0)
    with pytest.raises(_lib.WamctError) as e:
        c.set_subsets(3)
    assert e.value.status == _lib.E_UNSUPPORTED
    c3 = api.Context(synth.CONE_CONFIGS["cone32"]["geom"](), 2, "f32")
    with pytest.raises(_lib.WamctError) as e:
        c3.set_penalty(1.0)
    assert e.value.status == _lib.E_UNSUPPORTED
