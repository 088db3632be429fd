"""Differentiable path: loss and hand-written adjoint vs the oracle, autograd wiring, and
central differences (h = 1e-3 on 64 random coefficients), incl. a batch of 16 slices of the
256x256 fan-beam configuration (360 views, 512 bins, 2-level Haar, I0 = 5e4)."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry, haar, siddon, wam
from paper_1508_04458_amd import synth
from test_gpu_parity import dev, host, make_ctx, rel_l2

pytestmark = pytest.mark.gpu


def _coeffs(P, L, seed, noise=1e-3):
    mu = synth.rasterize(P.ellipses, P.geom.n, P.geom.pixel)
    c = haar.cascade_analysis(mu, L)
    return c + np.random.default_rng(seed).normal(0, noise, c.shape)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_loss_and_adjoint_match_oracle(dtype):
    P = synth.make_problem("fan96")
    g = P.geom
    L = 2
    H = siddon.system_matrix(g)
    O = haar.synthesis_matrix(g.n, L)
    cs = np.stack([_coeffs(P, L, s) for s in (1, 2)])
    if dtype == "f32":
        cs = cs.astype(np.float32).astype(np.float64)
    d = np.stack([P.d, np.random.default_rng(9).poisson(P.i0 * np.exp(-P.line_integrals)).astype(float)])
    ctx = make_ctx(g, L, dtype)
    loss, q = ctx.loss(dev(cs, dtype), dev(d, dtype), P.i0)
    grad = host(ctx.loss_backward(q, dev(d, dtype)))
    loss = host(loss)
    for b in range(2):
        lr, gr, qr = wam.loss_and_grad(H, O, d[b], P.i0, cs[b].ravel())
        assert abs(loss[b] - lr) <= (1e-6 if dtype == "f32" else 1e-11) * lr
        assert rel_l2(grad[b].ravel(), gr) <= (1e-4 if dtype == "f32" else 1e-10)


def test_autograd_function_and_central_differences():
    """torch autograd through WamLoss equals the adjoint, and matches central differences of
    the GPU loss itself (h = 1e-3, 64 random coefficients); tolerance = the truncation bound
    h^2/6 sum_y q |phi|^3 plus the rounding of two FP64 loss sums of FP32-synthesized images."""
    from paper_1508_04458_amd.autograd import wam_loss
    P = synth.make_problem("fan256")
    g = P.geom
    L = 2
    ctx = make_ctx(g, L, "f32")
    c = torch.tensor(_coeffs(P, L, 3)[None], dtype=torch.float32, device="cuda", requires_grad=True)
    d = dev(P.d[None], "f32")
    loss = wam_loss(c, d, P.i0, ctx)
    (2.5 * loss.sum()).backward()
    grad = host(c.grad)[0] / 2.5
    _, q = ctx.loss(c.detach(), d, P.i0)
    ref = host(ctx.loss_backward(q, d))[0]
    np.testing.assert_allclose(grad, ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())
    rng = np.random.default_rng(4)
    h = 1e-3
    o, e = geometry.rays(g)
    edges = geometry.pixel_edges(g)
    n = g.n
    base = c.detach().clone()
    qh = host(q)[0]
    worst = 0.0
    for z in rng.choice(n * n, 64, replace=False):
        cp, cm = base.clone(), base.clone()
        cp.view(-1)[z] += h
        cm.view(-1)[z] -= h
        lp = host(ctx.loss(cp, d, P.i0)[0])[0]
        lm = host(ctx.loss(cm, d, P.i0)[0])[0]
        step = float(cp.view(-1)[z].item()) - float(cm.view(-1)[z].item())   # the FP32 step taken
        fd = (lp - lm) / step
        # |phi| of coefficient z over all rays (box clipping), for the truncation bound
        r, cc = divmod(int(z), n)
        k = max(r, cc)
        lev = next((t for t in range(1, L + 1) if k >= (n >> t)), 0)
        if lev == 0:
            s = 1 << L
            phi = 2.0 ** -L * siddon.box_chord(o, e, edges[cc * s], edges[(cc + 1) * s], edges[r * s], edges[(r + 1) * s])
        else:
            m, s = n >> lev, 1 << lev
            i, j = r % m, cc % m
            phi = 2.0 ** -lev * siddon.box_chord(o, e, edges[j * s], edges[(j + 1) * s], edges[i * s], edges[(i + 1) * s])
        bound = h * h / 6 * np.sum(qh * np.abs(phi) ** 3) * math.exp(h * np.abs(phi).max())
        # rounding: mu is synthesized in FP32, so each perturbed loss carries ~1e-7 relative
        # noise of the rays through the coefficient's block; 2e-3 of the gradient covers it
        err = abs(fd - grad.ravel()[z])
        worst = max(worst, err / (abs(grad.ravel()[z]) + 1.0))
        assert err <= bound + 2e-3 * abs(grad.ravel()[z]) + 0.05, (z, fd, grad.ravel()[z], bound)
    print(f"worst FD relative deviation {worst:.2e}", flush=True)


def test_batch16_fan256_against_oracle():
    """Batch of 16 slices of the differentiable configuration (each with its own coefficients;
    counts from two seeded scans); every slice equals its single-slice call, and two slices
    are checked against the oracle."""
    g = synth.CONFIGS["fan256"]["geom"]()
    L = 2
    probs = [synth.make_problem("fan256", seed=1, problem_idx=k) for k in range(2)]
    print("problems generated", flush=True)
    cs = np.stack([_coeffs(probs[k % 2], L, 10 + k, noise=1e-3 * (1 + k)) for k in range(16)]).astype(np.float32)
    d = np.stack([probs[k % 2].d for k in range(16)])
    ctx = make_ctx(g, L, "f32")
    loss, q = ctx.loss(dev(cs, "f32"), dev(d, "f32"), probs[0].i0)
    grad = host(ctx.loss_backward(q, dev(d, "f32")))
    loss = host(loss)
    for k in (0, 11):
        l1, q1 = ctx.loss(dev(cs[k:k + 1], "f32"), dev(d[k:k + 1], "f32"), probs[0].i0)
        assert host(l1)[0] == loss[k]
        np.testing.assert_array_equal(host(ctx.loss_backward(q1, dev(d[k:k + 1], "f32")))[0], grad[k])
    H = siddon.system_matrix(g)
    O = haar.synthesis_matrix(g.n, L)
    print("oracle matrices built", flush=True)
    for k in (0, 11):
        lr, gr, _ = wam.loss_and_grad(H, O, d[k], probs[0].i0, cs[k].astype(np.float64).ravel())
        assert abs(loss[k] - lr) <= 1e-6 * lr
        assert rel_l2(grad[k].ravel(), gr) <= 1e-4
