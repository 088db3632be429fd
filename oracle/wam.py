"""Wavelet-domain alternating minimization, FP64 (test infrastructure; see oracle/__init__.py).

Written from the Introduction and Results sections of the paper, in its notation:

  * I(p||q) = sum_i p_i log(p_i / q_i) - p_i + q_i            (footnote to the Introduction)
  * q(mu)(y) = I0(y) exp(-sum_x h(y|x) mu(x))                    (Introduction)
  * mu = Omega beta, Phi = H Omega                               (eq. 1.2, text after eq. 1.4)
  * b(z) = sum_y d(y) phi(y|z)                                   (eq. 1.6)
  * Z0 = max_y sum_{z in Z_s} |phi(y|z)|                         (eq. 1.61)
  * b-hat+(z) = sum_{y: phi>0} q-hat(y) phi(y|z),
    b-hat-(z) = sum_{y: phi<0} q-hat(y) phi(y|z)  (<= 0)        (eq. 1.10)
  * new beta(z): the zero of
    b - b-hat+ exp(-Z0 (beta - beta-hat)) - b-hat- exp(Z0 (beta - beta-hat))   (eq. 1.9)
  * Algorithm 1 (unregularized wavelet AM) over a sequence of active sets Z_s^(j)
  * the tree rule of the Results section: start from approximation coefficients only; at
    the scheduled iterations synthesize the image, and every tree leaf containing a pixel
    whose value exceeds frac * max(image) is expanded by one level.

Readings where the paper is silent (each is listed with its reason in the design notes):
  beta(0) = 0; inactive coefficients are 0 and new ones start at 0; no non-negativity
  projection (Algorithm 1 applies none); Z0 is one scalar over all rays, recomputed when
  the tree changes; the tree is expanded *before* update j for each scheduled j; entries
  of Phi with |phi| <= 1e-12 * pixel are cancellation residue and are dropped; when eq. 1.9
  has no finite zero (b-hat+ = 0 with b >= 0 and b-hat- < 0 ... see `closed_form_update`)
  the coefficient is held and counted.
"""
import numpy as np
import scipy.sparse as sp

from . import haar


def idiv(d, q):
    """I-divergence I(d||q) with 0 log 0 = 0 (footnote to the Introduction)."""
    d = np.asarray(d, np.float64)
    q = np.asarray(q, np.float64)
    pos = d > 0
    out = np.sum(q - d)
    out += np.sum(d[pos] * np.log(d[pos] / q[pos]))
    return float(out)


def beer_mean(i0, p):
    """q(y) = I0(y) exp(-p(y)) (Introduction)."""
    return np.asarray(i0, np.float64) * np.exp(-np.asarray(p, np.float64))


def active_index(mask):
    return np.flatnonzero(np.asarray(mask).ravel())


def phi_matrix(H, Omega, mask, pixel):
    """Phi_s = H Omega restricted to the active columns (CSR, M x |Z_s|)."""
    act = active_index(mask)
    Phi = (H @ Omega[:, act]).tocsr()
    Phi.data[np.abs(Phi.data) <= 1e-12 * pixel] = 0.0
    Phi.eliminate_zeros()
    return Phi, act


def split_phi(Phi):
    """(Phi+, Phi-): the positive and negative entries of Phi (eq. 1.10)."""
    pos = Phi.copy()
    pos.data = np.maximum(pos.data, 0.0)
    pos.eliminate_zeros()
    neg = Phi.copy()
    neg.data = np.minimum(neg.data, 0.0)
    neg.eliminate_zeros()
    return pos, neg


def z0_of(Phi):
    """Z0 = max over rays of sum_{z in Z_s} |phi(y|z)| (eq. 1.61)."""
    return float(np.max(np.asarray(abs(Phi).sum(axis=1)).ravel()))


def closed_form_update(b, bp, bm, z0):
    """Zero of eq. 1.9 for each coefficient -> (delta = beta_new - beta_hat, held mask).

    With t = exp(-Z0 delta) > 0, eq. 1.9 = 0 reads bp t^2 - b t + bm = 0 (bp >= 0 >= bm).
      * bp > 0: the positive root t = (b + s) / (2 bp), s = sqrt(b^2 - 4 bp bm), written
        as 2 bm / (b - s) when b < 0 (same value, no cancellation); if t <= 0 (bm = 0
        and b <= 0) the surrogate has no finite minimizer.
      * bp = 0, bm < 0: the equation is linear, t = bm / b, finite only if b < 0.
      * bp = bm = 0: no ray sees the coefficient; delta = 0.
    Coefficients without a finite minimizer keep their value (delta = 0) and are
    reported in `held`."""
    b = np.asarray(b, np.float64)
    bp = np.asarray(bp, np.float64)
    bm = np.asarray(bm, np.float64)
    t = np.full(b.shape, np.nan)
    s = np.sqrt(b * b - 4.0 * bp * bm)
    quad = bp > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        t_pos = np.where(b >= 0, (b + s) / (2.0 * bp), 2.0 * bm / (b - s))
        t_lin = bm / b
    t = np.where(quad, t_pos, t)
    lin = (~quad) & (bm < 0)
    t = np.where(lin, t_lin, t)
    none = (~quad) & (bm == 0)
    ok = np.isfinite(t) & (t > 0)
    delta = np.zeros(b.shape)
    delta[ok] = -np.log(t[ok]) / z0
    held = ~ok & ~none
    return delta, held


# ------------------------------------------------------------------ roughness penalty (NEXT-3)
# The Introduction's objective adds lambda R(mu) with a roughness penalty whose form it does not
# give. Reading: R(mu) = 1/2 sum over horizontally and vertically adjacent pixel pairs of
# (mu_x - mu_x')^2. Its Hessian (a graph Laplacian) is below 8 I (Gershgorin: degree <= 4), and
# Omega is orthonormal, so at beta-hat R(Omega beta) <= R + g^T delta + (8 / 2) |delta|^2 with
# g = Omega^T grad R(mu-hat): a separable quadratic surrogate added to eq. 1.8's.
PENALTY_CURVATURE = 8.0


def roughness(mu):
    mu = np.asarray(mu, np.float64)
    dh = mu[:, 1:] - mu[:, :-1]
    dv = mu[1:, :] - mu[:-1, :]
    return 0.5 * float((dh * dh).sum() + (dv * dv).sum())


def roughness_grad(mu):
    """dR/dmu_x = sum over the 4-neighbours x' of x of (mu_x - mu_x')."""
    mu = np.asarray(mu, np.float64)
    g = np.zeros_like(mu)
    dh = mu[:, 1:] - mu[:, :-1]
    g[:, 1:] += dh
    g[:, :-1] -= dh
    dv = mu[1:, :] - mu[:-1, :]
    g[1:, :] += dv
    g[:-1, :] -= dv
    return g


def penalized_update(b, bp, bm, z0, lam, g, iters=200):
    """Minimizer of eq. 1.8's surrogate plus lam (g delta + 4 delta^2) for each coefficient:
    the root of G(delta) = b - bp exp(-Z0 delta) - bm exp(Z0 delta) + lam (g + 8 delta), an
    increasing function (bp >= 0 >= bm, lam > 0). G(0) fixes the side of the root and
    |delta| <= |G(0)| / (8 lam) bounds it; plain bisection on that bracket."""
    b, bp, bm, g = (np.asarray(x, np.float64) for x in (b, bp, bm, g))

    def G(dl):
        with np.errstate(over="ignore", invalid="ignore"):
            ep = np.where(bp != 0, bp * np.exp(-z0 * dl), 0.0)
            em = np.where(bm != 0, bm * np.exp(z0 * dl), 0.0)
        return b - ep - em + lam * (g + PENALTY_CURVATURE * dl)

    g0 = G(np.zeros_like(b))
    width = np.abs(g0) / (PENALTY_CURVATURE * lam)
    lo = np.where(g0 > 0, -width, 0.0)
    hi = np.where(g0 > 0, 0.0, width)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        neg = G(mid) < 0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    return 0.5 * (lo + hi)


def surrogate_increment(b, q_hat, Phi, z0, delta):
    """Surrogate of eq. 1.8 minus its value at delta = 0, for a step `delta` over Z_s:
    sum_z b(z) delta(z) + sum_y sum_z q(y) |phi|/Z0 (exp(-Z0 sign(phi) delta(z)) - 1)."""
    coo = Phi.tocoo()
    ph = coo.data
    arg = np.exp(-z0 * np.sign(ph) * delta[coo.col]) - 1.0
    return float(np.dot(b, delta) + np.sum(q_hat[coo.row] * np.abs(ph) / z0 * arg))


def expand_tree(beta, mask, levels, frac, Omega):
    """Tree rule of the Results section -> (new mask, number of nodes split).

    mu = Omega beta; threshold = frac * max(mu) (nothing expands if max(mu) <= 0). A leaf
    (a node at level >= 1 that is not split and whose parent is split, or a root) splits
    once when some pixel of its block exceeds the threshold (strict >). All decisions
    are taken on the old tree."""
    n = mask.shape[0]
    mu = (Omega @ np.asarray(beta, np.float64).ravel()).reshape(n, n)
    top = mu.max()
    new = mask.copy()
    if top <= 0:
        return new, 0
    thr = frac * top
    count = 0
    for lev in range(1, levels + 1):
        m = n >> lev
        s = 1 << lev
        split = haar.split_flags(mask, lev)
        if lev == levels:
            parent = np.ones((m, m), bool)
        else:
            parent = np.repeat(np.repeat(haar.split_flags(mask, lev + 1), 2, 0), 2, 1)
        leaf = ~split & parent
        block_max = mu.reshape(m, s, m, s).max(axis=(1, 3))
        grow = leaf & (block_max > thr)
        count += int(grow.sum())
        haar.set_split(new, lev, split | grow)
    return new, count


def expand_tree_gradient(beta, mask, levels, frac, Omega, H, d, i0):
    """Residual-gradient tree rule (an "other expansion rule" in the sense of the Conclusion)
    -> (new mask, number of nodes split).

    q-hat = I0 exp(-H Omega beta) (Beer's law), c = Omega^T H^T (d - q-hat): the derivative
    of I(d || q-hat) with respect to every coefficient (from eq. 1.6's form, dI/dbeta_z =
    sum_y phi(y|z) (d(y) - q-hat(y))). A leaf (as in expand_tree) scores max |c| over its
    node's three details; every leaf scoring above frac x the largest leaf score (strict >)
    splits once; nothing splits if every score is 0. Decisions on the old tree."""
    n = mask.shape[0]
    q = beer_mean(i0, H @ (Omega @ np.asarray(beta, np.float64).ravel()))
    c = (Omega.T @ (H.T @ (np.asarray(d, np.float64) - q))).reshape(n, n)
    scores, leaves = {}, {}
    for lev in range(1, levels + 1):
        m = n >> lev
        split = haar.split_flags(mask, lev)
        if lev == levels:
            parent = np.ones((m, m), bool)
        else:
            parent = np.repeat(np.repeat(haar.split_flags(mask, lev + 1), 2, 0), 2, 1)
        leaves[lev] = ~split & parent
        det = np.stack([c[:m, m:2 * m], c[m:2 * m, :m], c[m:2 * m, m:2 * m]])
        scores[lev] = np.where(leaves[lev], np.abs(det).max(axis=0), 0.0)
    top = max((s.max() for s in scores.values()), default=0.0)
    new = mask.copy()
    if not top > 0:
        return new, 0
    thr = frac * top
    count = 0
    for lev in range(1, levels + 1):
        grow = leaves[lev] & (scores[lev] > thr)
        count += int(grow.sum())
        haar.set_split(new, lev, haar.split_flags(mask, lev) | grow)
    return new, count


def wam_solve(H, n, levels, d, i0, n_iters, pixel, schedule=(), frac=0.1, masks=None,
              beta0=None, mask0=None, Omega=None, record_beta=False, rule="value", penalty=0.0):
    """Algorithm 1 with the tree rule of the Results section.

    H: CSR system matrix (M x n*n); d: counts; i0: scalar or per-ray incident counts.
    schedule: iterations j before whose update the tree is expanded by `expand_tree`
    (rule "value", the Results section) or `expand_tree_gradient` (rule "gradient").
    masks: optional {j: mask} giving Z_s^(j) explicitly (Algorithm 1 takes the sequence
    of active sets as an input); it overrides the rule at those j.
    Returns a dict with beta (Mallat, n x n), mu, idiv (n_iters + 1 values: I(d||q-hat^(j))
    before each update and after the last), the trees, Z0 and W = nnz(Phi_s) per tree, and
    the number of held coefficients. penalty = lambda > 0 minimizes I + lambda R(Omega beta)
    instead (roughness penalty above; `penalized_update` replaces the eq. 1.9 root; the result
    also holds the penalized objective before each update and after the last, `objective`)."""
    if Omega is None:
        Omega = haar.synthesis_matrix(n, levels)
    d = np.asarray(d, np.float64)
    beta = np.zeros(n * n) if beta0 is None else np.array(beta0, np.float64).ravel()
    mask = haar.approx_mask(n, levels) if mask0 is None else np.array(mask0, np.uint8)
    masks = masks or {}
    b_all = Omega.T @ (H.T @ d)                       # eq. 1.6, for every coefficient
    trace, trees, z0s, ws, held_total, betas, objective = [], [], [], [], 0, [], []
    Phi = None
    for j in range(n_iters):
        changed = False
        if j in masks:
            mask = np.array(masks[j], np.uint8)
            changed = True
        elif j in schedule:
            if rule == "gradient":
                mask, _ = expand_tree_gradient(beta, mask, levels, frac, Omega, H, d, i0)
            else:
                mask, _ = expand_tree(beta, mask, levels, frac, Omega)
            changed = True
        if Phi is None or changed:
            Phi, act = phi_matrix(H, Omega, mask, pixel)
            Php, Phm = split_phi(Phi)
            z0 = z0_of(Phi)
            trees.append((j, mask.copy()))
            z0s.append(z0)
            ws.append(int(Phi.nnz))
        q_hat = beer_mean(i0, Phi @ beta[act])
        trace.append(idiv(d, q_hat))
        bp = Php.T @ q_hat
        bm = Phm.T @ q_hat
        if penalty > 0:
            mu_hat = (Omega @ beta).reshape(n, n)
            objective.append(trace[-1] + penalty * roughness(mu_hat))
            g = (Omega.T @ roughness_grad(mu_hat).ravel())[act]
            delta = penalized_update(b_all[act], bp, bm, z0, penalty, g)
        else:
            delta, held = closed_form_update(b_all[act], bp, bm, z0)
            held_total += int(held.sum())
        beta[act] += delta
        if record_beta:
            betas.append(beta.copy())
    q_hat = beer_mean(i0, Phi @ beta[act]) if Phi is not None else beer_mean(i0, H @ (Omega @ beta))
    trace.append(idiv(d, q_hat))
    out = dict(beta=beta.reshape(n, n), mu=(Omega @ beta).reshape(n, n), idiv=np.array(trace),
               trees=trees, z0=z0s, w=ws, held=held_total, mask=mask, b=b_all.reshape(n, n))
    if record_beta:
        out["betas"] = betas
    if penalty > 0:
        objective.append(trace[-1] + penalty * roughness(out["mu"]))
        out["objective"] = np.array(objective)
    return out


def subset_rows(n_views, n_bins, n_subsets):
    """Rays of each ordered subset: subset s holds the views v with v mod S = s (interleaved
    views, each subset spanning the whole angular range), in view-major ray order."""
    if not 1 <= n_subsets <= n_views:
        raise ValueError("need 1 <= n_subsets <= n_views")
    return [(np.arange(s, n_views, n_subsets)[:, None] * n_bins + np.arange(n_bins)[None, :]).ravel()
            for s in range(n_subsets)]


def os_wam_solve(H, n, levels, d, i0, n_iters, pixel, n_views, n_subsets, schedule=(), frac=0.1,
                 Omega=None, record_sub=False, beta0=None, mask0=None):
    """Wavelet AM combined with ordered subsets (the combination the Conclusion names).

    The views are split into S interleaved subsets (`subset_rows`). Pass j applies the tree
    rule first when j is in `schedule`, then S sub-iterations; sub-iteration s is the update
    of Algorithm 1 with the data term restricted to the rays Y_s of subset s:
      q-hat = I0 exp(-Phi_s beta) on Y_s, b_s(z) = sum_{y in Y_s} d(y) phi(y|z) (eq. 1.6 on
      Y_s), b-hat+/- over Y_s (eq. 1.10), Z0_s = max_{y in Y_s} sum_z |phi(y|z)| (eq. 1.61
      on Y_s), and the zero of eq. 1.9 with these sums.
    Each sub-iteration is an exact AM step for I(d_s || q_s), so it cannot increase that
    subset's I-divergence; the full I-divergence is not guaranteed to fall.
    Returns beta, mu, idiv (n_iters + 1 values: I(d||q-hat) over all rays before each pass
    and after the last), trees, z0 (per tree: the S values Z0_s), the per-subset b_s, the
    held count and, with record_sub, (I(d_s||q_s) before, after) for every sub-iteration.
    beta0/mask0: starting coefficients and tree (default 0 and the approximation-only tree)."""
    if Omega is None:
        Omega = haar.synthesis_matrix(n, levels)
    d = np.asarray(d, np.float64)
    i0 = np.asarray(i0, np.float64)
    rows = subset_rows(n_views, H.shape[0] // n_views, n_subsets)
    i0_of = [i0 if i0.ndim == 0 else i0[r] for r in rows]
    b_sub = [Omega.T @ (H[r].T @ d[r]) for r in rows]
    beta = np.zeros(n * n) if beta0 is None else np.array(beta0, np.float64).ravel()
    mask = haar.approx_mask(n, levels) if mask0 is None else np.array(mask0, np.uint8)
    trace, trees, z0s, sub, held_total = [], [], [], [], 0
    Phi = None
    for j in range(n_iters):
        changed = False
        if j in schedule:
            mask, _ = expand_tree(beta, mask, levels, frac, Omega)
            changed = True
        if Phi is None or changed:
            Phi, act = phi_matrix(H, Omega, mask, pixel)
            parts = []
            for r in rows:
                Ps = Phi[r]
                Psp, Psm = split_phi(Ps)
                z = float(np.max(np.asarray(abs(Ps).sum(axis=1)).ravel()))
                if not z > 0:
                    raise ValueError("a subset has no ray crossing the image (Z0_s = 0)")
                parts.append((Ps, Psp, Psm, z))
            trees.append((j, mask.copy()))
            z0s.append([p[3] for p in parts])
        trace.append(idiv(d, beer_mean(i0, Phi @ beta[act])))
        for s, (Ps, Psp, Psm, z) in enumerate(parts):
            q_s = beer_mean(i0_of[s], Ps @ beta[act])
            before = idiv(d[rows[s]], q_s) if record_sub else None
            delta, held = closed_form_update(b_sub[s][act], Psp.T @ q_s, Psm.T @ q_s, z)
            held_total += int(held.sum())
            beta[act] += delta
            if record_sub:
                sub.append((before, idiv(d[rows[s]], beer_mean(i0_of[s], Ps @ beta[act]))))
    trace.append(idiv(d, beer_mean(i0, H @ (Omega @ beta))))
    out = dict(beta=beta.reshape(n, n), mu=(Omega @ beta).reshape(n, n), idiv=np.array(trace), trees=trees,
               z0=z0s, b_sub=[b.reshape(n, n) for b in b_sub], held=held_total, mask=mask)
    if record_sub:
        out["sub"] = sub
    return out


def volume_wam_solve(H, n, levels, ds, i0s, n_iters, pixel, schedule=(), frac=0.1, Omega=None,
                     betas0=None, mask0=None):
    """Algorithm 1 on a stack of z-slices that share one tree (Results: each z-slice is
    represented by a 2-D Haar transform, and the tree is expanded where the image summed
    over the slices exceeds frac times its maximum). Every slice has the 2-D scan H (rays
    stay in their slice), its own counts ds[p] and incident counts i0s[p]. Z0 is the
    maximum over all rays of the volume; with one tree and one geometry it is the same for
    every slice. Returns betas [P, n, n], the shared mask, idiv [P, n_iters + 1] per slice
    (before each update and after the last), trees, z0 per tree, held count."""
    if Omega is None:
        Omega = haar.synthesis_matrix(n, levels)
    P = len(ds)
    ds = [np.asarray(d, np.float64) for d in ds]
    betas = np.zeros((P, n * n)) if betas0 is None else np.array(betas0, np.float64).reshape(P, n * n)
    mask = haar.approx_mask(n, levels) if mask0 is None else np.array(mask0, np.uint8)
    b_all = [Omega.T @ (H.T @ d) for d in ds]
    trace = [[] for _ in range(P)]
    trees, z0s, held_total = [], [], 0
    Phi = None
    for j in range(n_iters):
        changed = False
        if j in schedule:
            # the image summed over slices is Omega applied to the summed coefficients
            mask, _ = expand_tree(betas.sum(axis=0), mask, levels, frac, Omega)
            changed = True
        if Phi is None or changed:
            Phi, act = phi_matrix(H, Omega, mask, pixel)
            Php, Phm = split_phi(Phi)
            z0 = z0_of(Phi)
            trees.append((j, mask.copy()))
            z0s.append(z0)
        for p in range(P):
            q_hat = beer_mean(i0s[p], Phi @ betas[p][act])
            trace[p].append(idiv(ds[p], q_hat))
            delta, held = closed_form_update(b_all[p][act], Php.T @ q_hat, Phm.T @ q_hat, z0)
            held_total += int(held.sum())
            betas[p][act] += delta
    for p in range(P):
        trace[p].append(idiv(ds[p], beer_mean(i0s[p], H @ (Omega @ betas[p]))))
    return dict(betas=betas.reshape(P, n, n), mask=mask, idiv=np.array(trace), trees=trees, z0=z0s,
                held=held_total)


def am_solve(H, n, d, i0, n_iters, pixel, mu0=None):
    """Unregularized image-domain AM (O'Sullivan-Benac): Algorithm 1 with Omega = I."""
    return wam_solve(H, n, 0, d, i0, n_iters, pixel, beta0=mu0)


def loss_and_grad(H, Omega, d, i0, c):
    """Coefficient-domain objective of eq. 1.3 with lambda = 0 and all coefficients
    free: loss(c) = I(d || I0 exp(-H Omega c)); gradient Omega^T H^T (d - q)."""
    q = beer_mean(i0, H @ (Omega @ c))
    return idiv(d, q), Omega.T @ (H.T @ (np.asarray(d, np.float64) - q)), q
