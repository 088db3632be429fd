"""Orthonormal Daubechies-4 wavelets on an n x n image with periodic boundary, FP64 (test
infrastructure; see oracle/__init__.py).

The Conclusion lists other wavelet families as future work; this is one: the compactly
supported orthonormal wavelet with two vanishing moments (four filter taps), in the same
2-D Mallat layout and tree structure as haar.py, so Algorithm 1 and the tree rule of the
Results section apply unchanged with this Omega (wam.wam_solve(..., Omega=synthesis_matrix)).

Filters (Daubechies' construction; scaling filter h normalised to sum sqrt 2):
  h = ((1 + s3), (3 + s3), (3 - s3), (1 - s3)) / (4 sqrt 2), s3 = sqrt 3,
  g[t] = (-1)^t h[3 - t]  (the wavelet filter).
1-D basis on a periodic grid of n points, level by level: level-0 scaling functions are the
unit vectors e_x; at level l (grid of n >> l positions)
  phi_{l,j} = sum_t h[t] phi_{l-1, (2j + t) mod (n >> (l-1))},
  psi_{l,j} = sum_t g[t] phi_{l-1, (2j + t) mod (n >> (l-1))},
so phi_{l,j} and psi_{l,j} are supported on the 3 * 2^l - 2 points 2^l j, 2^l j + 1, ...
(mod n). 2-D: the approximation of root (i, j) at beta[i, j] (i, j < n >> L) is
phi_L,i(y) phi_L,j(x); node (l, i, j) has D1 = phi_l,i(y) psi_l,j(x) at beta[i, m + j], D2 =
psi_l,i(y) phi_l,j(x) at beta[m + i, j] and D3 = psi_l,i(y) psi_l,j(x) at beta[m + i, m + j]
(m = n >> l; y is the row index). Requires n >> L >= 4 so that no support wraps onto itself.
"""
import numpy as np
import scipy.sparse as sp

S3 = np.sqrt(3.0)
H4 = np.array([1.0 + S3, 3.0 + S3, 3.0 - S3, 1.0 - S3]) / (4.0 * np.sqrt(2.0))
G4 = np.array([(-1.0) ** t * H4[3 - t] for t in range(4)])


def basis_1d(n, levels):
    """(phi, psi): lists over l = 0..levels of (n >> l) x n arrays whose row j is the level-l
    scaling (wavelet) function at position j (psi[0] unused)."""
    if n % (1 << levels) or (n >> levels) < 4:
        raise ValueError("n must be divisible by 2^levels with n >> levels >= 4")
    phi = [np.eye(n)]
    psi = [None]
    for l in range(1, levels + 1):
        m, mp = n >> l, n >> (l - 1)
        P = np.zeros((m, n))
        Q = np.zeros((m, n))
        for j in range(m):
            for t in range(4):
                P[j] += H4[t] * phi[l - 1][(2 * j + t) % mp]
                Q[j] += G4[t] * phi[l - 1][(2 * j + t) % mp]
        phi.append(P)
        psi.append(Q)
    return phi, psi


def synthesis_matrix(n, levels):
    """Omega (n*n x n*n, CSR): column z = the basis image of Mallat coefficient z, the outer
    product of its 1-D functions (row function along y, column function along x), assembled
    from their non-zero samples (entries below 1e-15 in magnitude dropped)."""
    phi, psi = basis_1d(n, levels)
    rows, cols, vals = [], [], []

    def put(r, c, fy, fx):
        iy, ix = np.flatnonzero(fy), np.flatnonzero(fx)
        rows.append((iy[:, None] * n + ix[None, :]).ravel())
        cols.append(np.full(iy.size * ix.size, r * n + c, np.int64))
        vals.append(np.outer(fy[iy], fx[ix]).ravel())

    m = n >> levels
    for i in range(m):
        for j in range(m):
            put(i, j, phi[levels][i], phi[levels][j])
    for l in range(1, levels + 1):
        m = n >> l
        for i in range(m):
            for j in range(m):
                put(i, m + j, phi[l][i], psi[l][j])
                put(m + i, j, psi[l][i], phi[l][j])
                put(m + i, m + j, psi[l][i], psi[l][j])
    v = np.concatenate(vals)
    keep = np.abs(v) >= 1e-15
    return sp.csr_matrix((v[keep], (np.concatenate(rows)[keep], np.concatenate(cols)[keep])), shape=(n * n, n * n))


def cascade_analysis(img, levels):
    """Textbook periodic filter bank (independent of synthesis_matrix): per level, rows then
    columns of the current approximation are filtered with h (low) and g (high) and
    downsampled by 2 (a[j] = sum_t h[t] x[(2j + t) mod len])."""
    a = np.array(img, np.float64)
    n = a.shape[0]
    out = np.zeros_like(a)

    def down(x, f, axis):
        L = x.shape[axis]
        idx = (2 * np.arange(L // 2)[:, None] + np.arange(4)[None, :]) % L
        xt = np.moveaxis(x, axis, -1)
        y = (xt[..., idx] * f).sum(-1)
        return np.moveaxis(y, -1, axis)

    for l in range(1, levels + 1):
        m = n >> l
        lo_x, hi_x = down(a, H4, 1), down(a, G4, 1)        # along x (columns index)
        ll, lh = down(lo_x, H4, 0), down(lo_x, G4, 0)      # then along y
        hl, hh = down(hi_x, H4, 0), down(hi_x, G4, 0)
        out[:m, m:2 * m] = hl          # D1: wavelet in x, scaling in y
        out[m:2 * m, :m] = lh          # D2: scaling in x, wavelet in y
        out[m:2 * m, m:2 * m] = hh     # D3
        a = ll
    out[:a.shape[0], :a.shape[0]] = a
    return out
