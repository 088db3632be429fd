"""Orthonormal multi-level 2-D Haar synthesis Omega, FP64 (test infrastructure).

mu = Omega beta (eq. 1.2). The paper uses a "Level 3 Haar" transform of each slice
(Results) without fixing normalisation or layout; this project reads it as the
orthonormal Haar basis (so Omega^T = Omega^-1 and analysis is Omega^T) in Mallat layout:

  * beta is an n x n array; at level l (1..L) let m = n >> l. Node (l, i, j) covers the
    pixel block rows [i 2^l, (i+1) 2^l), columns [j 2^l, (j+1) 2^l).
  * its three detail coefficients sit at beta[i, m+j] (D1), beta[m+i, j] (D2) and
    beta[m+i, m+j] (D3); the approximation coefficient of root (i, j) (level L) sits at
    beta[i, j] with i, j < n >> L.
  * basis functions: approximation = 2^-L on the root block; detail k of node (l,i,j) =
    2^-l s_k on the block, with quadrant signs over (top-left, top-right, bottom-left,
    bottom-right) s1 = (+,-,+,-), s2 = (+,+,-,-), s3 = (+,-,-,+); "top" is the smaller row.

Tree masks (the active set Z_s of the footnote to eq. 1.61) are uint8 n x n arrays in
the same layout; a node is "split" when its three details are active.
"""
import numpy as np
import scipy.sparse as sp


def synthesis_matrix(n, levels):
    """Omega as CSR (n*n x n*n): column z = basis image of Mallat coefficient z.

    Built pixel by pixel: pixel (r, c) receives 2^-L from the approximation coefficient
    of its root, and 2^-l s_k from detail k of the level-l node that contains it."""
    if n % (1 << levels):
        raise ValueError("image size must be divisible by 2^levels")
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    r, c = r.ravel(), c.ravel()
    pix = r * n + c
    rows, cols, vals = [pix], [(r >> levels) * n + (c >> levels)], [np.full(pix.size, 2.0 ** -levels)]
    for lev in range(1, levels + 1):
        m = n >> lev
        i, j = r >> lev, c >> lev
        s1 = np.where((c >> (lev - 1)) & 1, -1.0, 1.0)   # right half of the node: -
        s2 = np.where((r >> (lev - 1)) & 1, -1.0, 1.0)   # bottom half of the node: -
        for zr, zc, s in ((i, m + j, s1), (m + i, j, s2), (m + i, m + j, s1 * s2)):
            rows.append(pix)
            cols.append(zr * n + zc)
            vals.append(s * 2.0 ** -lev)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n * n, n * n))


def cascade_analysis(img, levels):
    """Textbook recursive 2x2 Haar analysis (independent of `synthesis_matrix`)."""
    a = np.array(img, dtype=np.float64)
    n = a.shape[0]
    out = np.zeros_like(a)
    for lev in range(1, levels + 1):
        m = n >> lev
        tl, tr = a[0::2, 0::2], a[0::2, 1::2]
        bl, br = a[1::2, 0::2], a[1::2, 1::2]
        out[:m, m:2 * m] = (tl - tr + bl - br) / 2
        out[m:2 * m, :m] = (tl + tr - bl - br) / 2
        out[m:2 * m, m:2 * m] = (tl - tr - bl + br) / 2
        a = (tl + tr + bl + br) / 2
    out[:a.shape[0], :a.shape[0]] = a
    return out


def cascade_synthesis(beta, levels):
    """Inverse of `cascade_analysis`, level by level from coarse to fine."""
    b = np.asarray(beta, dtype=np.float64)
    n = b.shape[0]
    nL = n >> levels
    a = b[:nL, :nL].copy()
    for lev in range(levels, 0, -1):
        m = n >> lev
        d1, d2, d3 = b[:m, m:2 * m], b[m:2 * m, :m], b[m:2 * m, m:2 * m]
        up = np.zeros((2 * m, 2 * m))
        up[0::2, 0::2] = (a + d1 + d2 + d3) / 2
        up[0::2, 1::2] = (a - d1 + d2 - d3) / 2
        up[1::2, 0::2] = (a + d1 - d2 - d3) / 2
        up[1::2, 1::2] = (a - d1 - d2 + d3) / 2
        a = up
    return a


# ------------------------------------------------------------------ tree masks

def approx_mask(n, levels):
    """Initial tree of the Results section: approximation coefficients only."""
    m = np.zeros((n, n), np.uint8)
    nL = n >> levels
    m[:nL, :nL] = 1
    return m


def full_mask(n):
    return np.ones((n, n), np.uint8)


def split_flags(mask, lev):
    """Boolean (n>>lev)^2 array: node (lev, i, j) has its details active."""
    n = mask.shape[0]
    m = n >> lev
    return mask[:m, m:2 * m].astype(bool)


def set_split(mask, lev, flags):
    n = mask.shape[0]
    m = n >> lev
    f = flags.astype(np.uint8)
    mask[:m, m:2 * m] = f
    mask[m:2 * m, :m] = f
    mask[m:2 * m, m:2 * m] = f


def valid_mask(mask, levels):
    """True when the mask is a tree: approximations active, details all-or-none per
    node, and a node split only if its parent is split (or it is a root)."""
    n = mask.shape[0]
    nL = n >> levels
    if not mask[:nL, :nL].all():
        return False
    if levels == 0:
        return bool(mask.all())
    for lev in range(1, levels + 1):
        m = n >> lev
        f = mask[:m, m:2 * m]
        if not (np.array_equal(f, mask[m:2 * m, :m]) and np.array_equal(f, mask[m:2 * m, m:2 * m])):
            return False
        if lev < levels:
            parent = np.repeat(np.repeat(split_flags(mask, lev + 1), 2, 0), 2, 1)
            if (f.astype(bool) & ~parent).any():
                return False
    return True


def leaf_level_map(mask, levels):
    """Per-pixel level of the tree leaf (block) that contains it, int [n, n]."""
    n = mask.shape[0]
    out = np.full((n, n), levels, np.int64)
    for lev in range(levels, 0, -1):
        f = np.repeat(np.repeat(split_flags(mask, lev), 1 << lev, 0), 1 << lev, 1)
        out = np.where(f & (out == lev), lev - 1, out)
    return out
