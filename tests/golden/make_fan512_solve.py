"""Write fan512_solve.npz: the FP64 oracle's complete solve of the fan512 scan (512x512 fan
beam, 720 views x 1024 bins, 3-level Haar tree, 100 iterations of Algorithm 1 with the tree
rule of the Results section at iterations 21, 43 and 85), stored for the GPU parity test
at the benchmark's full size.

The script calls only the oracle (oracle/) and the seeded input generator (synth), never the
HIP library. Run from the repository root:

    python tests/golden/make_fan512_solve.py

It takes about 4 minutes and 20 GB of memory (the system matrix has 3.0e8 nonzeros, the
largest Phi 2.9e8). Stored, for the scan drawn by synth.make_problem("fan512"):
  * d_sha256: SHA-256 of the counts as FP64 bytes (the test checks it regenerated the scan);
  * tree_at, masks: the tree sequence Z_s^(j) (tree k from update tree_at[k] on), as packed
    bits of the n x n Mallat masks;
  * idiv: I(d || q-hat) before each update and after the last (101 values, FP64);
  * z0, w: Z0 (eq. 1.61) and nnz(Phi) of each tree; held: coefficients held (no finite
    minimizer of eq. 1.8's surrogate) over the solve; n_split: nodes split per expansion;
  * beta_final: the final coefficients on the last tree's active set (FP64, in the order
    of the mask's nonzero positions);
  * beta_pre_k (k = 1, 2, 3): the coefficients the tree rule sees at expansion k (after
    update tree_at[k] - 1), on tree k - 1's active set.
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import haar, siddon, wam  # noqa: E402
from paper_1508_04458_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fan512_solve.npz")


def main():
    t0 = time.time()
    P = synth.make_problem("fan512")
    g = P.geom
    print(f"scan drawn ({time.time() - t0:.0f} s)", flush=True)
    H = siddon.system_matrix(g)
    print(f"H: {H.nnz} nonzeros ({time.time() - t0:.0f} s)", flush=True)
    O = haar.synthesis_matrix(g.n, P.levels)
    ref = wam.wam_solve(H, g.n, P.levels, P.d, P.i0, P.n_iters, g.pixel, schedule=P.schedule, Omega=O,
                        record_beta=True)
    print(f"solve done ({time.time() - t0:.0f} s): I-div {ref['idiv'][0]:.6e} -> {ref['idiv'][-1]:.6e}",
          flush=True)
    at = np.array([j for j, _ in ref["trees"]], np.int32)
    masks = [m for _, m in ref["trees"]]
    out = dict(
        d_sha256=np.array(hashlib.sha256(np.ascontiguousarray(P.d, np.float64).tobytes()).hexdigest()),
        tree_at=at,
        masks=np.stack([np.packbits(m.ravel().astype(np.uint8)) for m in masks]),
        idiv=np.asarray(ref["idiv"], np.float64),
        z0=np.asarray(ref["z0"], np.float64),
        w=np.asarray(ref["w"], np.int64),
        held=np.array(ref["held"], np.int64),
        beta_final=ref["beta"].ravel()[np.flatnonzero(masks[-1].ravel())],
    )
    n_split = []
    for k in range(1, len(at)):
        prev = masks[k - 1]
        beta = ref["betas"][at[k] - 1]
        out[f"beta_pre_{k}"] = beta[np.flatnonzero(prev.ravel())]
        _, cnt = wam.expand_tree(beta, prev, P.levels, 0.1, O)
        n_split.append(cnt)
    out["n_split"] = np.array(n_split, np.int64)
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e6:.2f} MB), trees at {at.tolist()}, W {out['w'].tolist()}, "
          f"held {int(out['held'])}, splits {n_split} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
