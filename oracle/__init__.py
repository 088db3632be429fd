"""FP64 CPU reference for wavelet-domain alternating minimization (AM) in transmission CT.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or execute this
package: only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of
`bench.py` use it. It shares no code with the HIP path (no kernels, headers, helpers,
tables or pre/post-processing) and imports nothing from it.

Source: Degirmenci, O'Sullivan, Politte, "Multiresolution Approach to Acceleration of
Iterative Image Reconstruction for X-Ray Imaging for Security Applications"
(arXiv 1508.04458).

  geometry.py  rays of a parallel- or fan-beam 2-D scan (no geometry is given in the
               paper; the conventions are stated in the module docstring)
  siddon.py    system matrix H: h(y|x) = length of ray y inside pixel x (Introduction,
               definition of the Beer's-law mean), by plane-crossing ray tracing, plus a
               brute-force per-box chord used to check it
  haar.py      orthonormal multi-level 2-D Haar synthesis matrix Omega, mu = Omega beta
               (eq. 1.2), Mallat layout, tree masks
  wam.py       Phi = H Omega, b (eq. 1.6), Z0 (eq. 1.61), b-hat+/- (eq. 1.10), the
               closed-form zero of eq. 1.9, Algorithm 1, the tree-expansion rule of the
               Results section, unregularized pixel AM (Omega = I), the I-divergence,
               the surrogate of eq. 1.8, the loss/gradient of the coefficient-domain
               problem (eq. 1.3 with lambda = 0), wavelet AM combined with ordered
               subsets of views (Conclusion), and z-slices sharing one tree chosen on
               the slice-summed image (Results)
  daub.py      orthonormal Daubechies-4 wavelets with periodic boundary in the same Mallat
               layout and tree structure (a "different wavelet type", Conclusion): Omega,
               the 1-D basis, and an independent textbook filter bank
  vol3d.py     cone-beam 3-D Siddon H, the 3-D Haar octree and its tree rule, and the
               Results section's per-slice representation of a volume (2-D Haar of every
               z-slice, one tree grown on the slice-summed image) on the same cone rays

Parity status: every function is pinned by the `-m "not gpu"` tests in
tests/test_oracle_*.py (closed forms, brute force, invariants, a hand-computed golden
fixture). The end-to-end reconstruction has no printed values in the paper to compare
with; it is pinned by those invariants (monotone I-divergence, the exact reduction of an
approximation-only tree to pixel AM on the coarse grid, fixed points), not by numbers
from the paper.
"""
from . import geometry, siddon, haar, wam, daub  # noqa: F401
