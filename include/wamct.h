/*
 * wamct: wavelet-tree alternating minimization (AM) for transmission CT on AMD MI355X.
 *
 * C ABI of the hot path of the method of Degirmenci, O'Sullivan and Politte,
 * "Multiresolution Approach to Acceleration of Iterative Image Reconstruction for X-Ray
 * Imaging for Security Applications" (arXiv 1508.04458). Every step runs in HIP kernels
 * for gfx950; the host code only validates, allocates at creation, and launches.
 *
 * Conventions (mm, mm^-1):
 *   image    n x n pixels of size `pixel`, centred on the origin, row-major [r][c];
 *            pixel (r, c) covers x in [(c - n/2) pixel, (c + 1 - n/2) pixel), y likewise with r.
 *   sinogram [view][bin], bin fastest; ray y = view * n_bins + bin through the bin centre.
 *            View v has angle a = angle0 + v * angle_span / n_views, bin b sits at
 *            u = (b - (n_bins - 1) / 2) * bin_pitch on the detector axis (-sin a, cos a).
 *            Parallel beam: the line x cos a + y sin a = u. Fan beam (flat detector): from
 *            the source sod (cos a, sin a) to the point -(sdd - sod)(cos a, sin a) + u (-sin a, cos a).
 *            A line on a pixel boundary belongs to the pixel on the + side, placed as exact
 *            arithmetic places it: cos a or sin a within 1e-12 of 0 is 0 (the angle is a
 *            multiple of pi/2), a direction component within 1e-12 of 0 is 0 (axis-parallel
 *            line), and such a line's offset within 1e-9 pixel of a boundary is on it.
 *   wavelets orthonormal 2-D Haar with `levels` levels in Mallat layout (an n x n array):
 *            at level l (1..L), with m = n >> l, node (l, i, j) covers pixel rows
 *            [i 2^l, (i+1) 2^l) and columns [j 2^l, (j+1) 2^l); its details sit at
 *            [i][m+j] (D1), [m+i][j] (D2), [m+i][m+j] (D3); the approximation of root (i, j)
 *            sits at [i][j], i, j < n >> L. Basis: approximation 2^-L on the root block;
 *            detail k = 2^-l s_k on the node block with quadrant signs over (top-left,
 *            top-right, bottom-left, bottom-right) s1 = (+,-,+,-), s2 = (+,+,-,-),
 *            s3 = (+,-,-,+), "top" = smaller row index.
 *   volume   (WAMCT_CONE) n x n x nz voxels of edge `pixel`, centred, layout [z][y][x], voxel
 *            (s, r, c) covering z in [(s - nz/2) pixel, (s + 1 - nz/2) pixel) (x, y as above).
 *            Circular orbit: source sod (cos a, sin a, 0); flat detector centred at
 *            -(sdd - sod)(cos a, sin a, 0), column axis (-sin a, cos a, 0), row axis (0, 0, 1);
 *            element (row rr, column cc) at (cc - (n_bins - 1)/2) bin_pitch,
 *            (rr - (n_rows - 1)/2) row_pitch; ray y = (view n_rows + rr) n_bins + cc.
 *            3-D Haar: orthonormal, separable, 3-D Mallat layout; node (l, k, i, j) covers
 *            the voxel block [k 2^l, (k+1) 2^l) x [i 2^l, ...) x [j 2^l, ...) (z, y, x); its
 *            seven details t = (tz, ty, tx) != 0 sit at [k + tz mz][i + ty m][j + tx m]
 *            (m = n >> l, mz = nz >> l), basis 2^(-3l/2) times, per flagged axis, +1 on the
 *            lower and -1 on the upper half; the approximation of root (k, i, j) sits at
 *            [k][i][j], basis 2^(-3L/2). A node splits into its seven details together.
 *   per-slice (WAMCT_CONE, wavelet_dims = 2) every z-slice s holds the 2-D Haar coefficients
 *            of its n x n image in the 2-D Mallat layout above ([s][y][x]); node (l, s, i, j)
 *            covers the voxels [i 2^l, (i+1) 2^l) x [j 2^l, ...) of slice s; the slices share
 *            one tree (the mask holds the same n x n tree in every slice); the tree rule
 *            synthesizes every slice, sums the images over the slices in FP64 and splits
 *            every leaf with a pixel of the summed image above frac x its maximum (Results).
 *            n must be divisible by 2^levels, nz need not.
 *   Daubechies-4 (wavelet = WAMCT_D4) the same Mallat layout and tree, with the orthonormal
 *            four-tap Daubechies basis, periodic in x and y: h = (1 + r, 3 + r, 3 - r, 1 - r) /
 *            (4 sqrt 2), r = sqrt 3, g[t] = (-1)^t h[3 - t]; level-0 scaling functions are the
 *            pixels, phi_l,j = sum_t h[t] phi_l-1,(2j+t) mod (n >> (l-1)) and psi_l,j likewise
 *            with g, supported on the 3 x 2^l - 2 pixels from 2^l j (mod n). Root (i, j): phi_L,i
 *            (y) phi_L,j (x) at [i][j]; node (l, i, j): D1 = phi_l,i(y) psi_l,j(x) at [i][m+j], D2 =
 *            psi_l,i(y) phi_l,j(x) at [m+i][j], D3 = psi_l,i(y) psi_l,j(x) at [m+i][m+j]. The tree
 *            rule splits a leaf when the largest pixel of its block (rows [i 2^l, (i+1) 2^l),
 *            columns likewise) exceeds frac x the image maximum. The mu of the forward pass and
 *            of the rule is synthesized per pixel; b-hat+/- and Z0 take each ray's chords through
 *            the basis function's support weighted by its value in each pixel.
 *   tree     the active set Z_s (footnote to eq. 1.61) is a uint8 n x n mask in Mallat
 *            layout: approximations always active; a node's three details are active
 *            together ("split"), and only if its parent is split or it is a root.
 *            levels = 0 is image-domain AM (Omega = I, every pixel active).
 *
 * Arrays: every bulk array argument is a DEVICE pointer owned by the caller, of the
 * context's element type (float for WAMCT_F32, double for WAMCT_F64) unless stated
 * otherwise; struct arguments are host memory, copied during the call. All work is
 * ordered on the stream given at creation; calls return after enqueueing unless they
 * return a host value, which synchronizes that stream.
 *
 * Stacks: a context holds `batch` (options) independent scans of its geometry, solved in
 * lockstep (same iteration count and expansion schedule; each scan has its own data, I0,
 * coefficients, tree, Z0 and held counter). Per-scan arrays are stacked scan-major:
 * "[S]" below is the batch size, so beta is [S][n*n], d is [S][n_views*n_bins] and an
 * I-divergence trace of n entries per scan is [S][n].
 *
 * Errors: every call returns a wamct_status and never aborts; wamct_last_error(ctx)
 * gives the message of the last failing call on that context (NULL ctx: the last
 * failure of wamct_create/wamct_validate in this thread).
 */
#ifndef WAMCT_H
#define WAMCT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WAMCT_OK = 0,
  WAMCT_E_INVALID = 1,     /* bad argument, geometry or data */
  WAMCT_E_UNSUPPORTED = 2, /* valid request the library does not implement */
  WAMCT_E_OOM = 3,         /* device allocation failed */
  WAMCT_E_HIP = 4,         /* HIP runtime error (message carries hipGetErrorString) */
  WAMCT_E_NUMERIC = 5,     /* non-finite values where finite ones are required */
  WAMCT_E_STATE = 6        /* call out of order (e.g. iterate before set_data) */
} wamct_status;

enum { WAMCT_PARALLEL = 0, WAMCT_FAN = 1, WAMCT_CONE = 2 };
enum { WAMCT_F32 = 0, WAMCT_F64 = 1 };

/* Scan geometry (the paper gives none; see the conventions above). */
typedef struct {
  int32_t kind;        /* WAMCT_PARALLEL or WAMCT_FAN */
  int32_t n;           /* image is n x n; 2 <= n <= 8192 */
  double pixel;        /* pixel size [mm], > 0 */
  int32_t n_views;     /* >= 1 */
  double angle0;       /* [rad] */
  double angle_span;   /* [rad]; view v at angle0 + v * angle_span / n_views */
  int32_t n_bins;      /* >= 1 */
  double bin_pitch;    /* [mm] at the detector, > 0 */
  double sod;          /* fan, cone: source to isocentre [mm], > image circumradius */
  double sdd;          /* fan, cone: source to detector [mm], > sod */
  int32_t nz;          /* cone: slices of the n x n x nz volume (1 <= nz <= 512); else ignored */
  int32_t n_rows;      /* cone: detector rows (>= 1); else ignored */
  double row_pitch;    /* cone: detector row pitch [mm] (> 0); else ignored */
} wamct_geometry;

typedef struct {
  int32_t levels;      /* Haar levels L, 0 <= L <= 8, n divisible by 2^L (Results: L = 3) */
  int32_t dtype;       /* WAMCT_F32 or WAMCT_F64: element type of every bulk array */
  int32_t geometry;    /* WAMCT_F32 or WAMCT_F64 (>= dtype): precision of the ray geometry,
                          chord lengths and per-ray/per-coefficient sums. WAMCT_F64 keeps
                          chords exact to ~1e-13 mm; WAMCT_F32 chords carry an absolute error
                          of about 1e-7 times the image half-diagonal. */
  int32_t batch;       /* scans in the stack, 1 <= batch <= 65535 */
  int32_t wavelet_dims;/* 0: the geometry's default (2-D Haar for parallel and fan beam, 3-D Haar
                          octree for the cone beam). 2 with the cone beam: the 2-D Haar transform
                          of every z-slice (Results: "each z-slice represented by a Level 3
                          Haar" with one tree for the volume), see "per-slice" below. 3 is valid
                          for the cone beam only. */
  int32_t wavelet;     /* WAMCT_HAAR (0) or WAMCT_D4 (1): the wavelet family of Omega. WAMCT_D4 is
                          the orthonormal Daubechies-4 basis with periodic boundary (Conclusion:
                          other wavelet types), see "Daubechies-4" below; it needs a parallel or
                          fan beam, batch = 1, levels >= 1 and n >> levels >= 4. */
} wamct_options;

enum { WAMCT_HAAR = 0, WAMCT_D4 = 1 };

enum {                 /* kernel classes reported by wamct_get_timing */
  WAMCT_K_SYNTH = 0,   /* mu = Omega beta over the active tree                      */
  WAMCT_K_FORWARD = 1, /* ray-driven projection over tree leaves, q = I0 exp(-p), I-div */
  WAMCT_K_UPDATE = 2,  /* node-driven sign-split backprojection + eq. 1.9 zero        */
  WAMCT_K_TREE = 3,    /* Z0, tree expansion, work-list compaction                  */
  WAMCT_K_OTHER = 4,   /* reductions, transforms, operator calls                    */
  WAMCT_NK = 5
};

/* Check geometry and options on the host only (no GPU use). Returns WAMCT_E_INVALID
 * with a message in msg (NUL-terminated, at most msg_len bytes; msg may be NULL). */
wamct_status wamct_validate(const wamct_geometry* geom, const wamct_options* opt,
                            char* msg, int32_t msg_len);

typedef struct wamct_ctx wamct_ctx;   /* opaque; owns every device work buffer */

/* Create a context on the current HIP device: validates, allocates every device buffer
 * the iteration needs (iterating allocates nothing), builds the ray table and the
 * approximation-only tree (Results: the initial tree) with beta = 0 (beta^(0) is an input
 * of Algorithm 1 whose value the paper does not give). `stream` is a hipStream_t
 * (NULL = default stream). On success *out owns the context (free with wamct_destroy).
 * A scan none of whose rays crosses the image has Z0 = 0 (eq. 1.61), for which the update
 * is undefined: creation then fails with WAMCT_E_INVALID. */
wamct_status wamct_create(const wamct_geometry* geom, const wamct_options* opt,
                          void* stream, wamct_ctx** out);
wamct_status wamct_destroy(wamct_ctx* ctx);
const char* wamct_last_error(const wamct_ctx* ctx);
const char* wamct_version(void);
wamct_status wamct_set_stream(wamct_ctx* ctx, void* stream);

/* Measured data of the Beer's-law model q(y) = I0(y) exp(-sum_x h(y|x) mu(x))
 * (Introduction). d: counts, [S][n_views * n_bins], finite and >= 0. i0: per-ray incident
 * counts of the same shape, or NULL to use one scalar per scan, i0_scalar (HOST double[S],
 * each finite and > 0; ignored when i0 is given). Both are COPIED into the context. Also
 * precomputes b(z) = sum_y d(y) phi(y|z) for every coefficient (eq. 1.6; Algorithm 1
 * "Precompute") as Omega^T (H^T d). Synchronizes (validation). */
wamct_status wamct_set_data(wamct_ctx* ctx, const void* d, const void* i0, const double* i0_scalar);

/* beta = 0 and the approximation-only tree. */
wamct_status wamct_reset(wamct_ctx* ctx);
/* Set beta (Mallat, [S][n*n]) and the tree masks (uint8 device array, [S][n*n]). Every mask
 * must be a valid tree (checked; E_INVALID otherwise); beta is zeroed outside it (inactive
 * coefficients are zero). Synchronizes. */
wamct_status wamct_set_state(wamct_ctx* ctx, const void* beta, const uint8_t* mask);
/* Copy beta and the mask out (either may be NULL); *iter_host (nullable) receives the
 * number of iterations applied since the last reset/set_state. */
wamct_status wamct_get_state(wamct_ctx* ctx, void* beta, uint8_t* mask, int32_t* iter_host);

/* n_iters iterations of Algorithm 1 on the current tree: q-hat = I0 exp(-Phi beta),
 * b-hat+/- (eq. 1.10), Z0 (eq. 1.61, recomputed only when the tree changed) and the
 * closed-form zero of eq. 1.9 for every active coefficient. idiv (nullable, device
 * double[S][n_iters]) receives I(d || q-hat^(j)) before each update (footnote to the
 * Introduction). Coefficients whose surrogate has no finite minimizer are held and
 * counted (wamct_tree_stats). E_STATE before wamct_set_data. */
wamct_status wamct_iterate(wamct_ctx* ctx, int32_t n_iters, double* idiv);

/* Tree rule of the Results section: synthesize mu, threshold = frac * max(mu) (FP64);
 * every leaf at level >= 1 with a pixel above the threshold (strict) gets its three
 * details activated at zero; one level per call; nothing if max(mu) <= 0. Per scan.
 * n_split_host (nullable, HOST int32[S]) receives the number of split nodes. Synchronizes. */
wamct_status wamct_expand(wamct_ctx* ctx, double frac, int32_t* n_split_host);

/* Algorithm 1 with the tree schedule: for j in [0, n_iters): expand (frac) first if j is
 * listed in expand_at (host int32[n_expand], ascending), then iterate once. idiv
 * (nullable, device double[S][n_iters + 1]) gets I(d || q-hat^(j)) for every j and after
 * the last update. Synchronizes once per expansion. */
wamct_status wamct_solve(wamct_ctx* ctx, int32_t n_iters, const int32_t* expand_at,
                         int32_t n_expand, double frac, double* idiv);

/* mu = Omega beta for the current state (eq. 1.2), mu: [S][n*n]. */
wamct_status wamct_synthesize(wamct_ctx* ctx, void* mu);
/* p = H mu for one arbitrary image mu [n*n] (pixel-level ray tracing), p: [n_rays]. */
wamct_status wamct_project(wamct_ctx* ctx, const void* mu, void* p);
/* img = H^T y for one sinogram, y: [n_rays], img: [n*n]. */
wamct_status wamct_backproject(wamct_ctx* ctx, const void* y, void* img);
/* Sign-split coefficient backprojections over the current tree (eq. 1.10):
 * bp(z) = sum_{phi(y|z) > 0} y phi(y|z) and bm(z) = sum_{phi(y|z) < 0} y phi(y|z) for
 * active z, 0 elsewhere; per scan over its own tree: y [S][n_rays], bp, bm: [S][n*n]. */
wamct_status wamct_backproject_split(wamct_ctx* ctx, const void* y, void* bp, void* bm);
/* q-hat = I0 exp(-Phi beta) of the current state into q [S][n_rays] (nullable), and
 * I(d || q-hat) into idiv (device double[S], nullable). E_STATE before set_data. */
wamct_status wamct_forward(wamct_ctx* ctx, void* q, double* idiv);
/* I(d || q) for q [S][n_rays] into out (device double[S]). */
wamct_status wamct_idiv(wamct_ctx* ctx, const void* q, double* out);
/* The precomputed b (eq. 1.6) for every coefficient, [S][n*n] Mallat. */
wamct_status wamct_get_b(wamct_ctx* ctx, void* b);
/* Host copies, per scan (HOST arrays of S), of the current tree's Z0 (eq. 1.61), W =
 * number of (ray, active coefficient) pairs with phi != 0, the number of active
 * coefficients, and the number of coefficient updates held since the last reset (any
 * pointer may be NULL). Synchronizes. */
wamct_status wamct_tree_stats(wamct_ctx* ctx, double* z0, int64_t* w, int64_t* n_active,
                              int64_t* n_held);

/* Differentiable coefficient-domain loss (eq. 1.3 with lambda = 0, every coefficient of the
 * `levels`-level Haar basis free), for a batch of scans that share this geometry:
 *   loss_b = I(d_b || I0 exp(-H Omega c_b)), b = 0..batch-1.
 * c: [batch][n*n] Mallat coefficients; d: [batch][n_rays] counts (not copied; the context's
 * own data are not used); i0: [batch][n_rays] or NULL for the scalar i0_scalar. loss: device
 * double[batch] (FP64 reduction). q: [batch][n_rays] receives q_b = I0 exp(-H Omega c_b), the
 * checkpoint the backward pass needs. Independent of the stack: does not touch beta, the
 * tree or the context's data. */
wamct_status wamct_loss(wamct_ctx* ctx, int32_t batch, const void* c, const void* d, const void* i0,
                        double i0_scalar, double* loss, void* q);
/* Adjoint of wamct_loss from its checkpoint: grad_b = s_b Omega^T H^T (d_b - q_b) (the
 * gradient of loss_b w.r.t. c_b, scaled by s_b = gscale[b], device double[batch], or 1 when
 * gscale is NULL). q, d as above; grad: [batch][n*n]. The residual d_b - q_b is staged in
 * the context's q-hat buffer, so a later wamct_forward must be called again to read q-hat. */
wamct_status wamct_loss_backward(wamct_ctx* ctx, int32_t batch, const void* q, const void* d,
                                 const double* gscale, void* grad);

/* Kernel timing with HIP events on the context's stream. classes: bit k set = record the
 * launches of kernel class k (WAMCT_K_*), each bracketed by two events; 0 stops recording;
 * WAMCT_TIME_ALL records every class; values outside [0, WAMCT_TIME_ALL] give E_INVALID.
 * The call synchronizes and clears the totals. Events add a few microseconds per recorded
 * launch, so record only the classes needed. wamct_get_timing synchronizes and returns, per
 * kernel class, the summed duration in ms and the launch count (arrays of WAMCT_NK). */
#define WAMCT_TIME_ALL ((1 << WAMCT_NK) - 1)
wamct_status wamct_timing(wamct_ctx* ctx, int32_t classes);
wamct_status wamct_get_timing(wamct_ctx* ctx, double* ms, int64_t* launches);

/* Tiling of the node-driven backprojection: a level segment whose items (over the whole
 * stack) number fewer than `lanes` has its views split into chunks so that about `lanes`
 * (item, view chunk) tasks run; 2^12 <= lanes <= 2^24, default 2^20 (2^23 for the cone beam,
 * whose 3-D update measured faster with more view chunks). A larger value may
 * reallocate the context's partial-sum buffer (synchronizes). Results do not depend on the
 * tiling beyond floating-point summation order. */
wamct_status wamct_set_tiling(wamct_ctx* ctx, int32_t lanes);
/* Lanes per ray of the tree's leaf walk (the forward pass over the leaves, Algorithm 1's
 * first step): each ray's path through the image is cut into `lanes` equal pieces walked by
 * neighbouring lanes and added (1, 2 or 4; 0 = chosen by the ray count of the launch: 4 below
 * 2^17 rays, 2 below 2^21, else 1). Results do not depend on it beyond floating-point
 * summation order. E_INVALID for other values; E_UNSUPPORTED for levels = 0 (one lane per ray
 * of the pixel walk) and the cone beam. wamct_get_walk_lanes gives the lanes in use. */
wamct_status wamct_set_walk_lanes(wamct_ctx* ctx, int32_t lanes);
wamct_status wamct_get_walk_lanes(wamct_ctx* ctx, int32_t* lanes);
wamct_status wamct_get_tiling(wamct_ctx* ctx, int32_t* lanes);

/* Ordered subsets of views (the combination with ordered subsets that the Conclusion names;
 * 1 <= n_subsets <= n_views, default 1 = Algorithm 1 as written). Subset k holds the views
 * v with v mod n_subsets = k. With n_subsets > 1 every iteration of wamct_iterate,
 * wamct_solve and batches becomes a pass of n_subsets updates; update k is the Algorithm 1
 * update with q-hat, b (eq. 1.6), b-hat+/- (eq. 1.10) and Z0 (eq. 1.61) all taken over the
 * rays of subset k, so it cannot increase that subset's I-divergence (the full I-divergence
 * is not guaranteed to fall). The idiv entries are I(d || q-hat) over all rays before each
 * pass (an extra full forward pass per iteration when idiv is not NULL) and after the last.
 * Precomputes b of every subset (now if data are set, else in wamct_set_data: [n_subsets]
 * extra coefficient arrays per scan) and a Z0 per subset at every tree change; E_INVALID if
 * a subset has no ray crossing the image. Synchronizes; may allocate. */
wamct_status wamct_set_subsets(wamct_ctx* ctx, int32_t n_subsets);
wamct_status wamct_get_subsets(wamct_ctx* ctx, int32_t* n_subsets);

/* Slices of one volume (Results: each z-slice has its own 2-D Haar transform and all
 * slices share one tree). shared = 1: the scans of the stack are slices with one tree,
 * which the tree rule grows on the FP64 image summed over the slices (every leaf with a
 * pixel of the summed image above frac times its maximum splits, in every slice); scan 0's
 * current tree is copied to every slice now and coefficients outside it are zeroed.
 * Z0 needs no change: with one tree and one geometry it is the same for every slice.
 * wamct_expand then reports the shared tree's split count for every slice. shared = 0
 * (default): every scan grows its own tree. */
wamct_status wamct_set_tree_sharing(wamct_ctx* ctx, int32_t shared);
wamct_status wamct_get_tree_sharing(wamct_ctx* ctx, int32_t* shared);

/* Tree rule used by wamct_expand, wamct_solve and batches.
 * WAMCT_RULE_VALUE (default; Results): every leaf containing a pixel of mu = Omega beta above
 * frac x max(mu) splits one level.
 * WAMCT_RULE_GRADIENT (an other expansion rule, as the Conclusion invites): with q-hat the
 * mean counts of the current beta, c = Omega^T H^T (d - q-hat) is the gradient of the
 * I-divergence with respect to every coefficient (eq. 1.6 applied to the residual); a leaf's
 * score is the largest |c| of its would-be details (the three details of its node), and
 * every leaf scoring above frac x the largest score splits one level (nothing if all scores
 * are 0); for the cone beam the same with the seven details of an octree node. Costs one
 * forward pass, one pixel (voxel) backprojection and one Haar analysis per scan and
 * expansion. Not with tree sharing (E_UNSUPPORTED). Synchronizes; a cone-beam context
 * allocates one coefficient volume when the rule is first selected. */
enum { WAMCT_RULE_VALUE = 0, WAMCT_RULE_GRADIENT = 1 };
wamct_status wamct_set_tree_rule(wamct_ctx* ctx, int32_t rule);
wamct_status wamct_get_tree_rule(wamct_ctx* ctx, int32_t* rule);

/* Roughness penalty (the Introduction's penalized objective I(d || q) + lambda R(mu), whose R the
 * paper does not spell out). Here R(mu) = 1/2 sum over horizontally and vertically adjacent
 * pixel pairs of (mu_x - mu_x')^2. With lambda > 0 every update minimizes eq. 1.8's surrogate
 * plus lambda times the separable quadratic surrogate R + g (beta - beta-hat) + 4 |beta -
 * beta-hat|^2 of R(Omega beta) (g = Omega^T grad R(mu-hat); 8 bounds the Hessian of R and Omega
 * is orthonormal), so I + lambda R cannot increase; per coefficient the minimizer is the root
 * of b - b-hat+ exp(-Z0 delta) - b-hat- exp(Z0 delta) + lambda (g + 8 delta), found in FP64 by
 * safeguarded Newton (no coefficient is held). lambda = 0 (default) is Algorithm 1. The
 * idiv traces still report I(d || q-hat). E_INVALID for lambda < 0 or not finite;
 * E_UNSUPPORTED with ordered subsets and for the cone beam. Synchronizes; the first lambda
 * > 0 allocates one coefficient image per scan. */
wamct_status wamct_set_penalty(wamct_ctx* ctx, double lambda);
wamct_status wamct_get_penalty(wamct_ctx* ctx, double* lambda);

/* Explicit tree sequence Z_s^(j): Algorithm 1 takes the sequence of active sets as an input
 * (the Results section grows it by the tree rule; wamct_solve does that when no schedule is
 * set). n_trees trees: before update j = at[k] of wamct_solve or wamct_batch_solve, tree k
 * becomes the active set of every scan. at: HOST int32[n_trees], >= 0 and strictly
 * ascending, counted from the first update of that solve. masks: DEVICE uint8
 * [n_trees][S][n*n] (cone beam: [n_trees][nz*n*n]), each a valid tree (E_INVALID
 * otherwise); they are copied into the context (allocates n_trees x S x n*n bytes) so the
 * solve needs no host round trip of the state: per tree change it enqueues the mask copy,
 * zeroes the coefficients outside the new tree (those it adds start at 0, as the tree rule's
 * do) and rebuilds Z0 (eq. 1.61) and the work lists, with the one host synchronization
 * every tree change has. With tree sharing, slice 0's tree is used for every slice. While a
 * schedule is set, wamct_solve needs n_expand = 0 (E_INVALID otherwise) and a batch applies
 * the context's schedule in place of its expansion list; n_trees = 0 clears the schedule.
 * wamct_iterate and wamct_expand ignore it. Synchronizes. */
wamct_status wamct_set_tree_schedule(wamct_ctx* ctx, int32_t n_trees, const int32_t* at, const uint8_t* masks);
/* Number of scheduled trees into *n_trees and their first min(cap, n) iterations into at
 * (HOST int32[cap], nullable). */
wamct_status wamct_get_tree_schedule(wamct_ctx* ctx, int32_t* n_trees, int32_t* at, int32_t cap);

/* ---------------------------------------------------------------- no-allocation call
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc) and hold no context: the I-divergence
 * of wamct_idiv, out[s] = I(d_s || q_s) = sum_y q_s(y) - d_s(y) + d_s(y) log(d_s(y) / q_s(y))
 * (0 log 0 = 0) for s < n_scans, from plain device arrays d, q ([n_scans][n_rays], float
 * for WAMCT_F32, double for WAMCT_F64) into out (device double[n_scans]), enqueued on
 * `stream` (hipStream_t, NULL = default). It runs the kernels of wamct_idiv (FP64 partial
 * sums of WAMCT_NOALLOC_RAYS_PER_PARTIAL rays, added in a fixed order), so the result equals
 * wamct_idiv's bit for bit. It allocates nothing: the partial sums live in a static device
 * buffer of WAMCT_NOALLOC_MAX_PARTIALS doubles (8 MiB) that every device the call runs on
 * holds until the process ends; its address is looked up once per device on the first
 * call there. n_scans x ceil(n_rays / WAMCT_NOALLOC_RAYS_PER_PARTIAL) may not exceed
 * WAMCT_NOALLOC_MAX_PARTIALS (E_INVALID; so up to 268 M rays in all). Calls on one device
 * share that buffer: calls that overlap in time on one device (other streams, other host
 * threads) race and must be ordered by the caller. Errors: E_INVALID for a bad dtype,
 * n_rays outside [1, 2^31 - 1], n_scans outside [1, 65535], NULL pointers or too many
 * partial sums; E_HIP for runtime failures. The message is wamct_last_error(NULL). */
#define WAMCT_NOALLOC_MAX_PARTIALS (1 << 20)
#define WAMCT_NOALLOC_RAYS_PER_PARTIAL 256
wamct_status wamct_idiv_noalloc(int32_t dtype, int64_t n_rays, int32_t n_scans, const void* d, const void* q,
                               double* out, void* stream);

/* ---------------------------------------------------------------- batches
 * Uneven batches: several contexts (different geometries, image sizes and view counts,
 * each a stack of scans) solved together. Each context is bound to one of n_streams
 * streams of the batch (longest processing time first by rays x image side x scans). With
 * use_graph != 0 one iteration of every context is captured into a HIP graph and replayed
 * for every iteration between two tree expansions; otherwise the iterations are launched
 * directly on the streams. The contexts stay owned by the caller, must outlive the batch
 * and must not be used concurrently with a batch call; `stream` (hipStream_t, NULL =
 * default) orders the batch after earlier work on it and later work after the batch, as do
 * the contexts' own streams. */
typedef struct wamct_batch wamct_batch;
wamct_status wamct_batch_create(int32_t n_ctx, wamct_ctx* const* ctxs, int32_t n_streams, int32_t use_graph,
                                void* stream, wamct_batch** out);
wamct_status wamct_batch_destroy(wamct_batch* batch);
/* Message of the last failing call on the batch (NULL batch: of wamct_batch_create). */
const char* wamct_batch_last_error(const wamct_batch* batch);
/* wamct_reset of every context, one host synchronization for the whole batch. */
wamct_status wamct_batch_reset(wamct_batch* batch);
/* wamct_solve of every context with the same schedule (n_iters, expand_at, frac).
 * idiv: HOST array of n_ctx device pointers (the array or any entry may be NULL); entry i
 * is double[S_i][n_iters + 1] for context i. A context with a tree schedule
 * (wamct_set_tree_schedule) follows it instead of the expansion list. Results equal those
 * of wamct_solve on each context alone. Synchronizes once per tree change. */
wamct_status wamct_batch_solve(wamct_batch* batch, int32_t n_iters, const int32_t* expand_at, int32_t n_expand,
                               double frac, double* const* idiv);
/* Autotuner of the launch shapes: for every context, n_trial iterations (after one untimed)
 * are timed with HIP events on the context's own stream, its state restored after every
 * trial: first at each candidate backprojection tiling (HOST int32[n_candidates]; NULL =
 * 2^18 .. 2^22), the fastest kept (wamct_set_tiling), then, for contexts with a leaf walk
 * (2-D, levels >= 1), at 1, 2 and 4 lanes per ray with that tiling, the fastest kept
 * (wamct_set_walk_lanes). chosen: HOST int32[n_ctx] (nullable) receives the tilings (the
 * lanes: wamct_get_walk_lanes). Tunes on each context's current tree. Synchronizes; may
 * allocate. */
wamct_status wamct_batch_autotune(wamct_batch* batch, int32_t n_trial, const int32_t* candidates,
                                  int32_t n_candidates, int32_t* chosen);
/* Stream index of each context (HOST int32[n_ctx]), graph launches so far, nodes of the
 * last captured graph and the number of captures (any pointer may be NULL). */
wamct_status wamct_batch_stats(wamct_batch* batch, int32_t* stream_of_ctx, int64_t* graph_launches,
                               int64_t* graph_nodes, int64_t* captures);

#ifdef __cplusplus
}
#endif
#endif
