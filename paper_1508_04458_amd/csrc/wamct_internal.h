// Internal interface between the C ABI (wamct_api.hip) and the kernels (wamct_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

namespace wamct {

constexpr int kMaxLevels = 8;
// Per-scan slots of the small device arrays of a context holding a stack of scans.
constexpr int kScal = 8;   // doubles: [0] Z0, [1] W, [2] max mu, [3] scratch, [4] scalar I0
constexpr int kInts = 32;  // ints: [0] held, [1] bad, [2] n_split, [3] iteration counter,
                           // [8] work items, [9 + k] items of level L - k

// Scan geometry as the kernels see it (see include/wamct.h for the conventions).
struct DevGeom {
  int kind;    // 0 parallel, 1 fan (flat detector)
  int n;       // image n x n
  int nv, nb;  // views, bins
  int L;       // Haar levels
  double pixel, pitch, sod, sdd;
  // views a launch works on: vs0 + vss k for k < nvs (every view: 0, 1, nv); ray arrays
  // stay indexed by the full [view][bin] layout
  int vs0, vss, nvs;
};

// Work item of the node-driven backprojection: one tree node or one box.
//   bit 31     : 1 = node with quadrant chords (three details, plus the approximation
//                when the node is a root), 0 = single box (root approximation or pixel)
//   bits 27-30 : level l
//   bits 13-25 : node row i
//   bits  0-12 : node column j
__host__ __device__ inline uint32_t item_pack(int quad, int l, int i, int j) {
  return (uint32_t(quad) << 31) | (uint32_t(l) << 27) | (uint32_t(i) << 13) | uint32_t(j);
}

enum GatherMode { kPlain = 0, kSplit = 1, kUpdate = 2 };

// Workgroups reach the 8 XCDs round-robin in launch order. The ray walks take their ray block
// through a rotation within each aligned group of 8 blocks: the j-th block an XCD receives is
// ray block 8 j + (xcd + (j >> p)) mod 8, so every XCD cycles through all parts of a view
// (without it, a view of 4 or 8 blocks sends its central, longest rays always to the same XCDs
// and the others idle) while the XCDs still work on neighbouring rays at any time. p = 0
// rotates at every group; a larger p keeps an XCD on the same part of consecutive views for
// 2^p groups (their rays reuse the records in that XCD's L2) and still balances a launch of
// many times 2^p groups. Walk grids are padded to a multiple of 8 (xcd_blocks); blocks past the
// rays write zero partial sums.
__host__ __device__ inline int xcd_rotate(int b, int p = 0) { return (b & ~7) | ((b + (b >> (3 + p))) & 7); }
inline int xcd_blocks(int64_t blocks) { return int((blocks + 7) / 8 * 8); }

// x[0] + x[stride] + ... + x[(n - 1) stride], added strictly in index order (the same
// rounding as a plain loop), with the loads issued eight at a time so that eight are in
// flight instead of one.
template <typename R>
__device__ inline R ordered_sum(const R* __restrict__ x, int n, size_t stride) {
  R s = R(0);
  int c = 0;
  for (; c + 8 <= n; c += 8) {
    R v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = x[size_t(c + k) * stride];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  for (; c < n; ++c) s += x[size_t(c) * stride];
  return s;
}

// v with its sign flipped where s is negative (s = -0.0 counts as negative): one integer op
// on the sign bit, for the direction-dependent signs of the Haar detail integrals.
__device__ inline double xsign(double v, double s) {
  return __longlong_as_double(__double_as_longlong(v) ^ (__double_as_longlong(s) & (1ll << 63)));
}
__device__ inline float xsign(float v, float s) {
  return __int_as_float(__float_as_int(v) ^ (__float_as_int(s) & int(0x80000000u)));
}

// Positive root t of bp t^2 - b t + bm = 0 (eq. 1.9 with t = exp(-Z0 (beta - beta_hat)))
// -> delta = -ln(t) / Z0. Cases (bp >= 0 >= bm): bp > 0 uses the cancellation-free form
// of the quadratic root; bp = 0 > bm is linear (t = bm / b); bp = bm = 0 means no ray sees
// the coefficient (delta = 0). No finite minimizer (t <= 0): hold and count.
template <typename R>
__device__ inline R am_delta(R b, R bp, R bm, R z0, int* held) {
  R t;
  if (bp > R(0)) {
    const R s = sqrt(fmax(b * b - R(4) * bp * bm, R(0)));
    t = b >= R(0) ? (b + s) / (R(2) * bp) : (R(2) * bm) / (b - s);
  } else if (bm < R(0)) {
    t = bm / b;
  } else {
    return R(0);
  }
  if (t > R(0) && isfinite(t)) return -log(t) / z0;
  atomicAdd(held, 1);
  return R(0);
}

// A run of work items of one level, processed with its views split into `chunks` ranges
// of `vpc` views (chunks = 1: one lane per item over all views). For a stack of scans the
// run of scan p is level index kseg of its per-scan counts (start and length read on the
// device) and `count` is the largest length over the stack; kseg < 0 means the fixed range
// [start, start + count) in every scan.
struct Segment {
  int kseg, start, count, level, chunks, vpc;
};
// Segments one gather takes (one per tree level, at most kMaxLevels; one for every pixel).
constexpr int kMaxGatherSegs = 12;
// Default lanes one level segment should occupy over the whole stack (about 64 wave64 per
// CU on 256 CUs, several rounds of the resident waves, so short and long tasks even out);
// tunable per context within [kMinTargetLanes, kMaxTargetLanes].
constexpr int kTargetLanes = 1 << 20;
constexpr int kMinTargetLanes = 1 << 12;
constexpr int kMaxTargetLanes = 1 << 24;
// Partial sums a chunked segment stores: 7 values of R per (scan, item, chunk group). The
// chunked segments of one gather store theirs side by side (one launch computes them all).
inline int64_t segment_part_elems(const Segment& sg, int n_scans) {
  if (sg.chunks <= 1) return 0;
  const int64_t groups = (sg.chunks + 3) / 4;
  return 7 * groups * int64_t(sg.count) * n_scans;
}

// Launchers. T is float or double. Every pointer is device memory unless noted.
template <typename T>
struct Launch {
  // Kernels taking S work on a stack of S scans: image-shaped arrays are [S][n*n],
  // sinogram-shaped arrays [S][n_views*n_bins], per-block partials [S][blocks].
  // mu = Omega beta (inactive coefficients are zero by invariant)
  static void synth(const DevGeom& g, const T* beta, T* mu, int S, hipStream_t s);
  // mu = Omega beta in both layouts the forward walk reads (row- and column-major)
  static void synth_layouts(const DevGeom& g, const T* beta, T* muR, T* muC, int S, hipStream_t s);
  // leaf records (value, level) of mu = Omega beta, row- and column-major
  static void synth_records(const DevGeom& g, const T* beta, const uint8_t* lev, void* leafR, void* leafC, int S,
                            hipStream_t s);
  static void transpose(int n, const T* in, T* out, hipStream_t s);
  // per-pixel leaf level from the tree mask
  static void levmap(const DevGeom& g, const uint8_t* mask, uint8_t* lev, int S, hipStream_t s);
  // I-divergence terms of a given q -> per-block partials. Returns the blocks per scan.
  static int idiv_terms(const DevGeom& g, const T* q, const T* d, double* part, int S, hipStream_t s);
  // b = Omega^T g for every coefficient (FP64 accumulation), one scan
  static void analysis(const DevGeom& g, const T* img, T* coef, hipStream_t s);
  // residual-gradient rule: per-leaf score max |coef| of its would-be details -> score
  // [S][n][n] at the node's first detail position (other entries untouched)
  static void grad_scores(const DevGeom& g, const uint8_t* mask, const T* coef, double* score, int S,
                          hipStream_t s);
  // q <- d - q over len values
  static void residual_inplace(const T* d, T* q, int64_t len, hipStream_t s);
  // gradient of the roughness penalty of the FP64 images mu64 [S][n][n] -> out [S][n][n]
  static void rough_grad(const DevGeom& g, const double* mu64, T* out, int S, hipStream_t s);
  // FP64 synthesis of the current beta and per-block maxima. Returns the blocks per scan.
  static int mu64(const DevGeom& g, const T* beta, double* mu64, double* part, int S, hipStream_t s);
  // zero beta outside the mask
  static void apply_mask(const DevGeom& g, T* beta, const uint8_t* mask, int S, hipStream_t s);
  // count non-finite or negative entries of x into *bad (int, accumulated)
  static void check(const T* x, int64_t len, bool allow_negative, int* bad, hipStream_t s);
  static void fill(T* x, int64_t len, T v, hipStream_t s);
  // r = gscale (d - q) (gscale: device double, null = 1)
  static void residual(const T* d, const T* q, const double* gscale, T* r, int64_t len, hipStream_t s);
};

// lanes per ray of the leaf walk chosen for a launch over `rays` rays (all scans)
int leaf_pieces(int64_t rays);

// Kernels whose ray arithmetic runs in R (float or double, R at least as wide as T).
template <typename T, typename R>
struct Geo {
  // per-ray table in R: A = (ox, oy, 1/ex, 1/ey), B = (ex, ey, 0, 0); origin = the point of
  // the ray closest to the image centre; views = per-view (cos a, sin a) in double.
  static void ray_table(const DevGeom& g, const double2* views, void* A, void* B, hipStream_t s);
  // per-view (cos a, sin a) in float, used only for the detector footprint of a box
  static void view_table(const DevGeom& g, const double2* views, void* vF, hipStream_t s);
  // pixel walk projection of muR/muC (row-/column-major copies of one image per scan). If
  // q != null: q = I0 exp(-p) (I0 = i0v per ray, else the scan's scalar i0s[scan * kScal])
  // and per-block FP64 partial sums of the I-divergence terms in `part`. If p != null the
  // line integrals are stored. Returns the blocks per scan.
  static int forward(const DevGeom& g, const void* A, const void* B, const T* muR, const T* muC, const T* d,
                     const T* i0v, const double* i0s, T* q, T* p, double* part, int S, hipStream_t s);
  // leaf walk over (value, level) records read from global memory
  // lanes: lanes per ray (1, 2 or 4; 0 = leaf_pieces of the launch's ray count)
  static int forward_records(const DevGeom& g, const void* A, const void* B, const void* leafR, const void* leafC,
                             const T* d, const T* i0v, const double* i0s, T* q, T* p, double* part, int S,
                             hipStream_t s, int lanes = 0);
  // node-driven backprojection of y over the segments of `items` (items null: every pixel
  // as a level-0 box), over the views of g's subset. counts: per-scan level counts (stride
  // kInts; null for fixed ranges); z0 per scan at stride z0stride, held at stride kInts;
  // `part` holds segment_part_elems. views: (cos, sin) per view in FP64 (fan-beam source).
  static void gather(const DevGeom& g, int mode, const void* vF, const double2* views, const void* A, const T* y,
                     const uint32_t* items, const int* counts, const Segment* segs, int n_segs, void* part,
                     T* beta, const T* b, const double* z0, int z0stride, int* held, T* bp, T* bm, T* out,
                     int S, hipStream_t s, const T* gpen = nullptr, double lam = 0.0);
};

// Daubechies-4 (periodic) basis tables on the device: per level l (1..L) the samples of the
// scaling function (f) and of the wavelet (g) at position 0, offsets 0 .. len[l] - 1 from the
// function's first pixel (len = 3 x 2^l - 2), starting at f + off[l] and g + off[l]. The
// function at position j is the same samples shifted by 2^l j (mod n).
struct D4Dev {
  const double* f;
  const double* g;
  int off[kMaxLevels + 1];
  int len[kMaxLevels + 1];
};
// Host samples of the tables (f, g concatenated over l = 1..L) and their offsets and lengths.
void d4_tables(int L, std::vector<double>& f, std::vector<double>& g, D4Dev& tb);
// Modes of the Daubechies-4 gather.
enum D4Mode { kD4Split = 0, kD4Update = 1, kD4Z0 = 2 };
template <typename T, typename R>
struct D4 {
  // mu = Omega beta in row-major muR and, when muC is not null, column-major muC (one scan)
  static void synth(const DevGeom& g, const D4Dev& tb, const T* beta, T* muR, T* muC, hipStream_t s);
  // FP64 mu = Omega beta and per-block maxima. Returns the number of blocks.
  static int mu64(const DevGeom& g, const D4Dev& tb, const T* beta, double* mu64, double* part, hipStream_t s);
  // coef = Omega^T img (FP64 accumulation)
  static void analysis(const DevGeom& g, const D4Dev& tb, const T* img, T* coef, hipStream_t s);
  // Node-driven backprojection of y over the work list (n_items read on the device, at most
  // max_items): kD4Split -> bp, bm; kD4Update -> beta += the eq. 1.9 zero (b, z0, held);
  // kD4Z0 -> zsum[ray] += sum |phi| over the list's coefficients (zsum zeroed by the caller)
  // and cnt[item] = number of non-zero phi of the item. A, B: the ray table of Geo.
  static void gather(const DevGeom& g, int mode, const D4Dev& tb, const double2* views, const void* A,
                     const void* B, const T* y, const uint32_t* items, const int* n_items, int max_items, T* beta,
                     const T* b, const double* z0, int* held, T* bp, T* bm, double* zsum, double* cnt,
                     hipStream_t s);
};

// Z0 and W of the current tree: per-ray FP64 sums of |phi| over active coefficients and
// counts of phi != 0; per-block partial max / sum. Returns the blocks per scan.
int z0_partials(const DevGeom& g, const double2* views, const uint8_t* lev, double* part_max,
                double* part_cnt, int S, hipStream_t s);
// Deterministic single-block reductions of per-block partials: out[0] = sum or max.
// per-block partial sums per scan that Launch<T>::idiv_terms writes for `rays` rays
int idiv_blocks(int64_t rays);
void reduce_sum(const double* part, int n, double* out, hipStream_t s);
void reduce_max(const double* part, int n, double* out, hipStream_t s);
// The same for a stack of S scans, one block per scan: scan p reduces part[p * pstride ..
// + n) into out[p * ostride + c], c = 0, or c = ctr[p * kInts] when ctr is not null (the
// counter is then incremented: the slot of the next call).
void reduce_stack(bool max, const double* part, int n, int64_t pstride, double* out, int64_t ostride, int* ctr,
                  int S, hipStream_t s);
// Work list of the node-driven backprojection (roots, then split nodes level by level,
// Morton order within a level), compacted with wave ballots; per scan counts[0] = number
// of items, counts[1 + k] = items of level L - k (k = 0..L; level 0 only when L = 0);
// counts at stride kInts, items at stride n*n.
// work lists of the active trees (items, per-scan counts at stride kInts); `scratch` holds
// list_scratch_ints(g, S) ints
int64_t list_scratch_ints(const DevGeom& g, int S);
void build_items(const DevGeom& g, const uint8_t* mask, uint32_t* items, int* counts, int S, int* scratch,
                 hipStream_t s);
// Tree rule: split every leaf of mask_old whose value exceeds frac * max (maxv at stride
// kScal, n_split at stride kInts). rule 0: the FP64 image mu64 (leaf-constant); rule 1: the
// leaf scores of grad_scores held in mu64 at each node's first detail position; rule 2: the
// largest pixel of mu64 over the leaf's block (images not constant on the leaves).
void expand(const DevGeom& g, const uint8_t* mask_old, uint8_t* mask, const double* mu64,
            const double* maxv, double frac, int* n_split, int S, hipStream_t s, int rule = 0);
// Sum of the FP64 images of S slices into slice 0 (slice order) and per-block maxima of the
// sum. Returns the number of blocks.
int sum_slices(const DevGeom& g, double* mu64, double* part, int S, hipStream_t s);
// Validity of S tree masks: *bad = number of violated constraints.
void check_mask(const DevGeom& g, const uint8_t* mask, int* bad, int S, hipStream_t s);
void fill_u8(uint8_t* x, int64_t len, uint8_t v, hipStream_t s);
void fill_i32(int* x, int64_t len, int v, hipStream_t s);
// x[k * stride] = v for k < count
void fill_i32_strided(int* x, int count, int stride, int v, hipStream_t s);
void approx_mask(const DevGeom& g, uint8_t* mask, int S, hipStream_t s);

}  // namespace wamct
