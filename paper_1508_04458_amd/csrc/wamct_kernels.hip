// HIP kernels of wavelet-tree alternating minimization for gfx950 (wave64).
//
// Method: Degirmenci, O'Sullivan, Politte, arXiv 1508.04458, Introduction (eqs. 1.2-1.10,
// Algorithm 1) and Results (tree rule). The system matrix is never stored: chord lengths
// h(y|x) (ray-pixel intersection lengths, Introduction) are recomputed on the fly, so the
// kernels are bound by vector ALU and cache gathers, not by streaming a matrix.
#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/wamct.h"
#include "wamct_internal.h"
#include "wamct_geom.h"
#include "wamct_worklist.h"

namespace wamct {
namespace {

template <typename T> struct V4;
template <> struct V4<float> { using t = float4; };
template <> struct V4<double> { using t = double4; };
template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

constexpr int kBlock = 256;
// wamct_idiv_noalloc sizes its static buffer by the rays one I-divergence partial covers
static_assert(kBlock == WAMCT_NOALLOC_RAYS_PER_PARTIAL, "partial-sum size of the I-divergence");

inline int blocks_for(int64_t n, int b = kBlock) { return int((n + b - 1) / b); }

// Slice of scan `off / size` of a stacked array (a null pointer stays null).
template <typename P>
__device__ inline P* at(P* x, int64_t off) { return x ? x + off : x; }

// Ray (index into the full [view][bin] layout) of the k-th ray of the launch's views.
__device__ inline int subset_ray(const DevGeom& g, int k) {
  const int j = k / g.nb;
  return (g.vs0 + g.vss * j) * g.nb + (k - j * g.nb);
}

// ------------------------------------------------------------------ reductions (wave64)

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// block of kBlock threads -> value in thread 0
template <bool MAX>
__device__ inline double block_reduce(double v) {
  __shared__ double sh[kBlock / 64];
  v = MAX ? wave_max(v) : wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int k = 1; k < kBlock / 64; ++k) r = MAX ? fmax(r, sh[k]) : r + sh[k];
    v = r;
  }
  return v;
}

// One block per scan; fixed assignment and order -> deterministic result. With a counter
// the result goes to slot ctr[scan] of the scan's row, and the counter moves on.
template <bool MAX>
__global__ __launch_bounds__(kBlock) void k_reduce(const double* __restrict__ part, int n, int64_t pstride,
                                                   double* __restrict__ out, int64_t ostride,
                                                   int* __restrict__ ctr) {
  const int p = blockIdx.x;
  part += p * pstride;
  double v;
  if (MAX) {
    v = -INFINITY;
    for (int k = threadIdx.x; k < n; k += kBlock) v = fmax(v, part[k]);
  } else {
    const int cnt = int(threadIdx.x) < n ? (n - 1 - int(threadIdx.x)) / kBlock + 1 : 0;
    v = ordered_sum(part + threadIdx.x, cnt, size_t(kBlock));
  }
  v = block_reduce<MAX>(v);
  if (threadIdx.x == 0) {
    int64_t o = p * ostride;
    if (ctr) {
      const int c = ctr[p * kInts];
      o += c;
      ctr[p * kInts] = c + 1;
    }
    out[o] = v;
  }
}

// ------------------------------------------------------------------ geometry

template <typename T>
__global__ __launch_bounds__(kBlock) void k_ray_table(DevGeom g, const double2* __restrict__ views,
                                                      typename V4<T>::t* __restrict__ A,
                                                      typename V4<T>::t* __restrict__ B) {
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= g.nv * g.nb) return;
  const int v = r / g.nb, b = r - v * g.nb;
  double ox, oy, ex, ey;
  ray_of(g, views[v], b, ox, oy, ex, ey);
  // an axis-parallel component (set to +-1e-12 by ray_of) gets an inverse that acts as
  // infinite: slab parameters (X - x) / e are then beyond any chord for every X off the
  // line's position, also when measured from the fan-beam source instead of the moved
  // origin, so the gather and the walks place the line in the same pixel row
  const double big = sizeof(T) == 8 ? 1e300 : 1e30;
  const double iex = fabs(ex) <= 1e-12 ? (ex < 0 ? -big : big) : 1.0 / ex;
  const double iey = fabs(ey) <= 1e-12 ? (ey < 0 ? -big : big) : 1.0 / ey;
  typename V4<T>::t a, bb;
  a.x = T(ox); a.y = T(oy); a.z = T(iex); a.w = T(iey);
  bb.x = T(ex); bb.y = T(ey); bb.z = T(0); bb.w = T(0);
  A[r] = a;
  B[r] = bb;
}

template <typename T>
__global__ void k_view_table(int nv, const double2* __restrict__ views, typename V2<T>::t* __restrict__ out) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= nv) return;
  typename V2<T>::t o;
  o.x = T(views[v].x); o.y = T(views[v].y);
  out[v] = o;
}

// ------------------------------------------------------------------ tree helpers

// node (l, i, j) split <=> its D1 detail is active (mask[i][m + j], m = n >> l)
__device__ inline bool is_split(const uint8_t* __restrict__ mask, int n, int l, int i, int j) {
  const int m = n >> l;
  return mask[i * n + (m + j)] != 0;
}

__device__ inline uint32_t morton_compact(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0f0f0f0fu;
  x = (x | (x >> 4)) & 0x00ff00ffu;
  x = (x | (x >> 8)) & 0x0000ffffu;
  return x;
}

// ------------------------------------------------------------------ synthesis (eq. 1.2)

// mu(r, c) = 2^-L beta_LL(root) + sum_l 2^-l (s1 D1 + s2 D2 + s3 D3) of the node at level l
// containing the pixel; inactive coefficients are zero, so this is Omega beta on Z_s.
template <typename T, typename R>
__device__ inline R synth_pixel(const T* __restrict__ beta, int n, int L, int r, int c) {
  R v = R(beta[(r >> L) * n + (c >> L)]) * R(1.0 / double(1 << L));
  for (int l = L; l >= 1; --l) {
    const int m = n >> l, i = r >> l, j = c >> l;
    const R d1 = R(beta[i * n + m + j]);
    const R d2 = R(beta[(m + i) * n + j]);
    const R d3 = R(beta[(m + i) * n + m + j]);
    const bool right = (c >> (l - 1)) & 1, bottom = (r >> (l - 1)) & 1;
    const R s1d1 = right ? -d1 : d1;
    const R s2d2 = bottom ? -d2 : d2;
    const R s3d3 = (right != bottom) ? -d3 : d3;
    v += (s1d1 + s2d2 + s3d3) * R(1.0 / double(1 << l));
  }
  return v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_synth(int n, int L, const T* __restrict__ beta, T* __restrict__ mu) {
  const int64_t off = int64_t(blockIdx.y) * n * n;
  beta += off;
  mu += off;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= n * n) return;
  mu[p] = synth_pixel<T, T>(beta, n, L, p / n, p % n);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mu64(int n, int L, const T* __restrict__ beta,
                                                 double* __restrict__ mu64, double* __restrict__ part) {
  const int64_t off = int64_t(blockIdx.y) * n * n;
  beta += off;
  mu64 += off;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  double v = -INFINITY;
  if (p < n * n) {
    v = synth_pixel<T, double>(beta, n, L, p / n, p % n);
    mu64[p] = v;
  }
  v = block_reduce<true>(v);
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = v;
}

// Slices sharing one tree (Results: the tree rule thresholds the image summed over the
// z-slices): mu64[i] = sum over the S slices of mu64[p][i] in slice order (FP64), written to
// slice 0, with per-block maxima of the sum.
__global__ __launch_bounds__(kBlock) void k_sum_slices(int64_t nn, int S, double* __restrict__ mu64,
                                                       double* __restrict__ part) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  double v = -INFINITY;
  if (i < nn) {
    v = 0.0;
    for (int p = 0; p < S; ++p) v += mu64[p * nn + i];
    mu64[i] = v;
  }
  v = block_reduce<true>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(kBlock) void k_levmap(int n, int L, const uint8_t* __restrict__ mask,
                                                   uint8_t* __restrict__ lev) {
  const int64_t off = int64_t(blockIdx.y) * n * n;
  mask += off;
  lev += off;
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= n * n) return;
  const int r = p / n, c = p % n;
  int l = L;
  while (l >= 1 && is_split(mask, n, l, r >> l, c >> l)) --l;
  lev[p] = uint8_t(l);
}

// ------------------------------------------------------------------ image layouts

// Leaf record of the forward walk, one word per pixel read with one load per step: the
// (leaf-constant) value at the pixel rounded to the nearest value whose 4 low mantissa
// bits are zero (relative rounding <= 2^-20 in FP32, 2^-49 in FP64), with the level of the
// tree leaf containing the pixel (0..8) stored in those 4 bits. Half the bytes of a
// (value, level) pair, so a wave's scattered loads touch fewer cache lines.
template <typename T>
struct Leaf;
template <>
struct Leaf<float> {
  uint32_t w;
  __device__ static Leaf make(float v, uint32_t lev) { return Leaf{((__float_as_uint(v) + 8u) & ~15u) | lev}; }
  __device__ float mu() const { return __uint_as_float(w & ~15u); }
  __device__ uint32_t lev() const { return w & 15u; }
};
template <>
struct Leaf<double> {
  uint64_t w;
  __device__ static Leaf make(double v, uint32_t lev) {
    return Leaf{((uint64_t(__double_as_longlong(v)) + 8u) & ~uint64_t(15)) | lev};
  }
  __device__ double mu() const { return __longlong_as_double((long long)(w & ~uint64_t(15))); }
  __device__ uint32_t lev() const { return uint32_t(w & 15u); }
};

// mu = Omega beta over 32x32 pixel tiles, written twice: row-major and column-major (the
// copy read by rays travelling mostly along x, whose lanes then step through consecutive
// addresses instead of one image row each). TREE: leaf records; otherwise plain values.
template <typename T, bool TREE>
__global__ __launch_bounds__(256) void k_synth_tiles(int n, int L, const T* __restrict__ beta,
                                                     const uint8_t* __restrict__ lev, T* __restrict__ muR,
                                                     T* __restrict__ muC, Leaf<T>* __restrict__ leafR,
                                                     Leaf<T>* __restrict__ leafC) {
  __shared__ T tile[32][33];
  __shared__ uint8_t ltile[32][33];
  const int64_t off = int64_t(blockIdx.z) * n * n;
  beta += off;
  lev = at(lev, off);
  muR = at(muR, off);
  muC = at(muC, off);
  leafR = at(leafR, off);
  leafC = at(leafC, off);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = r0 + ty + 8 * k, c = c0 + tx;
    if (r < n && c < n) {
      const T v = synth_pixel<T, T>(beta, n, L, r, c);
      tile[ty + 8 * k][tx] = v;
      if (TREE) {
        const uint8_t lv = lev[r * n + c];
        ltile[ty + 8 * k][tx] = lv;
        leafR[r * n + c] = Leaf<T>::make(v, lv);
      } else {
        muR[r * n + c] = v;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = c0 + ty + 8 * k, r = r0 + tx;
    if (r < n && c < n) {
      const T v = tile[tx][ty + 8 * k];
      if (TREE)
        leafC[c * n + r] = Leaf<T>::make(v, ltile[tx][ty + 8 * k]);
      else
        muC[c * n + r] = v;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_transpose(int n, const T* __restrict__ in, T* __restrict__ out) {
  __shared__ T tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = r0 + ty + 8 * k, c = c0 + tx;
    if (r < n && c < n) tile[ty + 8 * k][tx] = in[r * n + c];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = c0 + ty + 8 * k, r = r0 + tx;
    if (r < n && c < n) out[c * n + r] = tile[tx][ty + 8 * k];
  }
}

// ------------------------------------------------------------------ forward + Beer's law

// Pixel walk (image-domain AM and the projection operator). One lane per ray (consecutive
// lanes = consecutive bins of one view): p = sum_x h(y|x) mu(x) by incremental plane
// crossings (Siddon's parametric form, in R), then q-hat = I0 exp(-p) (Introduction;
// Algorithm 1 first step) and the FP64 term d log(d / q) - d + q of the I-divergence
// (0 log 0 = 0) with log q = log I0 - p. The pixel sequence does not depend on mu, so the
// walk runs KB steps ahead recording chord and address, then issues the KB loads together
// (KB loads in flight per lane instead of one dependent load per step). Rays travelling
// mostly along x read the column-major copy of the image, so neighbouring lanes touch
// consecutive addresses. K adjacent lanes share a ray: lane k walks the k-th of K equal parts
// of its parameter interval inside the image (from the pixel holding the part's start; a pixel
// one behind at a plane gives a zero chord and moves on), and the parts are added by a fixed
// shuffle.
template <typename T, typename R, int KB, int K>
__global__ __launch_bounds__(kBlock) void k_forward(DevGeom g, const typename V4<R>::t* __restrict__ A,
                                                    const typename V4<R>::t* __restrict__ B,
                                                    const T* __restrict__ muR, const T* __restrict__ muC,
                                                    const T* __restrict__ d, const T* __restrict__ i0v,
                                                    const double* __restrict__ i0s, T* __restrict__ q,
                                                    T* __restrict__ pout, double* __restrict__ part) {
  const int M = g.nv * g.nb;
  const int sc = blockIdx.y;
  {
    const int64_t oi = int64_t(sc) * g.n * g.n, orr = int64_t(sc) * M;
    muR += oi; muC += oi;
    d = at(d, orr); i0v = at(i0v, orr); q = at(q, orr); pout = at(pout, orr);
  }
  const int rb = xcd_rotate(blockIdx.x);
  const int lane_id = rb * kBlock + threadIdx.x;
  const int k = lane_id / K, piece = lane_id % K;
  const int r = subset_ray(g, k);
  double term = 0.0;
  const bool valid = k < g.nvs * g.nb;
  R acc = R(0);
  if (valid) {
    const typename V4<R>::t a = A[r];
    const typename V4<R>::t bb = B[r];
    const R ox = a.x, oy = a.y, iex = a.z, iey = a.w, ex = bb.x, ey = bb.y;
    const int n = g.n;
    const R pix = R(g.pixel), ipix = R(1.0 / g.pixel), hn = R(0.5 * n), half = R(0.5 * n * g.pixel);
    const R tx0 = (-half - ox) * iex, tx1 = (half - ox) * iex;
    const R ty0 = (-half - oy) * iey, ty1 = (half - oy) * iey;
    const R t_enter = fmax(fmin(tx0, tx1), fmin(ty0, ty1));
    const R t_exit = fmin(fmax(tx0, tx1), fmax(ty0, ty1));
    // this lane's part [t_in, t_out) of the path
    const R t_in = piece == 0 ? t_enter : t_enter + (t_exit - t_enter) * (R(piece) / R(K));
    const R t_out = piece == K - 1 ? t_exit : t_enter + (t_exit - t_enter) * (R(piece + 1) / R(K));
    if (t_exit > t_enter) {
      int ix = (int)floor(fmin(fmax((ox + t_in * ex) * ipix + hn, R(-1)), R(n)));
      int iy = (int)floor(fmin(fmax((oy + t_in * ey) * ipix + hn, R(-1)), R(n)));
      ix = imin(imax(ix, 0), n - 1);
      iy = imin(imax(iy, 0), n - 1);
      const bool px = ex > R(0), py = ey > R(0);
      const bool xmaj = fabs(ex) >= fabs(ey);
      const T* __restrict__ base = xmaj ? muC : muR;
      const int sx = px ? 1 : -1, sy = py ? 1 : -1;
      R t = t_in;
      bool alive = true;
      R tX = ((R(px ? ix + 1 : ix) - hn) * pix - ox) * iex;
      R tY = ((R(py ? iy + 1 : iy) - hn) * pix - oy) * iey;
      const R dtX = pix * fabs(iex), dtY = pix * fabs(iey);
      const int max_batches = (2 * n + 4) / KB + 1;
      for (int batch = 0; batch < max_batches && alive; ++batch) {
        R ch[KB];
        int ad[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          ad[k] = xmaj ? ix * n + iy : iy * n + ix;
          const bool sxs = tX <= tY;
          const R te = fmin(sxs ? tX : tY, t_out);
          const int nix = sxs ? ix + sx : ix, niy = sxs ? iy : iy + sy;
          ch[k] = alive ? fmax(te - t, R(0)) : R(0);
          const bool go = alive && te < t_out && (unsigned)nix < (unsigned)n && (unsigned)niy < (unsigned)n;
          if (go) {
            if (sxs) tX += dtX; else tY += dtY;
            t = te; ix = nix; iy = niy;
          }
          alive = go;
        }
        T mv[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) mv[k] = base[ad[k]];
#pragma unroll
        for (int k = 0; k < KB; ++k) acc += ch[k] * R(mv[k]);
      }
    }
  }
  // the K parts of a ray, added in a fixed order (every lane of the group gets the total)
#pragma unroll
  for (int o = 1; o < K; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if (valid && piece == 0) {
    const R p = acc;
    if (pout) pout[r] = T(p);
    if (q) {
      const double i0 = i0v ? double(i0v[r]) : i0s[sc * kScal];
      const double pd = double(p);
      const double qd = i0 * exp(-pd);
      q[r] = T(qd);
      const double dv = double(d[r]);
      term = qd - dv;
      if (dv > 0.0) term += dv * (log(dv) - (log(i0) - pd));
    }
  }
  if (part) {
    term = block_reduce<false>(term);
    if (threadIdx.x == 0) part[sc * gridDim.x + rb] = term;
  }
}

// Leaf walk (wavelet AM): p = sum over the tree leaves crossed of chord * mu_leaf
// (= sum_z phi(y|z) beta(z) on Z_s), then Beer's law and the I-divergence term as above.
// One (value, level) record per step; the next record is requested before the current
// chord is accumulated. From the pixel (ix, iy) inside the current leaf the exit is the
// nearer of the leaf's two exit planes; the next pixel is the neighbour across that plane,
// its other coordinate taken from the exit point (FP32 suffices: it is clamped into the old
// leaf's range and never moves backwards, so rounding at a corner only moves a vanishing
// chord between neighbours and cannot reverse the walk). Every step adds at least one to the
// crossed axis' pixel index and never lowers the other, and the walk stops once an index
// reaches n, so it ends after at most 2n steps for any levels in the records (no step
// counter). x-major rays read the column-major records.
// With K > 1, K adjacent lanes share a ray (for launches with too few rays to fill the
// GPU): lane k walks the k-th of K equal parameter pieces of the ray's path through the
// image from the pixel holding the piece's first point, and the K sums are added across
// the lanes.
template <typename T, typename R, int K>
__global__ __launch_bounds__(kBlock) void k_forward_rec(DevGeom g, const typename V4<R>::t* __restrict__ A,
                                                        const typename V4<R>::t* __restrict__ B,
                                                        const Leaf<T>* __restrict__ leafR,
                                                        const Leaf<T>* __restrict__ leafC,
                                                        const T* __restrict__ d, const T* __restrict__ i0v,
                                                        const double* __restrict__ i0s, T* __restrict__ q,
                                                        T* __restrict__ pout, double* __restrict__ part) {
  const int M = g.nv * g.nb;
  const int sc = blockIdx.y;
  {
    const int64_t oi = int64_t(sc) * g.n * g.n, orr = int64_t(sc) * M;
    leafR += oi; leafC += oi;
    d = at(d, orr); i0v = at(i0v, orr); q = at(q, orr); pout = at(pout, orr);
  }
  const int rb = xcd_rotate(blockIdx.x);
  const int lane_id = rb * kBlock + threadIdx.x;
  const int k = lane_id / K, piece = lane_id % K;
  const int r = subset_ray(g, k);
  double term = 0.0;
  R acc = R(0);
  if (k < g.nvs * g.nb) {
    const typename V4<R>::t a = A[r];
    const typename V4<R>::t bb = B[r];
    const R ox = a.x, oy = a.y, iex = a.z, iey = a.w, ex = bb.x, ey = bb.y;
    const int n = g.n;
    const R pix = R(g.pixel), ipix = R(1.0 / g.pixel), hn = R(0.5 * n), half = R(0.5 * n * g.pixel);
    const R tx0 = (-half - ox) * iex, tx1 = (half - ox) * iex;
    const R ty0 = (-half - oy) * iey, ty1 = (half - oy) * iey;
    const R t_in = fmax(fmin(tx0, tx1), fmin(ty0, ty1));
    const R t_end = fmin(fmax(tx0, tx1), fmax(ty0, ty1));
    if (t_end > t_in) {
      // this lane's piece [t_s, t_out) of the path
      const R t_s = piece == 0 ? t_in : t_in + (t_end - t_in) * (R(piece) / R(K));
      const R t_out = piece == K - 1 ? t_end : t_in + (t_end - t_in) * (R(piece + 1) / R(K));
      // major axis u (the one the ray travels along more; its records are contiguous in
      // the minor axis w) and minor axis w: the record of pixel (u, w) is base[u n + w].
      // The walk runs in a frame mirrored per axis so that both coordinates grow along the
      // ray (leaf boundaries stay aligned since 2^l divides n): pixel coordinate c0 + t ce,
      // plane k crossed at t = t0 + k dt.
      const bool xmaj = fabs(ex) >= fabs(ey);
      const Leaf<T>* __restrict__ base = xmaj ? leafC : leafR;
      const R eu = xmaj ? ex : ey, ew = xmaj ? ey : ex;
      const R ieu = xmaj ? iex : iey, iew = xmaj ? iey : iex;
      const R Ou = (xmaj ? ox : oy) * ipix + hn, Ow = (xmaj ? oy : ox) * ipix + hn;
      const R cu0 = eu < R(0) ? R(n) - Ou : Ou, cw0 = ew < R(0) ? R(n) - Ow : Ow;
      const R cue = fabs(eu) * ipix, cwe = fabs(ew) * ipix;
      const R dtu = fabs(ieu) * pix, dtw = fabs(iew) * pix;
      const R tu1 = (R(1) - cu0) * dtu, tw1 = (R(1) - cw0) * dtw;   // planes u = 1, w = 1
      // real index = c + s m of the mirrored one (c = 0, s = 1, or c = n - 1, s = -1), so the
      // record index (real u) n + (real w) is linear in the mirrored pixel
      const int su = eu < R(0) ? -1 : 1, sw = ew < R(0) ? -1 : 1;
      const int i0 = (eu < R(0) ? n - 1 : 0) * n + (ew < R(0) ? n - 1 : 0), du = su * n;
      auto idx = [&](int u, int w) { return unsigned(i0 + __mul24(du, imin(u, n - 1)) + __mul24(sw, imin(w, n - 1))); };
      int iu = imin(imax(int(fma(t_s, cue, cu0)), 0), n - 1);
      int iw = imin(imax(int(fma(t_s, cwe, cw0)), 0), n - 1);
      Leaf<T> rec = base[idx(iu, iw)];
      R t = t_s;
      for (;;) {   // ends: see the kernel's comment
        const int m = (1 << int(rec.lev())) - 1;
        const int hu = iu | m, hw = iw | m;   // last pixel of the leaf along u and w
        const R tU = fma(R(hu), dtu, tu1), tW = fma(R(hw), dtw, tw1);   // its upper planes
        const bool cu = tU <= tW;   // the leaf is left through a u plane
        // the planes lie ahead of t up to rounding (a chord an ulp below 0 where the ray
        // passes a corner; the pixel indices never move backwards)
        const R te = fmin(fmin(tU, tW), t_out);
        // the axis not crossed takes the exit point's pixel, clamped into the old leaf's
        // range and never moving backwards; the crossed axis steps to the neighbour leaf (its
        // exit point's pixel clamps to the leaf's last one)
        const int niu = imin(imax(int(fma(te, cue, cu0)), iu), hu) + int(cu);
        const int niw = imin(imax(int(fma(te, cwe, cw0)), iw), hw) + int(!cu);
        const bool go = te < t_out && niu < n && niw < n;
        const Leaf<T> nrec = base[idx(niu, niw)];
        acc += (te - t) * R(rec.mu());
        if (!go) break;
        t = te; iu = niu; iw = niw; rec = nrec;
      }
    }
  }
#pragma unroll
  for (int o = 1; o < K; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if (k < g.nvs * g.nb && piece == 0) {
    const R p = acc;
    if (pout) pout[r] = T(p);
    if (q) {
      const double i0 = i0v ? double(i0v[r]) : i0s[sc * kScal];
      const double pd = double(p);
      const double qd = i0 * exp(-pd);
      q[r] = T(qd);
      const double dv = double(d[r]);
      term = qd - dv;
      if (dv > 0.0) term += dv * (log(dv) - (log(i0) - pd));
    }
  }
  if (part) {
    term = block_reduce<false>(term);
    if (threadIdx.x == 0) part[sc * gridDim.x + rb] = term;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_idiv_terms(int M, const T* __restrict__ q, const T* __restrict__ d,
                                                       double* __restrict__ part) {
  q += int64_t(blockIdx.y) * M;
  d += int64_t(blockIdx.y) * M;
  const int r = blockIdx.x * kBlock + threadIdx.x;
  double term = 0.0;
  if (r < M) {
    const double qd = double(q[r]), dv = double(d[r]);
    term = qd - dv;
    if (dv > 0.0) term += dv * log(dv / qd);
  }
  term = block_reduce<false>(term);
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = term;
}

// ------------------------------------------------------------------ node-driven gather

// Sums of one work item over a range of views. For every view the item's box is projected
// onto the detector (its four corners bound the bins whose rays can hit it; FP32 suffices
// for this bound, which is widened by 1e-3 bin), and for each such ray the chord through
// the box is computed in R by slab clipping with the same ray table as the forward pass, and
// for a split node the quadrant combinations from the box interval and the ray's crossings of
// the box's mid-lines. Details of node (l, i, j) have phi = 2^-l sum_q s_k(q) chord(q); an
// approximation has 2^-L chord(box). The sign split of eq. 1.10 is taken per
// (ray, coefficient), so b-hat+ and b-hat- need no atomics.
template <typename R>
struct ItemSums {
  R acc;             // plain sum (box chord)
  R s0, s1, s2;      // per detail: signed sum
  R a0, a1, a2;      // per detail: sum of magnitudes (positive part (a + s) / 2, negative (s - a) / 2)
};

template <typename T, typename R, bool FAN>
__device__ inline ItemSums<R> item_sums_k(const DevGeom& g, const float2* __restrict__ vf,
                                        const double2* __restrict__ views, const typename V4<R>::t* __restrict__ A,
                                        const T* __restrict__ y, bool quad, int l, int i, int j, int v0, int v1) {
  const int n = g.n, s = 1 << l, nb = g.nb;
  const R pix = R(g.pixel), hn = R(0.5 * n);
  const R X0 = (R(j * s) - hn) * pix, X2 = (R((j + 1) * s) - hn) * pix;
  const R Y0 = (R(i * s) - hn) * pix, Y2 = (R((i + 1) * s) - hn) * pix;
  const R X1 = R(0.5) * (X0 + X2), Y1 = R(0.5) * (Y0 + Y2);
  const float fx0 = float(X0), fx2 = float(X2), fy0 = float(Y0), fy2 = float(Y2);
  const float ipitch = float(1.0 / g.pitch), ctr = float(0.5 * (nb - 1));
  const float sod = float(g.sod), sdd = float(g.sdd);
  // |phi| <= 1e-12 pixel is rounding residue of chord differences, taken as 0 (phi is 2^-l
  // times the quadrant combinations below); otherwise a coefficient whose rays all give
  // phi <= 0 would get a residue-sized b-hat+ and jump to the other branch of eq. 1.9
  const R tq = R(1e-12 * g.pixel * double(1 << l));
  ItemSums<R> r{R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
  for (int k = v0; k < v1; ++k) {
    const int v = g.vs0 + g.vss * k;   // k-th view of the launch's subset
    const float2 cs = vf[v];
    const float c = cs.x, sn = cs.y;
    float u00, u01, u10, u11;
    if (!FAN) {
      u00 = fx0 * c + fy0 * sn; u01 = fx2 * c + fy0 * sn; u10 = fx0 * c + fy2 * sn; u11 = fx2 * c + fy2 * sn;
    } else {
      // hardware reciprocal (1 ulp): the bound is widened by 1e-3 bin anyway
      u00 = sdd * (-fx0 * sn + fy0 * c) * __builtin_amdgcn_rcpf(sod - (fx0 * c + fy0 * sn));
      u01 = sdd * (-fx2 * sn + fy0 * c) * __builtin_amdgcn_rcpf(sod - (fx2 * c + fy0 * sn));
      u10 = sdd * (-fx0 * sn + fy2 * c) * __builtin_amdgcn_rcpf(sod - (fx0 * c + fy2 * sn));
      u11 = sdd * (-fx2 * sn + fy2 * c) * __builtin_amdgcn_rcpf(sod - (fx2 * c + fy2 * sn));
    }
    const float umin = fminf(fminf(u00, u01), fminf(u10, u11));
    const float umax = fmaxf(fmaxf(u00, u01), fmaxf(u10, u11));
    // bins whose centre lies in [umin, umax] widened by 1e-3 bin; clamped in floating
    // point first so the integer conversion can never overflow
    const float flo = fminf(fmaxf(umin * ipitch + ctr - 1e-3f, -1.f), float(nb));
    const float fhi = fminf(fmaxf(umax * ipitch + ctr + 1e-3f, -1.f), float(nb));
    const int blo = max(int(ceilf(flo)), 0);
    const int bhi = min(int(floorf(fhi)), nb - 1);
    const int base = v * nb;
    // Fan beam: every ray of the view passes through the source S = sod (c, s), so the
    // parameters are measured from S (a plane x = X at (X - Sx) / ex) and the differences
    // X - S are computed once per view; parallel beam: from each ray's own origin.
    R sx = R(0), sy = R(0);
    if (FAN) {
      const double2 cv = views[v];
      sx = R(g.sod * cv.x);
      sy = R(g.sod * cv.y);
    }
    const R dx0 = X0 - sx, dx1 = X1 - sx, dx2 = X2 - sx, dy0 = Y0 - sy, dy1 = Y1 - sy, dy2 = Y2 - sy;
    for (int bb = blo; bb <= bhi; ++bb) {
      const typename V4<R>::t a = A[base + bb];
      const R yv = R(y[base + bb]);
      // origin offset: 0 for the fan beam (parameters from S), the ray's origin otherwise
      const R ox = FAN ? R(0) : a.x, oy = FAN ? R(0) : a.y;
      const R tx0 = (dx0 - ox) * a.z, tx2 = (dx2 - ox) * a.z;
      const R ty0 = (dy0 - oy) * a.w, ty2 = (dy2 - oy) * a.w;
      if (!quad) {
        const R lo = fmax(fmin(tx0, tx2), fmin(ty0, ty2));
        const R hi = fmin(fmax(tx0, tx2), fmax(ty0, ty2));
        const R ch = hi - lo;
        r.acc += ch > tq ? yv * ch : R(0);
      } else {
        // Box interval [lo, hi] and the mid-line crossings clamped into it: along x the ray is
        // in the left half on one side of cx (before cx when it moves towards +x), so the
        // quadrant combinations (+ on the lower half) are lengths between the crossings:
        // x: s_x (2 cx - lo - hi), y: s_y (2 cy - lo - hi), xy: s_x s_y (hi - lo - 2 |cx - cy|),
        // with s the sign of the ray's direction along the axis.
        const R tx1 = (dx1 - ox) * a.z, ty1 = (dy1 - oy) * a.w;
        const R lo = fmax(fmin(tx0, tx2), fmin(ty0, ty2));
        const R hi = fmin(fmax(tx0, tx2), fmax(ty0, ty2));
        const R pb = hi - lo;
        // a ray that misses the box adds nothing (its values below stay finite, times 0)
        const R yq = pb > tq ? yv : R(0);
        const R cx = fmin(fmax(tx1, lo), hi), cy = fmin(fmax(ty1, lo), hi);
        const R lh = lo + hi;
        const R p1 = xsign(R(2) * cx - lh, a.z), p2 = xsign(R(2) * cy - lh, a.w);
        const R p3 = xsign(pb - R(2) * fabs(cx - cy), xsign(a.z, a.w));
        const R w1 = fabs(p1) > tq ? yq * p1 : R(0), w2 = fabs(p2) > tq ? yq * p2 : R(0);
        const R w3 = fabs(p3) > tq ? yq * p3 : R(0);
        r.acc += yq * pb;
        r.s0 += w1; r.a0 += fabs(w1);
        r.s1 += w2; r.a1 += fabs(w2);
        r.s2 += w3; r.a2 += fabs(w3);
      }
    }
  }
  return r;
}

template <typename T, typename R>
__device__ inline ItemSums<R> item_sums(const DevGeom& g, const float2* __restrict__ vf,
                                        const double2* __restrict__ views, const typename V4<R>::t* __restrict__ A,
                                        const T* __restrict__ y, bool quad, int l, int i, int j, int v0, int v1) {
  if (g.kind != 0) return item_sums_k<T, R, true>(g, vf, views, A, y, quad, l, i, j, v0, v1);
  return item_sums_k<T, R, false>(g, vf, views, A, y, quad, l, i, j, v0, v1);
}

__device__ inline uint32_t item_word(const uint32_t* __restrict__ items, int it, int n) {
  return items ? items[it] : item_pack(0, 0, it / n, it % n);
}

// Roughness-penalized update of one coefficient (FP64): the root of
//   G(delta) = b - bp exp(-Z0 delta) - bm exp(Z0 delta) + lam (g + 8 delta),
// the derivative of eq. 1.8's surrogate plus lam times the separable quadratic surrogate of the
// penalty (curvature 8 bounds the penalty's Hessian). G increases (bp >= 0 >= bm, lam > 0);
// G(0) fixes the side of the root and |delta| <= |G(0)| / (8 lam). Newton steps that leave the
// current bracket are replaced by bisection; at most 100 steps, stopping when a Newton step is
// below 1e-15 of the iterate (converged), the bracket shrinks to 1e-15 of its size or G is 0.
__device__ inline double pen_G(double dl, double b, double bp, double bm, double z0, double lam, double g,
                               double* dG) {
  const double ep = bp != 0.0 ? bp * exp(-z0 * dl) : 0.0;
  const double em = bm != 0.0 ? bm * exp(z0 * dl) : 0.0;
  *dG = z0 * (ep - em) + 8.0 * lam;
  return b - ep - em + lam * (g + 8.0 * dl);
}
__device__ inline double pen_delta(double b, double bp, double bm, double z0, double lam, double g) {
  double dG;
  const double g0 = pen_G(0.0, b, bp, bm, z0, lam, g, &dG);
  if (g0 == 0.0) return 0.0;
  const double w = fabs(g0) / (8.0 * lam);
  double lo = g0 > 0.0 ? -w : 0.0, hi = g0 > 0.0 ? 0.0 : w;
  double x = 0.0, gx = g0;
  const double tol = 1e-15 * w;
  for (int it = 0; it < 100 && hi - lo > tol; ++it) {
    const double step = gx / dG;
    if (fabs(step) <= 1e-15 * fabs(x)) return x;       // Newton has converged
    double nx = x - step;                              // Newton step from x
    if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);   // outside the bracket: bisect
    x = nx;
    gx = pen_G(x, b, bp, bm, z0, lam, g, &dG);
    if (gx == 0.0) return x;
    if (gx < 0.0) lo = x; else hi = x;
  }
  return x;
}

// Final write of one item's sums (scaled by 2^-l): H^T y (plain), b-hat+/- (split), or the
// closed-form zero of eq. 1.9 applied to beta (update).
template <typename T, typename R, int MODE>
__device__ inline void item_finish(const DevGeom& g, uint32_t w, const ItemSums<R>& r, T* __restrict__ beta,
                                   const T* __restrict__ bvec, const double* __restrict__ z0p, int* held,
                                   T* __restrict__ bp_out, T* __restrict__ bm_out, T* __restrict__ out,
                                   const T* __restrict__ gpen = nullptr, double lam = 0.0) {
  const int n = g.n;
  const bool quad = (w >> 31) != 0;
  const int l = int((w >> 27) & 15u);
  const int i = int((w >> 13) & 0x1fffu);
  const int j = int(w & 0x1fffu);
  const R sc = R(1.0 / double(1 << l));
  const int m = n >> l;
  if (MODE == kPlain) {
    out[i * n + j] = T(r.acc * sc);
    return;
  }
  const bool root = (l == g.L);
  if (MODE == kSplit) {
    if (root) {
      bp_out[i * n + j] = T(r.acc * sc);
      bm_out[i * n + j] = T(0);
    }
    if (quad) {
      const R h = R(0.5) * sc;
      bp_out[i * n + m + j] = T((r.a0 + r.s0) * h);
      bm_out[i * n + m + j] = T((r.s0 - r.a0) * h);
      bp_out[(m + i) * n + j] = T((r.a1 + r.s1) * h);
      bm_out[(m + i) * n + j] = T((r.s1 - r.a1) * h);
      bp_out[(m + i) * n + m + j] = T((r.a2 + r.s2) * h);
      bm_out[(m + i) * n + m + j] = T((r.s2 - r.a2) * h);
    }
    return;
  }
  const R z0 = R(*z0p);
  if (gpen) {   // roughness penalty: root of eq. 1.9's left side plus lam (g + 8 delta)
    const double z0d = *z0p;
    if (root) {
      const int z = i * n + j;
      beta[z] = T(double(beta[z]) + pen_delta(double(bvec[z]), double(r.acc * sc), 0.0, z0d, lam, double(gpen[z])));
    }
    if (quad) {
      const int z1 = i * n + m + j, z2 = (m + i) * n + j, z3 = (m + i) * n + m + j;
      const double h = 0.5 * double(sc);
      beta[z1] = T(double(beta[z1]) + pen_delta(double(bvec[z1]), double(r.a0 + r.s0) * h, double(r.s0 - r.a0) * h,
                                                z0d, lam, double(gpen[z1])));
      beta[z2] = T(double(beta[z2]) + pen_delta(double(bvec[z2]), double(r.a1 + r.s1) * h, double(r.s1 - r.a1) * h,
                                                z0d, lam, double(gpen[z2])));
      beta[z3] = T(double(beta[z3]) + pen_delta(double(bvec[z3]), double(r.a2 + r.s2) * h, double(r.s2 - r.a2) * h,
                                                z0d, lam, double(gpen[z3])));
    }
    return;
  }
  if (root) {
    const int z = i * n + j;
    beta[z] = T(R(beta[z]) + am_delta<R>(R(bvec[z]), r.acc * sc, R(0), z0, held));
  }
  if (quad) {
    const int z1 = i * n + m + j, z2 = (m + i) * n + j, z3 = (m + i) * n + m + j;
    const R h = R(0.5) * sc;
    beta[z1] = T(R(beta[z1]) + am_delta<R>(R(bvec[z1]), (r.a0 + r.s0) * h, (r.s0 - r.a0) * h, z0, held));
    beta[z2] = T(R(beta[z2]) + am_delta<R>(R(bvec[z2]), (r.a1 + r.s1) * h, (r.s1 - r.a1) * h, z0, held));
    beta[z3] = T(R(beta[z3]) + am_delta<R>(R(bvec[z3]), (r.a2 + r.s2) * h, (r.s2 - r.a2) * h, z0, held));
  }
}

// Arguments of the gather kernels. Scan p = blockIdx.y of a stack: its rays at y + p M,
// its items, coefficients and outputs at + p n^2, Z0 at z0 + p kScal, held counter at
// held + p kInts, partial sums at part + p pstride. The segment of scan p is level index
// kseg of its counts (start = sum of the earlier levels) or, with counts null, the fixed
// range [start, start + count); `count` is the largest segment length of the stack. Views
// are those of the launch's subset (g.vs0 + g.vss k, k < g.nvs), chunks count within them.
template <typename T, typename R>
struct GatherArgs {
  DevGeom g;
  const float2* vf;
  const double2* views;
  const typename V4<R>::t* A;
  const T* y;
  const uint32_t* items;
  const int* counts;
  int kseg, start, count, chunks, vpc;
  int64_t pstride;
  R* part;
  T* beta;
  const T* b;
  const double* z0;
  int z0stride;
  int* held;
  T *bp, *bm, *out;
  const T* gpen;   // roughness-penalty gradient Omega^T grad R per coefficient (null: no penalty)
  double lam;      // penalty weight lambda
};

template <typename T, typename R>
struct ScanView {
  const T* y;
  const uint32_t* items;
  T* beta;
  const T* b;
  const double* z0;
  int* held;
  T *bp, *bm, *out;
  const T* gpen;
  R* part;
  int start, count;
};

template <typename T, typename R>
__device__ inline ScanView<T, R> scan_view(const GatherArgs<T, R>& a) {
  const int p = blockIdx.y;
  const int64_t M = int64_t(a.g.nv) * a.g.nb, NN = int64_t(a.g.n) * a.g.n;
  ScanView<T, R> v;
  v.y = a.y + p * M;
  v.items = at(a.items, p * NN);
  v.beta = at(a.beta, p * NN);
  v.b = at(a.b, p * NN);
  v.z0 = at(a.z0, int64_t(p) * a.z0stride);
  v.held = at(a.held, int64_t(p) * kInts);
  v.bp = at(a.bp, p * NN);
  v.bm = at(a.bm, p * NN);
  v.out = at(a.out, p * NN);
  v.gpen = at(a.gpen, p * NN);
  v.part = at(a.part, p * a.pstride);
  v.start = a.start;
  v.count = a.count;
  if (a.counts) {
    const int* c = a.counts + p * kInts;
    int st = 0;
    for (int k = 0; k < a.kseg; ++k) st += c[k];
    v.start = st;
    v.count = c[a.kseg];
  }
  return v;
}

// Work blocks are dealt to the chip's 8 XCDs (each with its own L2) round-robin by block
// index. A block index b is mapped to work unit w so that each XCD gets one contiguous slice
// of the units, n_pad / 8 of them (n_pad = units rounded up to a multiple of 8; w >= units:
// an idle block): units close in the list (the same views, neighbouring items) then share
// one L2 instead of being fetched by all eight.
constexpr int kXcds = 8;
__device__ inline int xcd_unit(int b, int n_pad) { return (b % kXcds) * (n_pad / kXcds) + b / kXcds; }
inline int xcd_pad(int units) { return (units + kXcds - 1) / kXcds * kXcds; }

// One lane per item of a level segment, all views (used when the segment alone fills the GPU).
template <typename T, typename R, int MODE>
__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs<T, R> a) {
  const ScanView<T, R> v = scan_view(a);
  const int blk = xcd_unit(blockIdx.x, gridDim.x);
  const int k = blk * kBlock + threadIdx.x;
  if (k >= v.count) return;
  const uint32_t w = item_word(v.items, v.start + k, a.g.n);
  const ItemSums<R> r = item_sums<T, R>(a.g, a.vf, a.views, a.A, v.y, (w >> 31) != 0, int((w >> 27) & 15u),
                                        int((w >> 13) & 0x1fffu), int(w & 0x1fffu), 0, a.g.nvs);
  item_finish<T, R, MODE>(a.g, w, r, v.beta, v.b, v.z0, v.held, v.bp, v.bm, v.out, v.gpen, a.lam);
}

// (item, view chunk) tasks of the level segments whose items alone would leave the GPU idle,
// all chunked segments of a gather in one launch. A block of kChunkWaves waves takes 64
// consecutive (spatially adjacent) items of one segment; wave w handles view chunk
// kChunkWaves * group + w for all of them (uniform view range per wave). The chunk sums are
// added in LDS in wave order (deterministic) and written to the segment's
// part[group][slot][count] (count = the stack's largest segment length).
constexpr int kChunkWaves = 4;
constexpr int kMaxSegs = kMaxGatherSegs;

// The chunked segments of one launch, coarse levels first. Each segment owns a range of
// part-kernel blocks starting at a multiple of the XCD count (so a segment's blocks are
// dealt to the XCDs as in a launch of its own) and a range of finish blocks (64 items each).
struct SegTable {
  int n;
  int kseg[kMaxSegs], start[kMaxSegs], count[kMaxSegs], chunks[kMaxSegs], vpc[kMaxSegs];
  int64_t part_off[kMaxSegs];   // the segment's partial sums within a scan's block of part
  int blk0[kMaxSegs + 1];       // first part-kernel block; blk0[n] = blocks of the launch
  int fin0[kMaxSegs + 1];       // first finish block; fin0[n] = blocks of the launch
};

__device__ inline int seg_of(const int* first, int n, int b) {
  int k = 0;
  while (k + 1 < n && first[k + 1] <= b) ++k;
  return k;
}

template <typename T, typename R>
__device__ inline void select_segment(GatherArgs<T, R>& a, const SegTable& t, int k) {
  a.kseg = t.kseg[k];
  a.start = t.start[k];
  a.count = t.count[k];
  a.chunks = t.chunks[k];
  a.vpc = t.vpc[k];
  a.part = at(a.part, t.part_off[k]);
}

template <typename T, typename R>
__global__ __launch_bounds__(64 * kChunkWaves) void k_gather_part(GatherArgs<T, R> a, SegTable t) {
  __shared__ R sh[kChunkWaves][7][64];
  const int sg = seg_of(t.blk0, t.n, blockIdx.x);
  select_segment(a, t, sg);
  const ScanView<T, R> v = scan_view(a);
  const int n_item_groups = (a.count + 63) / 64;
  const int groups = (a.chunks + kChunkWaves - 1) / kChunkWaves;
  const int unit = xcd_unit(blockIdx.x - t.blk0[sg], t.blk0[sg + 1] - t.blk0[sg]);   // group * n_item_groups + ig
  if (unit >= groups * n_item_groups) return;
  const int ig = unit % n_item_groups, group = unit / n_item_groups;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int idx = ig * 64 + lane;
  const int chunk = group * kChunkWaves + wv;
  ItemSums<R> r{R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
  if (idx < v.count && chunk < a.chunks) {
    const uint32_t w = item_word(v.items, v.start + idx, a.g.n);
    const int v0 = chunk * a.vpc, v1 = min(a.g.nvs, v0 + a.vpc);
    r = item_sums<T, R>(a.g, a.vf, a.views, a.A, v.y, (w >> 31) != 0, int((w >> 27) & 15u), int((w >> 13) & 0x1fffu),
                        int(w & 0x1fffu), v0, v1);
  }
  sh[wv][0][lane] = r.acc;
  sh[wv][1][lane] = r.s0; sh[wv][2][lane] = r.s1; sh[wv][3][lane] = r.s2;
  sh[wv][4][lane] = r.a0; sh[wv][5][lane] = r.a1; sh[wv][6][lane] = r.a2;
  __syncthreads();
  for (int k = threadIdx.x; k < 7 * 64; k += 64 * kChunkWaves) {
    const int slot = k / 64, l2 = k % 64;
    const int it = ig * 64 + l2;
    if (it >= v.count) continue;
    R s = R(0);
#pragma unroll
    for (int w2 = 0; w2 < kChunkWaves; ++w2) s += sh[w2][slot][l2];
    v.part[(size_t(group) * 7 + slot) * a.count + it] = s;
  }
}

// Sum the chunk groups of each item in group order (deterministic): 7 waves of a block each
// add one slot for 64 consecutive items of one segment (coalesced), then one wave finishes
// the items. Every chunked segment of the gather in one launch.
template <typename T, typename R, int MODE>
__global__ __launch_bounds__(512) void k_gather_finish(GatherArgs<T, R> a, SegTable t) {
  __shared__ R sh[7][64];
  const int sg = seg_of(t.fin0, t.n, blockIdx.x);
  select_segment(a, t, sg);
  const ScanView<T, R> v = scan_view(a);
  const int lane = threadIdx.x & 63, slot = threadIdx.x >> 6;
  const int idx = (blockIdx.x - t.fin0[sg]) * 64 + lane;
  const int groups = (a.chunks + kChunkWaves - 1) / kChunkWaves;
  if (slot < 7) {
    sh[slot][lane] = idx < v.count ? ordered_sum(v.part + size_t(slot) * a.count + idx, groups, size_t(7) * a.count)
                                   : R(0);
  }
  __syncthreads();
  if (slot != 0 || idx >= v.count) return;
  const uint32_t w = item_word(v.items, v.start + idx, a.g.n);
  ItemSums<R> r{sh[0][lane], sh[1][lane], sh[2][lane], sh[3][lane], sh[4][lane], sh[5][lane], sh[6][lane]};
  item_finish<T, R, MODE>(a.g, w, r, v.beta, v.b, v.z0, v.held, v.bp, v.bm, v.out, v.gpen, a.lam);
}

// ------------------------------------------------------------------ Haar analysis

// coef(z) = sum over the support of basis function z of its value times img (Omega^T img),
// FP64 accumulation; Mallat position -> (level, band, node).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_analysis(int n, int L, const T* __restrict__ img, T* __restrict__ coef) {
  const int z = blockIdx.x * kBlock + threadIdx.x;
  if (z >= n * n) return;
  const int r = z / n, c = z % n;
  const int k = max(r, c);
  int l = 0;
  for (int t = 1; t <= L; ++t) {
    if (k >= (n >> t)) { l = t; break; }
  }
  double acc = 0.0;
  if (l == 0) {  // approximation of root (r, c)
    const int s = 1 << L;
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) acc += double(img[(r * s + a) * n + c * s + b]);
    acc *= 1.0 / double(s);
  } else {
    const int m = n >> l, s = 1 << l, h = s >> 1;
    const int band = (r < m) ? 1 : (c < m ? 2 : 3);
    const int i = r % m, j = c % m;
    for (int a = 0; a < s; ++a) {
      for (int b = 0; b < s; ++b) {
        const bool right = b >= h, bottom = a >= h;
        const bool neg = band == 1 ? right : (band == 2 ? bottom : (right != bottom));
        const double v = double(img[(i * s + a) * n + j * s + b]);
        acc += neg ? -v : v;
      }
    }
    acc *= 1.0 / double(s);
  }
  coef[z] = T(acc);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_apply_mask(int64_t len, T* __restrict__ beta,
                                                       const uint8_t* __restrict__ mask) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p < len && mask[p] == 0) beta[p] = T(0);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_check(const T* __restrict__ x, int64_t len, bool allow_neg,
                                                  int* __restrict__ bad) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= len) return;
  const T v = x[p];
  if (!isfinite(v) || (!allow_neg && v < T(0))) atomicAdd(bad, 1);
}

// r = g (d - q): the residual backprojected by the adjoint of the coefficient-domain loss
template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual(int64_t len, const T* __restrict__ d, const T* __restrict__ q,
                                                     const double* __restrict__ gscale, T* __restrict__ r) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= len) return;
  const double gs = gscale ? *gscale : 1.0;
  r[p] = T(gs * (double(d[p]) - double(q[p])));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* __restrict__ x, int64_t len, T v) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p < len) x[p] = v;
}

// ------------------------------------------------------------------ Z0 and W (eq. 1.61)

// Per ray in FP64: walk the leaves; every leaf chord adds s_k(quadrant) * chord to the
// three detail accumulators of each split ancestor (levels above the leaf), and chord to
// the approximation accumulator of its root. When the ray leaves a node (a bit at or above
// the node's level differs between the pixels of consecutive leaves), its |phi| =
// 2^-m |acc_k| are added to the ray's sum and the non-zero ones counted. Z0 is the maximum
// of the sums over rays; W the total count.
__device__ inline double flip_sign(double v, int neg) {
  return __longlong_as_double(__double_as_longlong(v) ^ (static_cast<long long>(neg) << 63));
}

template <int LT>
struct Z0Visitor {
  double tolm[LT + 1];    // count threshold per level, unscaled (index 0: root approximations)
  double sc[LT + 1];      // 2^-m per level (index 0: 2^-LT, the roots)
  double acc[LT + 1][3];
  double accLL;
  double sum;
  int cnt;
  int dirty;              // bit m: acc[m] holds chords of the current level-m node
  int px, py;             // pixel of the previous leaf (all bits set before the first)
  __device__ inline void flush_level(int m) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double a = fabs(acc[m][k]);
      sum = fma(a, sc[m], sum);
      cnt += (a > tolm[m]) ? 1 : 0;
      acc[m][k] = 0.0;
    }
  }
  __device__ inline void flush_ll() {
    sum = fma(accLL, sc[0], sum);
    cnt += (accLL > tolm[0]) ? 1 : 0;
    accLL = 0.0;
  }
  __device__ inline void operator()(int ix, int iy, int l, double chord) {
    const int dif = (ix ^ px) | (iy ^ py);
    px = ix; py = iy;
#pragma unroll
    for (int m = 1; m <= LT; ++m) {
      // a new node at level m: its sums enter the total (untouched sums are zero: nothing to add)
      if ((dif >> m) && (dirty >> m & 1)) {
        flush_level(m);
        dirty &= ~(1 << m);
      }
      if (m > l) {
        dirty |= 1 << m;
        const int right = (ix >> (m - 1)) & 1, bottom = (iy >> (m - 1)) & 1;
        const double cr = flip_sign(chord, right);
        acc[m][0] += cr;
        acc[m][1] += flip_sign(chord, bottom);
        acc[m][2] += flip_sign(cr, bottom);
      }
    }
    if (dif >> LT) flush_ll();
    accLL += chord;
  }
};

// The level count is a template parameter so the per-level accumulators stay in registers.
template <int LT>
__global__ __launch_bounds__(kBlock) void k_z0(DevGeom g, const double2* __restrict__ views,
                                               const uint8_t* __restrict__ lev, double* __restrict__ part_max,
                                               double* __restrict__ part_cnt) {
  lev += int64_t(blockIdx.y) * g.n * g.n;
  const int rb = xcd_rotate(blockIdx.x);
  const int k = rb * kBlock + threadIdx.x;
  double sum = 0.0, cnt = 0.0;
  if (k < g.nvs * g.nb) {
    const int r = subset_ray(g, k);
    const int v = r / g.nb, b = r - v * g.nb;
    double ox, oy, ex, ey;
    ray_of(g, views[v], b, ox, oy, ex, ey);
    Z0Visitor<LT> z;
    const double tol = 1e-9 * g.pixel;
    z.sc[0] = 1.0 / double(1 << LT);
    z.tolm[0] = tol * double(1 << LT);
#pragma unroll
    for (int m = 1; m <= LT; ++m) {
      z.sc[m] = 1.0 / double(1 << m);
      z.tolm[m] = tol * double(1 << m);
      z.acc[m][0] = z.acc[m][1] = z.acc[m][2] = 0.0;
    }
    z.accLL = 0.0; z.sum = 0.0; z.cnt = 0; z.dirty = 0; z.px = z.py = -1;
    walk<double, (LT > 0)>(g, ox, oy, ex, ey, 1.0 / ex, 1.0 / ey, lev, z);
#pragma unroll
    for (int m = 1; m <= LT; ++m) z.flush_level(m);
    z.flush_ll();
    sum = z.sum;
    cnt = double(z.cnt);
  }
  const double mx = block_reduce<true>(sum);
  __syncthreads();
  const double ct = block_reduce<false>(cnt);
  if (threadIdx.x == 0) {
    const int o = blockIdx.y * gridDim.x + rb;
    part_max[o] = mx;
    part_cnt[o] = ct;
  }
}

// ------------------------------------------------------------------ tree rule (Results)

// Leaf scores of the residual-gradient rule: for every leaf node (a node at level >= 1 not
// split whose parent is split, or a root) the largest |c| of its three would-be details, c =
// Omega^T H^T (d - q-hat) (the gradient of the I-divergence with respect to the detail
// coefficients), stored at the node's first detail position [i][m + j]; other positions
// keep their value (the caller fills zeros). Per scan: blockIdx.y.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_grad_scores(DevGeom g, const uint8_t* __restrict__ mask,
                                                        const T* __restrict__ coef, double* __restrict__ score) {
  const int n = g.n;
  {
    const int64_t off = int64_t(blockIdx.y) * n * n;
    mask += off; coef += off; score += off;
  }
  int k = blockIdx.x * kBlock + threadIdx.x;
  int l = 1;
  for (; l <= g.L; ++l) {
    const int m = n >> l;
    if (k < m * m) break;
    k -= m * m;
  }
  if (l > g.L) return;
  const int m = n >> l, i = k / m, j = k % m;
  if (is_split(mask, n, l, i, j)) return;
  if (l < g.L && !is_split(mask, n, l + 1, i >> 1, j >> 1)) return;
  const double c1 = fabs(double(coef[i * n + m + j])), c2 = fabs(double(coef[(m + i) * n + j]));
  const double c3 = fabs(double(coef[(m + i) * n + m + j]));
  score[i * n + m + j] = fmax(c1, fmax(c2, c3));
}

// Gradient of the roughness penalty R(mu) = 1/2 sum over 4-neighbour pixel pairs (mu_x -
// mu_x')^2: out_x = sum over the neighbours x' of x of (mu_x - mu_x'), from the FP64 image
// (per scan: blockIdx.y).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rough_grad(int n, const double* __restrict__ mu, T* __restrict__ out) {
  const int64_t off = int64_t(blockIdx.y) * n * n;
  mu += off;
  out += off;
  const int x = blockIdx.x * kBlock + threadIdx.x;
  if (x >= n * n) return;
  const int i = x / n, j = x - i * n;
  const double c = mu[x];
  double gsum = 0.0;
  if (j > 0) gsum += c - mu[x - 1];
  if (j < n - 1) gsum += c - mu[x + 1];
  if (i > 0) gsum += c - mu[x - n];
  if (i < n - 1) gsum += c - mu[x + n];
  out[x] = T(gsum);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual_inplace(int64_t len, const T* __restrict__ d, T* __restrict__ q) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k < len) q[k] = T(double(d[k]) - double(q[k]));
}

// Tree rule: rule 0 (Results) splits leaves whose leaf-constant value mu64 exceeds frac x max;
// rule 1 (residual gradient) splits leaves whose score (k_grad_scores, in `val`) exceeds
// frac x max score; rule 2 (the Results rule for bases that are not constant on the leaves)
// splits leaves with any pixel of mu64 above frac x max.
__global__ __launch_bounds__(kBlock) void k_expand(DevGeom g, const uint8_t* __restrict__ old,
                                                   uint8_t* __restrict__ mask, const double* __restrict__ mu64,
                                                   const double* __restrict__ maxv, double frac,
                                                   int* __restrict__ n_split, int rule) {
  const int n = g.n;
  {
    const int p = blockIdx.y;
    const int64_t off = int64_t(p) * n * n;
    old += off; mask += off; mu64 += off;
    maxv += p * kScal;
    n_split += p * kInts;
  }
  // flattened node index over levels 1..L
  int k = blockIdx.x * kBlock + threadIdx.x;
  int l = 1;
  for (; l <= g.L; ++l) {
    const int m = n >> l;
    if (k < m * m) break;
    k -= m * m;
  }
  if (l > g.L) return;
  const double top = *maxv;
  if (!(top > 0.0)) return;
  const int m = n >> l, i = k / m, j = k % m;
  if (is_split(old, n, l, i, j)) return;
  if (l < g.L && !is_split(old, n, l + 1, i >> 1, j >> 1)) return;
  const int s = 1 << l;
  // rule 0: leaf-constant value (any pixel of the block); rule 1: the node's score; rule 2:
  // the block's largest pixel
  double val;
  if (rule == 1) {
    val = mu64[i * n + m + j];
  } else if (rule == 2) {
    val = -INFINITY;
    for (int r = i * s; r < (i + 1) * s; ++r)
      for (int c = j * s; c < (j + 1) * s; ++c) val = fmax(val, mu64[int64_t(r) * n + c]);
  } else {
    val = mu64[(i * s) * n + j * s];
  }
  if (val > frac * top) {
    mask[i * n + m + j] = 1;
    mask[(m + i) * n + j] = 1;
    mask[(m + i) * n + m + j] = 1;
    atomicAdd(n_split, 1);
  }
}

__global__ __launch_bounds__(kBlock) void k_check_mask(DevGeom g, const uint8_t* __restrict__ mask,
                                                       int* __restrict__ bad) {
  const int z = blockIdx.x * kBlock + threadIdx.x;
  const int n = g.n;
  mask += int64_t(blockIdx.y) * n * n;
  if (z >= n * n) return;
  const int r = z / n, c = z % n, L = g.L;
  const int nL = n >> L;
  if (L == 0 || (r < nL && c < nL)) {
    if (mask[z] != 1) atomicAdd(bad, 1);
    return;
  }
  if (mask[z] > 1) { atomicAdd(bad, 1); return; }
  const int k = max(r, c);
  int l = 1;
  for (; l <= L; ++l)
    if (k >= (n >> l)) break;
  const int m = n >> l, i = r % m, j = c % m;
  const uint8_t f = mask[i * n + m + j];
  if (mask[z] != f) { atomicAdd(bad, 1); return; }
  if (f && l < L && !is_split(mask, n, l + 1, i >> 1, j >> 1)) atomicAdd(bad, 1);
}

__global__ void k_approx_mask(int n, int L, uint8_t* __restrict__ mask) {
  mask += int64_t(blockIdx.y) * n * n;
  const int z = blockIdx.x * kBlock + threadIdx.x;
  if (z >= n * n) return;
  const int nL = n >> L;
  mask[z] = (L == 0 || ((z / n) < nL && (z % n) < nL)) ? 1 : 0;
}

__global__ void k_fill_u8(uint8_t* x, int64_t len, uint8_t v) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p < len) x[p] = v;
}
__global__ void k_fill_i32(int* x, int64_t len, int v) {
  const int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (p < len) x[p] = v;
}
__global__ void k_fill_i32_strided(int* x, int count, int stride, int v) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < count) x[int64_t(k) * stride] = v;
}

}  // namespace

// ------------------------------------------------------------------ launchers

template <typename T>
void Launch<T>::synth(const DevGeom& g, const T* beta, T* mu, int S, hipStream_t s) {
  hipLaunchKernelGGL(k_synth<T>, dim3(blocks_for(int64_t(g.n) * g.n), S), dim3(kBlock), 0, s, g.n, g.L, beta, mu);
}
template <typename T>
void Launch<T>::levmap(const DevGeom& g, const uint8_t* mask, uint8_t* lev, int S, hipStream_t s) {
  hipLaunchKernelGGL(k_levmap, dim3(blocks_for(int64_t(g.n) * g.n), S), dim3(kBlock), 0, s, g.n, g.L, mask, lev);
}
template <typename T>
void Launch<T>::synth_layouts(const DevGeom& g, const T* beta, T* muR, T* muC, int S, hipStream_t s) {
  const dim3 grid((g.n + 31) / 32, (g.n + 31) / 32, S);
  hipLaunchKernelGGL((k_synth_tiles<T, false>), grid, dim3(256), 0, s, g.n, g.L, beta, nullptr, muR, muC,
                     (Leaf<T>*)nullptr, (Leaf<T>*)nullptr);
}
template <typename T>
void Launch<T>::synth_records(const DevGeom& g, const T* beta, const uint8_t* lev, void* leafR, void* leafC, int S,
                              hipStream_t s) {
  const dim3 grid((g.n + 31) / 32, (g.n + 31) / 32, S);
  hipLaunchKernelGGL((k_synth_tiles<T, true>), grid, dim3(256), 0, s, g.n, g.L, beta, lev, (T*)nullptr, (T*)nullptr,
                     (Leaf<T>*)leafR, (Leaf<T>*)leafC);
}
template <typename T>
void Launch<T>::transpose(int n, const T* in, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose<T>, dim3((n + 31) / 32, (n + 31) / 32), dim3(256), 0, s, n, in, out);
}
template <typename T>
int Launch<T>::idiv_terms(const DevGeom& g, const T* q, const T* d, double* part, int S, hipStream_t s) {
  const int M = g.nv * g.nb, nb = blocks_for(M);
  hipLaunchKernelGGL(k_idiv_terms<T>, dim3(nb, S), dim3(kBlock), 0, s, M, q, d, part);
  return nb;
}
template <typename T>
void Launch<T>::analysis(const DevGeom& g, const T* img, T* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_analysis<T>, dim3(blocks_for(int64_t(g.n) * g.n)), dim3(kBlock), 0, s, g.n, g.L, img, coef);
}
template <typename T>
int Launch<T>::mu64(const DevGeom& g, const T* beta, double* mu64, double* part, int S, hipStream_t s) {
  const int nb = blocks_for(int64_t(g.n) * g.n);
  hipLaunchKernelGGL(k_mu64<T>, dim3(nb, S), dim3(kBlock), 0, s, g.n, g.L, beta, mu64, part);
  return nb;
}
int sum_slices(const DevGeom& g, double* mu64, double* part, int S, hipStream_t s) {
  const int64_t nn = int64_t(g.n) * g.n;
  const int nb = blocks_for(nn);
  hipLaunchKernelGGL(k_sum_slices, dim3(nb), dim3(kBlock), 0, s, nn, S, mu64, part);
  return nb;
}
template <typename T>
void Launch<T>::apply_mask(const DevGeom& g, T* beta, const uint8_t* mask, int S, hipStream_t s) {
  const int64_t len = int64_t(g.n) * g.n * S;
  hipLaunchKernelGGL(k_apply_mask<T>, dim3(blocks_for(len)), dim3(kBlock), 0, s, len, beta, mask);
}
template <typename T>
void Launch<T>::check(const T* x, int64_t len, bool allow_negative, int* bad, hipStream_t s) {
  if (len <= 0) return;
  hipLaunchKernelGGL(k_check<T>, dim3(blocks_for(len)), dim3(kBlock), 0, s, x, len, allow_negative, bad);
}
template <typename T>
void Launch<T>::residual(const T* d, const T* q, const double* gscale, T* r, int64_t len, hipStream_t s) {
  if (len > 0) hipLaunchKernelGGL(k_residual<T>, dim3(blocks_for(len)), dim3(kBlock), 0, s, len, d, q, gscale, r);
}
template <typename T>
void Launch<T>::fill(T* x, int64_t len, T v, hipStream_t s) {
  if (len <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(len)), dim3(kBlock), 0, s, x, len, v);
}

template <typename T>
void Launch<T>::grad_scores(const DevGeom& g, const uint8_t* mask, const T* coef, double* score, int S,
                            hipStream_t s) {
  int64_t nodes = 0;
  for (int l = 1; l <= g.L; ++l) nodes += int64_t(g.n >> l) * (g.n >> l);
  if (nodes == 0) return;
  hipLaunchKernelGGL(k_grad_scores<T>, dim3(blocks_for(nodes), S), dim3(kBlock), 0, s, g, mask, coef, score);
}
template <typename T>
void Launch<T>::residual_inplace(const T* d, T* q, int64_t len, hipStream_t s) {
  if (len > 0) hipLaunchKernelGGL(k_residual_inplace<T>, dim3(blocks_for(len)), dim3(kBlock), 0, s, len, d, q);
}
template <typename T>
void Launch<T>::rough_grad(const DevGeom& g, const double* mu64, T* out, int S, hipStream_t s) {
  hipLaunchKernelGGL(k_rough_grad<T>, dim3(blocks_for(int64_t(g.n) * g.n), S), dim3(kBlock), 0, s, g.n, mu64, out);
}
template struct Launch<float>;
template struct Launch<double>;

template <typename T, typename R>
void Geo<T, R>::ray_table(const DevGeom& g, const double2* views, void* A, void* B, hipStream_t s) {
  const int M = g.nv * g.nb;
  hipLaunchKernelGGL(k_ray_table<R>, dim3(blocks_for(M)), dim3(kBlock), 0, s, g, views,
                     (typename V4<R>::t*)A, (typename V4<R>::t*)B);
}
template <typename T, typename R>
void Geo<T, R>::view_table(const DevGeom& g, const double2* views, void* vF, hipStream_t s) {
  hipLaunchKernelGGL(k_view_table<float>, dim3(blocks_for(g.nv)), dim3(kBlock), 0, s, g.nv, views, (float2*)vF);
}
template <typename T, typename R>
int Geo<T, R>::forward(const DevGeom& g, const void* A, const void* B, const T* muR, const T* muC, const T* d,
                       const T* i0v, const double* i0s, T* q, T* p, double* part, int S, hipStream_t s) {
  // lanes per ray as for the leaf walk (the launch's ray count over all scans)
  const int k = leaf_pieces(int64_t(g.nvs) * g.nb * S);
  const int nb = xcd_blocks(blocks_for(int64_t(g.nvs) * g.nb * k));
  auto a = (const typename V4<R>::t*)A;
  auto b = (const typename V4<R>::t*)B;
  if (k == 1)
    hipLaunchKernelGGL((k_forward<T, R, 8, 1>), dim3(nb, S), dim3(kBlock), 0, s, g, a, b, muR, muC, d, i0v, i0s, q, p, part);
  else if (k == 2)
    hipLaunchKernelGGL((k_forward<T, R, 8, 2>), dim3(nb, S), dim3(kBlock), 0, s, g, a, b, muR, muC, d, i0v, i0s, q, p, part);
  else
    hipLaunchKernelGGL((k_forward<T, R, 8, 4>), dim3(nb, S), dim3(kBlock), 0, s, g, a, b, muR, muC, d, i0v, i0s, q, p, part);
  return nb;
}
// rays per lane group: a launch with fewer than 2^21 rays splits each ray over 2 lanes, one
// with fewer than 2^17 over 4 (the GPU holds 2^19 lanes at 8 waves per SIMD; two half-length
// walks per ray also hide more of the record-load latency, measured faster for the 737K rays
// of a 720 x 1024 scan)
int leaf_pieces(int64_t rays) { return rays >= (int64_t(1) << 21) ? 1 : (rays >= (int64_t(1) << 17) ? 2 : 4); }

template <typename T, typename R>
int Geo<T, R>::forward_records(const DevGeom& g, const void* A, const void* B, const void* leafR, const void* leafC,
                               const T* d, const T* i0v, const double* i0s, T* q, T* p, double* part, int S,
                               hipStream_t s, int lanes) {
  const int64_t rays = int64_t(g.nvs) * g.nb * S;
  const int k = lanes > 0 ? lanes : leaf_pieces(rays);
  const int nb = xcd_blocks(blocks_for(int64_t(g.nvs) * g.nb * k));
  auto a = (const typename V4<R>::t*)A;
  auto b = (const typename V4<R>::t*)B;
  auto lr = (const Leaf<T>*)leafR;
  auto lc = (const Leaf<T>*)leafC;
  if (k == 1)
    hipLaunchKernelGGL((k_forward_rec<T, R, 1>), dim3(nb, S), dim3(kBlock), 0, s, g, a, b, lr, lc, d, i0v, i0s, q, p, part);
  else if (k == 2)
    hipLaunchKernelGGL((k_forward_rec<T, R, 2>), dim3(nb, S), dim3(kBlock), 0, s, g, a, b, lr, lc, d, i0v, i0s, q, p, part);
  else
    hipLaunchKernelGGL((k_forward_rec<T, R, 4>), dim3(nb, S), dim3(kBlock), 0, s, g, a, b, lr, lc, d, i0v, i0s, q, p, part);
  return nb;
}

namespace {
// Segments that fill the GPU with one lane per item run k_gather, one launch each; the
// chunked ones share one part launch and one finish launch.
template <typename T, typename R, int MODE>
void launch_segments(GatherArgs<T, R> a, const Segment* segs, int n_segs, int S, hipStream_t s) {
  SegTable t{};
  int64_t off = 0;
  for (int k = 0; k < n_segs; ++k) {
    const Segment& sg = segs[k];
    if (sg.count <= 0) continue;
    if (sg.chunks <= 1) {
      a.kseg = sg.kseg;
      a.start = sg.start;
      a.count = sg.count;
      a.chunks = sg.chunks;
      a.vpc = sg.vpc;
      hipLaunchKernelGGL((k_gather<T, R, MODE>), dim3(xcd_pad(blocks_for(a.count)), S), dim3(kBlock), 0, s, a);
      continue;
    }
    const int i = t.n++;
    const int groups = (sg.chunks + kChunkWaves - 1) / kChunkWaves;
    t.kseg[i] = sg.kseg;
    t.start[i] = sg.start;
    t.count[i] = sg.count;
    t.chunks[i] = sg.chunks;
    t.vpc[i] = sg.vpc;
    t.part_off[i] = off;
    off += segment_part_elems(sg, 1);
    t.blk0[i + 1] = t.blk0[i] + xcd_pad(((sg.count + 63) / 64) * groups);
    t.fin0[i + 1] = t.fin0[i] + (sg.count + 63) / 64;
  }
  if (t.n == 0) return;
  a.pstride = off;
  hipLaunchKernelGGL((k_gather_part<T, R>), dim3(t.blk0[t.n], S), dim3(64 * kChunkWaves), 0, s, a, t);
  hipLaunchKernelGGL((k_gather_finish<T, R, MODE>), dim3(t.fin0[t.n], S), dim3(512), 0, s, a, t);
}
}  // namespace

template <typename T, typename R>
void Geo<T, R>::gather(const DevGeom& g, int mode, const void* vF, const double2* views, const void* A, const T* y,
                       const uint32_t* items, const int* counts, const Segment* segs, int n_segs, void* part,
                       T* beta, const T* b, const double* z0, int z0stride, int* held, T* bp, T* bm, T* out,
                       int S, hipStream_t s, const T* gpen, double lam) {
  GatherArgs<T, R> a;
  a.gpen = gpen;
  a.lam = lam;
  a.g = g;
  a.vf = (const float2*)vF;
  a.views = views;
  a.A = (const typename V4<R>::t*)A;
  a.y = y;
  a.items = items;
  a.counts = counts;
  a.part = (R*)part;
  a.beta = beta;
  a.b = b;
  a.z0 = z0;
  a.z0stride = z0stride;
  a.held = held;
  a.bp = bp;
  a.bm = bm;
  a.out = out;
  if (n_segs > kMaxSegs) return;   // refused by the host
  if (mode == kPlain) launch_segments<T, R, kPlain>(a, segs, n_segs, S, s);
  else if (mode == kSplit) launch_segments<T, R, kSplit>(a, segs, n_segs, S, s);
  else launch_segments<T, R, kUpdate>(a, segs, n_segs, S, s);
}

template struct Geo<float, float>;
template struct Geo<float, double>;
template struct Geo<double, double>;

int z0_partials(const DevGeom& g, const double2* views, const uint8_t* lev, double* part_max,
                double* part_cnt, int S, hipStream_t s) {
  const int nb = xcd_blocks(blocks_for(int64_t(g.nvs) * g.nb));
  switch (g.L) {
#define Z0_CASE(K) \
    case K: hipLaunchKernelGGL(k_z0<K>, dim3(nb, S), dim3(kBlock), 0, s, g, views, lev, part_max, part_cnt); break;
    Z0_CASE(0) Z0_CASE(1) Z0_CASE(2) Z0_CASE(3) Z0_CASE(4) Z0_CASE(5) Z0_CASE(6) Z0_CASE(7) Z0_CASE(8)
#undef Z0_CASE
  }
  return nb;
}
int idiv_blocks(int64_t rays) { return blocks_for(rays); }
void reduce_sum(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce<false>, dim3(1), dim3(kBlock), 0, s, part, n, int64_t(0), out, int64_t(0),
                     (int*)nullptr);
}
void reduce_max(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce<true>, dim3(1), dim3(kBlock), 0, s, part, n, int64_t(0), out, int64_t(0),
                     (int*)nullptr);
}
void reduce_stack(bool max, const double* part, int n, int64_t pstride, double* out, int64_t ostride, int* ctr,
                  int S, hipStream_t s) {
  if (max)
    hipLaunchKernelGGL(k_reduce<true>, dim3(S), dim3(kBlock), 0, s, part, n, pstride, out, ostride, ctr);
  else
    hipLaunchKernelGGL(k_reduce<false>, dim3(S), dim3(kBlock), 0, s, part, n, pstride, out, ostride, ctr);
}
namespace {
// Node of Morton code `code` on level l of scan `scan`: kept by the filter of its pass.
struct ListSpec2 {
  const uint8_t* mask;
  int n;
  __device__ bool keep(int scan, int l, int filter, int64_t code, uint32_t& word) const {
    const int j = int(morton_compact(uint32_t(code))), i = int(morton_compact(uint32_t(code >> 1)));
    const int m = n >> l;
    if (i >= m || j >= m) return false;
    const bool sp = l > 0 && is_split(mask + int64_t(scan) * n * n, n, l, i, j);
    word = item_pack(sp ? 1 : 0, l, i, j);
    return filter == 2 || (filter == 0) == sp;
  }
};

// Levels coarse to fine; the roots' level lists its split roots first, then the others
// (waves of one kind). Count slot 1 + (L - l) per level; every pixel when L = 0.
PassTable list_passes(const DevGeom& g) {
  PassTable pt{};
  const int L = g.L;
  for (int l = L; l >= (L == 0 ? 0 : 1); --l) {
    const int m = g.n >> l;
    int pw = 1;
    while (pw < m) pw <<= 1;
    const int64_t codes = int64_t(pw) * pw;
    if (L == 0) {
      add_pass(pt, 0, 2, 1, codes);
    } else if (l == L) {
      add_pass(pt, l, 0, 1, codes);
      add_pass(pt, l, 1, 1, codes);
    } else {
      add_pass(pt, l, 0, 1 + (L - l), codes);
    }
  }
  return pt;
}
}  // namespace

int64_t list_scratch_ints(const DevGeom& g, int S) {
  const PassTable pt = list_passes(g);
  return 2 * int64_t(S) * pt.blk_start[pt.n_pass];
}
void build_items(const DevGeom& g, const uint8_t* mask, uint32_t* items, int* counts, int S, int* scratch,
                 hipStream_t s) {
  const PassTable pt = list_passes(g);
  const int nblk = pt.blk_start[pt.n_pass];
  int* bcount = scratch;
  int* boff = scratch + int64_t(S) * nblk;
  const ListSpec2 sp{mask, g.n};
  hipLaunchKernelGGL(k_list_count<ListSpec2>, dim3(nblk, S), dim3(kListThreads), 0, s, sp, pt, bcount);
  hipLaunchKernelGGL(k_list_scan, dim3(S), dim3(kListThreads), 0, s, pt, bcount, boff, counts, kInts);
  hipLaunchKernelGGL(k_list_write<ListSpec2>, dim3(nblk, S), dim3(kListThreads), 0, s, sp, pt, boff, items,
                     int64_t(g.n) * g.n);
}
void expand(const DevGeom& g, const uint8_t* mask_old, uint8_t* mask, const double* mu64,
            const double* maxv, double frac, int* n_split, int S, hipStream_t s, int rule) {
  int64_t nodes = 0;
  for (int l = 1; l <= g.L; ++l) nodes += int64_t(g.n >> l) * (g.n >> l);
  if (nodes == 0) return;
  hipLaunchKernelGGL(k_expand, dim3(blocks_for(nodes), S), dim3(kBlock), 0, s, g, mask_old, mask, mu64, maxv,
                     frac, n_split, rule);
}
void check_mask(const DevGeom& g, const uint8_t* mask, int* bad, int S, hipStream_t s) {
  hipLaunchKernelGGL(k_check_mask, dim3(blocks_for(int64_t(g.n) * g.n), S), dim3(kBlock), 0, s, g, mask, bad);
}
void fill_u8(uint8_t* x, int64_t len, uint8_t v, hipStream_t s) {
  if (len > 0) hipLaunchKernelGGL(k_fill_u8, dim3(blocks_for(len)), dim3(kBlock), 0, s, x, len, v);
}
void fill_i32(int* x, int64_t len, int v, hipStream_t s) {
  if (len > 0) hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(len)), dim3(kBlock), 0, s, x, len, v);
}
void fill_i32_strided(int* x, int count, int stride, int v, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_fill_i32_strided, dim3(blocks_for(count)), dim3(kBlock), 0, s, x, count, stride, v);
}
void approx_mask(const DevGeom& g, uint8_t* mask, int S, hipStream_t s) {
  hipLaunchKernelGGL(k_approx_mask, dim3(blocks_for(int64_t(g.n) * g.n), S), dim3(kBlock), 0, s, g.n, g.L, mask);
}

}  // namespace wamct
