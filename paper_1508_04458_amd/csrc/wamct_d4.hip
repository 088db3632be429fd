// Orthonormal Daubechies-4 wavelets (periodic boundary) for the 2-D scans: another wavelet
// family in the sense of the Conclusion, in the same Mallat layout and tree structure
// as the Haar basis, so Algorithm 1 (eqs. 1.6, 1.9, 1.10, 1.61) and the tree rule of the
// Results section run unchanged. The D4 basis functions are not constant on the tree's
// blocks, so there is no leaf walk: the forward pass synthesizes mu = Omega beta pixel by
// pixel and projects it with the pixel walk, and the sign-split backprojection walks every
// ray through the support of each active node (3 x 2^l - 2 pixels a side, wrapped at the
// image border) and weights each chord by the basis functions' values at that pixel.
//
// 1-D basis on a periodic grid of n pixels: level-0 scaling functions are the unit vectors;
// at level l, phi_{l,j} = sum_t h[t] phi_{l-1, 2j + t} and psi_{l,j} = sum_t g[t] phi_{l-1,
// 2j + t} (indices mod n >> (l-1)), h = (1 + r3, 3 + r3, 3 - r3, 1 - r3) / (4 sqrt 2), r3 =
// sqrt 3, g[t] = (-1)^t h[3 - t]. phi_{l,j} and psi_{l,j} are the same samples shifted by
// 2^l j: the tables hold them once per level (offsets 0 .. 3 x 2^l - 3 from 2^l j, mod n).
// 2-D: root approximation phi_L(y) phi_L(x) at [i][j]; node (l, i, j): D1 = phi_l(y) psi_l(x)
// at [i][m + j], D2 = psi_l(y) phi_l(x) at [m + i][j], D3 = psi_l(y) psi_l(x) at [m + i][m + j].
#include <hip/hip_runtime.h>
#include <math.h>

#include <cmath>
#include <vector>

#include "wamct_internal.h"

namespace wamct {

void d4_tables(int L, std::vector<double>& f, std::vector<double>& gt, D4Dev& tb) {
  const double r3 = std::sqrt(3.0), q = 4.0 * std::sqrt(2.0);
  const double h[4] = {(1.0 + r3) / q, (3.0 + r3) / q, (3.0 - r3) / q, (1.0 - r3) / q};
  double gw[4];
  for (int t = 0; t < 4; ++t) gw[t] = ((t & 1) ? -1.0 : 1.0) * h[3 - t];
  f.clear();
  gt.clear();
  // prev: level l-1 scaling function at position 0, samples at offsets 0 .. len-1 (level 0: a unit pulse)
  std::vector<double> prev(1, 1.0);
  int step_prev = 1;                   // shift between neighbouring level-(l-1) functions
  for (int l = 0; l <= kMaxLevels; ++l) tb.off[l] = tb.len[l] = 0;
  for (int l = 1; l <= L; ++l) {
    const int len = 3 * (1 << l) - 2;
    std::vector<double> P(size_t(len), 0.0), Q(size_t(len), 0.0);
    for (int t = 0; t < 4; ++t)
      for (size_t k = 0; k < prev.size(); ++k) {
        const size_t o = size_t(t) * size_t(step_prev) + k;
        P[o] += h[t] * prev[k];
        Q[o] += gw[t] * prev[k];
      }
    tb.off[l] = int(f.size());
    tb.len[l] = len;
    f.insert(f.end(), P.begin(), P.end());
    gt.insert(gt.end(), Q.begin(), Q.end());
    prev = P;
    step_prev <<= 1;
  }
}

namespace {

template <typename R> struct V4R;
template <> struct V4R<float> { using t = float4; };
template <> struct V4R<double> { using t = double4; };

constexpr int kD4Block = 256;
inline int d4_blocks(int64_t n) { return int((n + kD4Block - 1) / kD4Block); }

template <typename T>
__device__ inline double d4_coef(const T* __restrict__ beta, int64_t idx) { return double(beta[idx]); }

// mu(y, x) = sum over the active coefficients whose support holds the pixel (inactive ones are
// zero): per level the three positions i (rows) and j (columns) with an offset below the
// support length; rows written to muR [y][x] and, when muC is given, columns to muC [x][y].
template <typename T, typename O>
__global__ __launch_bounds__(kD4Block) void k_d4_synth(int n, int L, D4Dev tb, const T* __restrict__ beta,
                                                       O* __restrict__ muR, T* __restrict__ muC,
                                                       double* __restrict__ part) {
  const int64_t p = int64_t(blockIdx.x) * kD4Block + threadIdx.x;
  double v = -INFINITY;
  if (p < int64_t(n) * n) {
    const int y = int(p / n), x = int(p % n);
    v = 0.0;
    for (int l = L; l >= 1; --l) {
      const int m = n >> l, s = 1 << l, len = tb.len[l];
      const double* F = tb.f + tb.off[l];
      const double* G = tb.g + tb.off[l];
      for (int a = 0; a < 3; ++a) {
        const int i = ((y >> l) - a + m) % m;
        const int oy = ((y - s * i) % n + n) % n;
        if (oy >= len) continue;
        const double fy = F[oy], gy = G[oy];
        for (int b = 0; b < 3; ++b) {
          const int j = ((x >> l) - b + m) % m;
          const int ox = ((x - s * j) % n + n) % n;
          if (ox >= len) continue;
          const double fx = F[ox], gx = G[ox];
          v += fy * gx * d4_coef(beta, int64_t(i) * n + m + j) + gy * fx * d4_coef(beta, int64_t(m + i) * n + j) +
               gy * gx * d4_coef(beta, int64_t(m + i) * n + m + j);
          if (l == L) v += fy * fx * d4_coef(beta, int64_t(i) * n + j);
        }
      }
    }
    muR[p] = O(v);
    if (muC) muC[int64_t(x) * n + y] = T(v);
  }
  if (part) {   // per-block maxima of the FP64 image (the tree rule's threshold)
    __shared__ double sh[kD4Block / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = sh[0];
      for (int k = 1; k < kD4Block / 64; ++k) r = fmax(r, sh[k]);
      part[blockIdx.x] = r;
    }
  }
}

// coef(z) = sum over the support of z of img x basis (Omega^T img, FP64); Mallat position ->
// level, type and node as in the Haar analysis.
template <typename T>
__global__ __launch_bounds__(kD4Block) void k_d4_analysis(int n, int L, D4Dev tb, const T* __restrict__ img,
                                                          T* __restrict__ coef) {
  const int64_t p = int64_t(blockIdx.x) * kD4Block + threadIdx.x;
  if (p >= int64_t(n) * n) return;
  const int r = int(p / n), c = int(p % n);
  int l = L, t = 0;
  for (int lv = L; lv >= 1; --lv) {
    const int m = n >> lv;
    if (r < 2 * m && c < 2 * m) {
      t = (r >= m ? 2 : 0) | (c >= m ? 1 : 0);
      if (t != 0 || lv == L) { l = lv; break; }
    }
  }
  const int m = n >> l, s = 1 << l, len = tb.len[l];
  const int i = r % m, j = c % m;
  const double* Fy = (t & 2) ? tb.g + tb.off[l] : tb.f + tb.off[l];   // psi along y for D2, D3
  const double* Fx = (t & 1) ? tb.g + tb.off[l] : tb.f + tb.off[l];   // psi along x for D1, D3
  double acc = 0.0;
  for (int oy = 0; oy < len; ++oy) {
    const int yy = (s * i + oy) % n;
    double row = 0.0;
    for (int ox = 0; ox < len; ++ox) row += double(img[int64_t(yy) * n + (s * j + ox) % n]) * Fx[ox];
    acc += row * Fy[oy];
  }
  coef[p] = T(acc);
}

// One ray through one rectangle of pixels [xa, xb) x [ya, yb) of a basis function's support
// (table entry of pixel (px, py): px - xa + oxoff along x, py - ya + oyoff along y; T holds
// (phi, psi) pairs): v[0..3] += the chord in every pixel times phi(y) phi(x), phi(y) psi(x),
// psi(y) phi(x), psi(y) psi(x). Planes: x = k pixel lies at t = k sx + cx (sx = pixel / e_x,
// cx = (-n/2 pixel - o_x) / e_x), y likewise. The ray is clipped to the rectangle, the entry
// pixel (coordinate (t - cx) / sx in pixels) taken on the side the ray moves into, and the
// walk steps to the nearer of the next planes (a segment ending before it starts, after an
// entry pixel one off at a corner, adds nothing). The walk runs in the frame of the ray's
// major axis u (|s_u| <= |s_v|): along u it
// adds c phi(u) and c psi(u) to two run sums, which are multiplied by the minor axis' phi(v)
// and psi(v) when the walk crosses a v plane (and at the end).
__device__ inline void d4_piece(double sx, double cx, double sy, double cy, int xa, int xb, int ya, int yb,
                                int oxoff, int oyoff, const double2* __restrict__ T, double v[4]) {
  const double tx0 = fma(double(xa), sx, cx), tx1 = fma(double(xb), sx, cx);
  const double ty0 = fma(double(ya), sy, cy), ty1 = fma(double(yb), sy, cy);
  const double t_in = fmax(fmin(tx0, tx1), fmin(ty0, ty1));
  const double t_out = fmin(fmax(tx0, tx1), fmax(ty0, ty1));
  if (!(t_out > t_in)) return;
  const double fx = (t_in - cx) / sx, fy = (t_in - cy) / sy;
  int px = sx > 0.0 ? int(floor(fx)) : int(ceil(fx)) - 1;
  int py = sy > 0.0 ? int(floor(fy)) : int(ceil(fy)) - 1;
  px = px < xa ? xa : (px > xb - 1 ? xb - 1 : px);
  py = py < ya ? ya : (py > yb - 1 ? yb - 1 : py);
  const bool xmaj = fabs(sx) <= fabs(sy);
  int pu = xmaj ? px : py, pv = xmaj ? py : px;
  const int ua = xmaj ? xa : ya, un = xmaj ? xb - xa : yb - ya, uo = xmaj ? oxoff - xa : oyoff - ya;
  const int va = xmaj ? ya : xa, vn = xmaj ? yb - ya : xb - xa, vo = xmaj ? oyoff - ya : oxoff - xa;
  const double su = xmaj ? sx : sy, cu = xmaj ? cx : cy, sv = xmaj ? sy : sx, cv = xmaj ? cy : cx;
  const int du = su > 0.0 ? 1 : -1, dv = sv > 0.0 ? 1 : -1;
  const double nu = su > 0.0 ? 1.0 : 0.0, nv = sv > 0.0 ? 1.0 : 0.0;
  double tun = fma(double(pu) + nu, su, cu), tvn = fma(double(pv) + nv, sv, cv);
  double2 fu = T[pu + uo], fv = T[pv + vo];
  double t = t_in, Sf = 0.0, Sg = 0.0, a00 = 0.0, a01 = 0.0, a10 = 0.0, a11 = 0.0;
  for (;;) {
    const double te = fmin(fmin(tun, tvn), t_out);
    const double c = fmax(te - t, 0.0);
    Sf = fma(c, fu.x, Sf);
    Sg = fma(c, fu.y, Sg);
    t = fmax(t, te);
    if (te >= t_out) break;
    if (tun <= tvn) {
      pu += du;
      if (unsigned(pu - ua) >= unsigned(un)) break;
      tun = fma(double(pu) + nu, su, cu);
      fu = T[pu + uo];
    } else {
      a00 = fma(fv.x, Sf, a00);
      a01 = fma(fv.y, Sf, a01);
      a10 = fma(fv.x, Sg, a10);
      a11 = fma(fv.y, Sg, a11);
      Sf = 0.0;
      Sg = 0.0;
      pv += dv;
      if (unsigned(pv - va) >= unsigned(vn)) break;
      tvn = fma(double(pv) + nv, sv, cv);
      fv = T[pv + vo];
    }
  }
  a00 = fma(fv.x, Sf, a00);
  a01 = fma(fv.y, Sf, a01);
  a10 = fma(fv.x, Sg, a10);
  a11 = fma(fv.y, Sg, a11);
  // a10 = phi(v) psi(u), a01 = psi(v) phi(u)
  v[0] += a00;
  v[1] += xmaj ? a10 : a01;
  v[2] += xmaj ? a01 : a10;
  v[3] += a11;
}

// Bin range of view v whose rays can meet the box [X0, X1) x [Y0, Y1) (mm): projections of the
// four corners on the detector, widened by 1e-3 bin; empty when lo > hi.
__device__ inline void d4_bins(const DevGeom& g, double2 cs, double X0, double X1, double Y0, double Y1, int& lo,
                               int& hi) {
  double umin = 1e300, umax = -1e300;
  for (int k = 0; k < 4; ++k) {
    const double px = (k & 1) ? X1 : X0, py = (k & 2) ? Y1 : Y0;
    double u;
    if (g.kind == 0) {
      u = px * cs.x + py * cs.y;
    } else {
      const double depth = g.sod - (px * cs.x + py * cs.y);
      u = (-px * cs.y + py * cs.x) * g.sdd / depth;
    }
    umin = fmin(umin, u);
    umax = fmax(umax, u);
  }
  const double c0 = 0.5 * (g.nb - 1);
  const double flo = fmin(fmax(umin / g.pitch + c0 - 1e-3, -1.0), double(g.nb));
  const double fhi = fmin(fmax(umax / g.pitch + c0 + 1e-3, -1.0), double(g.nb));
  lo = max(int(ceil(flo)), 0);
  hi = min(int(floor(fhi)), g.nb - 1);
}

// The gather runs one work item per 64-lane block: items differ widely in cost (a split root
// has four coefficients, a level-1 node three over a support a quarter as wide), and a block of
// several items would hold its wave slots until its slowest item ends.
constexpr int kD4GatherBlock = 64;

// Rectangle q (0 .. count - 1) of a support of len x len pixels from (x0, y0), wrapped at the
// border n: q enumerates (upper or wrapped part in y) x (left or wrapped part in x), the
// wrapped parts present only when the support passes the border (wx, wy).
struct D4Rect {
  int xa, xb, ya, yb, ox, oy;
};
__device__ inline D4Rect d4_rect(int q, int x0, int y0, int len, int n, bool wx) {
  const int qx = wx ? (q & 1) : 0, qy = wx ? (q >> 1) : q;
  D4Rect r;
  r.ya = qy == 0 ? y0 : 0;
  r.yb = qy == 0 ? min(y0 + len, n) : y0 + len - n;
  r.oy = qy == 0 ? 0 : n - y0;
  r.xa = qx == 0 ? x0 : 0;
  r.xb = qx == 0 ? min(x0 + len, n) : x0 + len - n;
  r.ox = qx == 0 ? 0 : n - x0;
  return r;
}
// Whether the line crosses the rectangle (plane parameters as in d4_piece).
__device__ inline bool d4_hits(const D4Rect& r, double sx, double cx, double sy, double cy) {
  const double tx0 = fma(double(r.xa), sx, cx), tx1 = fma(double(r.xb), sx, cx);
  const double ty0 = fma(double(r.ya), sy, cy), ty1 = fma(double(r.yb), sy, cy);
  return fmin(fmax(tx0, tx1), fmax(ty0, ty1)) > fmax(fmin(tx0, tx1), fmin(ty0, ty1));
}

// One wave (one block) per work item (a root: its approximation, and its three details when
// split; a split node: its three details); lane k takes the views k, k + 64, ... and the wave's sums are
// combined by a fixed butterfly (deterministic). The support of the item's functions (len x
// len pixels from (2^l i, 2^l j), wrapped at the border into up to four rectangles) is
// projected per view to a bin range per rectangle; a ray is taken in the loop of the first
// rectangle it crosses (exact slab test) and walked through that rectangle and the later ones.
// kD4Split: b-hat+ and b-hat- of the item's coefficients (eq. 1.10; sign split per (ray,
// coefficient); |phi| <= 1e-12 pixel counted as 0) into bp and bm; kD4Update: the same sums,
// then the zero of eq. 1.9 (beta += delta); kD4Z0: per ray, sum |phi| over the item's
// coefficients added to zsum[ray] (atomics: eq. 1.61 needs each ray's total over all items)
// and the item's number of non-zero (ray, coefficient) pairs into cnt[item]. The basis tables
// are staged in LDS as (phi, psi) pairs (dynamic, one double2 per table entry). Rays come
// from the ray table's (origin, inverse direction). Registers are capped for four waves per
// SIMD (128 VGPRs, no spills; measured 1.2x faster than three waves at 146).
template <typename T, typename R, int MODE>
__global__ __launch_bounds__(kD4GatherBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_d4_gather(
    DevGeom g, D4Dev tb, int tab_len, const double2* __restrict__ views, const typename V4R<R>::t* __restrict__ A,
                                                        const T* __restrict__ y, const uint32_t* __restrict__ items,
                                                        const int* __restrict__ n_items, T* __restrict__ beta,
                                                        const T* __restrict__ b, const double* __restrict__ z0,
                                                        int* __restrict__ held, T* __restrict__ bp,
                                                        T* __restrict__ bm, double* __restrict__ zsum,
                                                        double* __restrict__ cnt) {
  const int it = blockIdx.x;
  const int lane = int(threadIdx.x);
  if (it >= *n_items) return;   // uniform over the block
  extern __shared__ double2 lds2[];
  for (int k = lane; k < tab_len; k += kD4GatherBlock) lds2[k] = make_double2(tb.f[k], tb.g[k]);
  __syncthreads();
  const uint32_t w = items[it];
  const bool quad = (w >> 31) != 0;
  const int l = int((w >> 27) & 15u), i = int((w >> 13) & 0x1fffu), j = int(w & 0x1fffu);
  const int n = g.n, m = n >> l, s = 1 << l;
  const bool root = l == g.L;
  const double tq = 1e-12 * g.pixel;
  const double pix = g.pixel, hn = 0.5 * n;
  const int len = tb.len[l];
  const double2* T2 = lds2 + tb.off[l];
  const int y0 = s * i, x0 = s * j;
  const bool wx = x0 + len > n, wy = y0 + len > n;
  const int nr = (wx ? 2 : 1) * (wy ? 2 : 1);
  double S[4] = {0, 0, 0, 0}, Aab[4] = {0, 0, 0, 0};
  double nz = 0.0;
  for (int v = lane; v < g.nv; v += 64) {
    const double2 cs = views[v];
    for (int q = 0; q < nr; ++q) {
      const D4Rect rq = d4_rect(q, x0, y0, len, n, wx);
      int lo, hi;
      d4_bins(g, cs, (rq.xa - hn) * pix, (rq.xb - hn) * pix, (rq.ya - hn) * pix, (rq.yb - hn) * pix, lo, hi);
      for (int bin = lo; bin <= hi; ++bin) {
        const int r = v * g.nb + bin;
        const auto a = A[r];
        const double ox = double(a.x), oy = double(a.y), iex = double(a.z), iey = double(a.w);
        const double sx = pix * iex, cx = (-hn * pix - ox) * iex, sy = pix * iey, cy = (-hn * pix - oy) * iey;
        if (nr > 1) {
          bool mine = d4_hits(rq, sx, cx, sy, cy);
          for (int q2 = 0; q2 < q && mine; ++q2) mine = !d4_hits(d4_rect(q2, x0, y0, len, n, wx), sx, cx, sy, cy);
          if (!mine) continue;
        }
        double vals[4] = {0, 0, 0, 0};
#pragma unroll 1
        for (int q2 = q; q2 < nr; ++q2) {
          const D4Rect r2 = d4_rect(q2, x0, y0, len, n, wx);
          d4_piece(sx, cx, sy, cy, r2.xa, r2.xb, r2.ya, r2.yb, r2.ox, r2.oy, T2, vals);
        }
        if (MODE == kD4Z0) {
          double zs = 0.0;
          if (root && fabs(vals[0]) > tq) { zs += fabs(vals[0]); nz += 1.0; }
          if (quad) {
#pragma unroll
            for (int k = 1; k < 4; ++k)
              if (fabs(vals[k]) > tq) { zs += fabs(vals[k]); nz += 1.0; }
          }
          if (zs > 0.0) atomicAdd(zsum + r, zs);
        } else {
          const double yv = double(y[r]);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const double wv = fabs(vals[k]) > tq ? yv * vals[k] : 0.0;
            S[k] += wv;
            Aab[k] += fabs(wv);
          }
        }
      }
    }
  }
  // butterfly over the wave: every lane ends with the same totals, added in the same order
  if (MODE == kD4Z0) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nz += __shfl_xor(nz, o, 64);
    if (lane == 0) cnt[it] = nz;
    return;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      S[k] += __shfl_xor(S[k], o, 64);
      Aab[k] += __shfl_xor(Aab[k], o, 64);
    }
  }
  // lane k writes coefficient k (the approximation only for a root, the details only when split)
  if (lane >= 4 || (lane == 0 ? !root : !quad)) return;
  const int64_t pos = lane == 0 ? int64_t(i) * n + j
                    : lane == 1 ? int64_t(i) * n + m + j
                    : lane == 2 ? int64_t(m + i) * n + j
                                : int64_t(m + i) * n + m + j;
  double Sk = S[0], Ak = Aab[0];
#pragma unroll
  for (int k = 1; k < 4; ++k)
    if (lane == k) { Sk = S[k]; Ak = Aab[k]; }
  const double p = 0.5 * (Ak + Sk), qn = 0.5 * (Sk - Ak);
  if (MODE == kD4Split) {
    bp[pos] = T(p);
    bm[pos] = T(qn);
  } else {
    beta[pos] = T(double(beta[pos]) + am_delta<double>(double(b[pos]), p, qn, *z0, held));
  }
}

}  // namespace

template <typename T, typename R>
void D4<T, R>::synth(const DevGeom& g, const D4Dev& tb, const T* beta, T* muR, T* muC, hipStream_t s) {
  const int64_t nn = int64_t(g.n) * g.n;
  hipLaunchKernelGGL((k_d4_synth<T, T>), dim3(d4_blocks(nn)), dim3(kD4Block), 0, s, g.n, g.L, tb, beta, muR, muC,
                     (double*)nullptr);
}
template <typename T, typename R>
int D4<T, R>::mu64(const DevGeom& g, const D4Dev& tb, const T* beta, double* mu64, double* part, hipStream_t s) {
  const int64_t nn = int64_t(g.n) * g.n;
  const int nb = d4_blocks(nn);
  hipLaunchKernelGGL((k_d4_synth<T, double>), dim3(nb), dim3(kD4Block), 0, s, g.n, g.L, tb, beta, mu64, (T*)nullptr,
                     part);
  return nb;
}
template <typename T, typename R>
void D4<T, R>::analysis(const DevGeom& g, const D4Dev& tb, const T* img, T* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_d4_analysis<T>, dim3(d4_blocks(int64_t(g.n) * g.n)), dim3(kD4Block), 0, s, g.n, g.L, tb, img,
                     coef);
}
template <typename T, typename R>
void D4<T, R>::gather(const DevGeom& g, int mode, const D4Dev& tb, const double2* views, const void* A,
                      const void* B, const T* y, const uint32_t* items, const int* n_items, int max_items, T* beta,
                      const T* b, const double* z0, int* held, T* bp, T* bm, double* zsum, double* cnt,
                      hipStream_t s) {
  if (max_items <= 0) return;
  auto a = (const typename V4R<R>::t*)A;
  (void)B;   // the walk needs the origin and inverse direction only
  const int tab_len = tb.off[g.L] + tb.len[g.L];
  const size_t lds = sizeof(double2) * size_t(tab_len);
  const dim3 grid(max_items);
  if (mode == kD4Split)
    hipLaunchKernelGGL((k_d4_gather<T, R, kD4Split>), grid, dim3(kD4GatherBlock), lds, s, g, tb, tab_len, views, a, y,
                       items, n_items, beta, b, z0, held, bp, bm, zsum, cnt);
  else if (mode == kD4Update)
    hipLaunchKernelGGL((k_d4_gather<T, R, kD4Update>), grid, dim3(kD4GatherBlock), lds, s, g, tb, tab_len, views, a,
                       y, items, n_items, beta, b, z0, held, bp, bm, zsum, cnt);
  else
    hipLaunchKernelGGL((k_d4_gather<T, R, kD4Z0>), grid, dim3(kD4GatherBlock), lds, s, g, tb, tab_len, views, a, y,
                       items, n_items, beta, b, z0, held, bp, bm, zsum, cnt);
}
template struct D4<float, float>;
template struct D4<float, double>;
template struct D4<double, double>;

}  // namespace wamct
