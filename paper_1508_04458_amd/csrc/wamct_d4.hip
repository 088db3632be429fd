// Orthonormal Daubechies-4 wavelets (periodic boundary) for the 2-D scans: a "different
// wavelet type" in the sense of the Conclusion, in the same Mallat layout and tree structure
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

// The sums of one ray through one node's support: vals[0..3] = the projections of phi phi
// (approximation), phi_y psi_x (D1), psi_y phi_x (D2), psi_y psi_x (D3) along the ray: the ray
// is clipped to the support (up to four boxes where the support wraps at the border) and
// walked pixel by pixel (plane crossings in parameter order), each chord weighted by the basis
// values at the pixel holding the chord's midpoint.
template <typename R>
__device__ inline void d4_ray(const DevGeom& g, const D4Dev& tb, int l, int x0, int y0, double ox, double oy,
                              double ex, double ey, double iex, double iey, double vals[4]) {
  const int n = g.n, len = tb.len[l];
  const double pix = g.pixel, hn = 0.5 * n;
  const double* F = tb.f + tb.off[l];
  const double* G = tb.g + tb.off[l];
  vals[0] = vals[1] = vals[2] = vals[3] = 0.0;
  for (int pyk = 0; pyk < 2; ++pyk) {
    // y piece: pixel rows [ya, yb) of the image, support offsets from oyoff
    const int ys = y0, ye = y0 + len;
    int ya, yb, oyoff;
    if (pyk == 0) { ya = ys; yb = ye < n ? ye : n; oyoff = 0; }
    else { if (ye <= n) break; ya = 0; yb = ye - n; oyoff = n - ys; }
    for (int pxk = 0; pxk < 2; ++pxk) {
      const int xs = x0, xe = x0 + len;
      int xa, xb, oxoff;
      if (pxk == 0) { xa = xs; xb = xe < n ? xe : n; oxoff = 0; }
      else { if (xe <= n) break; xa = 0; xb = xe - n; oxoff = n - xs; }
      const double X0 = (xa - hn) * pix, X1 = (xb - hn) * pix, Y0 = (ya - hn) * pix, Y1 = (yb - hn) * pix;
      const double tx0 = (X0 - ox) * iex, tx1 = (X1 - ox) * iex, ty0 = (Y0 - oy) * iey, ty1 = (Y1 - oy) * iey;
      const double t_in = fmax(fmin(tx0, tx1), fmin(ty0, ty1));
      const double t_out = fmin(fmax(tx0, tx1), fmax(ty0, ty1));
      if (!(t_out > t_in)) continue;
      // interior planes in parameter order: x planes xa+1 .. xb-1, y planes ya+1 .. yb-1
      const bool xpos = iex > 0.0, ypos = iey > 0.0;
      int kx = xpos ? xa + 1 : xb - 1, ky = ypos ? ya + 1 : yb - 1;
      const int kx_end = xpos ? xb : xa, ky_end = ypos ? yb : ya;
      double t = t_in;
      for (int step = 0; step < 2 * len + 4; ++step) {
        const double tx = kx != kx_end ? ((kx - hn) * pix - ox) * iex : INFINITY;
        const double ty = ky != ky_end ? ((ky - hn) * pix - oy) * iey : INFINITY;
        const double te = fmax(fmin(fmin(tx, ty), t_out), t);
        const double c = te - t;
        if (c > 0.0) {
          const double tm = t + 0.5 * c;
          int px = int(floor((ox + tm * ex) / pix + hn)), py = int(floor((oy + tm * ey) / pix + hn));
          px = px < xa ? xa : (px > xb - 1 ? xb - 1 : px);
          py = py < ya ? ya : (py > yb - 1 ? yb - 1 : py);
          const int offx = px - xa + oxoff, offy = py - ya + oyoff;
          const double fx = F[offx], gx = G[offx], fy = F[offy], gy = G[offy];
          vals[0] += c * fy * fx;
          vals[1] += c * fy * gx;
          vals[2] += c * gy * fx;
          vals[3] += c * gy * gx;
        }
        if (te >= t_out) break;
        if (tx <= ty) kx += xpos ? 1 : -1;
        else ky += ypos ? 1 : -1;
        t = te;
      }
    }
  }
}

// Bin range of view v whose rays can meet the box [X0, X1) x [Y0, Y1) (mm): projections of the
// four corners on the detector, widened by 1e-3 bin.
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
  lo = int(ceil(umin / g.pitch + c0 - 1e-3));
  hi = int(floor(umax / g.pitch + c0 + 1e-3));
  lo = lo < 0 ? 0 : lo;
  hi = hi > g.nb - 1 ? g.nb - 1 : hi;
}

// One lane per work item (a root: its approximation, and its three details when split; a
// split node: its three details), over every view. kD4Split: b-hat+ and b-hat- of the item's
// coefficients (eq. 1.10; the sign split per (ray, coefficient), |phi| <= 1e-12 pixel counted
// as 0) into bp and bm; kD4Update: the same sums, then the zero of eq. 1.9 (beta += delta);
// kD4Z0: per ray, sum |phi| over the item's coefficients added to zsum[ray] (atomics: eq.
// 1.61 needs each ray's total over all items) and the item's number of non-zero (ray,
// coefficient) pairs into cnt[item].
template <typename T, typename R, int MODE>
__global__ __launch_bounds__(kD4Block) void k_d4_gather(DevGeom g, D4Dev tb, const double2* __restrict__ views,
                                                        const typename V4R<R>::t* __restrict__ A,
                                                        const typename V4R<R>::t* __restrict__ B,
                                                        const T* __restrict__ y, const uint32_t* __restrict__ items,
                                                        const int* __restrict__ n_items, T* __restrict__ beta,
                                                        const T* __restrict__ b,
                                                        const double* __restrict__ z0, int* __restrict__ held,
                                                        T* __restrict__ bp, T* __restrict__ bm,
                                                        double* __restrict__ zsum, double* __restrict__ cnt) {
  const int it = blockIdx.x * kD4Block + threadIdx.x;
  if (it >= *n_items) return;
  const uint32_t w = items[it];
  const bool quad = (w >> 31) != 0;
  const int l = int((w >> 27) & 15u), i = int((w >> 13) & 0x1fffu), j = int(w & 0x1fffu);
  const int n = g.n, m = n >> l, s = 1 << l;
  const bool root = l == g.L;
  const double tq = 1e-12 * g.pixel;
  double S[4] = {0, 0, 0, 0}, Aab[4] = {0, 0, 0, 0};
  double nz = 0.0;
  const double hn = 0.5 * n, pix = g.pixel;
  const int len = tb.len[l];
  for (int v = 0; v < g.nv; ++v) {
    const double2 cs = views[v];
    for (int pyk = 0; pyk < 2; ++pyk) {
      const int ye = s * i + len;
      if (pyk == 1 && ye <= n) break;
      const int ya = pyk == 0 ? s * i : 0, yb = pyk == 0 ? (ye < n ? ye : n) : ye - n;
      for (int pxk = 0; pxk < 2; ++pxk) {
        const int xe = s * j + len;
        if (pxk == 1 && xe <= n) break;
        const int xa = pxk == 0 ? s * j : 0, xb = pxk == 0 ? (xe < n ? xe : n) : xe - n;
        int lo, hi;
        d4_bins(g, cs, (xa - hn) * pix, (xb - hn) * pix, (ya - hn) * pix, (yb - hn) * pix, lo, hi);
        for (int bin = lo; bin <= hi; ++bin) {
          // rays meeting several pieces of the support are summed once per ray below: take
          // the ray only from the first piece its bin range reaches
          bool seen = false;
          for (int qy = 0; qy <= pyk && !seen; ++qy)
            for (int qx = 0; qx < 2 && !seen; ++qx) {
              if (qy == pyk && qx >= pxk) break;
              if (qx == 1 && xe <= n) break;
              if (qy == 1 && ye <= n) break;
              const int ya2 = qy == 0 ? s * i : 0, yb2 = qy == 0 ? (ye < n ? ye : n) : ye - n;
              const int xa2 = qx == 0 ? s * j : 0, xb2 = qx == 0 ? (xe < n ? xe : n) : xe - n;
              int lo2, hi2;
              d4_bins(g, cs, (xa2 - hn) * pix, (xb2 - hn) * pix, (ya2 - hn) * pix, (yb2 - hn) * pix, lo2, hi2);
              seen = bin >= lo2 && bin <= hi2;
            }
          if (seen) continue;
          const int r = v * g.nb + bin;
          const auto a = A[r];
          const auto bb = B[r];
          double vals[4];
          d4_ray<R>(g, tb, l, s * j, s * i, double(a.x), double(a.y), double(bb.x), double(bb.y), double(a.z),
                    double(a.w), vals);
          const bool use[4] = {root, quad, quad, quad};
          if (MODE == kD4Z0) {
            double zs = 0.0;
            for (int k = 0; k < 4; ++k)
              if (use[k] && fabs(vals[k]) > tq) { zs += fabs(vals[k]); nz += 1.0; }
            if (zs > 0.0) atomicAdd(zsum + r, zs);
          } else {
            const double yv = double(y[r]);
            for (int k = 0; k < 4; ++k) {
              const double wv = use[k] && fabs(vals[k]) > tq ? yv * vals[k] : 0.0;
              S[k] += wv;
              Aab[k] += fabs(wv);
            }
          }
        }
      }
    }
  }
  if (MODE == kD4Z0) {
    cnt[it] = nz;
    return;
  }
  const int64_t pos[4] = {int64_t(i) * n + j, int64_t(i) * n + m + j, int64_t(m + i) * n + j,
                          int64_t(m + i) * n + m + j};
  for (int k = 0; k < 4; ++k) {
    if (!(k == 0 ? root : quad)) continue;
    const double p = 0.5 * (Aab[k] + S[k]), q = 0.5 * (S[k] - Aab[k]);
    if (MODE == kD4Split) {
      bp[pos[k]] = T(p);
      bm[pos[k]] = T(q);
    } else {
      beta[pos[k]] = T(double(beta[pos[k]]) + am_delta<double>(double(b[pos[k]]), p, q, *z0, held));
    }
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
  auto bb = (const typename V4R<R>::t*)B;
  const dim3 grid(d4_blocks(max_items));
  if (mode == kD4Split)
    hipLaunchKernelGGL((k_d4_gather<T, R, kD4Split>), grid, dim3(kD4Block), 0, s, g, tb, views, a, bb, y, items,
                       n_items, beta, b, z0, held, bp, bm, zsum, cnt);
  else if (mode == kD4Update)
    hipLaunchKernelGGL((k_d4_gather<T, R, kD4Update>), grid, dim3(kD4Block), 0, s, g, tb, views, a, bb, y, items,
                       n_items, beta, b, z0, held, bp, bm, zsum, cnt);
  else
    hipLaunchKernelGGL((k_d4_gather<T, R, kD4Z0>), grid, dim3(kD4Block), 0, s, g, tb, views, a, bb, y, items,
                       n_items, beta, b, z0, held, bp, bm, zsum, cnt);
}
template struct D4<float, float>;
template struct D4<float, double>;
template struct D4<double, double>;

}  // namespace wamct
