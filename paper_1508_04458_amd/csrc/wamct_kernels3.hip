// HIP kernels of wavelet-tree AM on a 3-D volume for gfx950: circular cone beam with a flat
// detector, and either a 3-D Haar octree (seven details per node) or the 2-D Haar transform
// of every z-slice with one quadtree shared by the slices (three details per node, a node one
// voxel deep; the Results section's representation of its volumes).
//
// Method: Degirmenci, O'Sullivan, Politte, arXiv 1508.04458, Introduction (eqs. 1.2-1.10,
// Algorithm 1) and Results (tree rule), applied to voxels and octree nodes. As in 2-D the
// system matrix is never stored: chords through voxels, leaves and node octants are
// recomputed from the ray table, so the kernels are bound by vector ALU and cache gathers.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "wamct_internal3.h"
#include "wamct_worklist.h"

namespace wamct {
namespace {

constexpr int kB = 256;
// Groups of 8 walk blocks an XCD keeps the same part of the detector rows (2^8 groups: 512
// consecutive views of a row; the records they cross stay in its L2).
constexpr int kRotate3 = 8;
inline int blocks3(int64_t n, int b = kB) { return int((n + b - 1) / b); }

// Workgroups are dealt to the 8 XCDs round-robin (block b runs on XCD b mod 8), each XCD with
// its own L2. The one-lane-per-item gather maps block b of a padded grid to the work unit
// (b mod 8) (grid / 8) + b / 8, so every XCD takes one contiguous range of items (a compact
// region of the volume, whose rays it then finds in its L2). The leaf walks and the
// view-chunked gather keep the round-robin order: there every XCD works on the same views at
// the same time, which shares the last-level cache and balances the load.
constexpr int kXcd3 = 8;

// Ray of launch index k in the walks: k runs over (detector row, view, column), so the rays
// in flight at any time belong to one detector row of many views and traverse one band of
// z-slabs (a fraction of the volume) rather than the whole volume of one view.
__device__ inline int64_t row_major_ray(const DevGeom3& g, int64_t k) {
  const int64_t per_row = int64_t(g.nv) * g.nc;
  const int row = int(k / per_row);
  const int64_t rem = k - row * per_row;
  const int v = int(rem / g.nc), col = int(rem - int64_t(v) * g.nc);
  return (int64_t(v) * g.nr + row) * g.nc + col;
}
__device__ inline int xcd_unit3(int b, int grid) { return (b % kXcd3) * (grid / kXcd3) + b / kXcd3; }
inline int xcd_pad3(int units) { return (units + kXcd3 - 1) / kXcd3 * kXcd3; }

__device__ inline int imin3(int a, int b) { return a < b ? a : b; }
__device__ inline int imax3(int a, int b) { return a > b ? a : b; }

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
template <bool MAX>
__device__ inline double breduce(double v) {
  __shared__ double sh[kB / 64];
  v = MAX ? wmax(v) : wsum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int k = 1; k < kB / 64; ++k) r = MAX ? fmax(r, sh[k]) : r + sh[k];
    v = r;
  }
  return v;
}

// ------------------------------------------------------------------ geometry

// A coordinate in voxel units within 1e-9 of an integer (a voxel boundary) is taken as on it.
__device__ inline double edge_snap3(double f) {
  const double r = rint(f);
  return fabs(f - r) <= 1e-9 ? r : f;
}

// Ray of detector element (row, col) of view v for the leaf walks, from the per-view factors
// the gather also uses (no per-ray table): the line starts at the source S = sod (c, s, 0)
// and runs along D = (-sdd c - u s, -sdd s + u c, w) (u, w: column and row offsets on the
// detector), unit direction e = D / |D|, 1/e from the factors 1/Dx, 1/Dy (per view and column)
// and 1/Dz (per row) times |D| (per row and column). A component of D within 1e-12 sdd of 0
// (the factor is then +-1e300) is exactly 0: e is axis-parallel there, with a positive
// reciprocal (no mirroring), and the source's coordinate on that axis, within 1e-9 voxel of a
// boundary taken as on it, decides the slab: a line on a boundary lies in the voxel on the +
// side (half-open voxels), as in the gather, which also measures from the source.
struct Ray3 {
  double X, Y, Z;        // source in voxel coordinates (0 .. n, 0 .. nz across the volume)
  double ex, ey, ez;     // unit direction
  double iex, iey, iez;  // 1 / e (1e300 on an axis-parallel component)
};
__device__ inline Ray3 ray_from_factors(const DevGeom3& g, const RayF3& f, int64_t r) {
  const int64_t per_view = int64_t(g.nr) * g.nc;
  const int v = int(r / per_view);
  const int rem = int(r - int64_t(v) * per_view);
  const int row = rem / g.nc, col = rem - row * g.nc;
  const double2 cs = f.views[v];
  const double2 cd = f.colt[int64_t(v) * g.nc + col];
  const double idz = f.rowt[row];
  const double nd = f.nrm[rem];
  const double u = (col - 0.5 * (g.nc - 1)) * g.cpitch, w = (row - 0.5 * (g.nr - 1)) * g.rpitch;
  const double dx = -g.sdd * cs.x - u * cs.y, dy = -g.sdd * cs.y + u * cs.x;
  const double ind = 1.0 / nd;
  const bool snx = fabs(cd.x) >= 1e299, sny = fabs(cd.y) >= 1e299, snz = fabs(idz) >= 1e299;
  const double ipix = 1.0 / g.pixel;
  Ray3 q;
  q.X = g.sod * cs.x * ipix + 0.5 * g.n;
  q.Y = g.sod * cs.y * ipix + 0.5 * g.n;
  q.Z = 0.5 * g.nz;
  q.ex = snx ? 0.0 : dx * ind;
  q.ey = sny ? 0.0 : dy * ind;
  q.ez = snz ? 0.0 : w * ind;
  q.iex = snx ? 1e300 : cd.x * nd;
  q.iey = sny ? 1e300 : cd.y * nd;
  q.iez = snz ? 1e300 : idz * nd;
  if (snx) q.X = edge_snap3(q.X);
  if (sny) q.Y = edge_snap3(q.Y);
  if (snz) q.Z = edge_snap3(q.Z);
  return q;
}

// ------------------------------------------------------------------ octree helpers

// node (l, k, i, j) split <=> its tx detail is active: mask[k][i][m + j], m = n >> l
__device__ inline bool split3(const uint8_t* __restrict__ mask, int n, int l, int k, int i, int j) {
  const int m = n >> l;
  return mask[(int64_t(k) * n + i) * n + m + j] != 0;
}

__device__ inline uint32_t morton3_compact(uint32_t x) {
  x &= 0x09249249u;
  x = (x | (x >> 2)) & 0x030c30c3u;
  x = (x | (x >> 4)) & 0x0300f00fu;
  x = (x | (x >> 8)) & 0x030000ffu;
  x = (x | (x >> 16)) & 0x000003ffu;
  return x;
}

// Detail slot d (0..6) has the type t = d + 1 with bits (tz, ty, tx) = (t >> 2, t >> 1, t) & 1,
// at [k + tz mz][i + ty m][j + tx m]; its basis is 2^(-3l/2) prod over flagged axes of
// (+1 lower half, -1 upper half).
__device__ inline int64_t detail_pos(int n, int nz, int l, int d, int k, int i, int j) {
  const int t = d + 1, m = n >> l, mz = nz >> l;
  return (int64_t(k + ((t >> 2) & 1) * mz) * n + (i + ((t >> 1) & 1) * m)) * n + (j + (t & 1) * m);
}

__device__ inline double scale3(int l) { return exp2(-1.5 * double(l)); }

// Per-slice 2-D Haar (wd = 2) uses the detail slots d = 0, 1, 2 (types t = 1, 2, 3: tz = 0, so
// detail_pos gives [k][i][m + j], [k][m + i][j], [k][m + i][m + j] in slice k: the 2-D Mallat
// positions of D1, D2, D3) and the basis 2^-l; the octree all seven and 2^(-3l/2).
template <int WD> __device__ constexpr int n_details() { return WD == 3 ? 7 : 3; }
template <int WD> __device__ inline double scale_w(int l) { return WD == 3 ? scale3(l) : exp2(-double(l)); }

// mu(voxel) = scale(L) beta_LL(root) + sum over levels of scale(l) sum_d sign_d beta_d
template <typename T, typename R, int WD>
__device__ inline R synth_voxel(const T* __restrict__ beta, int n, int nz, int L, int s, int r, int c) {
  R v = R(beta[(int64_t(s >> node_zshift(WD, L)) * n + (r >> L)) * n + (c >> L)]) * R(scale_w<WD>(L));
  for (int l = L; l >= 1; --l) {
    const int k = s >> node_zshift(WD, l), i = r >> l, j = c >> l;
    const int oct = (WD == 3 ? ((s >> (l - 1)) & 1) << 2 : 0) | (((r >> (l - 1)) & 1) << 1) | ((c >> (l - 1)) & 1);
    R acc = R(0);
#pragma unroll
    for (int d = 0; d < n_details<WD>(); ++d) {
      const R b = R(beta[detail_pos(n, nz, l, d, k, i, j)]);
      acc += (__popc(uint32_t((d + 1) & oct)) & 1) ? -b : b;
    }
    v += acc * R(scale_w<WD>(l));
  }
  return v;
}
template <typename T, typename R>
__device__ inline R synth_voxel_g(const DevGeom3& g, const T* __restrict__ beta, int s, int r, int c) {
  return g.wd == 2 ? synth_voxel<T, R, 2>(beta, g.n, g.nz, g.L, s, r, c)
                   : synth_voxel<T, R, 3>(beta, g.n, g.nz, g.L, s, r, c);
}

// Leaf record: value rounded to 4 free low mantissa bits that hold the leaf level.
template <typename T> struct Rec3;
template <> struct Rec3<float> {
  uint32_t w;
  __device__ static Rec3 make(float v, uint32_t lev) { return Rec3{((__float_as_uint(v) + 8u) & ~15u) | lev}; }
  __device__ float mu() const { return __uint_as_float(w & ~15u); }
  __device__ uint32_t lev() const { return w & 15u; }
};
template <> struct Rec3<double> {
  uint64_t w;
  __device__ static Rec3 make(double v, uint32_t lev) {
    return Rec3{((uint64_t(__double_as_longlong(v)) + 8u) & ~uint64_t(15)) | lev};
  }
  __device__ double mu() const { return __longlong_as_double((long long)(w & ~uint64_t(15))); }
  __device__ uint32_t lev() const { return uint32_t(w & 15u); }
};

template <typename T>
__global__ __launch_bounds__(kB) void k3_synth_records(DevGeom3 g, const T* __restrict__ beta,
                                                       const uint8_t* __restrict__ lev, Rec3<T>* __restrict__ recR,
                                                       Rec3<T>* __restrict__ recC) {
  const int64_t p = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int n = g.n;
  if (p >= int64_t(n) * n * g.nz) return;
  const int s = int(p / (int64_t(n) * n)), r = int((p / n) % n), c = int(p % n);
  const T v = lev ? synth_voxel_g<T, T>(g, beta, s, r, c) : beta[p];
  const uint32_t l = lev ? lev[p] : 0u;
  recR[p] = Rec3<T>::make(v, l);
  recC[(int64_t(s) * n + c) * n + r] = Rec3<T>::make(v, l);
}

template <typename T>
__global__ __launch_bounds__(kB) void k3_synth(DevGeom3 g, const T* __restrict__ beta, T* __restrict__ mu) {
  const int64_t p = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int n = g.n;
  if (p >= int64_t(n) * n * g.nz) return;
  mu[p] = synth_voxel_g<T, T>(g, beta, int(p / (int64_t(n) * n)), int((p / n) % n), int(p % n));
}

template <typename T>
__global__ __launch_bounds__(kB) void k3_mu64(DevGeom3 g, const T* __restrict__ beta, double* __restrict__ mu64,
                                              double* __restrict__ part) {
  const int64_t p = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int n = g.n;
  double v = -INFINITY;
  if (p < int64_t(n) * n * g.nz) {
    v = synth_voxel_g<T, double>(g, beta, int(p / (int64_t(n) * n)), int((p / n) % n), int(p % n));
    mu64[p] = v;
  }
  v = breduce<true>(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ __launch_bounds__(kB) void k3_levmap(DevGeom3 g, const uint8_t* __restrict__ mask,
                                                uint8_t* __restrict__ lev, uint8_t* __restrict__ levC) {
  const int64_t p = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int n = g.n;
  if (p >= int64_t(n) * n * g.nz) return;
  const int s = int(p / (int64_t(n) * n)), r = int((p / n) % n), c = int(p % n);
  int l = g.L;
  while (l >= 1 && split3(mask, n, l, s >> node_zshift(g.wd, l), r >> l, c >> l)) --l;
  lev[p] = uint8_t(l);
  if (levC) levC[(int64_t(s) * n + c) * n + r] = uint8_t(l);
}

// coef(z) = sum over the support of basis function z of its value times vol (Omega^T vol),
// FP64; Mallat position -> (level, detail type, node)
template <typename T>
__global__ __launch_bounds__(kB) void k3_analysis(DevGeom3 g, const T* __restrict__ vol, T* __restrict__ coef) {
  const int64_t p = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int n = g.n, nz = g.nz, L = g.L;
  if (p >= int64_t(n) * n * nz) return;
  const int z = int(p / (int64_t(n) * n)), y = int((p / n) % n), x = int(p % n);
  const bool oc = g.wd == 3;   // octree; else 2-D Haar of slice z
  int l = 0, t = 0;
  for (int lv = L; lv >= 1; --lv) {
    const int m = n >> lv, mz = oc ? nz >> lv : nz;
    if ((!oc || z < 2 * mz) && y < 2 * m && x < 2 * m) {
      t = (oc && z >= mz ? 4 : 0) | (y >= m ? 2 : 0) | (x >= m ? 1 : 0);
      if (t != 0 || lv == L) { l = lv; break; }
    }
  }
  double acc = 0.0;
  if (t == 0) {  // approximation of root (z, y, x) (or a voxel when L = 0)
    const int s = 1 << L, sz = oc ? s : 1;
    for (int a = 0; a < sz; ++a)
      for (int b = 0; b < s; ++b)
        for (int c = 0; c < s; ++c) acc += double(vol[(int64_t(z * sz + a) * n + y * s + b) * n + x * s + c]);
    acc *= oc ? scale3(L) : exp2(-double(L));
  } else {
    const int m = n >> l, mz = oc ? nz >> l : nz, s = 1 << l, h = s >> 1, sz = oc ? s : 1;
    const int k = z % mz, i = y % m, j = x % m;
    for (int a = 0; a < sz; ++a)
      for (int b = 0; b < s; ++b)
        for (int c = 0; c < s; ++c) {
          const int oct = (oc && a >= h ? 4 : 0) | ((b >= h) << 1) | (c >= h);
          const double v = double(vol[(int64_t(k * sz + a) * n + i * s + b) * n + j * s + c]);
          acc += (__popc(uint32_t(t & oct)) & 1) ? -v : v;
        }
    acc *= oc ? scale3(l) : exp2(-double(l));
  }
  coef[p] = T(acc);
}

template <typename T>
__global__ __launch_bounds__(kB) void k3_apply_mask(int64_t len, T* __restrict__ beta, const uint8_t* __restrict__ m) {
  const int64_t p = int64_t(blockIdx.x) * kB + threadIdx.x;
  if (p < len && m[p] == 0) beta[p] = T(0);
}

// Validity of an octree mask: *bad counts violated constraints (roots active; 0/1 values;
// a node's seven details equal; a split node's parent split).
__global__ __launch_bounds__(kB) void k3_check_mask(DevGeom3 g, const uint8_t* __restrict__ mask,
                                                    int* __restrict__ bad) {
  const int64_t p = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int n = g.n, nz = g.nz, L = g.L;
  if (p >= int64_t(n) * n * nz) return;
  const int z = int(p / (int64_t(n) * n)), y = int((p / n) % n), x = int(p % n);
  const bool oc = g.wd == 3;   // octree; else one quadtree shared by the slices
  if (!oc && mask[p] != mask[int64_t(y) * n + x]) { atomicAdd(bad, 1); return; }
  if ((!oc || z < (nz >> L)) && y < (n >> L) && x < (n >> L)) {
    if (mask[p] != 1) atomicAdd(bad, 1);
    return;
  }
  if (mask[p] > 1) { atomicAdd(bad, 1); return; }
  int l = 0;
  for (int lv = L; lv >= 1; --lv)
    if ((!oc || z < 2 * (nz >> lv)) && y < 2 * (n >> lv) && x < 2 * (n >> lv)) { l = lv; break; }
  if (l == 0) { atomicAdd(bad, 1); return; }
  const int m = n >> l, mz = oc ? nz >> l : nz;
  const int k = z % mz, i = y % m, j = x % m;
  const bool f = split3(mask, n, l, k, i, j);
  if ((mask[p] != 0) != f) { atomicAdd(bad, 1); return; }
  if (f && l < L && !split3(mask, n, l + 1, oc ? k >> 1 : k, i >> 1, j >> 1)) atomicAdd(bad, 1);
}

__global__ void k3_approx_mask(DevGeom3 g, uint8_t* __restrict__ mask) {
  const int64_t p = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int n = g.n;
  if (p >= int64_t(n) * n * g.nz) return;
  const int z = int(p / (int64_t(n) * n)), y = int((p / n) % n), x = int(p % n);
  mask[p] = (z < (g.nz >> node_zshift(g.wd, g.L)) && y < (n >> g.L) && x < (n >> g.L)) ? 1 : 0;
}

// slices 1 .. nz-1 of the mask take slice 0 (wd = 2: one tree shared by every slice)
__global__ void k3_bcast_slice0(DevGeom3 g, uint8_t* __restrict__ mask) {
  const int64_t nn = int64_t(g.n) * g.n;
  const int64_t p = nn + int64_t(blockIdx.x) * kB + threadIdx.x;
  if (p >= nn * g.nz) return;
  mask[p] = mask[p % nn];
}

// ------------------------------------------------------------------ forward (leaf walk)

// Octree leaf walk of one ray (cubes of side 2^l voxels, l from the voxel's record). The walk
// runs in a frame mirrored per axis so that every direction component is >= 0 (leaf
// boundaries stay aligned since 2^l divides n and nz): a leaf is left through the nearest of
// its three upper faces; the crossed axis steps to the neighbouring leaf, the two others take
// the exit point's voxel, clamped into the old leaf's range and never moving backwards.
// Voxel indices fit in 32 bits (n, nz <= 512). WD = 2: leaves are 2^l x 2^l x 1 blocks of
// one slice (their z face is the voxel's).
template <int WD>
struct Walker3 {
  double x0, y0, z0;   // mirrored voxel coordinates of the ray at t = 0
  double ux, uy, uz;   // voxels per unit t along each axis
  double kx, ky, kz;   // t per voxel along each axis
  double cx, cy, cz;   // t at mirrored coordinate 0
  double cx1, cy1, cz1;  // t at mirrored coordinate 1
  double t, t_out;
  int x, y, z;         // current voxel, mirrored frame
  int xx, xy, xz;      // real index = (mirrored ^ x) + a: (0, 0), or (-1, size) for size - 1 - mirrored
  int ax, ay, az;
  int n, nz;

  __device__ bool init(const DevGeom3& g, const Ray3& q) {
    n = g.n; nz = g.nz;
    const double ipix = 1.0 / g.pixel;
    const double X = q.X, Y = q.Y, Z = q.Z;
    const double ex = q.ex, ey = q.ey, ez = q.ez, iex = q.iex, iey = q.iey, iez = q.iez;
    x0 = ex < 0.0 ? double(n) - X : X;
    y0 = ey < 0.0 ? double(n) - Y : Y;
    z0 = ez < 0.0 ? double(nz) - Z : Z;
    ux = fabs(ex) * ipix; uy = fabs(ey) * ipix; uz = fabs(ez) * ipix;
    kx = fabs(iex) * g.pixel; ky = fabs(iey) * g.pixel; kz = fabs(iez) * g.pixel;
    xx = ex < 0.0 ? -1 : 0; ax = ex < 0.0 ? n : 0;
    xy = ey < 0.0 ? -1 : 0; ay = ey < 0.0 ? n : 0;
    xz = ez < 0.0 ? -1 : 0; az = ez < 0.0 ? nz : 0;
    cx = -x0 * kx; cy = -y0 * ky; cz = -z0 * kz;
    cx1 = cx + kx; cy1 = cy + ky; cz1 = cz + kz;
    const double t_in = fmax(fmax(cx, cy), cz);
    t_out = fmin(fmin((double(n) - x0) * kx, (double(n) - y0) * ky), (double(nz) - z0) * kz);
    if (!(t_out > t_in)) return false;
    t = t_in;
    x = min(max(int(fma(t_in, ux, x0)), 0), n - 1);
    y = min(max(int(fma(t_in, uy, y0)), 0), n - 1);
    z = min(max(int(fma(t_in, uz, z0)), 0), nz - 1);
    return true;
  }
  int i0, dx, dy, dz;  // record index = i0 + dx x + dy y + dz z (mirrored voxel), see layout
  __device__ int real_x(int m) const { return (m ^ xx) + ax; }
  __device__ int real_y(int m) const { return (m ^ xy) + ay; }
  __device__ int real_z(int m) const { return (m ^ xz) + az; }
  __device__ int rx() const { return real_x(x); }
  __device__ int ry() const { return real_y(y); }
  __device__ int rz() const { return real_z(z); }
  // Per-voxel arrays in [z][x][y] (x-major) or [z][y][x] order: along each axis the real index
  // is c + s m of the mirrored one (c = 0, s = 1, or c = size - 1, s = -1), so the flat index
  // is linear in the mirrored coordinates with signed per-ray strides.
  __device__ void layout(bool xmaj) {
    const int cxr = ax + xx, cyr = ay + xy, czr = az + xz;
    const int sx = 2 * xx + 1, sy = 2 * xy + 1, sz = 2 * xz + 1;
    i0 = xmaj ? (czr * n + cxr) * n + cyr : (czr * n + cyr) * n + cxr;
    dx = xmaj ? sx * n : sx;
    dy = xmaj ? sy : sy * n;
    dz = sz * n * n;
  }
  // flat index of mirrored voxel (x, y, z), clamped into the volume (a walk's last step may
  // leave it)
  __device__ unsigned index(int x_, int y_, int z_) const {
    return unsigned(i0 + __mul24(dx, min(x_, n - 1)) + __mul24(dy, min(y_, n - 1)) + __mul24(dz, min(z_, nz - 1)));
  }
  // Leaves the current leaf (level l): chord = parameter length inside it; returns whether the
  // walk goes on (then x, y, z is a voxel of the next leaf; else possibly out of range).
  __device__ bool step(int l, double& chord) {
    const int m = (1 << l) - 1;
    // last voxel of the leaf along each axis (leaf boundaries are multiples of 2^l)
    const int hx = x | m, hy = y | m, hz = WD == 3 ? (z | m) : z;
    const double tX = fma(double(hx), kx, cx1), tY = fma(double(hy), ky, cy1);
    const double tZ = fma(double(hz), kz, cz1);
    const bool ax0 = tX <= tY && tX <= tZ;
    const bool ax1 = !ax0 && tY <= tZ;
    // the leaf's faces lie inside the volume, so te <= t_out and te >= t up to rounding (a
    // chord of an ulp below 0 where the ray passes an edge; the voxel indices never move
    // backwards and the index test below ends the walk at the volume's faces)
    const double te = fmin(tX, fmin(tY, tZ));
    chord = te - t;
    int nx = min(max(int(fma(te, ux, x0)), x), hx);
    int ny = min(max(int(fma(te, uy, y0)), y), hy);
    int nzv = min(max(int(fma(te, uz, z0)), z), hz);
    // the crossed axis moves to the next leaf (the clamped exit voxel there is hx, hy or hz):
    // every step adds one to one index and lowers none, so a walk that stops once an index
    // leaves the volume ends after at most 2 n + nz steps, for any leaf levels below 32
    nx += int(ax0);
    ny += int(ax1);
    nzv += int(!ax0 && !ax1);
    t = te; x = nx; y = ny; z = nzv;
    return te < t_out && nx < n && ny < n && nzv < nz;
  }
};

// Per ray: p = sum over the leaves crossed of chord * leaf value; then Beer's law and the FP64
// I-divergence term. x-major rays read the [z][x][y] records (neighbouring lanes,
// neighbouring rays of a detector row, then touch neighbouring addresses).
template <typename T, int WD>
__global__ __launch_bounds__(kB) void k3_forward(DevGeom3 g, RayF3 f,
                                                 const Rec3<T>* __restrict__ recR, const Rec3<T>* __restrict__ recC,
                                                 const T* __restrict__ d, const T* __restrict__ i0v,
                                                 const double* __restrict__ i0s, T* __restrict__ q,
                                                 T* __restrict__ pout, double* __restrict__ part) {
  const int blk = xcd_rotate(blockIdx.x, kRotate3);
  const int64_t k = int64_t(blk) * kB + threadIdx.x;
  const int64_t M = int64_t(g.nv) * g.nr * g.nc;
  double term = 0.0;
  if (k < M) {
    const int64_t r = row_major_ray(g, k);
    const Ray3 ray = ray_from_factors(g, f, r);
    Walker3<WD> w;
    double acc = 0.0;
    if (w.init(g, ray)) {
      const int n = g.n;
      const bool xmaj = fabs(ray.ex) >= fabs(ray.ey);
      const Rec3<T>* __restrict__ base = xmaj ? recC : recR;
      w.layout(xmaj);
      Rec3<T> rec = base[w.index(w.x, w.y, w.z)];
      for (;;) {   // ends within 2 n + nz steps (Walker3::step)
        double chord;
        const bool go = w.step(int(rec.lev()), chord);
        const Rec3<T> nrec = base[w.index(w.x, w.y, w.z)];
        acc += chord * double(rec.mu());
        if (!go) break;
        rec = nrec;
      }
    }
    if (pout) pout[r] = T(acc);
    if (q) {
      const double i0 = i0v ? double(i0v[r]) : *i0s;
      const double qd = i0 * exp(-acc);
      q[r] = T(qd);
      const double dv = double(d[r]);
      term = qd - dv;
      if (dv > 0.0) term += dv * (log(dv) - (log(i0) - acc));
    }
  }
  if (part) {
    term = breduce<false>(term);
    if (threadIdx.x == 0) part[blk] = term;
  }
}

// ------------------------------------------------------------------ node-driven gather

template <typename R>
struct Sums3 {
  R v[kSlots3];   // [0] plain sum, [1 + d] signed sum of detail d, [8 + d] sum of its magnitudes
};

// Rays of one view, factorised: every ray of view v leaves the source S = sod (c, s, 0)
// along D = (-sdd c - u s, -sdd s + u c, w) (u: column offset, w: row offset on the
// detector), so the parameter of the plane x = X is (X - Sx) / Dx with 1/Dx, 1/Dy per
// (view, column) and 1/Dz per row. Parameter differences are lengths / |D|, and
// |D| = sqrt(sdd^2 + u^2 + w^2) depends on (row, column) only; the ray values are scaled by
// |D| before the gather. A component within 1e-12 sdd of 0 gets the reciprocal +-1e300 (a
// line parallel to that axis: inside a slab or not, as decided by the source's coordinate).
__device__ inline double inv_or_big(double x, double scale) {
  return fabs(x) < 1e-12 * scale ? (x < 0.0 ? -1e300 : 1e300) : 1.0 / x;
}

__global__ __launch_bounds__(kB) void k3_ray_factors(DevGeom3 g, const double2* __restrict__ views,
                                                     double2* __restrict__ colt, double* __restrict__ rowt,
                                                     double* __restrict__ nrm) {
  const int64_t t = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int64_t nvc = int64_t(g.nv) * g.nc, nrc = int64_t(g.nr) * g.nc;
  if (t < nvc) {
    const int v = int(t / g.nc), col = int(t - int64_t(v) * g.nc);
    const double c = views[v].x, s = views[v].y, u = (col - 0.5 * (g.nc - 1)) * g.cpitch;
    colt[t] = make_double2(inv_or_big(-g.sdd * c - u * s, g.sdd), inv_or_big(-g.sdd * s + u * c, g.sdd));
  }
  if (t < nrc) {
    const int row = int(t / g.nc), col = int(t - int64_t(row) * g.nc);
    const double u = (col - 0.5 * (g.nc - 1)) * g.cpitch, w = (row - 0.5 * (g.nr - 1)) * g.rpitch;
    nrm[t] = sqrt(g.sdd * g.sdd + u * u + w * w);
    if (col == 0) rowt[row] = inv_or_big(w, g.sdd);
  }
}

// out[ray] = y[ray] |D| (the ray values of the factorised gather)
template <typename T>
__global__ __launch_bounds__(kB) void k3_scale_rays(DevGeom3 g, const T* __restrict__ y,
                                                    const double* __restrict__ nrm, T* __restrict__ out) {
  const int64_t r = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int64_t nrc = int64_t(g.nr) * g.nc;
  if (r >= nrc * g.nv) return;
  out[r] = T(double(y[r]) * nrm[r % nrc]);
}

// Sums of one item over views [v0, v1). Per view the item box's eight corners are projected
// onto the detector (FP32 with the hardware reciprocal, widened by 1e-3 element) to bound the
// rows and columns whose rays can cross it; per such ray the parameter interval of the box
// comes from slab clipping in FP64 (z slabs once per row), and the seven detail values (the
// 2x2x2 Haar combinations of the octant chords) from the box interval and the ray's three
// mid-plane crossings. Per detail the signed sum S and the sum of magnitudes A are kept: the
// positive part is (A + S) / 2 and the negative part (S - A) / 2 (per (ray, coefficient) sign
// split, eq. 1.10).
// WD = 2 (2-D Haar per slice): the node box is one voxel deep, split nodes take the three
// details of its four quadrants (one z slab, the x and y crossings; scale 2^-l).
template <typename T, bool SPLIT, int WD>
__device__ inline Sums3<double> item_sums3(const DevGeom3& g, const double2* __restrict__ views,
                                           const double2* __restrict__ colt, const double* __restrict__ rowt,
                                           const T* __restrict__ y, int l, int k, int i, int j, int v0, int v1) {
  const int n = g.n, nz = g.nz, s = 1 << l, sz = WD == 3 ? s : 1;
  const double pix = g.pixel, hn = 0.5 * n, hz = 0.5 * nz;
  const double X0 = (double(j * s) - hn) * pix, X2 = (double((j + 1) * s) - hn) * pix;
  const double Y0 = (double(i * s) - hn) * pix, Y2 = (double((i + 1) * s) - hn) * pix;
  const double Z0 = (double(k * sz) - hz) * pix, Z2 = (double((k + 1) * sz) - hz) * pix;
  const double X1 = 0.5 * (X0 + X2), Y1 = 0.5 * (Y0 + Y2), Z1 = 0.5 * (Z0 + Z2);
  const float sod = float(g.sod), sdd = float(g.sdd);
  const float icp = float(1.0 / g.cpitch), irp = float(1.0 / g.rpitch);
  const float cc0 = float(0.5 * (g.nc - 1)), rc0 = float(0.5 * (g.nr - 1));
  // |phi| <= 1e-12 pixel is rounding residue of chord differences, taken as 0 (phi is
  // 2^(-3l/2) times the butterfly outputs, in parameter units of the unnormalised ray
  // direction: chords there are mm / |D|, and |D| >= sdd)
  const double tq = 1e-12 * g.pixel / scale_w<WD>(l) / g.sdd;
  Sums3<double> r;
#pragma unroll
  for (int q = 0; q < kSlots3; ++q) r.v[q] = 0.0;
  for (int v = v0; v < v1; ++v) {
    const double2 cs = views[v];
    const float c = float(cs.x), sn = float(cs.y);
    float umin = 1e30f, umax = -1e30f, wmin = 1e30f, wmax = -1e30f;
#pragma unroll
    for (int corner = 0; corner < 8; ++corner) {
      const float px = float((corner & 1) ? X2 : X0), py = float((corner & 2) ? Y2 : Y0);
      const float pz = float((corner & 4) ? Z2 : Z0);
      const float depth = sod - (px * c + py * sn);                  // distance from the source along the axis
      const float f = sdd * __builtin_amdgcn_rcpf(depth);
      const float u = (-px * sn + py * c) * f, w = pz * f;
      umin = fminf(umin, u); umax = fmaxf(umax, u); wmin = fminf(wmin, w); wmax = fmaxf(wmax, w);
    }
    const float fc0 = fminf(fmaxf(umin * icp + cc0 - 1e-3f, -1.f), float(g.nc));
    const float fc1 = fminf(fmaxf(umax * icp + cc0 + 1e-3f, -1.f), float(g.nc));
    const float fr0 = fminf(fmaxf(wmin * irp + rc0 - 1e-3f, -1.f), float(g.nr));
    const float fr1 = fminf(fmaxf(wmax * irp + rc0 + 1e-3f, -1.f), float(g.nr));
    const int clo = max(int(ceilf(fc0)), 0), chi = min(int(floorf(fc1)), g.nc - 1);
    const int rlo = max(int(ceilf(fr0)), 0), rhi = min(int(floorf(fr1)), g.nr - 1);
    const double Sx = g.sod * cs.x, Sy = g.sod * cs.y;
    const double ax0 = X0 - Sx, ax1 = X1 - Sx, ax2 = X2 - Sx;
    const double ay0 = Y0 - Sy, ay1 = Y1 - Sy, ay2 = Y2 - Sy;
    const double2* __restrict__ cv = colt + int64_t(v) * g.nc;
    for (int row = rlo; row <= rhi; ++row) {
      const double iz = rowt[row];
      const double tz0 = Z0 * iz, tz2 = Z2 * iz;
      const T* __restrict__ yr = y + (int64_t(v) * g.nr + row) * g.nc;
      if (!SPLIT) {
        const double zlo = fmin(tz0, tz2), zhi = fmax(tz0, tz2);
        const auto chord = [&](double2 cd) {
          const double tx0 = ax0 * cd.x, tx2 = ax2 * cd.x, ty0 = ay0 * cd.y, ty2 = ay2 * cd.y;
          const double lo = fmax(fmax(fmin(tx0, tx2), fmin(ty0, ty2)), zlo);
          const double hi = fmin(fmin(fmax(tx0, tx2), fmax(ty0, ty2)), zhi);
          return hi - lo;
        };
        // columns four at a time with all eight loads issued before the first use (one
        // memory wait per four rays instead of two per ray); sums in column order
        int col = clo;
        for (; col + 3 <= chi; col += 4) {
          double2 cd[4];
          T yy[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) { cd[u] = cv[col + u]; yy[u] = yr[col + u]; }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double chd = chord(cd[u]);
            r.v[0] += chd > tq ? double(yy[u]) * chd : 0.0;
          }
        }
        for (; col <= chi; ++col) {
          const double chd = chord(cv[col]);
          r.v[0] += chd > tq ? double(yr[col]) * chd : 0.0;
        }
        continue;
      }
      // Per ray: the box's parameter interval [lo, hi] and the mid-plane crossings clamped
      // into it. Along an axis the ray is in the lower half on one side of its crossing c
      // (before c when it moves up that axis, after c otherwise), so the signed length of a
      // product of half indicators (+ lower, - upper) is a sum of lengths between the sorted
      // crossings: one axis s (2 c - lo - hi), two axes s s' (hi - lo - 2 |c - c'|), three
      // axes s s' s'' (2 (c1 - c2 + c3) - lo - hi) with c1 <= c2 <= c3 and s the sign of the
      // ray's direction along the axis. These are the butterfly outputs of the octant chords
      // without forming the chords.
      const double zlo = fmin(tz0, tz2), zhi = fmax(tz0, tz2);
      const double tz1 = WD == 3 ? Z1 * iz : 0.0;
      for (int col = clo; col <= chi; ++col) {
        const double2 cd = cv[col];
        const double tx0 = ax0 * cd.x, tx1 = ax1 * cd.x, tx2 = ax2 * cd.x;
        const double ty0 = ay0 * cd.y, ty1 = ay1 * cd.y, ty2 = ay2 * cd.y;
        const double lo = fmax(fmax(fmin(tx0, tx2), fmin(ty0, ty2)), zlo);
        const double hi = fmin(fmin(fmax(tx0, tx2), fmax(ty0, ty2)), zhi);
        const double box = hi - lo;
        // a ray that misses the box (or grazes it within the residue) adds nothing; the values
        // below stay finite for it and are multiplied by 0
        const double yl = double(yr[col]);
        const double yv = box > tq ? yl : 0.0;
        const double cx = fmin(fmax(tx1, lo), hi), cy = fmin(fmax(ty1, lo), hi);
        const double lh = lo + hi;
        const double sxy = xsign(cd.x, cd.y);   // sign of the product of the x and y directions
        double det[7];
        det[0] = xsign(2.0 * cx - lh, cd.x);
        det[1] = xsign(2.0 * cy - lh, cd.y);
        det[2] = xsign(box - 2.0 * fabs(cx - cy), sxy);
        if (WD == 3) {
          const double cz = fmin(fmax(tz1, lo), hi);
          const double med = fmax(fmin(cx, cy), fmin(fmax(cx, cy), cz));
          det[3] = xsign(2.0 * cz - lh, iz);
          det[4] = xsign(xsign(box - 2.0 * fabs(cx - cz), cd.x), iz);
          det[5] = xsign(xsign(box - 2.0 * fabs(cy - cz), cd.y), iz);
          det[6] = xsign(xsign(2.0 * (cx + cy + cz - 2.0 * med) - lh, sxy), iz);
        }
        r.v[0] += yv * box;
#pragma unroll
        for (int d = 0; d < n_details<WD>(); ++d) {
          const double wv = fabs(det[d]) > tq ? yv * det[d] : 0.0;
          r.v[1 + d] += wv;
          r.v[8 + d] += fabs(wv);
        }
      }
    }
  }
  return r;
}

// am_delta as in 2-D (eq. 1.9 zero; held when no finite minimizer)
__device__ inline double am_delta3(double b, double bp, double bm, double z0, int* held) {
  double t;
  if (bp > 0.0) {
    const double sq = sqrt(fmax(b * b - 4.0 * bp * bm, 0.0));
    t = b >= 0.0 ? (b + sq) / (2.0 * bp) : (2.0 * bm) / (b - sq);
  } else if (bm < 0.0) {
    t = bm / b;
  } else {
    return 0.0;
  }
  if (t > 0.0 && isfinite(t)) return -log(t) / z0;
  atomicAdd(held, 1);
  return 0.0;
}

template <typename T>
struct GArgs3 {
  DevGeom3 g;
  const double2* views;
  const double2* colt;
  const double* rowt;
  const T* y;
  const uint32_t* items;
  const int* counts;
  int kseg, start, count, chunks, vpc;
  double* part;
  T* beta;
  const T* b;
  const double* z0;
  int* held;
  T *bp, *bm, *out;
};

__device__ inline uint32_t item3_word(const uint32_t* __restrict__ items, int64_t it, int n) {
  if (items) return items[it];
  // every voxel as a level-0 box
  const int64_t nn = int64_t(n) * n;
  return item3_pack(0, 0, int(it / nn), int((it / n) % n), int(it % n));
}

template <typename T>
__device__ inline void seg_range3(const GArgs3<T>& a, int& start, int& count) {
  start = a.start;
  count = a.count;
  if (a.counts) {
    start = 0;
    for (int q = 0; q < a.kseg; ++q) start += a.counts[q];
    count = a.counts[a.kseg];
  }
}

template <typename T, int MODE, int WD>
__device__ inline void item_finish3(const GArgs3<T>& a, uint32_t w, const Sums3<double>& r) {
  const int n = a.g.n, nz = a.g.nz;
  const bool split = (w >> 31) != 0;
  const int l = int((w >> 27) & 15u);
  const int k = int((w >> 18) & 0x1ffu), i = int((w >> 9) & 0x1ffu), j = int(w & 0x1ffu);
  const double sc = scale_w<WD>(l);
  const int64_t root = (int64_t(k) * n + i) * n + j;
  if (MODE == kPlain) {
    a.out[root] = T(r.v[0] * sc);
    return;
  }
  const bool is_root = l == a.g.L;
  if (MODE == kSplit) {
    if (is_root) { a.bp[root] = T(r.v[0] * sc); a.bm[root] = T(0); }
    if (split)
      for (int d = 0; d < n_details<WD>(); ++d) {
        const int64_t z = detail_pos(n, nz, l, d, k, i, j);
        a.bp[z] = T(0.5 * (r.v[8 + d] + r.v[1 + d]) * sc);
        a.bm[z] = T(0.5 * (r.v[1 + d] - r.v[8 + d]) * sc);
      }
    return;
  }
  const double z0 = *a.z0;
  if (is_root) a.beta[root] = T(double(a.beta[root]) + am_delta3(double(a.b[root]), r.v[0] * sc, 0.0, z0, a.held));
  if (split)
    for (int d = 0; d < n_details<WD>(); ++d) {
      const int64_t z = detail_pos(n, nz, l, d, k, i, j);
      const double bp = 0.5 * (r.v[8 + d] + r.v[1 + d]) * sc, bm = 0.5 * (r.v[1 + d] - r.v[8 + d]) * sc;
      a.beta[z] = T(double(a.beta[z]) + am_delta3(double(a.b[z]), bp, bm, z0, a.held));
    }
}

template <typename T, int MODE, bool SPLIT, int WD>
__global__ __launch_bounds__(kB) void k3_gather(GArgs3<T> a) {
  int start, count;
  seg_range3(a, start, count);
  const int it = xcd_unit3(blockIdx.x, gridDim.x) * kB + threadIdx.x;
  if (it >= count) return;
  const uint32_t w = item3_word(a.items, start + it, a.g.n);
  const Sums3<double> r = item_sums3<T, SPLIT, WD>(a.g, a.views, a.colt, a.rowt, a.y, int((w >> 27) & 15u),
                                                   int((w >> 18) & 0x1ffu), int((w >> 9) & 0x1ffu), int(w & 0x1ffu),
                                                   0, a.g.nv);
  item_finish3<T, MODE, WD>(a, w, r);
}

// (item, view chunk) tasks: a block of 4 waves takes 64 items; wave w handles view chunk
// 4 group + w; the four chunk sums are added in LDS in wave order and stored per group.
// Capped at 128 VGPRs (4 waves per SIMD instead of 3; a few values spill): measured 3 %
// faster on the 512x512x256 cone update.
template <typename T, bool SPLIT, int WD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k3_gather_part(GArgs3<T> a) {
  __shared__ double sh[4][kSlots3][64];
  int start, count;
  seg_range3(a, start, count);
  // Block 8 j + x runs on XCD x (round-robin dispatch): it takes view-chunk group j / per and
  // item group x per + j mod per (item groups padded to 8 per, the padding without items), so
  // at any time an XCD works on one compact region of the volume, whose rays overlap in its L2
  const int n_ig = (a.count + 63) / 64, per = (n_ig + 7) >> 3;
  const int jj = int(blockIdx.x >> 3);
  const int group = jj / per, ig = int(blockIdx.x & 7) * per + jj % per;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int idx = ig * 64 + lane, chunk = group * 4 + wv;
  Sums3<double> r;
#pragma unroll
  for (int q = 0; q < kSlots3; ++q) r.v[q] = 0.0;
  if (idx < count && chunk < a.chunks) {
    const uint32_t w = item3_word(a.items, start + idx, a.g.n);
    const int v0 = chunk * a.vpc, v1 = min(a.g.nv, v0 + a.vpc);
    r = item_sums3<T, SPLIT, WD>(a.g, a.views, a.colt, a.rowt, a.y, int((w >> 27) & 15u), int((w >> 18) & 0x1ffu),
                                 int((w >> 9) & 0x1ffu), int(w & 0x1ffu), v0, v1);
  }
#pragma unroll
  for (int q = 0; q < kSlots3; ++q) sh[wv][q][lane] = r.v[q];
  __syncthreads();
  for (int t = threadIdx.x; t < kSlots3 * 64; t += 256) {
    const int slot = t / 64, l2 = t % 64;
    const int it = ig * 64 + l2;
    if (it >= count) continue;
    a.part[(size_t(group) * kSlots3 + slot) * a.count + it] = sh[0][slot][l2] + sh[1][slot][l2] + sh[2][slot][l2] +
                                                               sh[3][slot][l2];
  }
}

// adds the chunk groups of each item in group order, then the item's final step
template <typename T, int MODE, int WD>
__global__ __launch_bounds__(1024) void k3_gather_finish(GArgs3<T> a) {
  __shared__ double sh[kSlots3][64];
  int start, count;
  seg_range3(a, start, count);
  const int lane = threadIdx.x & 63, slot = threadIdx.x >> 6;
  const int idx = blockIdx.x * 64 + lane;
  const int groups = (a.chunks + 3) / 4;
  if (slot < kSlots3) {
    sh[slot][lane] = idx < count ? ordered_sum(a.part + size_t(slot) * a.count + idx, groups,
                                               size_t(kSlots3) * a.count)
                                 : 0.0;
  }
  __syncthreads();
  if (slot != 0 || idx >= count) return;
  const uint32_t w = item3_word(a.items, start + idx, a.g.n);
  Sums3<double> r;
#pragma unroll
  for (int q = 0; q < kSlots3; ++q) r.v[q] = sh[q][lane];
  item_finish3<T, MODE, WD>(a, w, r);
}

// ------------------------------------------------------------------ Z0 and W (eq. 1.61)

__device__ inline double flip_sign(double v, int neg) {
  return __longlong_as_double(__double_as_longlong(v) ^ (static_cast<long long>(neg) << 63));
}

// Per ray in FP64: walk the octree leaves; every leaf chord adds sign_d(octant) * chord to
// the seven signed detail sums of each split ancestor, and chord to its root's approximation
// sum; when the ray leaves a node (a bit at or above the node's level differs between the
// voxels of consecutive leaves), 2^(-3m/2) |sum| of its details enter the ray's total and
// the non-zero ones are counted (threshold 1e-9 pixel on the scaled value). Z0 = max over
// rays of the totals, W = total count.
// WD = 2 (2-D Haar per slice): three details per node (the types with tz = 0), scale 2^-m,
// and a node belongs to one slice: a change of slice starts new nodes at every level.
template <int LT, int WD>
struct Z0Vis3 {
  static constexpr int ND = WD == 3 ? 7 : 3;
  double tolm[LT + 1];     // count threshold per level, unscaled (index 0: root approximations)
  double sc[LT + 1];       // scale of the level-m basis (index 0: scale of level LT, the roots)
  double acc[LT + 1][ND];
  double accLL;
  double sum;
  int cnt;
  int dirty;               // bit m: acc[m] holds chords of the current level-m node
  int px, py, pz;          // voxel of the previous leaf (all bits set before the first)
  __device__ void flush(int m) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const double a = fabs(acc[m][d]);
      sum = fma(a, sc[m], sum);
      cnt += a > tolm[m] ? 1 : 0;
      acc[m][d] = 0.0;
    }
  }
  __device__ void flushLL() {
    sum = fma(accLL, sc[0], sum);
    cnt += accLL > tolm[0] ? 1 : 0;
    accLL = 0.0;
  }
  __device__ void visit(int ix, int iy, int iz, int l, double chord) {
    const int dif = WD == 3 ? (ix ^ px) | (iy ^ py) | (iz ^ pz) : ((ix ^ px) | (iy ^ py) | (iz != pz ? ~0 : 0));
    px = ix; py = iy; pz = iz;
#pragma unroll
    for (int m = 1; m <= LT; ++m) {
      // a new node at level m: its sums enter the total (untouched sums are zero: nothing to add)
      if ((dif >> m) && (dirty >> m & 1)) {
        flush(m);
        dirty &= ~(1 << m);
      }
      if (m > l) {
        dirty |= 1 << m;
        const int bx = (ix >> (m - 1)) & 1, by = (iy >> (m - 1)) & 1;
        const double cx = flip_sign(chord, bx), cy = flip_sign(chord, by), cxy = flip_sign(cx, by);
        acc[m][0] += cx;                    // types (tz, ty, tx) = 001 .. 111
        acc[m][1] += cy;
        acc[m][2] += cxy;
        if (WD == 3) {
          const int bz = (iz >> (m - 1)) & 1;
          acc[m][3 % ND] += flip_sign(chord, bz);
          acc[m][4 % ND] += flip_sign(cx, bz);
          acc[m][5 % ND] += flip_sign(cy, bz);
          acc[m][6 % ND] += flip_sign(cxy, bz);
        }
      }
    }
    if (dif >> LT) flushLL();
    accLL += chord;
  }
};

template <int LT, int WD>
__global__ __launch_bounds__(kB) void k3_z0(DevGeom3 g, RayF3 f, const uint8_t* __restrict__ lev,
                                            const uint8_t* __restrict__ levC, double* __restrict__ part_max,
                                            double* __restrict__ part_cnt) {
  const int blk = xcd_rotate(blockIdx.x, kRotate3);
  const int64_t k = int64_t(blk) * kB + threadIdx.x;
  const int64_t M = int64_t(g.nv) * g.nr * g.nc;
  double sum = 0.0, cnt = 0.0;
  if (k < M) {
    const int64_t r = row_major_ray(g, k);
    const Ray3 ray = ray_from_factors(g, f, r);
    Z0Vis3<LT, WD> z;
    const double tol = 1e-9 * g.pixel;
    z.sum = 0.0; z.cnt = 0; z.accLL = 0.0; z.dirty = 0;
    z.px = z.py = z.pz = -1;
    z.sc[0] = scale_w<WD>(LT);
    z.tolm[0] = tol / z.sc[0];
#pragma unroll
    for (int m = 1; m <= LT; ++m) {
      z.sc[m] = scale_w<WD>(m);
      z.tolm[m] = tol / z.sc[m];
#pragma unroll
      for (int d = 0; d < Z0Vis3<LT, WD>::ND; ++d) z.acc[m][d] = 0.0;
    }
    Walker3<WD> w;
    if (w.init(g, ray)) {
      const int n = g.n;
      // x-major rays read the [z][x][y] level map (neighbouring lanes, neighbouring addresses)
      const bool xmaj = fabs(ray.ex) >= fabs(ray.ey);
      const uint8_t* __restrict__ lv = xmaj ? levC : lev;
      // leaf level at mirrored voxel (x, y, z), clamped into range (past the last leaf the
      // value is loaded and not used)
      w.layout(xmaj);
      auto level = [&](int x, int y, int zz) {
        if (LT == 0) return 0;
        return int(lv[w.index(x, y, zz)]);
      };
      int l = level(w.x, w.y, w.z);
      for (;;) {   // ends within 2 n + nz steps (Walker3::step)
        const int ix = w.rx(), iy = w.ry(), iz = w.rz();
        double chord;
        const bool go = w.step(l, chord);
        const int ln = level(w.x, w.y, w.z);   // the next leaf's level, in flight during the visit
        z.visit(ix, iy, iz, l, chord);
        if (!go) break;
        l = ln;
      }
#pragma unroll
      for (int m = 1; m <= LT; ++m) z.flush(m);
      z.flushLL();
    }
    sum = z.sum;
    cnt = double(z.cnt);
  }
  const double mx = breduce<true>(sum);
  __syncthreads();
  const double ct = breduce<false>(cnt);
  if (threadIdx.x == 0) { part_max[blk] = mx; part_cnt[blk] = ct; }
}

// ------------------------------------------------------------------ tree rule and work lists

// Leaf scores of the residual-gradient rule: for every leaf node the largest |c| of its seven
// would-be details (c = Omega^T H^T (d - q-hat)), stored at its first detail position.
template <typename T>
__global__ __launch_bounds__(kB) void k3_grad_scores(DevGeom3 g, const uint8_t* __restrict__ mask,
                                                     const T* __restrict__ coef, double* __restrict__ score) {
  int64_t k = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int n = g.n, nz = g.nz;
  int l = 1;
  for (; l <= g.L; ++l) {
    const int64_t cntl = int64_t(nz >> l) * (n >> l) * (n >> l);
    if (k < cntl) break;
    k -= cntl;
  }
  if (l > g.L) return;
  const int m = n >> l;
  const int kz = int(k / (int64_t(m) * m)), i = int((k / m) % m), j = int(k % m);
  if (split3(mask, n, l, kz, i, j)) return;
  if (l < g.L && !split3(mask, n, l + 1, kz >> 1, i >> 1, j >> 1)) return;
  double sc = 0.0;
#pragma unroll
  for (int d = 0; d < 7; ++d) sc = fmax(sc, fabs(double(coef[detail_pos(n, nz, l, d, kz, i, j)])));
  score[detail_pos(n, nz, l, 0, kz, i, j)] = sc;
}

// Tree rule: rule 0 (Results) on the leaf-constant FP64 image mu64, rule 1 (residual
// gradient) on the leaf scores held in mu64 at each node's first detail position.
__global__ __launch_bounds__(kB) void k3_expand(DevGeom3 g, const uint8_t* __restrict__ old,
                                                uint8_t* __restrict__ mask, const double* __restrict__ mu64,
                                                const double* __restrict__ maxv, double frac,
                                                int* __restrict__ n_split, int rule) {
  int64_t k = int64_t(blockIdx.x) * kB + threadIdx.x;
  const int n = g.n, nz = g.nz;
  int l = 1;
  for (; l <= g.L; ++l) {
    const int64_t cntl = int64_t(nz >> l) * (n >> l) * (n >> l);
    if (k < cntl) break;
    k -= cntl;
  }
  if (l > g.L) return;
  const double top = *maxv;
  if (!(top > 0.0)) return;
  const int m = n >> l;
  const int kz = int(k / (int64_t(m) * m)), i = int((k / m) % m), j = int(k % m);
  if (split3(old, n, l, kz, i, j)) return;
  if (l < g.L && !split3(old, n, l + 1, kz >> 1, i >> 1, j >> 1)) return;
  const int s = 1 << l;
  const double val = rule == 0 ? mu64[(int64_t(kz * s) * n + i * s) * n + j * s]   // leaf-constant
                               : mu64[detail_pos(n, nz, l, 0, kz, i, j)];
  if (val > frac * top) {
    for (int d = 0; d < 7; ++d) mask[detail_pos(n, nz, l, d, kz, i, j)] = 1;
    atomicAdd(n_split, 1);
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

template <typename T>
int Geo3<T>::forward(const DevGeom3& g, const RayF3& f, const void* recR, const void* recC, const T* d,
                     const T* i0v, const double* i0s, T* q, T* p, double* part, hipStream_t s) {
  const int nb = xcd_blocks(blocks3(int64_t(g.nv) * g.nr * g.nc));
  if (g.wd == 2)
    hipLaunchKernelGGL((k3_forward<T, 2>), dim3(nb), dim3(kB), 0, s, g, f, (const Rec3<T>*)recR, (const Rec3<T>*)recC,
                       d, i0v, i0s, q, p, part);
  else
    hipLaunchKernelGGL((k3_forward<T, 3>), dim3(nb), dim3(kB), 0, s, g, f, (const Rec3<T>*)recR, (const Rec3<T>*)recC,
                       d, i0v, i0s, q, p, part);
  return nb;
}
template <typename T>
void Geo3<T>::ray_factors(const DevGeom3& g, const double2* views, double2* colt, double* rowt, double* nrm,
                          hipStream_t s) {
  const int64_t t = std::max(int64_t(g.nv) * g.nc, int64_t(g.nr) * g.nc);
  hipLaunchKernelGGL(k3_ray_factors, dim3(blocks3(t)), dim3(kB), 0, s, g, views, colt, rowt, nrm);
}
template <typename T>
void Geo3<T>::scale_rays(const DevGeom3& g, const T* y, const double* nrm, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k3_scale_rays<T>, dim3(blocks3(int64_t(g.nv) * g.nr * g.nc)), dim3(kB), 0, s, g, y, nrm, out);
}
template <typename T, int MODE, bool SPLIT, int WD>
static void gather_seg3(const GArgs3<T>& a, const Segment& sg, hipStream_t s) {
  if (sg.chunks <= 1) {
    hipLaunchKernelGGL((k3_gather<T, MODE, SPLIT, WD>), dim3(xcd_pad3(blocks3(sg.count))), dim3(kB), 0, s, a);
    return;
  }
  const int groups = (sg.chunks + 3) / 4;
  const int per = ((sg.count + 63) / 64 + 7) >> 3;   // item groups per XCD (k3_gather_part)
  hipLaunchKernelGGL((k3_gather_part<T, SPLIT, WD>), dim3(8 * per * groups), dim3(256), 0, s, a);
  hipLaunchKernelGGL((k3_gather_finish<T, MODE, WD>), dim3((sg.count + 63) / 64), dim3(1024), 0, s, a);
}
template <typename T, int MODE>
static void gather_mode3(const GArgs3<T>& a, const Segment& sg, bool split, hipStream_t s) {
  if (a.g.wd == 2) {
    if (split) gather_seg3<T, MODE, true, 2>(a, sg, s);
    else gather_seg3<T, MODE, false, 2>(a, sg, s);
  } else {
    if (split) gather_seg3<T, MODE, true, 3>(a, sg, s);
    else gather_seg3<T, MODE, false, 3>(a, sg, s);
  }
}
template <typename T>
void Geo3<T>::gather(const DevGeom3& g, int mode, const double2* views, const double2* colt, const double* rowt,
                     const T* y, const uint32_t* items, const int* counts, const Segment* segs, int n_segs, void* part,
                     T* beta, const T* b, const double* z0, int* held, T* bp, T* bm, T* out, hipStream_t s) {
  GArgs3<T> a;
  a.g = g; a.views = views; a.colt = colt; a.rowt = rowt; a.y = y;
  a.items = items; a.counts = counts; a.part = (double*)part;
  a.beta = beta; a.b = b; a.z0 = z0; a.held = held; a.bp = bp; a.bm = bm; a.out = out;
  for (int k = 0; k < n_segs; ++k) {
    const Segment& sg = segs[k];
    if (sg.count <= 0) continue;
    a.kseg = sg.kseg; a.start = sg.start; a.count = sg.count; a.chunks = sg.chunks; a.vpc = sg.vpc;
    // work-list segment 1 holds the roots that are not split; every other segment of a
    // work list holds nodes with octant chords; no work list: voxels as plain boxes
    const bool split = items != nullptr && sg.kseg != 1;
    if (mode == kPlain) gather_mode3<T, kPlain>(a, sg, split, s);
    else if (mode == kSplit) gather_mode3<T, kSplit>(a, sg, split, s);
    else gather_mode3<T, kUpdate>(a, sg, split, s);
  }
}
template <typename T>
void Geo3<T>::synth_records(const DevGeom3& g, const T* beta, const uint8_t* lev, void* recR, void* recC,
                            hipStream_t s) {
  hipLaunchKernelGGL(k3_synth_records<T>, dim3(blocks3(int64_t(g.n) * g.n * g.nz)), dim3(kB), 0, s, g, beta, lev,
                     (Rec3<T>*)recR, (Rec3<T>*)recC);
}
template <typename T>
void Geo3<T>::synth(const DevGeom3& g, const T* beta, T* mu, hipStream_t s) {
  hipLaunchKernelGGL(k3_synth<T>, dim3(blocks3(int64_t(g.n) * g.n * g.nz)), dim3(kB), 0, s, g, beta, mu);
}
template <typename T>
int Geo3<T>::mu64(const DevGeom3& g, const T* beta, double* mu64, double* part, hipStream_t s) {
  const int nb = blocks3(int64_t(g.n) * g.n * g.nz);
  hipLaunchKernelGGL(k3_mu64<T>, dim3(nb), dim3(kB), 0, s, g, beta, mu64, part);
  return nb;
}
template <typename T>
void Geo3<T>::analysis(const DevGeom3& g, const T* vol, T* coef, hipStream_t s) {
  hipLaunchKernelGGL(k3_analysis<T>, dim3(blocks3(int64_t(g.n) * g.n * g.nz)), dim3(kB), 0, s, g, vol, coef);
}
template <typename T>
void Geo3<T>::apply_mask(const DevGeom3& g, T* beta, const uint8_t* mask, hipStream_t s) {
  const int64_t len = int64_t(g.n) * g.n * g.nz;
  hipLaunchKernelGGL(k3_apply_mask<T>, dim3(blocks3(len)), dim3(kB), 0, s, len, beta, mask);
}
template <typename T>
void Geo3<T>::grad_scores(const DevGeom3& g, const uint8_t* mask, const T* coef, double* score, hipStream_t s) {
  int64_t nodes = 0;
  for (int l = 1; l <= g.L; ++l) nodes += int64_t(g.nz >> l) * (g.n >> l) * (g.n >> l);
  if (nodes == 0) return;
  hipLaunchKernelGGL(k3_grad_scores<T>, dim3(blocks3(nodes)), dim3(kB), 0, s, g, mask, coef, score);
}
template struct Geo3<float>;
template struct Geo3<double>;

int z0_partials3(const DevGeom3& g, const RayF3& f, const uint8_t* lev, const uint8_t* levC, double* part_max,
                 double* part_cnt, hipStream_t s) {
  const int nb = xcd_blocks(blocks3(int64_t(g.nv) * g.nr * g.nc));
  switch (g.L) {
#define Z3_CASE(K)                                                                                        \
    case K:                                                                                               \
      if (g.wd == 2)                                                                                      \
        hipLaunchKernelGGL((k3_z0<K, 2>), dim3(nb), dim3(kB), 0, s, g, f, lev, levC, part_max, part_cnt); \
      else                                                                                                \
        hipLaunchKernelGGL((k3_z0<K, 3>), dim3(nb), dim3(kB), 0, s, g, f, lev, levC, part_max, part_cnt); \
      break;
    Z3_CASE(0) Z3_CASE(1) Z3_CASE(2) Z3_CASE(3) Z3_CASE(4)
#undef Z3_CASE
  }
  return nb;
}
void levmap3(const DevGeom3& g, const uint8_t* mask, uint8_t* lev, uint8_t* levC, hipStream_t s) {
  hipLaunchKernelGGL(k3_levmap, dim3(blocks3(int64_t(g.n) * g.n * g.nz)), dim3(kB), 0, s, g, mask, lev, levC);
}
namespace {
struct ListSpec3 {
  const uint8_t* mask;
  int n, nz, wd;
  __device__ bool keep(int, int l, int filter, int64_t code, uint32_t& word) const {
    const int j = int(morton3_compact(uint32_t(code)));
    const int i = int(morton3_compact(uint32_t(code >> 1)));
    const int k = int(morton3_compact(uint32_t(code >> 2)));
    const int m = n >> l, mz = nz >> node_zshift(wd, l);
    if (i >= m || j >= m || k >= mz) return false;
    const bool sp = l > 0 && split3(mask, n, l, k, i, j);
    word = item3_pack(sp ? 1 : 0, l, k, i, j);
    return filter == 2 || (filter == 0) == sp;
  }
};

// Segments (count slot 1 + segment): split roots, unsplit roots, then the split nodes of
// levels L - 1 .. 1; with L = 0 the first is empty and the second holds every voxel.
PassTable list_passes3(const DevGeom3& g) {
  PassTable pt{};
  const int L = g.L;
  const int n_seg = L >= 1 ? L + 1 : 2;
  for (int sgi = 0; sgi < n_seg; ++sgi) {
    const int l = sgi <= 1 ? L : L - (sgi - 1);
    const int m = g.n >> l, mz = g.nz >> node_zshift(g.wd, l);
    int pw = 1;
    while (pw < m || pw < mz) pw <<= 1;
    const int filter = sgi == 1 ? 1 : 0;
    const int64_t codes = (l == 0 && filter == 0) ? 0 : int64_t(pw) * pw * pw;
    add_pass(pt, l, filter, 1 + sgi, codes);
  }
  return pt;
}
}  // namespace

int64_t list_scratch_ints3(const DevGeom3& g) {
  const PassTable pt = list_passes3(g);
  return 2 * int64_t(pt.blk_start[pt.n_pass]);
}
void build_items3(const DevGeom3& g, const uint8_t* mask, uint32_t* items, int* counts, int* scratch,
                  hipStream_t s) {
  const PassTable pt = list_passes3(g);
  const int nblk = pt.blk_start[pt.n_pass];
  int* bcount = scratch;
  int* boff = scratch + nblk;
  const ListSpec3 sp{mask, g.n, g.nz, g.wd};
  hipLaunchKernelGGL(k_list_count<ListSpec3>, dim3(nblk, 1), dim3(kListThreads), 0, s, sp, pt, bcount);
  hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(kListThreads), 0, s, pt, bcount, boff, counts, kInts);
  hipLaunchKernelGGL(k_list_write<ListSpec3>, dim3(nblk, 1), dim3(kListThreads), 0, s, sp, pt, boff, items,
                     int64_t(0));
}
void expand3(const DevGeom3& g, const uint8_t* mask_old, uint8_t* mask, const double* mu64, const double* maxv,
             double frac, int* n_split, hipStream_t s, int rule) {
  int64_t nodes = 0;
  for (int l = 1; l <= g.L; ++l) nodes += int64_t(g.nz >> l) * (g.n >> l) * (g.n >> l);
  if (nodes == 0) return;
  hipLaunchKernelGGL(k3_expand, dim3(blocks3(nodes)), dim3(kB), 0, s, g, mask_old, mask, mu64, maxv, frac, n_split,
                     rule);
}
void check_mask3(const DevGeom3& g, const uint8_t* mask, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k3_check_mask, dim3(blocks3(int64_t(g.n) * g.n * g.nz)), dim3(kB), 0, s, g, mask, bad);
}
void broadcast_slice3(const DevGeom3& g, uint8_t* mask, hipStream_t s) {
  const int64_t rest = int64_t(g.n) * g.n * (g.nz - 1);
  if (rest > 0) hipLaunchKernelGGL(k3_bcast_slice0, dim3(blocks3(rest)), dim3(kB), 0, s, g, mask);
}
void approx_mask3(const DevGeom3& g, uint8_t* mask, hipStream_t s) {
  hipLaunchKernelGGL(k3_approx_mask, dim3(blocks3(int64_t(g.n) * g.n * g.nz)), dim3(kB), 0, s, g, mask);
}

}  // namespace wamct
