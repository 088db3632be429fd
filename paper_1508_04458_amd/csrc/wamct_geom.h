// Ray geometry and the leaf walk, shared by the kernels (and usable on the host, which is
// how the walk's arithmetic is checked against the CPU reference without a GPU).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "wamct_internal.h"

namespace wamct {

__host__ __device__ inline int imin(int a, int b) { return a < b ? a : b; }
__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }

// A coordinate in pixel units within 1e-9 of an integer (a pixel boundary) is taken as on it.
__host__ __device__ inline double edge_snap(double f) {
  const double r = rint(f);
  return fabs(f - r) <= 1e-9 ? r : f;
}

// Ray (origin, unit direction) of view v, bin b in FP64 (conventions in include/wamct.h).
__host__ __device__ inline void ray_of(const DevGeom& g, double2 cs, int b, double& ox, double& oy,
                              double& ex, double& ey) {
  const double u = (b - 0.5 * (g.nb - 1)) * g.pitch;
  const double c = cs.x, s = cs.y;
  if (g.kind == 0) {
    ox = u * c; oy = u * s; ex = -s; ey = c;
  } else {
    const double sx = g.sod * c, sy = g.sod * s;
    const double px = -(g.sdd - g.sod) * c - u * s, py = -(g.sdd - g.sod) * s + u * c;
    double dx = px - sx, dy = py - sy;
    const double inv = 1.0 / sqrt(dx * dx + dy * dy);
    ex = dx * inv; ey = dy * inv; ox = sx; oy = sy;
  }
  // A direction within 1e-12 of an axis is treated as exactly axis-parallel: the line is
  // moved to the centre of the pixel row (column) holding the ray's origin (the fan-beam
  // source, or the parallel-beam foot point u (c, s)), which leaves every chord unchanged
  // and puts a line lying on a boundary into the pixel on the + side (half-open pixels; an
  // origin within 1e-9 pixel of a boundary is on it, as exact arithmetic would place it);
  // it keeps a 1e-12 tilt so that 1/e is finite for the walks (the ray table stores an
  // inverse that acts as infinite).
  const double hn = 0.5 * g.n;
  const bool snap_y = fabs(ey) < 1e-12, snap_x = fabs(ex) < 1e-12;
  const double py0 = (floor(edge_snap(oy / g.pixel + hn)) + 0.5 - hn) * g.pixel;
  const double px0 = (floor(edge_snap(ox / g.pixel + hn)) + 0.5 - hn) * g.pixel;
  if (snap_y) ey = ey < 0 ? -1e-12 : 1e-12;
  if (snap_x) ex = ex < 0 ? -1e-12 : 1e-12;
  // move the origin to the point of the line closest to the image centre (|t| stays
  // below the image half-diagonal inside the image, which keeps FP32 chords accurate)
  const double tc = -(ox * ex + oy * ey);
  ox += tc * ex; oy += tc * ey;
  if (snap_y) oy = py0;
  if (snap_x) ox = px0;
}

// Walk one ray through the leaves of the tree (or through pixels when !TREE) and call
// f(ix, iy, level, chord) for every leaf it crosses, in order. The walk runs in a frame
// mirrored per axis so that both coordinates grow along the ray (leaf boundaries stay aligned
// because 2^L divides n): the current position is a pixel inside the current leaf; the exit
// parameter of the leaf is the nearer of its two upper planes, and the next pixel is the
// neighbour across that plane, its other coordinate taken at the exit point and clamped into
// the leaf's range (monotone even when rounding puts the exit point on a corner). Every step
// adds at least one to the crossed axis' index and lowers neither, and the walk stops once an
// index reaches n, so it ends after at most 2n steps for any levels below 32 in the map.
template <typename R, bool TREE, typename F>
__host__ __device__ inline void walk(const DevGeom& g, R ox, R oy, R ex, R ey, R iex, R iey,
                            const uint8_t* lev, F& f) {
  const int n = g.n;
  const R ipix = R(1.0 / g.pixel), hn = R(0.5 * n);
  const R X = ox * ipix + hn, Y = oy * ipix + hn;                 // pixel coordinates at t = 0
  const R x0 = ex < R(0) ? R(n) - X : X, y0 = ey < R(0) ? R(n) - Y : Y;
  const R ux = fabs(ex) * ipix, uy = fabs(ey) * ipix;             // pixels per unit t
  const R kx = fabs(iex) * R(g.pixel), ky = fabs(iey) * R(g.pixel);   // t per pixel
  const R cx = -x0 * kx, cy = -y0 * ky;                           // t at mirrored coordinate 0
  const R cx1 = (R(1) - x0) * kx, cy1 = (R(1) - y0) * ky;         // t at mirrored coordinate 1
  // real index = c + s m of the mirrored one (c = 0, s = 1, or c = n - 1, s = -1)
  const int sx = ex < R(0) ? -1 : 1, cxr = ex < R(0) ? n - 1 : 0;
  const int sy = ey < R(0) ? -1 : 1, cyr = ey < R(0) ? n - 1 : 0;
  const R t_in = fmax(cx, cy);
  const R t_out = fmin(fma(R(n), kx, cx), fma(R(n), ky, cy));
  if (!(t_out > t_in)) return;
  int x = imin(imax(int(fma(t_in, ux, x0)), 0), n - 1);
  int y = imin(imax(int(fma(t_in, uy, y0)), 0), n - 1);
  R t = t_in;
  // leaf level of the mirrored pixel (x, y), clamped into range: row-major index linear in
  // the mirrored coordinates
  const int i0 = cyr * n + cxr, dy = sy * n;
  auto level = [&](int xm, int ym) { return TREE ? int(lev[i0 + dy * imin(ym, n - 1) + sx * imin(xm, n - 1)]) : 0; };
  int l = level(x, y);
  for (;;) {
    const int rx = cxr + sx * x, ry = cyr + sy * y;
    const int m = (1 << l) - 1;
    const int hx = x | m, hy = y | m;   // last pixel of the leaf along x and y
    const R tX = fma(R(hx), kx, cx1), tY = fma(R(hy), ky, cy1);   // its upper planes
    const bool cross_x = tX <= tY;
    // the planes lie inside the image and ahead of t, up to rounding (a chord an ulp below 0
    // where the ray passes a corner; the pixel indices never move backwards)
    const R te = fmin(tX, tY);
    const int xn = imin(imax(int(fma(te, ux, x0)), x), hx) + int(cross_x);
    const int yn = imin(imax(int(fma(te, uy, y0)), y), hy) + int(!cross_x);
    const int ln = level(xn, yn);   // the next leaf's level, in flight while f runs
    f(rx, ry, l, te - t);
    if (te >= t_out || xn >= n || yn >= n) break;
    x = xn;
    y = yn;
    t = te;
    l = ln;
  }
}

}  // namespace wamct
