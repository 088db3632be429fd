// Ray geometry and the leaf walk, shared by the kernels (and usable on the host, which is
// how the walk's arithmetic is checked against the CPU reference without a GPU).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "wamct_internal.h"

namespace wamct {

__host__ __device__ inline int imin(int a, int b) { return a < b ? a : b; }
__host__ __device__ inline int imax(int a, int b) { return a > b ? a : b; }

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
  // move the origin to the point of the line closest to the image centre (|t| stays
  // below the image half-diagonal inside the image, which keeps FP32 chords accurate)
  const double tc = -(ox * ex + oy * ey);
  ox += tc * ex; oy += tc * ey;
  // A direction within 1e-12 of an axis is treated as exactly axis-parallel: the line is
  // moved to the centre of the pixel row (column) that contains it, which leaves every
  // chord unchanged and puts a line lying on a boundary into the pixel on the + side
  // (half-open pixels), and it gets a 1e-12 tilt so 1/e stays finite; the tilt moves it by
  // less than 1e-8 pixel across any image this library accepts.
  const double hn = 0.5 * g.n;
  if (fabs(ey) < 1e-12) {
    oy = (floor(oy / g.pixel + hn) + 0.5 - hn) * g.pixel;
    ey = ey < 0 ? -1e-12 : 1e-12;
  }
  if (fabs(ex) < 1e-12) {
    ox = (floor(ox / g.pixel + hn) + 0.5 - hn) * g.pixel;
    ex = ex < 0 ? -1e-12 : 1e-12;
  }
}

// Walk one ray through the leaves of the tree (or through pixels when !TREE) and call
// f(ix, iy, level, chord) for every leaf it crosses, in order. The current position is a
// pixel (ix, iy) inside the current leaf; the exit parameter of the leaf is the nearer of
// its two exit planes, and the next pixel is the neighbour across that plane (its other
// coordinate clamped into the leaf's range, which keeps the walk monotone even when
// rounding puts the exit point on a corner). Every step moves to a new leaf, so at most
// 2n steps occur; the loop bound 4n + 8 only guards against malformed input.
template <typename R, bool TREE, typename F>
__host__ __device__ inline void walk(const DevGeom& g, R ox, R oy, R ex, R ey, R iex, R iey,
                            const uint8_t* lev, F& f) {
  const int n = g.n;
  const R pix = R(g.pixel), ipix = R(1.0 / g.pixel), hn = R(0.5 * n), half = R(0.5 * n * g.pixel);
  const R tx0 = (-half - ox) * iex, tx1 = (half - ox) * iex;
  const R ty0 = (-half - oy) * iey, ty1 = (half - oy) * iey;
  const R t_in = fmax(fmin(tx0, tx1), fmin(ty0, ty1));
  const R t_out = fmin(fmax(tx0, tx1), fmax(ty0, ty1));
  if (!(t_out > t_in)) return;
  int ix = (int)floor(fmin(fmax((ox + t_in * ex) * ipix + hn, R(-1)), R(n)));
  int iy = (int)floor(fmin(fmax((oy + t_in * ey) * ipix + hn, R(-1)), R(n)));
  ix = imin(imax(ix, 0), n - 1);
  iy = imin(imax(iy, 0), n - 1);
  const bool px = ex > R(0), py = ey > R(0);
  R t = t_in;
  for (int step = 0; step < 4 * n + 8; ++step) {
    const int l = TREE ? int(lev[iy * n + ix]) : 0;
    const int s = 1 << l;
    const int bx0 = (ix >> l) << l, by0 = (iy >> l) << l;
    const int X = px ? bx0 + s : bx0;
    const int Y = py ? by0 + s : by0;
    const R tX = ((R(X) - hn) * pix - ox) * iex;
    const R tY = ((R(Y) - hn) * pix - oy) * iey;
    R te = fmin(fmin(tX, tY), t_out);
    te = fmax(te, t);
    f(ix, iy, l, te - t);
    if (te >= t_out) break;
    // the other coordinate never moves backwards (monotone walk) and stays in the leaf
    if (tX <= tY) {
      ix = px ? bx0 + s : bx0 - 1;
      if (TREE) {
        const int rr = (int)floor(fmin(fmax((oy + te * ey) * ipix + hn, R(-1)), R(n)));
        iy = py ? imin(imax(rr, iy), by0 + s - 1) : imax(imin(rr, iy), by0);
      }
    } else {
      iy = py ? by0 + s : by0 - 1;
      if (TREE) {
        const int cc = (int)floor(fmin(fmax((ox + te * ex) * ipix + hn, R(-1)), R(n)));
        ix = px ? imin(imax(cc, ix), bx0 + s - 1) : imax(imin(cc, ix), bx0);
      }
    }
    if ((unsigned)ix >= (unsigned)n || (unsigned)iy >= (unsigned)n) break;
    t = te;
  }
}

}  // namespace wamct
