// Internal interface of the 3-D path (circular cone beam, 3-D Haar octree) between the C
// ABI (wamct_api3.hip) and its kernels (wamct_kernels3.hip). Conventions: include/wamct.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wamct_internal.h"

namespace wamct {

// Cone-beam scan and volume as the kernels see them.
struct DevGeom3 {
  int n, nz;        // volume n x n x nz, layout [z][y][x]
  int nv, nr, nc;   // views, detector rows, detector columns
  int L;            // Haar levels
  int wd;           // wavelet dimensions: 3 = 3-D Haar octree, 2 = 2-D Haar per z-slice (one
                    // tree for every slice; a node is one voxel deep, its z index the slice)
  double pixel, cpitch, rpitch, sod, sdd;
};

// z shift of a level-l node: octree nodes halve in z as well, per-slice nodes do not
__host__ __device__ inline int node_zshift(int wd, int l) { return wd == 3 ? l : 0; }

// Work item of the 3-D node-driven backprojection: one octree node or one box.
//   bit 31     : 1 = node with octant chords (seven details, plus the approximation when the
//                node is a root), 0 = single box (root approximation or voxel)
//   bits 27-30 : level l
//   bits 18-26 : node z index k, bits 9-17 : y index i, bits 0-8 : x index j
__host__ __device__ inline uint32_t item3_pack(int split, int l, int k, int i, int j) {
  return (uint32_t(split) << 31) | (uint32_t(l) << 27) | (uint32_t(k) << 18) | (uint32_t(i) << 9) | uint32_t(j);
}

// Sums of one 3-D item: the plain sum and, per detail, the signed sum and the sum of magnitudes.
constexpr int kSlots3 = 15;

// Per-view ray factors of the scan (device arrays): views = (cos a, sin a) per view,
// colt [nv][nc] = (1/Dx, 1/Dy), rowt [nr] = 1/Dz, nrm [nr][nc] = |D| for D = detector element -
// source (a component within 1e-12 sdd of 0 has the factor +-1e300). The walks and the gather
// build every ray from them.
struct RayF3 {
  const double2* views;
  const double2* colt;
  const double* rowt;
  const double* nrm;
};

template <typename T>
struct Geo3 {
  // Leaf walk over (value | level) records (row layout [z][y][x] and [z][x][y]): p = sum of
  // chord * leaf value; if q != null, q = I0 exp(-p) (I0 per ray or the scalar *i0s) and
  // per-block FP64 partials of the I-divergence terms in `part`; if p != null p is stored.
  // Returns the number of blocks.
  static int forward(const DevGeom3& g, const RayF3& f, const void* recR, const void* recC, const T* d,
                     const T* i0v, const double* i0s, T* q, T* p, double* part, hipStream_t s);
  // Per-view ray factors of the gather: colt [nv][nc] = (1/Dx, 1/Dy), rowt [nr] = 1/Dz,
  // nrm [nr][nc] = |D| for D = detector element - source.
  static void ray_factors(const DevGeom3& g, const double2* views, double2* colt, double* rowt, double* nrm,
                          hipStream_t s);
  // out = y |D| per ray (the ray values the gather takes)
  static void scale_rays(const DevGeom3& g, const T* y, const double* nrm, T* out, hipStream_t s);
  // Node-driven backprojection of the scaled ray values y over item segments (items null:
  // every voxel as a level-0 box); part holds 15 partial sums per (chunk group, item).
  static void gather(const DevGeom3& g, int mode, const double2* views, const double2* colt, const double* rowt,
                     const T* y, const uint32_t* items, const int* counts, const Segment* segs, int n_segs,
                     void* part, T* beta, const T* b, const double* z0, int* held, T* bp, T* bm, T* out,
                     hipStream_t s);
  // leaf records of mu = Omega beta (both layouts); with L = 0 in g and lev null, records of
  // the volume `beta` itself at level 0
  static void synth_records(const DevGeom3& g, const T* beta, const uint8_t* lev, void* recR, void* recC,
                            hipStream_t s);
  static void synth(const DevGeom3& g, const T* beta, T* mu, hipStream_t s);
  // FP64 synthesis and per-block maxima; returns the number of blocks
  static int mu64(const DevGeom3& g, const T* beta, double* mu64, double* part, hipStream_t s);
  static void analysis(const DevGeom3& g, const T* vol, T* coef, hipStream_t s);
  static void apply_mask(const DevGeom3& g, T* beta, const uint8_t* mask, hipStream_t s);
  // residual-gradient rule: per-leaf score max |coef| over its seven would-be details, at the
  // node's first detail position of score (other entries untouched)
  static void grad_scores(const DevGeom3& g, const uint8_t* mask, const T* coef, double* score, hipStream_t s);
};

// wd = 2: mask slices 1 .. nz-1 = slice 0 (the tree every slice shares)
void broadcast_slice3(const DevGeom3& g, uint8_t* mask, hipStream_t s);

// Z0 and W of the current octree (per ray FP64 walk); returns the number of blocks.
// lev: per-voxel leaf level [z][y][x]; levC the same in [z][x][y] (read by x-major rays)
int z0_partials3(const DevGeom3& g, const RayF3& f, const uint8_t* lev, const uint8_t* levC, double* part_max,
                 double* part_cnt, hipStream_t s);
void levmap3(const DevGeom3& g, const uint8_t* mask, uint8_t* lev, uint8_t* levC, hipStream_t s);
// Work list in segments: split roots, roots not split (every voxel when L = 0), then split
// nodes level by level (L - 1 down to 1), 3-D Morton order within a segment; counts[0] =
// items, counts[1 + k] = items of segment k.
// octree work list (items, counts); `scratch` holds list_scratch_ints3(g) ints
int64_t list_scratch_ints3(const DevGeom3& g);
void build_items3(const DevGeom3& g, const uint8_t* mask, uint32_t* items, int* counts, int* scratch,
                  hipStream_t s);
// rule 0: leaf-constant values of mu64; rule 1: leaf scores of grad_scores held in mu64
void expand3(const DevGeom3& g, const uint8_t* mask_old, uint8_t* mask, const double* mu64, const double* maxv,
             double frac, int* n_split, hipStream_t s, int rule = 0);
void approx_mask3(const DevGeom3& g, uint8_t* mask, hipStream_t s);
// *bad += number of violated octree constraints of the mask
void check_mask3(const DevGeom3& g, const uint8_t* mask, int* bad, hipStream_t s);

}  // namespace wamct
