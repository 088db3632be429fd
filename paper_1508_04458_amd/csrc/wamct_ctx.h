// The context interface shared by the 2-D (wamct_api.hip) and 3-D (wamct_api3.hip)
// implementations of the C ABI in include/wamct.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/wamct.h"

namespace wamct {
std::string fmt(const char* f, ...) __attribute__((format(printf, 1, 2)));

// (cos a, sin a) of a view with values within 1e-12 of zero set to exactly zero (the partner
// then exactly +-1): a view angle that is a multiple of pi/2 in exact arithmetic puts the
// source (or the parallel-beam foot point) on an axis, which the ~1e-16 rounding of cos and
// sin would move off it; lines on pixel boundaries then fall on the + side as stated.
inline void view_cos_sin(double a, double& c, double& s) {
  c = std::cos(a);
  s = std::sin(a);
  const bool cz = std::fabs(c) < 1e-12, sz = std::fabs(s) < 1e-12;
  if (cz) { c = 0.0; s = s < 0 ? -1.0 : 1.0; }
  if (sz) { s = 0.0; c = c < 0 ? -1.0 : 1.0; }
}
}  // namespace wamct

struct wamct_ctx {
  std::string err;
  // explicit tree sequence Z_s^(j) (an input of Algorithm 1): tree k becomes the active set
  // before update sched_at[k] of a solve (ascending); empty: the tree rule decides
  std::vector<int32_t> sched_at;
  virtual ~wamct_ctx() {}
  // index k of the scheduled tree that takes effect before update j, or -1
  int sched_index(int j) const {
    const auto it = std::lower_bound(sched_at.begin(), sched_at.end(), j);
    return (it != sched_at.end() && *it == j) ? int(it - sched_at.begin()) : -1;
  }
  // host check of a schedule's iteration list ("" = valid)
  static std::string check_sched(int32_t n, const int32_t* at, const void* masks) {
    if (n < 0) return "n_trees must be >= 0";
    if (n > 0 && (!at || !masks)) return "at and masks must not be NULL";
    for (int k = 0; k < n; ++k) {
      if (at[k] < 0) return "tree schedule iterations must be >= 0";
      if (k > 0 && at[k] <= at[k - 1]) return "tree schedule iterations must ascend strictly";
    }
    return "";
  }
  virtual wamct_status init(const wamct_geometry&, const wamct_options&, hipStream_t) = 0;
  virtual wamct_status set_stream(hipStream_t) = 0;
  virtual wamct_status set_data(const void*, const void*, const double*) = 0;
  virtual wamct_status reset() = 0;
  virtual wamct_status set_state(const void*, const uint8_t*) = 0;
  virtual wamct_status get_state(void*, uint8_t*, int32_t*) = 0;
  virtual wamct_status iterate(int32_t, double*) = 0;
  virtual wamct_status expand_tree(double, int32_t*) = 0;
  virtual wamct_status solve(int32_t, const int32_t*, int32_t, double, double*) = 0;
  virtual wamct_status synthesize(void*) = 0;
  virtual wamct_status project(const void*, void*) = 0;
  virtual wamct_status backproject(const void*, void*) = 0;
  virtual wamct_status backproject_split(const void*, void*, void*) = 0;
  virtual wamct_status forward(void*, double*) = 0;
  virtual wamct_status idiv(const void*, double*) = 0;
  virtual wamct_status get_b(void*) = 0;
  virtual wamct_status tree_stats(double*, int64_t*, int64_t*, int64_t*) = 0;
  virtual wamct_status loss(int32_t, const void*, const void*, const void*, double, double*, void*) = 0;
  virtual wamct_status loss_backward(int32_t, const void*, const void*, const double*, void*) = 0;
  virtual wamct_status timing(int32_t) = 0;
  virtual wamct_status get_timing(double*, int64_t*) = 0;
  virtual wamct_status set_tiling(int32_t) = 0;
  virtual int32_t tiling() const = 0;
  // lanes per ray of the leaf walk (0 = chosen by the launch size); 2-D trees only
  virtual wamct_status set_walk_lanes(int32_t) { return fail(WAMCT_E_UNSUPPORTED, "no leaf-walk lanes to set"); }
  virtual int32_t walk_lanes() const { return 0; }
  virtual wamct_status set_subsets(int32_t) = 0;
  virtual int32_t subsets() const = 0;
  virtual wamct_status set_tree_sharing(int32_t) = 0;
  virtual int32_t tree_sharing() const = 0;
  virtual wamct_status set_tree_rule(int32_t) = 0;
  virtual int32_t tree_rule() const = 0;
  virtual wamct_status set_penalty(double) = 0;
  virtual double penalty() const = 0;
  virtual wamct_status set_tree_schedule(int32_t, const int32_t*, const uint8_t*) = 0;
  // tree k of the schedule becomes the current tree (stream-ordered; then enq_tree)
  virtual wamct_status enq_schedule(hipStream_t, int) = 0;
  // stream-ordered pieces used by batches (no host synchronization inside)
  virtual int n_scans() const = 0;
  virtual hipStream_t stream() const = 0;
  virtual double work() const = 0;
  virtual bool has_data_() const = 0;
  virtual bool tree_dirty_() const = 0;
  virtual wamct_status enq_tree(hipStream_t) = 0;
  virtual wamct_status finish_tree(int32_t*) = 0;
  virtual wamct_status enq_reset(hipStream_t) = 0;
  virtual wamct_status enq_expand(hipStream_t, double) = 0;
  virtual wamct_status enq_begin(hipStream_t) = 0;
  virtual wamct_status enq_iteration(hipStream_t, double*, int64_t, bool) = 0;
  virtual wamct_status enq_final(hipStream_t, double*, int64_t, bool) = 0;
  virtual wamct_status save_state(hipStream_t) = 0;
  virtual wamct_status restore_state(hipStream_t) = 0;
  virtual void count_iters(int) = 0;
  wamct_status fail(wamct_status s, const std::string& m) {
    err = m;
    return s;
  }
};

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(WAMCT_E_HIP, wamct::fmt("%s: %s", #expr, hipGetErrorString(e_)));            \
  } while (0)
#define LAUNCHED()                                                                     \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess) return fail(WAMCT_E_HIP, wamct::fmt("kernel launch: %s", hipGetErrorString(e_))); \
  } while (0)
#define CHECKED(expr)                                                                  \
  do {                                                                                 \
    wamct_status r_ = (expr);                                                          \
    if (r_ != WAMCT_OK) return r_;                                                     \
  } while (0)


namespace wamct {
// 3-D context (circular cone beam, 3-D Haar octree): validation message ("" = valid) and
// factory; defined in wamct_api3.hip.
std::string validate3(const wamct_geometry* g, const wamct_options* o);
wamct_ctx* make_ctx3(const wamct_options& o);
}  // namespace wamct
