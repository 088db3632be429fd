// The context interface shared by the 2-D (wamct_api.hip) and 3-D (wamct_api3.hip)
// implementations of the C ABI in include/wamct.h.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/wamct.h"

namespace wamct {
std::string fmt(const char* f, ...) __attribute__((format(printf, 1, 2)));
}  // namespace wamct

struct wamct_ctx {
  std::string err;
  virtual ~wamct_ctx() {}
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
  virtual wamct_status set_subsets(int32_t) = 0;
  virtual int32_t subsets() const = 0;
  virtual wamct_status set_tree_sharing(int32_t) = 0;
  virtual int32_t tree_sharing() const = 0;
  virtual wamct_status set_tree_rule(int32_t) = 0;
  virtual int32_t tree_rule() const = 0;
  virtual wamct_status set_penalty(double) = 0;
  virtual double penalty() const = 0;
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
