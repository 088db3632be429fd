// C ABI of wavelet-tree AM (include/wamct.h): validation, buffers, and the order of
// kernel launches for Algorithm 1 and the tree rule (arXiv 1508.04458, Introduction and
// Results). Device memory is allocated only in wamct_create; iterating allocates nothing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>

#include "../../include/wamct.h"
#include "wamct_internal.h"

using namespace wamct;

namespace {
thread_local std::string g_last_error;

const char* kVersion = "wamct 0.1 (gfx950)";

std::string fmt(const char* f, ...) __attribute__((format(printf, 1, 2)));
std::string fmt(const char* f, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, f);
  vsnprintf(buf, sizeof buf, f, ap);
  va_end(ap);
  return buf;
}

std::string validate(const wamct_geometry* g, const wamct_options* o) {
  if (!g || !o) return "geometry and options must not be NULL";
  if (g->kind != WAMCT_PARALLEL && g->kind != WAMCT_FAN) return fmt("unknown geometry kind %d", g->kind);
  if (g->n < 2 || g->n > 8192) return fmt("image size n = %d outside [2, 8192]", g->n);
  if (!(g->pixel > 0) || !std::isfinite(g->pixel)) return "pixel size must be finite and > 0";
  if (g->n_views < 1 || g->n_bins < 1) return "n_views and n_bins must be >= 1";
  if (int64_t(g->n_views) * g->n_bins > (int64_t(1) << 31) - 1) return "too many rays";
  if (!(g->bin_pitch > 0) || !std::isfinite(g->bin_pitch)) return "bin pitch must be finite and > 0";
  if (!std::isfinite(g->angle0) || !std::isfinite(g->angle_span)) return "angles must be finite";
  if (g->kind == WAMCT_FAN) {
    const double rc = 0.5 * g->n * g->pixel * std::sqrt(2.0);
    if (!(g->sod > rc)) return fmt("fan beam needs sod (%g) > image circumradius (%g)", g->sod, rc);
    if (!(g->sdd > g->sod) || !std::isfinite(g->sdd)) return "fan beam needs finite sdd > sod";
  }
  if (o->levels < 0 || o->levels > kMaxLevels) return fmt("levels = %d outside [0, %d]", o->levels, kMaxLevels);
  if (g->n % (1 << o->levels)) return fmt("n = %d is not divisible by 2^levels = %d", g->n, 1 << o->levels);
  if (o->dtype != WAMCT_F32 && o->dtype != WAMCT_F64) return fmt("unknown dtype %d", o->dtype);
  if (o->geometry != WAMCT_F32 && o->geometry != WAMCT_F64) return fmt("unknown geometry precision %d", o->geometry);
  if (o->geometry == WAMCT_F32 && o->dtype == WAMCT_F64) return "geometry precision must be at least dtype";
  return "";
}
}  // namespace

struct wamct_ctx {
  std::string err;
  virtual ~wamct_ctx() {}
  virtual wamct_status init(const wamct_geometry&, const wamct_options&, hipStream_t) = 0;
  virtual wamct_status set_stream(hipStream_t) = 0;
  virtual wamct_status set_data(const void*, const void*, double) = 0;
  virtual wamct_status reset() = 0;
  virtual wamct_status set_state(const void*, const uint8_t*) = 0;
  virtual wamct_status get_state(void*, uint8_t*, int32_t*) = 0;
  virtual wamct_status iterate(int32_t, double*) = 0;
  virtual wamct_status expand_tree(double, int32_t*) = 0;
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
  wamct_status fail(wamct_status s, const std::string& m) {
    err = m;
    return s;
  }
};

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(WAMCT_E_HIP, fmt("%s: %s", #expr, hipGetErrorString(e_)));            \
  } while (0)
#define LAUNCHED()                                                                     \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess) return fail(WAMCT_E_HIP, fmt("kernel launch: %s", hipGetErrorString(e_))); \
  } while (0)

namespace {

template <typename T, typename R>
struct Ctx final : wamct_ctx {
  DevGeom g{};
  hipStream_t st = nullptr;
  int64_t M = 0, NN = 0;
  int max_items = 0, nb_rays = 0, nb_pix = 0;
  // device buffers
  double2* views = nullptr;
  void* vT = nullptr;
  void* A = nullptr;
  void* B = nullptr;
  T *d = nullptr, *i0v = nullptr, *q = nullptr;
  T *beta = nullptr, *b = nullptr, *mu = nullptr, *muT = nullptr, *img = nullptr;
  void *leafR = nullptr, *leafC = nullptr;  // leaf records (value, level) for the tree walk
  uint8_t *mask = nullptr, *mask_old = nullptr, *lev = nullptr;
  uint32_t* items = nullptr;
  double *partd = nullptr, *part2 = nullptr, *mu64 = nullptr, *scal = nullptr;  // scal: [0]=z0 [1]=w [2]=max [3]=tmp
  int* ints = nullptr;  // [0]=held [1]=bad [2]=n_split; [8] = item count, [9 + k] = items of level L - k
  void* part = nullptr;  // chunked gather partial sums
  std::vector<Segment> segs, pix_segs;
  std::vector<void*> allocs;
  // host state
  double i0s = 1.0;
  bool has_data = false, tree_dirty = true;
  int n_items = 0;
  int32_t iters = 0;
  // timing
  bool timing_on = false;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double tot_ms[WAMCT_NK] = {0};
  int64_t tot_n[WAMCT_NK] = {0};

  ~Ctx() override {
    if (st) hipStreamSynchronize(st);
    for (auto& r : recs) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
    for (auto e : pool) hipEventDestroy(e);
    for (void* p : allocs) hipFree(p);
  }

  template <typename P>
  wamct_status alloc(P*& p, int64_t count) {
    void* v = nullptr;
    wamct_status r = alloc_bytes(v, size_t(count > 0 ? count : 1) * sizeof(P));
    p = static_cast<P*>(v);
    return r;
  }
  wamct_status alloc_bytes(void*& v, size_t bytes) {
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(WAMCT_E_OOM, fmt("hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e)));
    }
    allocs.push_back(v);
    return WAMCT_OK;
  }

  // ---------------------------------------------------------------- timing helpers
  hipEvent_t ev() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
  }
  void harvest() {
    for (auto& r : recs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) { tot_ms[r.kind] += ms; tot_n[r.kind] += 1; }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
  struct Scope {
    Ctx* c; int kind; hipEvent_t a = nullptr;
    Scope(Ctx* c_, int k) : c(c_), kind(k) {
      if (c->timing_on) { a = c->ev(); hipEventRecord(a, c->st); }
    }
    ~Scope() {
      if (a) {
        hipEvent_t b = c->ev();
        hipEventRecord(b, c->st);
        c->recs.push_back({kind, a, b});
        if (c->recs.size() > 4096) { hipEventSynchronize(b); c->harvest(); }
      }
    }
  };

  // Split the views of a level segment into chunks when its items alone cannot fill the GPU.
  Segment make_segment(int start, int count, int level) const {
    Segment sg{start, count, level, 1, g.nv};
    if (count < kTargetLanes) {
      int chunks = std::min(g.nv, (kTargetLanes + count - 1) / count);
      const int vpc = (g.nv + chunks - 1) / chunks;
      chunks = (g.nv + vpc - 1) / vpc;
      sg.chunks = chunks;
      sg.vpc = vpc;
    }
    return sg;
  }

  // ---------------------------------------------------------------- setup
  wamct_status init(const wamct_geometry& G, const wamct_options& O, hipStream_t s) override {
    st = s;
    g.kind = G.kind; g.n = G.n; g.nv = G.n_views; g.nb = G.n_bins; g.L = O.levels;
    g.pixel = G.pixel; g.pitch = G.bin_pitch; g.sod = G.sod; g.sdd = G.sdd;
    M = int64_t(g.nv) * g.nb;
    NN = int64_t(g.n) * g.n;
    nb_rays = int((M + 255) / 256);
    nb_pix = int((NN + 255) / 256);
    max_items = int(NN);
    wamct_status r;
    if ((r = alloc(views, g.nv))) return r;
    if ((r = alloc_bytes(vT, sizeof(float) * 2 * size_t(g.nv)))) return r;
    if ((r = alloc_bytes(A, sizeof(R) * 4 * size_t(M))) || (r = alloc_bytes(B, sizeof(R) * 4 * size_t(M)))) return r;
    if ((r = alloc(d, M)) || (r = alloc(i0v, M)) || (r = alloc(q, M))) return r;
    if ((r = alloc(beta, NN)) || (r = alloc(b, NN)) || (r = alloc(mu, NN)) || (r = alloc(img, NN))) return r;
    if ((r = alloc(muT, NN))) return r;
    if (g.L > 0 && ((r = alloc_bytes(leafR, 2 * sizeof(T) * size_t(NN))) ||
                    (r = alloc_bytes(leafC, 2 * sizeof(T) * size_t(NN)))))
      return r;
    if ((r = alloc(mask, NN)) || (r = alloc(mask_old, NN)) || (r = alloc(lev, NN))) return r;
    if ((r = alloc(items, max_items)) || (r = alloc(mu64, NN))) return r;
    const int np = std::max(nb_rays, nb_pix) + 1;
    if ((r = alloc(partd, np)) || (r = alloc(part2, np)) || (r = alloc(scal, 8)) || (r = alloc(ints, 32))) return r;
    if ((r = alloc_bytes(part, sizeof(R) * 7 * 2 * size_t(kTargetLanes)))) return r;
    pix_segs = {make_segment(0, int(NN), 0)};
    i0v_used = false;
    std::vector<double2> hv(g.nv);
    for (int v = 0; v < g.nv; ++v) {
      const double a = G.angle0 + v * (G.angle_span / G.n_views);
      hv[v] = make_double2(std::cos(a), std::sin(a));
    }
    HIPCHK(hipMemcpyAsync(views, hv.data(), sizeof(double2) * g.nv, hipMemcpyHostToDevice, st));
    Geo<T, R>::view_table(g, views, vT, st);
    Geo<T, R>::ray_table(g, views, A, B, st);
    fill_i32(ints, 32, 0, st);
    Launch<T>::fill(q, M, T(0), st);
    LAUNCHED();
    HIPCHK(hipStreamSynchronize(st));
    return reset();
  }
  bool i0v_used = false;

  wamct_status set_stream(hipStream_t s) override {
    HIPCHK(hipStreamSynchronize(st));
    st = s;
    return WAMCT_OK;
  }

  wamct_status set_data(const void* dd, const void* ii, double i0) override {
    if (!dd) return fail(WAMCT_E_INVALID, "d must not be NULL");
    if (!ii && !(i0 > 0 && std::isfinite(i0))) return fail(WAMCT_E_INVALID, "scalar I0 must be finite and > 0");
    HIPCHK(hipMemcpyAsync(d, dd, sizeof(T) * M, hipMemcpyDeviceToDevice, st));
    if (ii) HIPCHK(hipMemcpyAsync(i0v, ii, sizeof(T) * M, hipMemcpyDeviceToDevice, st));
    fill_i32(ints + 1, 1, 0, st);
    Launch<T>::check(d, M, false, ints + 1, st);
    int bad_d = 0, bad_i = 0;
    HIPCHK(hipMemcpyAsync(&bad_d, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad_d) return fail(WAMCT_E_INVALID, fmt("%d counts are negative or not finite", bad_d));
    if (ii) {
      fill_i32(ints + 1, 1, 0, st);
      Launch<T>::check(i0v, M, false, ints + 1, st);
      HIPCHK(hipMemcpyAsync(&bad_i, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (bad_i) return fail(WAMCT_E_INVALID, fmt("%d I0 values are negative or not finite", bad_i));
    }
    i0v_used = ii != nullptr;
    i0s = ii ? 1.0 : i0;
    // eq. 1.6: b = Phi^T d = Omega^T (H^T d) for every coefficient
    {
      Scope sc(this, WAMCT_K_OTHER);
      Geo<T, R>::gather(g, kPlain, vT, A, d, nullptr, pix_segs.data(), int(pix_segs.size()), part, nullptr,
                        nullptr, nullptr, nullptr, nullptr, nullptr, img, st);
      Launch<T>::analysis(g, img, b, st);
    }
    LAUNCHED();
    has_data = true;
    return WAMCT_OK;
  }

  wamct_status rebuild_tree() {
    {
      Scope sc(this, WAMCT_K_TREE);
      build_items(g, mask, items, ints + 8, st);
      Launch<T>::levmap(g, mask, lev, st);
      const int nbk = z0_partials(g, views, lev, partd, part2, st);
      reduce_max(partd, nbk, scal + 0, st);
      reduce_sum(part2, nbk, scal + 1, st);
    }
    LAUNCHED();
    int cnt[2 + kMaxLevels] = {0};
    HIPCHK(hipMemcpyAsync(cnt, ints + 8, sizeof cnt, hipMemcpyDeviceToHost, st));
    double z0 = 0;
    HIPCHK(hipMemcpyAsync(&z0, scal + 0, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    n_items = cnt[0];
    segs.clear();
    int start = 0;
    const int n_levels = g.L == 0 ? 1 : g.L;
    for (int k = 0; k < n_levels; ++k) {
      const int c = cnt[1 + k];
      if (c > 0) segs.push_back(make_segment(start, c, g.L - k));
      start += c;
    }
    if (!(z0 > 0) || !std::isfinite(z0)) return fail(WAMCT_E_INVALID, "Z0 = 0: no ray crosses the image");
    tree_dirty = false;
    return WAMCT_OK;
  }

  wamct_status reset() override {
    Launch<T>::fill(beta, NN, T(0), st);
    approx_mask(g, mask, st);
    fill_i32(ints, 1, 0, st);
    LAUNCHED();
    iters = 0;
    tree_dirty = true;
    return rebuild_tree();
  }

  wamct_status set_state(const void* bt, const uint8_t* mk) override {
    if (!bt || !mk) return fail(WAMCT_E_INVALID, "beta and mask must not be NULL");
    HIPCHK(hipMemcpyAsync(mask_old, mk, NN, hipMemcpyDeviceToDevice, st));
    fill_i32(ints + 1, 1, 0, st);
    check_mask(g, mask_old, ints + 1, st);
    Launch<T>::check((const T*)bt, NN, true, ints + 1, st);
    LAUNCHED();
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad) return fail(WAMCT_E_INVALID, fmt("state rejected: %d invalid tree entries or non-finite coefficients", bad));
    HIPCHK(hipMemcpyAsync(mask, mask_old, NN, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(beta, bt, sizeof(T) * NN, hipMemcpyDeviceToDevice, st));
    Launch<T>::apply_mask(g, beta, mask, st);
    fill_i32(ints, 1, 0, st);
    LAUNCHED();
    iters = 0;
    tree_dirty = true;
    return rebuild_tree();
  }

  wamct_status get_state(void* bt, uint8_t* mk, int32_t* it) override {
    if (bt) HIPCHK(hipMemcpyAsync(bt, beta, sizeof(T) * NN, hipMemcpyDeviceToDevice, st));
    if (mk) HIPCHK(hipMemcpyAsync(mk, mask, NN, hipMemcpyDeviceToDevice, st));
    if (it) *it = iters;
    return WAMCT_OK;
  }

  // one forward pass of the current state: mu, q-hat and the I-divergence partials
  int forward_pass() {
    const bool tree = g.L > 0;
    if (tree) {
      {
        Scope sc(this, WAMCT_K_SYNTH);
        Launch<T>::synth_records(g, beta, lev, leafR, leafC, st);
      }
      Scope sc(this, WAMCT_K_FORWARD);
      return Geo<T, R>::forward_records(g, A, B, leafR, leafC, d, i0v_used ? i0v : nullptr, i0s, q, nullptr, partd,
                                        st);
    }
    {
      Scope sc(this, WAMCT_K_SYNTH);
      Launch<T>::synth_layouts(g, beta, mu, muT, st);
    }
    Scope sc(this, WAMCT_K_FORWARD);
    return Geo<T, R>::forward(g, A, B, mu, muT, d, i0v_used ? i0v : nullptr, i0s, q, nullptr, partd, st);
  }

  wamct_status iterate(int32_t n, double* idv) override {
    if (!has_data) return fail(WAMCT_E_STATE, "iterate before set_data");
    if (n < 0) return fail(WAMCT_E_INVALID, "n_iters must be >= 0");
    if (tree_dirty) { wamct_status r = rebuild_tree(); if (r) return r; }
    for (int k = 0; k < n; ++k) {
      const int nbk = forward_pass();
      {
        Scope sc(this, WAMCT_K_OTHER);
        reduce_sum(partd, nbk, idv ? idv + k : scal + 3, st);
      }
      {
        Scope sc(this, WAMCT_K_UPDATE);
        Geo<T, R>::gather(g, kUpdate, vT, A, q, items, segs.data(), int(segs.size()), part, beta, b, scal + 0,
                          ints + 0, nullptr, nullptr, nullptr, st);
      }
      ++iters;
    }
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status expand_tree(double frac, int32_t* n_split) override {
    if (!(frac >= 0) || !std::isfinite(frac)) return fail(WAMCT_E_INVALID, "frac must be finite and >= 0");
    int ns = 0;
    if (g.L > 0) {
      {
        Scope sc(this, WAMCT_K_TREE);
        const int nbk = Launch<T>::mu64(g, beta, mu64, partd, st);
        reduce_max(partd, nbk, scal + 2, st);
        HIPCHK(hipMemcpyAsync(mask_old, mask, NN, hipMemcpyDeviceToDevice, st));
        fill_i32(ints + 2, 1, 0, st);
        expand(g, mask_old, mask, mu64, scal + 2, frac, ints + 2, st);
      }
      LAUNCHED();
      HIPCHK(hipMemcpyAsync(&ns, ints + 2, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (ns > 0) {
        tree_dirty = true;
        wamct_status r = rebuild_tree();
        if (r) return r;
      }
    }
    if (n_split) *n_split = ns;
    return WAMCT_OK;
  }

  wamct_status synthesize(void* out) override {
    if (!out) return fail(WAMCT_E_INVALID, "mu must not be NULL");
    Scope sc(this, WAMCT_K_SYNTH);
    Launch<T>::synth(g, beta, (T*)out, st);
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status project(const void* m, void* p) override {
    if (!m || !p) return fail(WAMCT_E_INVALID, "mu and p must not be NULL");
    Scope sc(this, WAMCT_K_OTHER);
    Launch<T>::transpose(g.n, (const T*)m, muT, st);
    Geo<T, R>::forward(g, A, B, (const T*)m, muT, nullptr, nullptr, 1.0, nullptr, (T*)p, nullptr, st);
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status backproject(const void* y, void* out) override {
    if (!y || !out) return fail(WAMCT_E_INVALID, "y and img must not be NULL");
    Scope sc(this, WAMCT_K_OTHER);
    Geo<T, R>::gather(g, kPlain, vT, A, (const T*)y, nullptr, pix_segs.data(), int(pix_segs.size()), part,
                      nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, (T*)out, st);
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status backproject_split(const void* y, void* bp, void* bm) override {
    if (!y || !bp || !bm) return fail(WAMCT_E_INVALID, "y, bp and bm must not be NULL");
    if (tree_dirty) { wamct_status r = rebuild_tree(); if (r) return r; }
    Scope sc(this, WAMCT_K_OTHER);
    Launch<T>::fill((T*)bp, NN, T(0), st);
    Launch<T>::fill((T*)bm, NN, T(0), st);
    Geo<T, R>::gather(g, kSplit, vT, A, (const T*)y, items, segs.data(), int(segs.size()), part, nullptr,
                      nullptr, nullptr, nullptr, (T*)bp, (T*)bm, nullptr, st);
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status forward(void* qo, double* idv) override {
    if (!has_data) return fail(WAMCT_E_STATE, "forward before set_data");
    if (tree_dirty) { wamct_status r = rebuild_tree(); if (r) return r; }
    const int nbk = forward_pass();
    if (idv) reduce_sum(partd, nbk, idv, st);
    if (qo) HIPCHK(hipMemcpyAsync(qo, q, sizeof(T) * M, hipMemcpyDeviceToDevice, st));
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status idiv(const void* qq, double* out) override {
    if (!has_data) return fail(WAMCT_E_STATE, "idiv before set_data");
    if (!qq || !out) return fail(WAMCT_E_INVALID, "q and out must not be NULL");
    Scope sc(this, WAMCT_K_OTHER);
    const int nbk = Launch<T>::idiv_terms(g, (const T*)qq, d, partd, st);
    reduce_sum(partd, nbk, out, st);
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status get_b(void* out) override {
    if (!has_data) return fail(WAMCT_E_STATE, "get_b before set_data");
    if (!out) return fail(WAMCT_E_INVALID, "b must not be NULL");
    HIPCHK(hipMemcpyAsync(out, b, sizeof(T) * NN, hipMemcpyDeviceToDevice, st));
    return WAMCT_OK;
  }

  wamct_status tree_stats(double* z0, int64_t* w, int64_t* n_active, int64_t* n_held) override {
    if (tree_dirty) { wamct_status r = rebuild_tree(); if (r) return r; }
    double sc[2] = {0, 0};
    int held = 0;
    HIPCHK(hipMemcpyAsync(sc, scal, sizeof sc, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&held, ints, sizeof(int), hipMemcpyDeviceToHost, st));
    std::vector<uint8_t> hm;
    if (n_active) {
      hm.resize(NN);
      HIPCHK(hipMemcpyAsync(hm.data(), mask, NN, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    if (z0) *z0 = sc[0];
    if (w) *w = int64_t(llround(sc[1]));
    if (n_held) *n_held = held;
    if (n_active) {
      int64_t c = 0;
      for (uint8_t v : hm) c += v;
      *n_active = c;
    }
    return WAMCT_OK;
  }

  // Coefficient-domain loss (eq. 1.3 with lambda = 0, every coefficient free):
  // loss_b = I(d_b || I0 exp(-H Omega c_b)) for a batch of scans of this geometry.
  wamct_status loss(int32_t batch, const void* c, const void* dd, const void* i0p, double i0sc, double* lossd,
                    void* qout) override {
    if (batch < 0) return fail(WAMCT_E_INVALID, "batch must be >= 0");
    if (batch > 0 && (!c || !dd || !lossd || !qout)) return fail(WAMCT_E_INVALID, "c, d, loss and q must not be NULL");
    if (!i0p && !(i0sc > 0 && std::isfinite(i0sc))) return fail(WAMCT_E_INVALID, "scalar I0 must be finite and > 0");
    for (int k = 0; k < batch; ++k) {
      const T* ck = (const T*)c + size_t(k) * NN;
      const T* dk = (const T*)dd + size_t(k) * M;
      const T* ik = i0p ? (const T*)i0p + size_t(k) * M : nullptr;
      T* qk = (T*)qout + size_t(k) * M;
      {
        Scope sc(this, WAMCT_K_SYNTH);
        Launch<T>::synth_layouts(g, ck, mu, muT, st);
      }
      int nbk;
      {
        Scope sc(this, WAMCT_K_FORWARD);
        nbk = Geo<T, R>::forward(g, A, B, mu, muT, dk, ik, i0sc, qk, nullptr, partd, st);
      }
      Scope sc(this, WAMCT_K_OTHER);
      reduce_sum(partd, nbk, lossd + k, st);
    }
    LAUNCHED();
    return WAMCT_OK;
  }

  // Hand-written adjoint: grad_b = s_b Omega^T H^T (d_b - q_b) from the saved q_b (s_b = the
  // incoming gradient of loss_b, null = 1).
  wamct_status loss_backward(int32_t batch, const void* qq, const void* dd, const double* gscale,
                             void* grad) override {
    if (batch < 0) return fail(WAMCT_E_INVALID, "batch must be >= 0");
    if (batch > 0 && (!qq || !dd || !grad)) return fail(WAMCT_E_INVALID, "q, d and grad must not be NULL");
    for (int k = 0; k < batch; ++k) {
      Scope sc(this, WAMCT_K_UPDATE);
      Launch<T>::residual((const T*)dd + size_t(k) * M, (const T*)qq + size_t(k) * M, gscale ? gscale + k : nullptr,
                          q, M, st);
      Geo<T, R>::gather(g, kPlain, vT, A, q, nullptr, pix_segs.data(), int(pix_segs.size()), part, nullptr, nullptr,
                        nullptr, nullptr, nullptr, nullptr, img, st);
      Launch<T>::analysis(g, img, (T*)grad + size_t(k) * NN, st);
    }
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status timing(int32_t on) override {
    HIPCHK(hipStreamSynchronize(st));
    harvest();
    for (int k = 0; k < WAMCT_NK; ++k) { tot_ms[k] = 0; tot_n[k] = 0; }
    timing_on = on != 0;
    return WAMCT_OK;
  }

  wamct_status get_timing(double* ms, int64_t* n) override {
    HIPCHK(hipStreamSynchronize(st));
    harvest();
    for (int k = 0; k < WAMCT_NK; ++k) {
      if (ms) ms[k] = tot_ms[k];
      if (n) n[k] = tot_n[k];
    }
    return WAMCT_OK;
  }
};

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

wamct_status wamct_validate(const wamct_geometry* geom, const wamct_options* opt, char* msg, int32_t msg_len) {
  std::string e = validate(geom, opt);
  if (msg && msg_len > 0) {
    std::snprintf(msg, size_t(msg_len), "%s", e.c_str());
  }
  if (!e.empty()) {
    g_last_error = e;
    return WAMCT_E_INVALID;
  }
  return WAMCT_OK;
}

wamct_status wamct_create(const wamct_geometry* geom, const wamct_options* opt, void* stream, wamct_ctx** out) {
  if (!out) { g_last_error = "out must not be NULL"; return WAMCT_E_INVALID; }
  *out = nullptr;
  std::string e = validate(geom, opt);
  if (!e.empty()) { g_last_error = e; return WAMCT_E_INVALID; }
  wamct_ctx* c = nullptr;
  if (opt->dtype == WAMCT_F64) c = new Ctx<double, double>();
  else if (opt->geometry == WAMCT_F32) c = new Ctx<float, float>();
  else c = new Ctx<float, double>();
  wamct_status s = c->init(*geom, *opt, static_cast<hipStream_t>(stream));
  if (s != WAMCT_OK) {
    g_last_error = c->err;
    delete c;
    return s;
  }
  *out = c;
  return WAMCT_OK;
}

wamct_status wamct_destroy(wamct_ctx* ctx) {
  delete ctx;
  return WAMCT_OK;
}

const char* wamct_last_error(const wamct_ctx* ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }
const char* wamct_version(void) { return kVersion; }

#define CTX_CALL(call)                                   \
  do {                                                   \
    if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; } \
    return ctx->call;                                    \
  } while (0)

wamct_status wamct_set_stream(wamct_ctx* ctx, void* stream) { CTX_CALL(set_stream(static_cast<hipStream_t>(stream))); }
wamct_status wamct_set_data(wamct_ctx* ctx, const void* d, const void* i0, double i0s) { CTX_CALL(set_data(d, i0, i0s)); }
wamct_status wamct_reset(wamct_ctx* ctx) { CTX_CALL(reset()); }
wamct_status wamct_set_state(wamct_ctx* ctx, const void* beta, const uint8_t* mask) { CTX_CALL(set_state(beta, mask)); }
wamct_status wamct_get_state(wamct_ctx* ctx, void* beta, uint8_t* mask, int32_t* it) { CTX_CALL(get_state(beta, mask, it)); }
wamct_status wamct_iterate(wamct_ctx* ctx, int32_t n, double* idiv) { CTX_CALL(iterate(n, idiv)); }
wamct_status wamct_expand(wamct_ctx* ctx, double frac, int32_t* n_split) { CTX_CALL(expand_tree(frac, n_split)); }
wamct_status wamct_synthesize(wamct_ctx* ctx, void* mu) { CTX_CALL(synthesize(mu)); }
wamct_status wamct_project(wamct_ctx* ctx, const void* mu, void* p) { CTX_CALL(project(mu, p)); }
wamct_status wamct_backproject(wamct_ctx* ctx, const void* y, void* img) { CTX_CALL(backproject(y, img)); }
wamct_status wamct_backproject_split(wamct_ctx* ctx, const void* y, void* bp, void* bm) { CTX_CALL(backproject_split(y, bp, bm)); }
wamct_status wamct_forward(wamct_ctx* ctx, void* q, double* idiv) { CTX_CALL(forward(q, idiv)); }
wamct_status wamct_idiv(wamct_ctx* ctx, const void* q, double* out) { CTX_CALL(idiv(q, out)); }
wamct_status wamct_get_b(wamct_ctx* ctx, void* b) { CTX_CALL(get_b(b)); }
wamct_status wamct_tree_stats(wamct_ctx* ctx, double* z0, int64_t* w, int64_t* na, int64_t* nh) { CTX_CALL(tree_stats(z0, w, na, nh)); }
wamct_status wamct_timing(wamct_ctx* ctx, int32_t enable) { CTX_CALL(timing(enable)); }
wamct_status wamct_loss(wamct_ctx* ctx, int32_t batch, const void* c, const void* d, const void* i0, double i0s,
                        double* loss, void* q) { CTX_CALL(loss(batch, c, d, i0, i0s, loss, q)); }
wamct_status wamct_loss_backward(wamct_ctx* ctx, int32_t batch, const void* q, const void* d, const double* gscale,
                                 void* grad) { CTX_CALL(loss_backward(batch, q, d, gscale, grad)); }
wamct_status wamct_get_timing(wamct_ctx* ctx, double* ms, int64_t* n) { CTX_CALL(get_timing(ms, n)); }

wamct_status wamct_solve(wamct_ctx* ctx, int32_t n_iters, const int32_t* expand_at, int32_t n_expand, double frac,
                         double* idiv) {
  if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; }
  if (n_iters < 0 || n_expand < 0 || (n_expand > 0 && !expand_at))
    return ctx->fail(WAMCT_E_INVALID, "bad iteration count or expansion schedule");
  for (int k = 1; k < n_expand; ++k)
    if (expand_at[k] <= expand_at[k - 1]) return ctx->fail(WAMCT_E_INVALID, "expansion schedule must ascend");
  int e = 0;
  int j = 0;
  while (j < n_iters) {
    while (e < n_expand && expand_at[e] < j) ++e;
    if (e < n_expand && expand_at[e] == j) {
      wamct_status s = ctx->expand_tree(frac, nullptr);
      if (s) return s;
      ++e;
    }
    // run up to the next scheduled expansion in one call
    int stop = n_iters;
    if (e < n_expand && expand_at[e] < stop) stop = expand_at[e];
    wamct_status s = ctx->iterate(stop - j, idiv ? idiv + j : nullptr);
    if (s) return s;
    j = stop;
  }
  return ctx->forward(nullptr, idiv ? idiv + n_iters : nullptr);
}

}  // extern "C"
