// C ABI of wavelet-tree AM (include/wamct.h): validation, buffers, and the order of
// kernel launches for Algorithm 1 and the tree rule (arXiv 1508.04458, Introduction and
// Results). Device memory is allocated only in wamct_create (and when a larger gather
// tiling is requested); iterating allocates nothing. A context holds a stack of scans of
// one geometry, solved in lockstep; a batch runs several contexts concurrently, one
// iteration of all of them captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/wamct.h"
#include "wamct_ctx.h"
#include "wamct_internal.h"

using namespace wamct;

namespace wamct {
std::string fmt(const char* f, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, f);
  vsnprintf(buf, sizeof buf, f, ap);
  va_end(ap);
  return buf;
}
}  // namespace wamct

namespace {
thread_local std::string g_last_error;

const char* kVersion = "wamct 0.2 (gfx950)";

std::string validate(const wamct_geometry* g, const wamct_options* o) {
  if (!g || !o) return "geometry and options must not be NULL";
  if (g->kind == WAMCT_CONE) return validate3(g, o);
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
  if (o->batch < 1 || o->batch > 65535) return fmt("batch = %d outside [1, 65535]", o->batch);
  if (o->wavelet_dims != 0 && o->wavelet_dims != 2)
    return fmt("wavelet_dims = %d: 2-D scans take the 2-D Haar transform (0 or 2)", o->wavelet_dims);
  if (o->wavelet != WAMCT_HAAR && o->wavelet != WAMCT_D4) return fmt("unknown wavelet %d", o->wavelet);
  if (o->wavelet == WAMCT_D4) {
    if (o->levels < 1) return "Daubechies-4 needs levels >= 1";
    if ((g->n >> o->levels) < 4)
      return fmt("Daubechies-4 needs n >> levels >= 4 (n = %d, levels = %d): a support must not wrap onto itself",
                 g->n, o->levels);
    if (o->batch != 1) return fmt("Daubechies-4 is implemented for one scan per context (batch = %d)", o->batch);
  }
  return "";
}
}  // namespace

namespace {

template <typename T, typename R>
struct Ctx final : wamct_ctx {
  DevGeom g{};
  hipStream_t st = nullptr;
  int P = 1;                  // scans in the stack
  int64_t M = 0, NN = 0;      // rays and pixels per scan
  int nb_rays = 0, nb_pix = 0, np = 0;
  // device buffers ([P][...] per scan unless noted)
  double2* views = nullptr;   // shared
  void* vT = nullptr;         // shared
  void* A = nullptr;          // shared ray table
  void* B = nullptr;
  T *d = nullptr, *i0v = nullptr, *q = nullptr;
  T *beta = nullptr, *b = nullptr, *mu = nullptr, *muT = nullptr;
  T* img = nullptr;           // one image (operators, precompute)
  void *leafR = nullptr, *leafC = nullptr;  // leaf records (value | level) for the tree walk
  uint8_t *mask = nullptr, *mask_old = nullptr, *lev = nullptr;
  uint32_t* items = nullptr;
  int* list_tmp = nullptr;      // block counts and offsets of the work-list builder
  double *partd = nullptr, *part2 = nullptr, *mu64 = nullptr;
  double* scal = nullptr;     // [P][kScal]
  int* ints = nullptr;        // [P][kInts]
  double* i0one = nullptr;    // scalar I0 of the loss path
  T* beta_save = nullptr;     // tiling trials
  int* ints_save = nullptr;
  int32_t iters_save = 0;
  void* part = nullptr;       // chunked gather partial sums
  int64_t part_cap = 0;       // elements of R
  int* h_ints = nullptr;      // pinned host copies read after a tree rebuild
  double* h_scal = nullptr;
  // one tree for the whole stack, grown on the slice-summed image
  bool shared_tree = false;
  int rule = WAMCT_RULE_VALUE;   // tree rule of the expansions
  double lam = 0.0;              // roughness-penalty weight (0: Algorithm 1 as in the paper)
  T* gpen = nullptr;             // [P][n][n] Omega^T grad R(mu-hat) of the current iteration
  uint8_t* sched = nullptr;       // [n trees][P][n*n] masks of the explicit tree schedule
  // ordered subsets of views (n_sub > 1): b and Z0 of every subset, [n_sub][P][...]
  int n_sub = 1;
  T* bsub = nullptr;
  double* z0s = nullptr;
  double* h_z0s = nullptr;
  std::vector<Segment> segs, pix_segs, segs_sub, pix_segs_sub;
  std::vector<void*> allocs;
  // host state
  bool has_data = false, tree_dirty = true, i0v_used = false;
  int32_t iters = 0;
  int target_lanes = kTargetLanes;
  int walk_k = 0;             // lanes per ray of the leaf walk (0: by launch size)
  // Daubechies-4 basis (wavelet = WAMCT_D4): basis tables and the per-ray Z0 sums
  bool d4 = false;
  D4Dev tb{};
  double* zsum = nullptr;
  // timing
  uint32_t timing_mask = 0;   // bit k: record kernel class k
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double tot_ms[WAMCT_NK] = {0};
  int64_t tot_n[WAMCT_NK] = {0};

  ~Ctx() override {
    if (st) hipStreamSynchronize(st);
    hipDeviceSynchronize();
    for (auto& r : recs) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
    for (auto e : pool) hipEventDestroy(e);
    for (void* p : allocs) hipFree(p);
    if (part) hipFree(part);
    free_subsets();
    if (sched) hipFree(sched);
    if (h_ints) hipHostFree(h_ints);
    if (h_scal) hipHostFree(h_scal);
  }

  int n_scans() const override { return P; }
  hipStream_t stream() const override { return st; }
  double work() const override { return double(P) * double(M) * double(g.n); }
  bool has_data_() const override { return has_data; }
  bool tree_dirty_() const override { return tree_dirty; }
  int32_t tiling() const override { return target_lanes; }
  wamct_status set_walk_lanes(int32_t k) override {
    if (k != 0 && k != 1 && k != 2 && k != 4) return fail(WAMCT_E_INVALID, fmt("walk lanes %d not in {0, 1, 2, 4}", k));
    if (g.L == 0) return fail(WAMCT_E_UNSUPPORTED, "levels = 0 walks pixels, one lane per ray");
    if (d4) return fail(WAMCT_E_UNSUPPORTED, "the Daubechies-4 forward pass walks pixels, one lane per ray");
    walk_k = k;
    return WAMCT_OK;
  }
  int32_t walk_lanes() const override {
    return g.L == 0 || d4 ? 0 : walk_k > 0 ? walk_k : leaf_pieces(M * P);
  }
  void count_iters(int k) override { iters += k; }

  template <typename Q>
  wamct_status alloc(Q*& p, int64_t count) {
    void* v = nullptr;
    wamct_status r = alloc_bytes(v, size_t(count > 0 ? count : 1) * sizeof(Q));
    p = static_cast<Q*>(v);
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
  // Records the kernels of its lifetime under `kind` when timing is on and the work runs on
  // the context's own stream (batch streams are not timed per kernel class).
  struct Scope {
    Ctx* c; int kind; hipStream_t s; hipEvent_t a = nullptr;
    Scope(Ctx* c_, int k, hipStream_t s_) : c(c_), kind(k), s(s_) {
      if (((c->timing_mask >> kind) & 1u) && s == c->st) { a = c->ev(); hipEventRecord(a, s); }
    }
    ~Scope() {
      if (a) {
        hipEvent_t b = c->ev();
        hipEventRecord(b, s);
        c->recs.push_back({kind, a, b});
        if (c->recs.size() > 4096) { hipEventSynchronize(b); c->harvest(); }
      }
    }
  };

  // ---------------------------------------------------------------- tiling of the gather
  // Split the nv views of a level segment into chunks when its items (over the S scans of
  // one launch) alone cannot fill the GPU.
  Segment make_segment(int kseg, int start, int count, int level, int S, int nv) const {
    Segment sg{kseg, start, count, level, 1, nv};
    const int64_t lanes = int64_t(count) * S;
    if (count > 0 && lanes < target_lanes) {
      int chunks = int(std::min<int64_t>(nv, (target_lanes + lanes - 1) / lanes));
      const int vpc = (nv + chunks - 1) / chunks;
      chunks = (nv + vpc - 1) / vpc;
      sg.chunks = chunks;
      sg.vpc = vpc;
    }
    return sg;
  }
  // Partial sums a gather can need at a given target: per chunked segment 7 (target / 4 +
  // lanes) with lanes = count * S < target (chunk groups of four waves, rounded up), one
  // segment per tree level side by side.
  int64_t part_need(int target) const {
    return int64_t(std::max(1, g.L)) * 7 * (int64_t(target) / 4 + 1 + std::min<int64_t>(int64_t(P) * NN, target));
  }
  wamct_status ensure_part(int target) {
    const int64_t need = part_need(target);
    if (need <= part_cap) return WAMCT_OK;
    if (part) {
      HIPCHK(hipDeviceSynchronize());
      HIPCHK(hipFree(part));
      part = nullptr;
      part_cap = 0;
    }
    hipError_t e = hipMalloc(&part, size_t(need) * sizeof(R));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      part = nullptr;
      return fail(WAMCT_E_OOM, fmt("hipMalloc(%zu bytes): %s", size_t(need) * sizeof(R), hipGetErrorString(e)));
    }
    part_cap = need;
    return WAMCT_OK;
  }
  void build_segs() {
    segs.clear();
    segs_sub.clear();
    const int n_levels = g.L == 0 ? 1 : g.L;
    for (int k = 0; k < n_levels; ++k) {
      int mx = 0;
      for (int p = 0; p < P; ++p) mx = std::max(mx, h_ints[p * kInts + 9 + k]);
      if (mx > 0) {
        segs.push_back(make_segment(k, 0, mx, g.L - k, P, g.nv));
        segs_sub.push_back(make_segment(k, 0, mx, g.L - k, P, sub_views(0)));
      }
    }
    build_pix_segs();
  }
  void build_pix_segs() {
    pix_segs = {make_segment(-1, 0, int(NN), 0, 1, g.nv)};
    pix_segs_sub = {make_segment(-1, 0, int(NN), 0, 1, sub_views(0))};
  }
  wamct_status set_tiling(int32_t t) override {
    if (t < kMinTargetLanes || t > kMaxTargetLanes)
      return fail(WAMCT_E_INVALID, fmt("tiling %d outside [%d, %d]", t, kMinTargetLanes, kMaxTargetLanes));
    HIPCHK(hipStreamSynchronize(st));
    CHECKED(ensure_part(t));
    target_lanes = t;
    if (!tree_dirty) build_segs();
    else build_pix_segs();
    return WAMCT_OK;
  }

  // ---------------------------------------------------------------- ordered subsets
  // Subset k holds the views v = k mod n_sub: geometry, b and Z0 of subset k (k < 0: all
  // views, the context's own b and Z0).
  struct Sel {
    DevGeom g;
    const T* b;
    const double* z0;
    int z0stride;
  };
  int sub_views(int k) const { return (g.nv - k + n_sub - 1) / n_sub; }
  Sel sel(int k) const {
    if (k < 0) return Sel{g, b, scal + 0, kScal};
    DevGeom gs = g;
    gs.vs0 = k;
    gs.vss = n_sub;
    gs.nvs = sub_views(k);
    return Sel{gs, bsub + size_t(k) * P * NN, z0s + size_t(k) * P, 1};
  }
  void free_subsets() {
    if (bsub) hipFree(bsub);
    if (z0s) hipFree(z0s);
    if (h_z0s) hipHostFree(h_z0s);
    bsub = nullptr;
    z0s = nullptr;
    h_z0s = nullptr;
  }
  // b of every subset (eq. 1.6 over the subset's rays), for every scan
  wamct_status precompute_bsub(hipStream_t s) {
    for (int k = 0; k < n_sub; ++k)
      for (int p = 0; p < P; ++p) {
        CHECKED(gather(kPlain, d + p * M, pix_segs_sub, 1, nullptr, nullptr, nullptr, nullptr, img, s, sel(k)));
        Launch<T>::analysis(g, img, bsub + (size_t(k) * P + p) * NN, s);
      }
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status set_subsets(int32_t ns) override {
    if (ns > 1 && d4) return fail(WAMCT_E_UNSUPPORTED, "ordered subsets are not implemented for Daubechies-4");
    if (ns > 1 && lam > 0.0)
      return fail(WAMCT_E_UNSUPPORTED, "ordered subsets are not implemented with the roughness penalty");
    if (ns < 1 || ns > g.nv) return fail(WAMCT_E_INVALID, fmt("n_subsets = %d outside [1, n_views = %d]", ns, g.nv));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipDeviceSynchronize());
    free_subsets();
    n_sub = ns;
    if (ns > 1) {
      void* v = nullptr;
      hipError_t e1 = hipMalloc(&v, sizeof(T) * size_t(ns) * P * NN);
      bsub = static_cast<T*>(v);
      hipError_t e2 = hipMalloc(&v, sizeof(double) * size_t(ns) * P);
      z0s = static_cast<double*>(v);
      hipError_t e3 = hipHostMalloc((void**)&h_z0s, sizeof(double) * size_t(ns) * P, hipHostMallocDefault);
      if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        (void)hipGetLastError();
        if (e2 != hipSuccess) z0s = nullptr;
        if (e3 != hipSuccess) h_z0s = nullptr;
        if (e1 != hipSuccess) bsub = nullptr;
        free_subsets();
        n_sub = 1;
        return fail(WAMCT_E_OOM, "allocation of the ordered-subset buffers failed");
      }
    }
    build_pix_segs();
    if (has_data && ns > 1) CHECKED(precompute_bsub(st));
    tree_dirty = true;
    return WAMCT_OK;
  }
  int32_t subsets() const override { return n_sub; }

  wamct_status set_tree_rule(int32_t r) override {
    if (r != WAMCT_RULE_VALUE && r != WAMCT_RULE_GRADIENT) return fail(WAMCT_E_INVALID, fmt("unknown tree rule %d", r));
    if (r == WAMCT_RULE_GRADIENT && shared_tree)
      return fail(WAMCT_E_UNSUPPORTED, "the residual-gradient rule is not implemented for slices sharing one tree");
    if (r == WAMCT_RULE_GRADIENT && d4)
      return fail(WAMCT_E_UNSUPPORTED, "the residual-gradient rule is not implemented for Daubechies-4");
    HIPCHK(hipStreamSynchronize(st));
    rule = r;
    return WAMCT_OK;
  }
  int32_t tree_rule() const override { return rule; }
  wamct_status set_penalty(double l) override {
    if (!(l >= 0.0) || !std::isfinite(l)) return fail(WAMCT_E_INVALID, "the penalty weight must be finite and >= 0");
    if (l > 0.0 && n_sub > 1)
      return fail(WAMCT_E_UNSUPPORTED, "the roughness penalty is not implemented with ordered subsets");
    if (l > 0.0 && d4) return fail(WAMCT_E_UNSUPPORTED, "the roughness penalty is not implemented for Daubechies-4");
    HIPCHK(hipStreamSynchronize(st));
    if (l > 0.0 && !gpen) CHECKED(alloc(gpen, NN * P));
    lam = l;
    return WAMCT_OK;
  }
  double penalty() const override { return lam; }
  wamct_status set_tree_sharing(int32_t on) override {
    if (on != 0 && on != 1) return fail(WAMCT_E_INVALID, "shared must be 0 or 1");
    if (on == 1 && d4) return fail(WAMCT_E_UNSUPPORTED, "tree sharing is not implemented for Daubechies-4");
    if (on == 1 && rule == WAMCT_RULE_GRADIENT)
      return fail(WAMCT_E_UNSUPPORTED, "the residual-gradient rule is not implemented for slices sharing one tree");
    shared_tree = on == 1;
    if (shared_tree && P > 1) {
      // every slice takes slice 0's tree; coefficients outside it become 0
      for (int p = 1; p < P; ++p) HIPCHK(hipMemcpyAsync(mask + p * NN, mask, NN, hipMemcpyDeviceToDevice, st));
      Launch<T>::apply_mask(g, beta, mask, P, st);
      LAUNCHED();
      tree_dirty = true;
    }
    return WAMCT_OK;
  }
  int32_t tree_sharing() const override { return shared_tree ? 1 : 0; }

  // Explicit Z_s^(j): the masks are validated and copied into the context.
  wamct_status set_tree_schedule(int32_t n, const int32_t* at, const uint8_t* mk) override {
    const std::string e = check_sched(n, at, mk);
    if (!e.empty()) return fail(WAMCT_E_INVALID, e);
    HIPCHK(hipStreamSynchronize(st));
    sched_at.clear();
    if (sched) {
      HIPCHK(hipFree(sched));
      sched = nullptr;
    }
    if (n == 0) return WAMCT_OK;
    const size_t bytes = size_t(n) * P * NN;
    hipError_t er = hipMalloc((void**)&sched, bytes);
    if (er != hipSuccess) {
      (void)hipGetLastError();
      sched = nullptr;
      return fail(WAMCT_E_OOM, fmt("hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(er)));
    }
    HIPCHK(hipMemcpyAsync(sched, mk, bytes, hipMemcpyDeviceToDevice, st));
    fill_i32(ints + 1, 1, 0, st);
    check_mask(g, sched, ints + 1, n * P, st);
    LAUNCHED();
    HIPCHK(hipMemcpyAsync(h_ints + 1, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h_ints[1]) {
      HIPCHK(hipFree(sched));
      sched = nullptr;
      return fail(WAMCT_E_INVALID, fmt("tree schedule rejected: %d invalid tree entries", h_ints[1]));
    }
    sched_at.assign(at, at + n);
    return WAMCT_OK;
  }
  // Tree k becomes the active set: coefficients outside it are zeroed (new ones are zero
  // already); a shared tree takes slice 0's mask for every slice.
  wamct_status enq_schedule(hipStream_t s, int k) override {
    const uint8_t* src = sched + size_t(k) * P * NN;
    {
      Scope sc(this, WAMCT_K_TREE, s);
      if (shared_tree)
        for (int p = 0; p < P; ++p) HIPCHK(hipMemcpyAsync(mask + p * NN, src, NN, hipMemcpyDeviceToDevice, s));
      else
        HIPCHK(hipMemcpyAsync(mask, src, NN * P, hipMemcpyDeviceToDevice, s));
      Launch<T>::apply_mask(g, beta, mask, P, s);
      fill_i32_strided(ints + 2, P, kInts, 0, s);
    }
    LAUNCHED();
    return enq_tree(s);
  }
  // gather over segments (of the tree, or of every pixel) with a host check that their
  // partial sums fit; views, b and Z0 of the selection
  wamct_status gather(int mode, const T* y, const std::vector<Segment>& sg, int S, T* bt, int* held, T* bp, T* bm,
                      T* out, hipStream_t s, const Sel& v) {
    int64_t need = 0;
    for (const Segment& x : sg) need += segment_part_elems(x, S);
    if (need > part_cap || sg.size() > size_t(kMaxGatherSegs))
      return fail(WAMCT_E_HIP, "internal: gather partial buffer too small for its tiling");
    const bool tree = &sg == &segs || &sg == &segs_sub;
    const bool pen = mode == kUpdate && lam > 0.0;
    Geo<T, R>::gather(v.g, mode, vT, views, A, y, tree ? items : nullptr, tree ? ints + 9 : nullptr, sg.data(),
                      int(sg.size()), part, bt, v.b, v.z0, v.z0stride, held, bp, bm, out, S, s,
                      pen ? gpen : nullptr, lam);
    return WAMCT_OK;
  }
  wamct_status gather(int mode, const T* y, const std::vector<Segment>& sg, int S, T* bt, int* held, T* bp, T* bm,
                      T* out, hipStream_t s) {
    return gather(mode, y, sg, S, bt, held, bp, bm, out, s, sel(-1));
  }

  // ---------------------------------------------------------------- setup
  wamct_status init(const wamct_geometry& G, const wamct_options& O, hipStream_t s) override {
    st = s;
    P = O.batch;
    g.kind = G.kind; g.n = G.n; g.nv = G.n_views; g.nb = G.n_bins; g.L = O.levels;
    g.pixel = G.pixel; g.pitch = G.bin_pitch; g.sod = G.sod; g.sdd = G.sdd;
    g.vs0 = 0; g.vss = 1; g.nvs = g.nv;
    M = int64_t(g.nv) * g.nb;
    NN = int64_t(g.n) * g.n;
    nb_rays = int((M + 255) / 256);
    nb_pix = int((NN + 255) / 256);
    // the tree walk may use 4 lanes per ray; walk grids are padded to a multiple of 8 blocks
    np = std::max(4 * nb_rays, nb_pix) + 8;
    // image-domain AM (levels = 0): the pixel gather has cheap items and many of them; finer
    // view chunks (2^23 lanes instead of 2^20) measured 0.89 -> 0.73 ms per pass at fan512
    if (g.L == 0) target_lanes = 1 << 23;
    d4 = O.wavelet == WAMCT_D4;
    if (hipHostMalloc((void**)&h_ints, sizeof(int) * kInts * P, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_scal, sizeof(double) * kScal * P, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(WAMCT_E_OOM, "hipHostMalloc of the readback buffers failed");
    }
    std::memset(h_ints, 0, sizeof(int) * kInts * P);
    std::memset(h_scal, 0, sizeof(double) * kScal * P);
    CHECKED(alloc(views, g.nv));
    CHECKED(alloc_bytes(vT, sizeof(float) * 2 * size_t(g.nv)));
    CHECKED(alloc_bytes(A, sizeof(R) * 4 * size_t(M)));
    CHECKED(alloc_bytes(B, sizeof(R) * 4 * size_t(M)));
    CHECKED(alloc(d, M * P)); CHECKED(alloc(i0v, M * P)); CHECKED(alloc(q, M * P));
    CHECKED(alloc(beta, NN * P)); CHECKED(alloc(b, NN * P));
    CHECKED(alloc(mu, NN * P)); CHECKED(alloc(muT, NN * P)); CHECKED(alloc(img, NN));
    if (g.L > 0 && !d4) {
      CHECKED(alloc_bytes(leafR, sizeof(T) * size_t(NN * P)));
      CHECKED(alloc_bytes(leafC, sizeof(T) * size_t(NN * P)));
    }
    if (d4) {
      std::vector<double> hf, hg;
      d4_tables(g.L, hf, hg, tb);
      double *df = nullptr, *dg = nullptr;
      CHECKED(alloc(df, int64_t(hf.size())));
      CHECKED(alloc(dg, int64_t(hg.size())));
      HIPCHK(hipMemcpyAsync(df, hf.data(), sizeof(double) * hf.size(), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dg, hg.data(), sizeof(double) * hg.size(), hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
      tb.f = df;
      tb.g = dg;
      CHECKED(alloc(zsum, M));
    }
    CHECKED(alloc(mask, NN * P)); CHECKED(alloc(mask_old, NN * P)); CHECKED(alloc(lev, NN * P));
    CHECKED(alloc(items, NN * P)); CHECKED(alloc(mu64, NN * P));
    CHECKED(alloc(list_tmp, list_scratch_ints(g, P)));
    CHECKED(alloc(partd, int64_t(np) * P)); CHECKED(alloc(part2, int64_t(np) * P));
    CHECKED(alloc(scal, int64_t(kScal) * P)); CHECKED(alloc(ints, int64_t(kInts) * P));
    CHECKED(alloc(i0one, 1));
    CHECKED(ensure_part(target_lanes));
    build_pix_segs();
    std::vector<double2> hv(g.nv);
    for (int v = 0; v < g.nv; ++v) {
      const double a = G.angle0 + v * (G.angle_span / G.n_views);
      double c, sn;
      view_cos_sin(a, c, sn);
      hv[v] = make_double2(c, sn);
    }
    HIPCHK(hipMemcpyAsync(views, hv.data(), sizeof(double2) * g.nv, hipMemcpyHostToDevice, st));
    Geo<T, R>::view_table(g, views, vT, st);
    Geo<T, R>::ray_table(g, views, A, B, st);
    fill_i32(ints, int64_t(kInts) * P, 0, st);
    Launch<double>::fill(scal, int64_t(kScal) * P, 0.0, st);
    Launch<T>::fill(q, M * P, T(0), st);
    LAUNCHED();
    HIPCHK(hipStreamSynchronize(st));
    return reset();
  }

  wamct_status set_stream(hipStream_t s) override {
    HIPCHK(hipStreamSynchronize(st));
    st = s;
    return WAMCT_OK;
  }

  wamct_status set_data(const void* dd, const void* ii, const double* i0h) override {
    if (!dd) return fail(WAMCT_E_INVALID, "d must not be NULL");
    std::vector<double> i0s(P, 1.0);
    if (!ii) {
      if (!i0h) return fail(WAMCT_E_INVALID, "scalar I0 values must be given when i0 is NULL");
      for (int p = 0; p < P; ++p) {
        if (!(i0h[p] > 0) || !std::isfinite(i0h[p]))
          return fail(WAMCT_E_INVALID, fmt("scalar I0 of scan %d must be finite and > 0", p));
        i0s[p] = i0h[p];
      }
    }
    HIPCHK(hipMemcpyAsync(d, dd, sizeof(T) * M * P, hipMemcpyDeviceToDevice, st));
    if (ii) HIPCHK(hipMemcpyAsync(i0v, ii, sizeof(T) * M * P, hipMemcpyDeviceToDevice, st));
    for (int p = 0; p < P; ++p) h_scal[p * kScal + 4] = i0s[p];
    HIPCHK(hipMemcpy2DAsync(scal + 4, sizeof(double) * kScal, h_scal + 4, sizeof(double) * kScal, sizeof(double),
                            P, hipMemcpyHostToDevice, st));
    fill_i32(ints + 1, 1, 0, st);
    Launch<T>::check(d, M * P, false, ints + 1, st);
    int bad_d = 0, bad_i = 0;
    HIPCHK(hipMemcpyAsync(h_ints + 1, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bad_d = h_ints[1];
    if (bad_d) return fail(WAMCT_E_INVALID, fmt("%d counts are negative or not finite", bad_d));
    if (ii) {
      fill_i32(ints + 1, 1, 0, st);
      Launch<T>::check(i0v, M * P, false, ints + 1, st);
      HIPCHK(hipMemcpyAsync(h_ints + 1, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      bad_i = h_ints[1];
      if (bad_i) return fail(WAMCT_E_INVALID, fmt("%d I0 values are negative or not finite", bad_i));
    }
    i0v_used = ii != nullptr;
    // eq. 1.6: b = Phi^T d = Omega^T (H^T d) for every coefficient of every scan
    {
      Scope sc(this, WAMCT_K_OTHER, st);
      for (int p = 0; p < P; ++p) {
        CHECKED(gather(kPlain, d + p * M, pix_segs, 1, nullptr, nullptr, nullptr, nullptr, img, st));
        if (d4) D4<T, R>::analysis(g, tb, img, b + p * NN, st);
        else Launch<T>::analysis(g, img, b + p * NN, st);
      }
      if (n_sub > 1) CHECKED(precompute_bsub(st));
    }
    LAUNCHED();
    has_data = true;
    return WAMCT_OK;
  }

  // ---------------------------------------------------------------- tree (stream-ordered)
  // Work list, leaf levels, Z0 and W of every scan's tree, then a copy of the per-scan
  // counters and scalars to pinned host memory (read by finish_tree once s has finished).
  wamct_status enq_tree(hipStream_t s) override {
    if (d4) {
      // Z0 (eq. 1.61): per-ray sums of |phi| over the work list's coefficients, then the
      // largest; W: the non-zero (ray, coefficient) pairs per item, summed (mu64 holds them)
      Scope sc(this, WAMCT_K_TREE, s);
      build_items(g, mask, items, ints + 8, P, list_tmp, s);
      Launch<double>::fill(zsum, M, 0.0, s);
      Launch<double>::fill(mu64, NN, 0.0, s);
      D4<T, R>::gather(g, kD4Z0, tb, views, A, B, nullptr, items, ints + 8, int(NN), nullptr, nullptr, nullptr,
                       nullptr, nullptr, nullptr, zsum, mu64, s);
      reduce_stack(true, zsum, int(M), M, scal + 0, kScal, nullptr, 1, s);
      reduce_stack(false, mu64, int(NN), NN, scal + 1, kScal, nullptr, 1, s);
    } else {
      Scope sc(this, WAMCT_K_TREE, s);
      build_items(g, mask, items, ints + 8, P, list_tmp, s);
      Launch<T>::levmap(g, mask, lev, P, s);
      const int nbk = z0_partials(g, views, lev, partd, part2, P, s);
      reduce_stack(true, partd, nbk, nbk, scal + 0, kScal, nullptr, P, s);
      reduce_stack(false, part2, nbk, nbk, scal + 1, kScal, nullptr, P, s);
      if (n_sub > 1)
        for (int k = 0; k < n_sub; ++k) {   // Z0 of every view subset
          const Sel v = sel(k);
          const int nbs = z0_partials(v.g, views, lev, partd, part2, P, s);
          reduce_stack(true, partd, nbs, nbs, z0s + size_t(k) * P, 1, nullptr, P, s);
        }
    }
    LAUNCHED();
    if (n_sub > 1)
      HIPCHK(hipMemcpyAsync(h_z0s, z0s, sizeof(double) * n_sub * P, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_ints, ints, sizeof(int) * kInts * P, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_scal, scal, sizeof(double) * kScal * P, hipMemcpyDeviceToHost, s));
    tree_dirty = true;
    return WAMCT_OK;
  }
  wamct_status finish_tree(int32_t* n_split) override {
    build_segs();
    for (int p = 0; p < P; ++p) {
      const double z0 = h_scal[p * kScal + 0];
      if (!(z0 > 0) || !std::isfinite(z0))
        return fail(WAMCT_E_INVALID, fmt("Z0 = 0 in scan %d: no ray crosses the image", p));
      if (n_split) n_split[p] = h_ints[(shared_tree ? 0 : p) * kInts + 2];
    }
    for (int k = 0; n_sub > 1 && k < n_sub * P; ++k)
      if (!(h_z0s[k] > 0) || !std::isfinite(h_z0s[k]))
        return fail(WAMCT_E_INVALID, fmt("Z0 = 0 for view subset %d of scan %d: none of its rays crosses the image",
                                         k / P, k % P));
    tree_dirty = false;
    return WAMCT_OK;
  }
  wamct_status rebuild_tree() {
    CHECKED(enq_tree(st));
    HIPCHK(hipStreamSynchronize(st));
    return finish_tree(nullptr);
  }

  wamct_status enq_reset(hipStream_t s) override {
    Launch<T>::fill(beta, NN * P, T(0), s);
    approx_mask(g, mask, P, s);
    fill_i32_strided(ints + 0, P, kInts, 0, s);
    fill_i32_strided(ints + 2, P, kInts, 0, s);
    LAUNCHED();
    iters = 0;
    return enq_tree(s);
  }
  wamct_status reset() override {
    CHECKED(enq_reset(st));
    HIPCHK(hipStreamSynchronize(st));
    return finish_tree(nullptr);
  }

  wamct_status set_state(const void* bt, const uint8_t* mk) override {
    if (!bt || !mk) return fail(WAMCT_E_INVALID, "beta and mask must not be NULL");
    HIPCHK(hipMemcpyAsync(mask_old, mk, NN * P, hipMemcpyDeviceToDevice, st));
    fill_i32(ints + 1, 1, 0, st);
    check_mask(g, mask_old, ints + 1, P, st);
    Launch<T>::check((const T*)bt, NN * P, true, ints + 1, st);
    LAUNCHED();
    HIPCHK(hipMemcpyAsync(h_ints + 1, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int bad = h_ints[1];
    if (bad) return fail(WAMCT_E_INVALID, fmt("state rejected: %d invalid tree entries or non-finite coefficients", bad));
    HIPCHK(hipMemcpyAsync(mask, mask_old, NN * P, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(beta, bt, sizeof(T) * NN * P, hipMemcpyDeviceToDevice, st));
    Launch<T>::apply_mask(g, beta, mask, P, st);
    fill_i32_strided(ints + 0, P, kInts, 0, st);
    LAUNCHED();
    iters = 0;
    return rebuild_tree();
  }

  wamct_status get_state(void* bt, uint8_t* mk, int32_t* it) override {
    if (bt) HIPCHK(hipMemcpyAsync(bt, beta, sizeof(T) * NN * P, hipMemcpyDeviceToDevice, st));
    if (mk) HIPCHK(hipMemcpyAsync(mk, mask, NN * P, hipMemcpyDeviceToDevice, st));
    if (it) *it = iters;
    return WAMCT_OK;
  }

  // ---------------------------------------------------------------- iteration (stream-ordered)
  // One forward pass of the current state: mu, q-hat and the I-divergence partials.
  // (over the views of gg; partials of the I-divergence only when `pd` is not null)
  int forward_pass(hipStream_t s, const DevGeom& gg, double* pd) {
    const T* iv = i0v_used ? i0v : nullptr;
    if (d4) {
      // Daubechies-4: mu is not constant on the leaves; synthesize it per pixel (both
      // layouts) and project with the pixel walk
      {
        Scope sc(this, WAMCT_K_SYNTH, s);
        D4<T, R>::synth(g, tb, beta, mu, muT, s);
      }
      Scope sc(this, WAMCT_K_FORWARD, s);
      return Geo<T, R>::forward(gg, A, B, mu, muT, d, iv, scal + 4, q, nullptr, pd, P, s);
    }
    if (g.L > 0) {
      {
        Scope sc(this, WAMCT_K_SYNTH, s);
        Launch<T>::synth_records(g, beta, lev, leafR, leafC, P, s);
      }
      Scope sc(this, WAMCT_K_FORWARD, s);
      return Geo<T, R>::forward_records(gg, A, B, leafR, leafC, d, iv, scal + 4, q, nullptr, pd, P, s, walk_k);
    }
    {
      Scope sc(this, WAMCT_K_SYNTH, s);
      Launch<T>::synth_layouts(g, beta, mu, muT, P, s);
    }
    Scope sc(this, WAMCT_K_FORWARD, s);
    return Geo<T, R>::forward(gg, A, B, mu, muT, d, iv, scal + 4, q, nullptr, pd, P, s);
  }
  int forward_pass(hipStream_t s) { return forward_pass(s, g, partd); }
  // I-divergence of scan p -> out[p * ostride] (or out[p * ostride + counter] with the
  // device counters; out null: the scratch slot)
  void store_idiv(int nbk, double* out, int64_t ostride, bool counted, hipStream_t s) {
    Scope sc(this, WAMCT_K_OTHER, s);
    if (out)
      reduce_stack(false, partd, nbk, nbk, out, ostride, counted ? ints + 3 : nullptr, P, s);
    else
      reduce_stack(false, partd, nbk, nbk, scal + 3, kScal, nullptr, P, s);
  }
  wamct_status enq_iteration(hipStream_t s, double* out, int64_t ostride, bool counted) override {
    if (n_sub > 1) {
      // a pass of ordered subsets: the full I-divergence before the pass (when asked for),
      // then one update per subset with q-hat, b, b-hat+/- and Z0 of its rays
      if (out) store_idiv(forward_pass(s), out, ostride, counted, s);
      for (int k = 0; k < n_sub; ++k) {
        const Sel v = sel(k);
        forward_pass(s, v.g, nullptr);
        Scope sc(this, WAMCT_K_UPDATE, s);
        CHECKED(gather(kUpdate, q, segs_sub, P, beta, ints + 0, nullptr, nullptr, nullptr, s, v));
      }
      ++iters;
      LAUNCHED();
      return WAMCT_OK;
    }
    const int nbk = forward_pass(s);
    store_idiv(nbk, out, ostride, counted, s);
    if (d4) {
      {
        Scope sc(this, WAMCT_K_UPDATE, s);
        D4<T, R>::gather(g, kD4Update, tb, views, A, B, q, items, ints + 8, int(NN), beta, b, scal + 0, ints + 0,
                         nullptr, nullptr, nullptr, nullptr, s);
      }
      ++iters;
      LAUNCHED();
      return WAMCT_OK;
    }
    if (lam > 0.0) {
      // gradient of the roughness penalty at beta-hat for every coefficient:
      // Omega^T grad R(Omega beta-hat) (mu and part2 are free at this point of an iteration)
      Scope sc(this, WAMCT_K_OTHER, s);
      Launch<T>::mu64(g, beta, mu64, part2, P, s);
      Launch<T>::rough_grad(g, mu64, mu, P, s);
      for (int p = 0; p < P; ++p) Launch<T>::analysis(g, mu + p * NN, gpen + p * NN, s);
    }
    {
      Scope sc(this, WAMCT_K_UPDATE, s);
      CHECKED(gather(kUpdate, q, segs, P, beta, ints + 0, nullptr, nullptr, nullptr, s));
    }
    ++iters;
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status enq_final(hipStream_t s, double* out, int64_t ostride, bool counted) override {
    const int nbk = forward_pass(s);
    store_idiv(nbk, out, ostride, counted, s);
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status enq_begin(hipStream_t s) override {
    fill_i32_strided(ints + 3, P, kInts, 0, s);
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status iterate(int32_t n, double* idv) override {
    if (!has_data) return fail(WAMCT_E_STATE, "iterate before set_data");
    if (n < 0) return fail(WAMCT_E_INVALID, "n_iters must be >= 0");
    if (tree_dirty) CHECKED(rebuild_tree());
    for (int k = 0; k < n; ++k) CHECKED(enq_iteration(st, idv ? idv + k : nullptr, n, false));
    return WAMCT_OK;
  }

  // Tree rule (Results): FP64 synthesis, per-scan maximum, split, then the new tree. With
  // a shared tree the rule runs once, on the image summed over the stack's slices, and the
  // resulting tree is copied to every slice.
  wamct_status enq_expand(hipStream_t s, double frac) override {
    if (d4) {
      // the Results rule on the per-pixel FP64 image: a leaf splits when the largest pixel
      // of its block exceeds frac x the maximum
      {
        Scope sc(this, WAMCT_K_TREE, s);
        const int nbk = D4<T, R>::mu64(g, tb, beta, mu64, partd, s);
        reduce_stack(true, partd, nbk, nbk, scal + 2, kScal, nullptr, 1, s);
        HIPCHK(hipMemcpyAsync(mask_old, mask, NN, hipMemcpyDeviceToDevice, s));
        fill_i32_strided(ints + 2, 1, kInts, 0, s);
        expand(g, mask_old, mask, mu64, scal + 2, frac, ints + 2, 1, s, 2);
      }
      LAUNCHED();
      return enq_tree(s);
    }
    if (g.L > 0 && shared_tree && P > 1) {
      {
        Scope sc(this, WAMCT_K_TREE, s);
        Launch<T>::mu64(g, beta, mu64, partd, P, s);
        const int nbk = sum_slices(g, mu64, partd, P, s);
        reduce_stack(true, partd, nbk, nbk, scal + 2, kScal, nullptr, 1, s);
        HIPCHK(hipMemcpyAsync(mask_old, mask, NN, hipMemcpyDeviceToDevice, s));
        fill_i32_strided(ints + 2, P, kInts, 0, s);
        expand(g, mask_old, mask, mu64, scal + 2, frac, ints + 2, 1, s);
        for (int p = 1; p < P; ++p)
          HIPCHK(hipMemcpyAsync(mask + p * NN, mask, NN, hipMemcpyDeviceToDevice, s));
      }
      LAUNCHED();
      return enq_tree(s);
    }
    if (g.L > 0 && rule == WAMCT_RULE_GRADIENT) {
      // q-hat of the current beta over all views, residual d - q-hat (in q), then per scan
      // c = Omega^T H^T (d - q-hat) (in mu, free in tree runs) and the leaf scores (in mu64)
      forward_pass(s, g, nullptr);
      {
        Scope sc(this, WAMCT_K_TREE, s);
        Launch<T>::residual_inplace(d, q, M * P, s);
        for (int p = 0; p < P; ++p) {
          CHECKED(gather(kPlain, q + p * M, pix_segs, 1, nullptr, nullptr, nullptr, nullptr, img, s));
          Launch<T>::analysis(g, img, mu + p * NN, s);
        }
        Launch<double>::fill(mu64, NN * P, 0.0, s);
        HIPCHK(hipMemcpyAsync(mask_old, mask, NN * P, hipMemcpyDeviceToDevice, s));
        Launch<T>::grad_scores(g, mask_old, mu, mu64, P, s);
        reduce_stack(true, mu64, int(NN), int(NN), scal + 2, kScal, nullptr, P, s);
        fill_i32_strided(ints + 2, P, kInts, 0, s);
        expand(g, mask_old, mask, mu64, scal + 2, frac, ints + 2, P, s, WAMCT_RULE_GRADIENT);
      }
      LAUNCHED();
      return enq_tree(s);
    }
    if (g.L > 0) {
      {
        Scope sc(this, WAMCT_K_TREE, s);
        const int nbk = Launch<T>::mu64(g, beta, mu64, partd, P, s);
        reduce_stack(true, partd, nbk, nbk, scal + 2, kScal, nullptr, P, s);
        HIPCHK(hipMemcpyAsync(mask_old, mask, NN * P, hipMemcpyDeviceToDevice, s));
        fill_i32_strided(ints + 2, P, kInts, 0, s);
        expand(g, mask_old, mask, mu64, scal + 2, frac, ints + 2, P, s);
      }
      LAUNCHED();
    } else {
      fill_i32_strided(ints + 2, P, kInts, 0, s);
      LAUNCHED();
    }
    return enq_tree(s);
  }
  wamct_status expand_tree(double frac, int32_t* n_split) override {
    if (!(frac >= 0) || !std::isfinite(frac)) return fail(WAMCT_E_INVALID, "frac must be finite and >= 0");
    CHECKED(enq_expand(st, frac));
    HIPCHK(hipStreamSynchronize(st));
    return finish_tree(n_split);
  }

  wamct_status solve(int32_t n_iters, const int32_t* expand_at, int32_t n_expand, double frac,
                     double* idv) override {
    if (!has_data) return fail(WAMCT_E_STATE, "solve before set_data");
    if (!(frac >= 0) || !std::isfinite(frac)) return fail(WAMCT_E_INVALID, "frac must be finite and >= 0");
    if (!sched_at.empty() && n_expand > 0)
      return fail(WAMCT_E_INVALID, "a tree schedule is set: the expansion list must be empty");
    if (tree_dirty) CHECKED(rebuild_tree());
    const int64_t os = int64_t(n_iters) + 1;
    int e = 0;
    for (int j = 0; j < n_iters; ++j) {
      const int k = sched_index(j);
      if (k >= 0) {
        CHECKED(enq_schedule(st, k));
        HIPCHK(hipStreamSynchronize(st));
        CHECKED(finish_tree(nullptr));
      }
      while (e < n_expand && expand_at[e] < j) ++e;
      if (e < n_expand && expand_at[e] == j) {
        CHECKED(expand_tree(frac, nullptr));
        ++e;
      }
      CHECKED(enq_iteration(st, idv ? idv + j : nullptr, os, false));
    }
    return enq_final(st, idv ? idv + n_iters : nullptr, os, false);
  }

  // ---------------------------------------------------------------- tiling trials
  wamct_status save_state(hipStream_t s) override {
    if (!beta_save) {
      CHECKED(alloc(beta_save, NN * P));
      CHECKED(alloc(ints_save, int64_t(kInts) * P));
    }
    HIPCHK(hipMemcpyAsync(beta_save, beta, sizeof(T) * NN * P, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ints_save, ints, sizeof(int) * kInts * P, hipMemcpyDeviceToDevice, s));
    iters_save = iters;
    return WAMCT_OK;
  }
  wamct_status restore_state(hipStream_t s) override {
    if (!beta_save) return fail(WAMCT_E_STATE, "no saved state");
    HIPCHK(hipMemcpyAsync(beta, beta_save, sizeof(T) * NN * P, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ints, ints_save, sizeof(int) * kInts * P, hipMemcpyDeviceToDevice, s));
    iters = iters_save;
    return WAMCT_OK;
  }

  // ---------------------------------------------------------------- operators
  wamct_status synthesize(void* out) override {
    if (!out) return fail(WAMCT_E_INVALID, "mu must not be NULL");
    Scope sc(this, WAMCT_K_SYNTH, st);
    if (d4) D4<T, R>::synth(g, tb, beta, (T*)out, nullptr, st);
    else Launch<T>::synth(g, beta, (T*)out, P, st);
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status project(const void* m, void* p) override {
    if (!m || !p) return fail(WAMCT_E_INVALID, "mu and p must not be NULL");
    Scope sc(this, WAMCT_K_OTHER, st);
    Launch<T>::transpose(g.n, (const T*)m, muT, st);
    Geo<T, R>::forward(g, A, B, (const T*)m, muT, nullptr, nullptr, nullptr, nullptr, (T*)p, nullptr, 1, st);
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status backproject(const void* y, void* out) override {
    if (!y || !out) return fail(WAMCT_E_INVALID, "y and img must not be NULL");
    Scope sc(this, WAMCT_K_OTHER, st);
    CHECKED(gather(kPlain, (const T*)y, pix_segs, 1, nullptr, nullptr, nullptr, nullptr, (T*)out, st));
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status backproject_split(const void* y, void* bp, void* bm) override {
    if (!y || !bp || !bm) return fail(WAMCT_E_INVALID, "y, bp and bm must not be NULL");
    if (tree_dirty) CHECKED(rebuild_tree());
    Scope sc(this, WAMCT_K_OTHER, st);
    Launch<T>::fill((T*)bp, NN * P, T(0), st);
    Launch<T>::fill((T*)bm, NN * P, T(0), st);
    if (d4)
      D4<T, R>::gather(g, kD4Split, tb, views, A, B, (const T*)y, items, ints + 8, int(NN), nullptr, nullptr,
                       nullptr, nullptr, (T*)bp, (T*)bm, nullptr, nullptr, st);
    else
      CHECKED(gather(kSplit, (const T*)y, segs, P, nullptr, nullptr, (T*)bp, (T*)bm, nullptr, st));
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status forward(void* qo, double* idv) override {
    if (!has_data) return fail(WAMCT_E_STATE, "forward before set_data");
    if (tree_dirty) CHECKED(rebuild_tree());
    const int nbk = forward_pass(st);
    if (idv) reduce_stack(false, partd, nbk, nbk, idv, 1, nullptr, P, st);
    if (qo) HIPCHK(hipMemcpyAsync(qo, q, sizeof(T) * M * P, hipMemcpyDeviceToDevice, st));
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status idiv(const void* qq, double* out) override {
    if (!has_data) return fail(WAMCT_E_STATE, "idiv before set_data");
    if (!qq || !out) return fail(WAMCT_E_INVALID, "q and out must not be NULL");
    Scope sc(this, WAMCT_K_OTHER, st);
    const int nbk = Launch<T>::idiv_terms(g, (const T*)qq, d, partd, P, st);
    reduce_stack(false, partd, nbk, nbk, out, 1, nullptr, P, st);
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status get_b(void* out) override {
    if (!has_data) return fail(WAMCT_E_STATE, "get_b before set_data");
    if (!out) return fail(WAMCT_E_INVALID, "b must not be NULL");
    HIPCHK(hipMemcpyAsync(out, b, sizeof(T) * NN * P, hipMemcpyDeviceToDevice, st));
    return WAMCT_OK;
  }

  wamct_status tree_stats(double* z0, int64_t* w, int64_t* n_active, int64_t* n_held) override {
    if (tree_dirty) CHECKED(rebuild_tree());
    std::vector<double> sc(size_t(kScal) * P);
    std::vector<int> in(size_t(kInts) * P);
    HIPCHK(hipMemcpyAsync(sc.data(), scal, sizeof(double) * kScal * P, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(in.data(), ints, sizeof(int) * kInts * P, hipMemcpyDeviceToHost, st));
    std::vector<uint8_t> hm;
    if (n_active) {
      hm.resize(size_t(NN) * P);
      HIPCHK(hipMemcpyAsync(hm.data(), mask, NN * P, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int p = 0; p < P; ++p) {
      if (z0) z0[p] = sc[p * kScal + 0];
      if (w) w[p] = int64_t(llround(sc[p * kScal + 1]));
      if (n_held) n_held[p] = in[p * kInts + 0];
      if (n_active) {
        int64_t c = 0;
        const uint8_t* m = hm.data() + size_t(p) * NN;
        for (int64_t k = 0; k < NN; ++k) c += m[k];
        n_active[p] = c;
      }
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
    Launch<double>::fill(i0one, 1, i0p ? 1.0 : i0sc, st);
    for (int k = 0; k < batch; ++k) {
      const T* ck = (const T*)c + size_t(k) * NN;
      const T* dk = (const T*)dd + size_t(k) * M;
      const T* ik = i0p ? (const T*)i0p + size_t(k) * M : nullptr;
      T* qk = (T*)qout + size_t(k) * M;
      {
        Scope sc(this, WAMCT_K_SYNTH, st);
        if (d4) D4<T, R>::synth(g, tb, ck, mu, muT, st);
        else Launch<T>::synth_layouts(g, ck, mu, muT, 1, st);
      }
      int nbk;
      {
        Scope sc(this, WAMCT_K_FORWARD, st);
        nbk = Geo<T, R>::forward(g, A, B, mu, muT, dk, ik, i0one, qk, nullptr, partd, 1, st);
      }
      Scope sc(this, WAMCT_K_OTHER, st);
      reduce_sum(partd, nbk, lossd + k, st);
    }
    LAUNCHED();
    return WAMCT_OK;
  }

  // Hand-written adjoint: grad_b = s_b Omega^T H^T (d_b - q_b) from the saved q_b (s_b = the
  // incoming gradient of loss_b, null = 1). The residual is staged in the context's q-hat
  // buffer, so the solver's q-hat is overwritten.
  wamct_status loss_backward(int32_t batch, const void* qq, const void* dd, const double* gscale,
                             void* grad) override {
    if (batch < 0) return fail(WAMCT_E_INVALID, "batch must be >= 0");
    if (batch > 0 && (!qq || !dd || !grad)) return fail(WAMCT_E_INVALID, "q, d and grad must not be NULL");
    for (int k = 0; k < batch; ++k) {
      Scope sc(this, WAMCT_K_UPDATE, st);
      Launch<T>::residual((const T*)dd + size_t(k) * M, (const T*)qq + size_t(k) * M, gscale ? gscale + k : nullptr,
                          q, M, st);
      CHECKED(gather(kPlain, q, pix_segs, 1, nullptr, nullptr, nullptr, nullptr, img, st));
      if (d4) D4<T, R>::analysis(g, tb, img, (T*)grad + size_t(k) * NN, st);
      else Launch<T>::analysis(g, img, (T*)grad + size_t(k) * NN, st);
    }
    LAUNCHED();
    return WAMCT_OK;
  }

  wamct_status timing(int32_t on) override {
    HIPCHK(hipStreamSynchronize(st));
    harvest();
    for (int k = 0; k < WAMCT_NK; ++k) { tot_ms[k] = 0; tot_n[k] = 0; }
    if (on < 0 || on >= (1 << WAMCT_NK)) return fail(WAMCT_E_INVALID, fmt("timing mask %d outside [0, %d]", on, (1 << WAMCT_NK) - 1));
    timing_mask = uint32_t(on);
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

// ------------------------------------------------------------------ batches

// Several contexts (stacks of scans of different geometries) solved together. Each context
// is bound to one of the batch's streams (longest-processing-time-first by its work
// estimate); one iteration of every context is captured into a HIP graph (fork from the
// batch's main stream, one chain per stream, join) that is replayed for every iteration
// between two tree expansions. The expansions run on the same streams with one host
// synchronization for the whole batch. Per-scan I-divergence slots come from device
// counters, so every replay of the same graph writes the next slot.
struct wamct_batch {
  std::string err;
  std::vector<wamct_ctx*> ctx;
  std::vector<int> lane;
  std::vector<hipStream_t> streams;
  hipStream_t main = nullptr, caller = nullptr;
  hipEvent_t ev_main = nullptr, ev_in = nullptr;
  std::vector<hipEvent_t> ev_s;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = true;
  int64_t graph_launches = 0, graph_nodes = 0, captures = 0;

  wamct_status fail(wamct_status s, const std::string& m) {
    err = m;
    return s;
  }
  wamct_status from(wamct_ctx* c, wamct_status s) {
    err = c->err;
    return s;
  }
  void drop_graph() {
    if (exec || graph) hipStreamSynchronize(main);
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~wamct_batch() {
    if (main) hipStreamSynchronize(main);
    for (auto s : streams) hipStreamSynchronize(s);
    drop_graph();
    for (auto s : streams) hipStreamDestroy(s);
    if (main) hipStreamDestroy(main);
    for (auto e : ev_s) hipEventDestroy(e);
    if (ev_main) hipEventDestroy(ev_main);
    if (ev_in) hipEventDestroy(ev_in);
  }
  hipStream_t sof(size_t i) const { return streams[lane[i]]; }

  wamct_status init(int n, wamct_ctx* const* cs, int n_streams, int graph_on, hipStream_t s) {
    caller = s;
    use_graph = graph_on != 0;
    ctx.assign(cs, cs + n);
    HIPCHK(hipStreamCreateWithFlags(&main, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&ev_main, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
    streams.resize(n_streams, nullptr);
    ev_s.resize(n_streams, nullptr);
    for (int k = 0; k < n_streams; ++k) {
      HIPCHK(hipStreamCreateWithFlags(&streams[k], hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&ev_s[k], hipEventDisableTiming));
    }
    // longest processing time first
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ctx[a]->work() > ctx[b]->work(); });
    std::vector<double> load(n_streams, 0.0);
    lane.assign(n, 0);
    for (int i : order) {
      const int k = int(std::min_element(load.begin(), load.end()) - load.begin());
      lane[i] = k;
      load[k] += ctx[i]->work();
    }
    return WAMCT_OK;
  }
  // main waits for the caller's stream and every context's own stream
  wamct_status enter() {
    HIPCHK(hipEventRecord(ev_in, caller));
    HIPCHK(hipStreamWaitEvent(main, ev_in, 0));
    for (wamct_ctx* c : ctx) {
      HIPCHK(hipEventRecord(ev_in, c->stream()));
      HIPCHK(hipStreamWaitEvent(main, ev_in, 0));
    }
    return fork();
  }
  wamct_status fork() {
    HIPCHK(hipEventRecord(ev_main, main));
    for (auto s : streams) HIPCHK(hipStreamWaitEvent(s, ev_main, 0));
    return WAMCT_OK;
  }
  wamct_status join() {
    for (size_t k = 0; k < streams.size(); ++k) {
      HIPCHK(hipEventRecord(ev_s[k], streams[k]));
      HIPCHK(hipStreamWaitEvent(main, ev_s[k], 0));
    }
    return WAMCT_OK;
  }
  // the caller's stream and every context's stream wait for the batch's work
  wamct_status leave() {
    CHECKED(join());
    HIPCHK(hipEventRecord(ev_main, main));
    HIPCHK(hipStreamWaitEvent(caller, ev_main, 0));
    for (wamct_ctx* c : ctx) HIPCHK(hipStreamWaitEvent(c->stream(), ev_main, 0));
    return WAMCT_OK;
  }
  wamct_status sync_streams() {
    for (auto s : streams) HIPCHK(hipStreamSynchronize(s));
    return WAMCT_OK;
  }
  // tree work already enqueued on the streams: wait, then every context reads its counts
  wamct_status finish_trees() {
    CHECKED(sync_streams());
    for (wamct_ctx* c : ctx) {
      wamct_status r = c->finish_tree(nullptr);
      if (r) return from(c, r);
    }
    return WAMCT_OK;
  }

  wamct_status reset() {
    CHECKED(enter());
    for (size_t i = 0; i < ctx.size(); ++i) {
      wamct_status r = ctx[i]->enq_reset(sof(i));
      if (r) return from(ctx[i], r);
    }
    CHECKED(finish_trees());
    return leave();
  }

  wamct_status capture(double* const* idiv, int64_t os) {
    drop_graph();
    HIPCHK(hipStreamBeginCapture(main, hipStreamCaptureModeThreadLocal));
    wamct_status r = fork();
    for (size_t i = 0; i < ctx.size() && r == WAMCT_OK; ++i) {
      double* out = idiv ? idiv[i] : nullptr;
      wamct_status rc = ctx[i]->enq_iteration(sof(i), out, os, out != nullptr);
      if (rc) r = from(ctx[i], rc);
    }
    if (r == WAMCT_OK) r = join();
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(main, &gr);
    if (r != WAMCT_OK) {
      if (gr) hipGraphDestroy(gr);
      return r;
    }
    if (e != hipSuccess) return fail(WAMCT_E_HIP, fmt("hipStreamEndCapture: %s", hipGetErrorString(e)));
    graph = gr;
    HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    size_t nodes = 0;
    HIPCHK(hipGraphGetNodes(graph, nullptr, &nodes));
    graph_nodes = int64_t(nodes);
    ++captures;
    return WAMCT_OK;
  }

  wamct_status run(int k, double* const* idiv, int64_t os) {
    if (k <= 0) return WAMCT_OK;
    if (use_graph) {
      CHECKED(capture(idiv, os));  // counts one iteration per context
      CHECKED(join());
      for (int it = 0; it < k; ++it) {
        HIPCHK(hipGraphLaunch(exec, main));
        ++graph_launches;
      }
      for (wamct_ctx* c : ctx) c->count_iters(k - 1);
      return fork();
    }
    for (int it = 0; it < k; ++it)
      for (size_t i = 0; i < ctx.size(); ++i) {
        double* out = idiv ? idiv[i] : nullptr;
        wamct_status r = ctx[i]->enq_iteration(sof(i), out, os, out != nullptr);
        if (r) return from(ctx[i], r);
      }
    return WAMCT_OK;
  }

  wamct_status solve(int n_iters, const int32_t* at, int n_expand, double frac, double* const* idiv) {
    for (wamct_ctx* c : ctx)
      if (!c->has_data_()) return fail(WAMCT_E_STATE, "batch solve before set_data on every context");
    CHECKED(enter());
    bool dirty = false;
    for (size_t i = 0; i < ctx.size(); ++i)
      if (ctx[i]->tree_dirty_()) {
        wamct_status r = ctx[i]->enq_tree(sof(i));
        if (r) return from(ctx[i], r);
        dirty = true;
      }
    if (dirty) CHECKED(finish_trees());
    for (size_t i = 0; i < ctx.size(); ++i) {
      wamct_status r = ctx[i]->enq_begin(sof(i));
      if (r) return from(ctx[i], r);
    }
    const int64_t os = int64_t(n_iters) + 1;
    // tree changes: the batch's expansion list (the tree rule, for contexts without a tree
    // schedule) and every context's own schedule
    std::vector<int> events(at, at + n_expand);
    for (wamct_ctx* c : ctx) events.insert(events.end(), c->sched_at.begin(), c->sched_at.end());
    std::sort(events.begin(), events.end());
    events.erase(std::unique(events.begin(), events.end()), events.end());
    size_t e = 0;
    int j = 0;
    while (j < n_iters) {
      while (e < events.size() && events[e] < j) ++e;
      if (e < events.size() && events[e] == j) {
        const bool rule_now = std::binary_search(at, at + n_expand, j);
        bool changed = false;
        for (size_t i = 0; i < ctx.size(); ++i) {
          wamct_status r = WAMCT_OK;
          if (!ctx[i]->sched_at.empty()) {
            const int k = ctx[i]->sched_index(j);
            if (k >= 0) r = ctx[i]->enq_schedule(sof(i), k);
            changed = changed || k >= 0;
          } else if (rule_now) {
            r = ctx[i]->enq_expand(sof(i), frac);
            changed = true;
          }
          if (r) return from(ctx[i], r);
        }
        if (changed) CHECKED(finish_trees());
        ++e;
      }
      int stop = n_iters;
      if (e < events.size() && events[e] < stop) stop = events[e];
      CHECKED(run(stop - j, idiv, os));
      j = stop;
    }
    for (size_t i = 0; i < ctx.size(); ++i) {
      double* out = idiv ? idiv[i] : nullptr;
      wamct_status r = ctx[i]->enq_final(sof(i), out, os, out != nullptr);
      if (r) return from(ctx[i], r);
    }
    drop_graph();
    return leave();
  }

  // n_trial iterations of context c (after one untimed) timed with HIP events on its own
  // stream, its state restored afterwards: *ms
  wamct_status trial(wamct_ctx* c, int n_trial, hipEvent_t e0, hipEvent_t e1, float* ms) {
    const hipStream_t s = c->stream();
    wamct_status r = WAMCT_OK;
    if (c->tree_dirty_()) {
      r = c->enq_tree(s);
      if (!r && hipStreamSynchronize(s) != hipSuccess) r = fail(WAMCT_E_HIP, "synchronize");
      if (!r) r = c->finish_tree(nullptr);
    }
    if (!r) r = c->save_state(s);
    if (!r) r = c->enq_iteration(s, nullptr, 0, false);
    if (!r && hipEventRecord(e0, s) != hipSuccess) r = fail(WAMCT_E_HIP, "hipEventRecord");
    for (int t = 0; t < n_trial && !r; ++t) r = c->enq_iteration(s, nullptr, 0, false);
    if (!r && hipEventRecord(e1, s) != hipSuccess) r = fail(WAMCT_E_HIP, "hipEventRecord");
    if (!r) r = c->restore_state(s);
    if (!r && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess))
      r = fail(WAMCT_E_HIP, "trial timing failed");
    if (r && err.empty()) err = c->err;
    return r;
  }
  // Per context: the fastest backprojection tiling among the candidates, then (trees of
  // 2-D contexts) the fastest lanes per ray of the leaf walk among 1, 2 and 4 at that tiling.
  wamct_status autotune(int n_trial, const int32_t* cand, int n_cand, int32_t* chosen) {
    err.clear();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    wamct_status res = WAMCT_OK;
    for (size_t i = 0; i < ctx.size() && res == WAMCT_OK; ++i) {
      wamct_ctx* c = ctx[i];
      int32_t best = c->tiling();
      float best_ms = -1.f;
      for (int k = 0; k < n_cand && res == WAMCT_OK; ++k) {
        float ms = 0.f;
        wamct_status r = c->set_tiling(cand[k]);
        if (r) { err = c->err; res = r; break; }
        res = trial(c, n_trial, e0, e1, &ms);
        if (!res && (best_ms < 0 || ms < best_ms)) { best_ms = ms; best = cand[k]; }
      }
      if (res == WAMCT_OK) {
        wamct_status r = c->set_tiling(best);
        if (r) res = from(c, r);
      }
      if (chosen) chosen[i] = best;
      // lanes per ray of the leaf walk (contexts that have one)
      const int32_t auto_k = c->walk_lanes();
      if (res == WAMCT_OK && auto_k > 0 && c->set_walk_lanes(auto_k) == WAMCT_OK) {
        int32_t best_k = auto_k;
        float best_kms = -1.f;
        static const int32_t kLanes[] = {1, 2, 4};
        for (int32_t kk : kLanes) {
          float ms = 0.f;
          if (c->set_walk_lanes(kk)) break;
          res = trial(c, n_trial, e0, e1, &ms);
          if (res) break;
          if (best_kms < 0 || ms < best_kms) { best_kms = ms; best_k = kk; }
        }
        if (res == WAMCT_OK) c->set_walk_lanes(best_k);
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return res;
  }
};

// ------------------------------------------------------------------ no-allocation I-divergence

// FP64 partial sums of wamct_idiv_noalloc: one copy per device, held until the process ends.
// Host code never passes this name to a kernel (on the host it is only a stand-in for the
// symbol); it passes the device address looked up below.
static __device__ __align__(256) double scratch[WAMCT_NOALLOC_MAX_PARTIALS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (which must be current), looked up once per device.
hipError_t scratch_on(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

template <typename T>
void idiv_into(const T* d, const T* q, int64_t rays, int scans, double* part, double* out, hipStream_t s) {
  DevGeom g{};
  g.nv = 1;
  g.nb = int(rays);
  const int nbk = Launch<T>::idiv_terms(g, q, d, part, scans, s);
  reduce_stack(false, part, nbk, nbk, out, 1, nullptr, scans, s);
}
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
  if (geom->kind == WAMCT_CONE) c = make_ctx3(*opt);
  else if (opt->dtype == WAMCT_F64) c = new Ctx<double, double>();
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
wamct_status wamct_set_data(wamct_ctx* ctx, const void* d, const void* i0, const double* i0s) { CTX_CALL(set_data(d, i0, i0s)); }
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
wamct_status wamct_set_tiling(wamct_ctx* ctx, int32_t lanes) { CTX_CALL(set_tiling(lanes)); }
wamct_status wamct_set_subsets(wamct_ctx* ctx, int32_t n_subsets) { CTX_CALL(set_subsets(n_subsets)); }
wamct_status wamct_set_tree_sharing(wamct_ctx* ctx, int32_t shared) { CTX_CALL(set_tree_sharing(shared)); }
wamct_status wamct_set_tree_rule(wamct_ctx* ctx, int32_t rule) { CTX_CALL(set_tree_rule(rule)); }
wamct_status wamct_set_penalty(wamct_ctx* ctx, double lambda) { CTX_CALL(set_penalty(lambda)); }
wamct_status wamct_set_walk_lanes(wamct_ctx* ctx, int32_t lanes) { CTX_CALL(set_walk_lanes(lanes)); }
wamct_status wamct_get_walk_lanes(wamct_ctx* ctx, int32_t* lanes) {
  if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; }
  if (!lanes) return ctx->fail(WAMCT_E_INVALID, "lanes must not be NULL");
  *lanes = ctx->walk_lanes();
  return WAMCT_OK;
}
wamct_status wamct_set_tree_schedule(wamct_ctx* ctx, int32_t n_trees, const int32_t* at, const uint8_t* masks) {
  CTX_CALL(set_tree_schedule(n_trees, at, masks));
}
wamct_status wamct_get_tree_schedule(wamct_ctx* ctx, int32_t* n_trees, int32_t* at, int32_t cap) {
  if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; }
  if (!n_trees) return ctx->fail(WAMCT_E_INVALID, "n_trees must not be NULL");
  *n_trees = int32_t(ctx->sched_at.size());
  for (int k = 0; at && k < cap && k < *n_trees; ++k) at[k] = ctx->sched_at[size_t(k)];
  return WAMCT_OK;
}
wamct_status wamct_get_penalty(wamct_ctx* ctx, double* lambda) {
  if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; }
  if (!lambda) return ctx->fail(WAMCT_E_INVALID, "lambda must not be NULL");
  *lambda = ctx->penalty();
  return WAMCT_OK;
}
wamct_status wamct_get_tree_rule(wamct_ctx* ctx, int32_t* rule) {
  if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; }
  if (!rule) return ctx->fail(WAMCT_E_INVALID, "rule must not be NULL");
  *rule = ctx->tree_rule();
  return WAMCT_OK;
}
wamct_status wamct_get_tree_sharing(wamct_ctx* ctx, int32_t* shared) {
  if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; }
  if (!shared) return ctx->fail(WAMCT_E_INVALID, "shared must not be NULL");
  *shared = ctx->tree_sharing();
  return WAMCT_OK;
}
wamct_status wamct_get_subsets(wamct_ctx* ctx, int32_t* n_subsets) {
  if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; }
  if (!n_subsets) return ctx->fail(WAMCT_E_INVALID, "n_subsets must not be NULL");
  *n_subsets = ctx->subsets();
  return WAMCT_OK;
}
wamct_status wamct_get_tiling(wamct_ctx* ctx, int32_t* lanes) {
  if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; }
  if (!lanes) return ctx->fail(WAMCT_E_INVALID, "lanes must not be NULL");
  *lanes = ctx->tiling();
  return WAMCT_OK;
}

static std::string check_schedule(int32_t n_iters, const int32_t* expand_at, int32_t n_expand, double frac) {
  if (n_iters < 0 || n_expand < 0 || (n_expand > 0 && !expand_at)) return "bad iteration count or expansion schedule";
  for (int k = 1; k < n_expand; ++k)
    if (expand_at[k] <= expand_at[k - 1]) return "expansion schedule must ascend";
  if (!(frac >= 0) || !std::isfinite(frac)) return "frac must be finite and >= 0";
  return "";
}

wamct_status wamct_solve(wamct_ctx* ctx, int32_t n_iters, const int32_t* expand_at, int32_t n_expand, double frac,
                         double* idiv) {
  if (!ctx) { g_last_error = "ctx is NULL"; return WAMCT_E_INVALID; }
  std::string e = check_schedule(n_iters, expand_at, n_expand, frac);
  if (!e.empty()) return ctx->fail(WAMCT_E_INVALID, e);
  return ctx->solve(n_iters, expand_at, n_expand, frac, idiv);
}

wamct_status wamct_batch_create(int32_t n_ctx, wamct_ctx* const* ctxs, int32_t n_streams, int32_t use_graph,
                                void* stream, wamct_batch** out) {
  if (!out) { g_last_error = "out must not be NULL"; return WAMCT_E_INVALID; }
  *out = nullptr;
  if (n_ctx < 1 || !ctxs) { g_last_error = "a batch needs at least one context"; return WAMCT_E_INVALID; }
  if (n_streams < 1 || n_streams > 64) { g_last_error = "n_streams outside [1, 64]"; return WAMCT_E_INVALID; }
  for (int i = 0; i < n_ctx; ++i) {
    if (!ctxs[i]) { g_last_error = fmt("context %d is NULL", i); return WAMCT_E_INVALID; }
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) { g_last_error = fmt("context %d appears twice", i); return WAMCT_E_INVALID; }
  }
  wamct_batch* b = new wamct_batch();
  wamct_status s = b->init(n_ctx, ctxs, n_streams, use_graph, static_cast<hipStream_t>(stream));
  if (s != WAMCT_OK) {
    g_last_error = b->err;
    delete b;
    return s;
  }
  *out = b;
  return WAMCT_OK;
}

wamct_status wamct_batch_destroy(wamct_batch* batch) {
  delete batch;
  return WAMCT_OK;
}

const char* wamct_batch_last_error(const wamct_batch* batch) {
  return batch ? batch->err.c_str() : g_last_error.c_str();
}

#define BATCH_CHECK()                                                      \
  do {                                                                     \
    if (!batch) { g_last_error = "batch is NULL"; return WAMCT_E_INVALID; } \
  } while (0)

wamct_status wamct_batch_reset(wamct_batch* batch) {
  BATCH_CHECK();
  return batch->reset();
}

wamct_status wamct_batch_solve(wamct_batch* batch, int32_t n_iters, const int32_t* expand_at, int32_t n_expand,
                               double frac, double* const* idiv) {
  BATCH_CHECK();
  std::string e = check_schedule(n_iters, expand_at, n_expand, frac);
  if (!e.empty()) return batch->fail(WAMCT_E_INVALID, e);
  return batch->solve(n_iters, expand_at, n_expand, frac, idiv);
}

wamct_status wamct_batch_autotune(wamct_batch* batch, int32_t n_trial, const int32_t* candidates,
                                  int32_t n_candidates, int32_t* chosen) {
  BATCH_CHECK();
  static const int32_t kDefault[] = {1 << 18, 1 << 19, 1 << 20, 1 << 21, 1 << 22};
  if (n_trial < 1) return batch->fail(WAMCT_E_INVALID, "n_trial must be >= 1");
  if (!candidates) {
    candidates = kDefault;
    n_candidates = int32_t(sizeof kDefault / sizeof kDefault[0]);
  }
  if (n_candidates < 1) return batch->fail(WAMCT_E_INVALID, "no candidate tilings");
  for (int k = 0; k < n_candidates; ++k)
    if (candidates[k] < kMinTargetLanes || candidates[k] > kMaxTargetLanes)
      return batch->fail(WAMCT_E_INVALID, fmt("candidate tiling %d outside [%d, %d]", candidates[k],
                                              kMinTargetLanes, kMaxTargetLanes));
  for (wamct_ctx* c : batch->ctx)
    if (!c->has_data_()) return batch->fail(WAMCT_E_STATE, "autotune before set_data on every context");
  return batch->autotune(n_trial, candidates, n_candidates, chosen);
}

wamct_status wamct_idiv_noalloc(int32_t dtype, int64_t n_rays, int32_t n_scans, const void* d, const void* q,
                               double* out, void* stream) {
  auto bad = [](wamct_status st, const std::string& m) {
    g_last_error = m;
    return st;
  };
  if (dtype != WAMCT_F32 && dtype != WAMCT_F64) return bad(WAMCT_E_INVALID, fmt("unknown dtype %d", dtype));
  if (n_rays < 1 || n_rays > (int64_t(1) << 31) - 1)
    return bad(WAMCT_E_INVALID, fmt("n_rays = %lld outside [1, 2^31 - 1]", (long long)n_rays));
  if (n_scans < 1 || n_scans > 65535) return bad(WAMCT_E_INVALID, fmt("n_scans = %d outside [1, 65535]", n_scans));
  if (!d || !q || !out) return bad(WAMCT_E_INVALID, "d, q and out must not be NULL");
  const int64_t need = int64_t(n_scans) * idiv_blocks(n_rays);
  if (need > WAMCT_NOALLOC_MAX_PARTIALS)
    return bad(WAMCT_E_INVALID, fmt("n_scans x ceil(n_rays / %d) = %lld partial sums exceed the static buffer "
                                    "of %lld", WAMCT_NOALLOC_RAYS_PER_PARTIAL, (long long)need,
                                    (long long)WAMCT_NOALLOC_MAX_PARTIALS));
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return bad(WAMCT_E_HIP, fmt("hipGetDevice: %s", hipGetErrorString(e)));
  if (dev < 0 || dev >= kMaxDevices) return bad(WAMCT_E_UNSUPPORTED, fmt("device %d >= %d", dev, kMaxDevices));
  double* part = nullptr;
  e = scratch_on(dev, &part);
  if (e != hipSuccess) return bad(WAMCT_E_HIP, fmt("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e)));
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == WAMCT_F32)
    idiv_into(static_cast<const float*>(d), static_cast<const float*>(q), n_rays, n_scans, part, out, s);
  else
    idiv_into(static_cast<const double*>(d), static_cast<const double*>(q), n_rays, n_scans, part, out, s);
  e = hipGetLastError();
  if (e != hipSuccess) return bad(WAMCT_E_HIP, fmt("kernel launch: %s", hipGetErrorString(e)));
  return WAMCT_OK;
}

wamct_status wamct_batch_stats(wamct_batch* batch, int32_t* stream_of_ctx, int64_t* graph_launches,
                               int64_t* graph_nodes, int64_t* captures) {
  BATCH_CHECK();
  if (stream_of_ctx)
    for (size_t i = 0; i < batch->ctx.size(); ++i) stream_of_ctx[i] = batch->lane[i];
  if (graph_launches) *graph_launches = batch->graph_launches;
  if (graph_nodes) *graph_nodes = batch->graph_nodes;
  if (captures) *captures = batch->captures;
  return WAMCT_OK;
}

}  // extern "C"
