// C ABI of wavelet-tree AM on a 3-D volume (include/wamct.h, geometry kind WAMCT_CONE):
// validation, buffers and the order of kernel launches for Algorithm 1 and the tree rule
// (arXiv 1508.04458, Introduction and Results) with a circular cone-beam scan and a 3-D Haar
// octree. One scan per context; device memory is allocated in wamct_create (and when a
// larger gather tiling is requested); iterating allocates nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "wamct_ctx.h"
#include "wamct_internal3.h"

using namespace wamct;

namespace wamct {

std::string validate3(const wamct_geometry* g, const wamct_options* o) {
  if (g->n < 2 || g->n > 512) return fmt("cone beam: n = %d outside [2, 512]", g->n);
  if (g->nz < 1 || g->nz > 512) return fmt("cone beam: nz = %d outside [1, 512]", g->nz);
  if (!(g->pixel > 0) || !std::isfinite(g->pixel)) return "pixel size must be finite and > 0";
  if (g->n_views < 1 || g->n_bins < 1 || g->n_rows < 1) return "n_views, n_bins and n_rows must be >= 1";
  if (int64_t(g->n_views) * g->n_bins * g->n_rows > (int64_t(1) << 34)) return "too many rays";
  if (!(g->bin_pitch > 0) || !(g->row_pitch > 0) || !std::isfinite(g->bin_pitch) || !std::isfinite(g->row_pitch))
    return "detector pitches must be finite and > 0";
  if (!std::isfinite(g->angle0) || !std::isfinite(g->angle_span)) return "angles must be finite";
  const double rc = 0.5 * g->n * g->pixel * std::sqrt(2.0);
  if (!(g->sod > rc)) return fmt("cone beam needs sod (%g) > the volume's circumradius in x-y (%g)", g->sod, rc);
  if (!(g->sdd > g->sod) || !std::isfinite(g->sdd)) return "cone beam needs finite sdd > sod";
  if (o->levels < 0 || o->levels > 4) return fmt("cone beam: levels = %d outside [0, 4]", o->levels);
  if (o->wavelet_dims != 0 && o->wavelet_dims != 2 && o->wavelet_dims != 3)
    return fmt("cone beam: wavelet_dims = %d outside {0, 2, 3}", o->wavelet_dims);
  if (o->wavelet != WAMCT_HAAR)
    return fmt("cone beam: wavelet = %d, only the Haar basis (0) is implemented for the cone beam", o->wavelet);
  if (o->wavelet_dims == 2) {
    if (g->n % (1 << o->levels)) return fmt("n = %d must be divisible by 2^levels = %d", g->n, 1 << o->levels);
  } else if (g->n % (1 << o->levels) || g->nz % (1 << o->levels)) {
    return fmt("n = %d and nz = %d must be divisible by 2^levels = %d", g->n, g->nz, 1 << o->levels);
  }
  if (o->dtype != WAMCT_F32 && o->dtype != WAMCT_F64) return fmt("unknown dtype %d", o->dtype);
  if (o->geometry != WAMCT_F64) return "cone beam: ray geometry is FP64 only";
  if (o->batch != 1) return "cone beam: one scan per context (batch = 1)";
  return "";
}

}  // namespace wamct

namespace {

template <typename T>
struct Ctx3 final : wamct_ctx {
  DevGeom3 g{};
  hipStream_t st = nullptr;
  int64_t M = 0, N = 0;
  int np = 0;
  double2* views = nullptr;
  T *d = nullptr, *i0v = nullptr, *q = nullptr, *beta = nullptr, *b = nullptr, *img = nullptr;
  T* yn = nullptr;                 // ray values scaled by |D| for the gather
  T* coefg = nullptr;              // Omega^T H^T (d - q-hat) of the residual-gradient rule
  int rule = WAMCT_RULE_VALUE;     // tree rule of the expansions
  uint8_t* sched = nullptr;        // [n trees][N] masks of the explicit tree schedule
  double2* colt = nullptr;         // [nv][nc] (1/Dx, 1/Dy)
  double *rowt = nullptr, *nrm = nullptr;  // [nr] 1/Dz, [nr][nc] |D|
  void *recR = nullptr, *recC = nullptr;
  uint8_t *mask = nullptr, *mask_old = nullptr, *lev = nullptr, *levC = nullptr;  // levC: [z][x][y]
  uint32_t* items = nullptr;
  int* list_tmp = nullptr;      // block counts and offsets of the work-list builder
  double *partd = nullptr, *part2 = nullptr, *mu64 = nullptr, *scal = nullptr;  // [0] Z0 [1] W [2] max [3] tmp [4] I0
  int* ints = nullptr;  // [0] held [1] bad [2] n_split [3] iteration counter [8] items [9 + k] level counts
  T* beta_save = nullptr;
  int* ints_save = nullptr;
  int32_t iters_save = 0;
  void* part = nullptr;
  int64_t part_cap = 0;
  int* h_ints = nullptr;
  double* h_scal = nullptr;
  std::vector<Segment> segs, vox_segs;
  std::vector<void*> allocs;
  bool has_data = false, tree_dirty = true, i0v_used = false;
  int32_t iters = 0;
  // gather tiling target: the 3-D update favours more view chunks than the 2-D one (measured
  // on the 512x512x256 cone workload: 84 ms per update pass at 2^20 lanes, 76 ms at 2^23)
  int target_lanes = 1 << 23;
  uint32_t timing_mask = 0;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double tot_ms[WAMCT_NK] = {0};
  int64_t tot_n[WAMCT_NK] = {0};

  ~Ctx3() override {
    if (st) hipStreamSynchronize(st);
    hipDeviceSynchronize();
    for (auto& r : recs) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
    for (auto e : pool) hipEventDestroy(e);
    for (void* p : allocs) hipFree(p);
    if (part) hipFree(part);
    if (sched) hipFree(sched);
    if (h_ints) hipHostFree(h_ints);
    if (h_scal) hipHostFree(h_scal);
  }

    RayF3 rayf() const { return RayF3{views, colt, rowt, nrm}; }
  // one z-slice as a 2-D image (the 2-D tree helpers take the slices as a stack)
  DevGeom slice_geom() const {
    DevGeom g2{};
    g2.kind = 1; g2.n = g.n; g2.L = g.L; g2.pixel = g.pixel;
    g2.nv = 1; g2.nb = 1; g2.vs0 = 0; g2.vss = 1; g2.nvs = 1;
    return g2;
  }
template <typename Q>
  wamct_status alloc(Q*& p, int64_t count) {
    void* v = nullptr;
    const size_t bytes = size_t(count > 0 ? count : 1) * sizeof(Q);
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(WAMCT_E_OOM, fmt("hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e)));
    }
    allocs.push_back(v);
    p = static_cast<Q*>(v);
    return WAMCT_OK;
  }

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
    Ctx3* c; int kind; hipStream_t s; hipEvent_t a = nullptr;
    Scope(Ctx3* c_, int k, hipStream_t s_) : c(c_), kind(k), s(s_) {
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

  // ---------------------------------------------------------------- gather tiling
  Segment make_segment(int kseg, int start, int count, int level) const {
    Segment sg{kseg, start, count, level, 1, g.nv};
    if (count > 0 && count < target_lanes) {
      int chunks = std::min(g.nv, (target_lanes + count - 1) / count);
      const int vpc = (g.nv + chunks - 1) / chunks;
      chunks = (g.nv + vpc - 1) / vpc;
      sg.chunks = chunks;
      sg.vpc = vpc;
    }
    return sg;
  }
  // a segment of c items has chunks <= min(nv, ceil(target / c)) and groups = ceil(chunks / 4),
  // so groups x c <= min(nv N, target) / 4 + min(N, target)
  int64_t part_need(int target) const {
    const int64_t t = std::min<int64_t>(target, int64_t(g.nv) * N);
    return int64_t(kSlots3) * (t / 4 + 1 + std::min<int64_t>(N, target));
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
    hipError_t e = hipMalloc(&part, size_t(need) * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      part = nullptr;
      return fail(WAMCT_E_OOM, fmt("hipMalloc(%zu bytes): %s", size_t(need) * sizeof(double), hipGetErrorString(e)));
    }
    part_cap = need;
    return WAMCT_OK;
  }
  // work-list segments: 0 split roots, 1 roots not split, 2 + m split nodes of level L - 1 - m
  void build_segs() {
    segs.clear();
    const int n_seg = g.L >= 1 ? g.L + 1 : 2;
    for (int k = 0; k < n_seg; ++k) {
      const int c = h_ints[9 + k];
      if (c > 0) segs.push_back(make_segment(k, 0, c, k <= 1 ? g.L : g.L - (k - 1)));
    }
    vox_segs = {make_segment(-1, 0, int(N), 0)};
  }
  wamct_status gather(int mode, const T* y, const std::vector<Segment>& sg, T* bt, int* held, T* bp, T* bm, T* out,
                      hipStream_t s) {
    for (const Segment& x : sg)
      if (x.chunks > 1 && int64_t(kSlots3) * ((x.chunks + 3) / 4) * x.count > part_cap)
        return fail(WAMCT_E_HIP, "internal: gather partial buffer too small for its tiling");
    const bool tree = &sg == &segs;
    Geo3<T>::scale_rays(g, y, nrm, yn, s);
    Geo3<T>::gather(g, mode, views, colt, rowt, yn, tree ? items : nullptr, tree ? ints + 9 : nullptr, sg.data(),
                    int(sg.size()), part, bt, b, scal + 0, held, bp, bm, out, s);
    return WAMCT_OK;
  }

  // ---------------------------------------------------------------- setup
  wamct_status init(const wamct_geometry& G, const wamct_options& O, hipStream_t s) override {
    st = s;
    g.n = G.n; g.nz = G.nz; g.nv = G.n_views; g.nr = G.n_rows; g.nc = G.n_bins; g.L = O.levels;
    g.wd = O.wavelet_dims == 2 ? 2 : 3;
    g.pixel = G.pixel; g.cpitch = G.bin_pitch; g.rpitch = G.row_pitch; g.sod = G.sod; g.sdd = G.sdd;
    M = int64_t(g.nv) * g.nr * g.nc;
    N = int64_t(g.n) * g.n * g.nz;
    np = int(std::max((M + 255) / 256, (N + 255) / 256)) + 8;   // walk grids: multiples of 8 blocks
    if (hipHostMalloc((void**)&h_ints, sizeof(int) * kInts, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_scal, sizeof(double) * kScal, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(WAMCT_E_OOM, "hipHostMalloc of the readback buffers failed");
    }
    std::memset(h_ints, 0, sizeof(int) * kInts);
    std::memset(h_scal, 0, sizeof(double) * kScal);
    CHECKED(alloc(views, g.nv));
    CHECKED(alloc(d, M)); CHECKED(alloc(i0v, M)); CHECKED(alloc(q, M)); CHECKED(alloc(yn, M));
    CHECKED(alloc(colt, int64_t(g.nv) * g.nc)); CHECKED(alloc(rowt, g.nr)); CHECKED(alloc(nrm, int64_t(g.nr) * g.nc));
    CHECKED(alloc(beta, N)); CHECKED(alloc(b, N)); CHECKED(alloc(img, N)); CHECKED(alloc(mu64, N));
    T *rr = nullptr, *rc = nullptr;
    CHECKED(alloc(rr, N)); CHECKED(alloc(rc, N));
    recR = rr; recC = rc;
    CHECKED(alloc(mask, N)); CHECKED(alloc(mask_old, N)); CHECKED(alloc(lev, N)); CHECKED(alloc(levC, N));
    CHECKED(alloc(items, N));
    CHECKED(alloc(list_tmp, list_scratch_ints3(g)));
    CHECKED(alloc(partd, np)); CHECKED(alloc(part2, np)); CHECKED(alloc(scal, kScal)); CHECKED(alloc(ints, kInts));
    CHECKED(ensure_part(target_lanes));
    vox_segs = {make_segment(-1, 0, int(N), 0)};
    std::vector<double2> hv(g.nv);
    for (int v = 0; v < g.nv; ++v) {
      const double a = G.angle0 + v * (G.angle_span / G.n_views);
      double c, sn;
      view_cos_sin(a, c, sn);
      hv[v] = make_double2(c, sn);
    }
    HIPCHK(hipMemcpyAsync(views, hv.data(), sizeof(double2) * g.nv, hipMemcpyHostToDevice, st));
    Geo3<T>::ray_factors(g, views, colt, rowt, nrm, st);
    fill_i32(ints, kInts, 0, st);
    Launch<double>::fill(scal, kScal, 0.0, st);
    Launch<T>::fill(q, M, T(0), st);
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
    double i0s = 1.0;
    if (!ii) {
      if (!i0h || !(i0h[0] > 0) || !std::isfinite(i0h[0])) return fail(WAMCT_E_INVALID, "scalar I0 must be finite and > 0");
      i0s = i0h[0];
    }
    HIPCHK(hipMemcpyAsync(d, dd, sizeof(T) * M, hipMemcpyDeviceToDevice, st));
    if (ii) HIPCHK(hipMemcpyAsync(i0v, ii, sizeof(T) * M, hipMemcpyDeviceToDevice, st));
    Launch<double>::fill(scal + 4, 1, i0s, st);
    fill_i32(ints + 1, 1, 0, st);
    Launch<T>::check(d, M, false, ints + 1, st);
    if (ii) Launch<T>::check(i0v, M, false, ints + 1, st);
    LAUNCHED();
    HIPCHK(hipMemcpyAsync(h_ints + 1, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h_ints[1]) return fail(WAMCT_E_INVALID, fmt("%d counts or I0 values are negative or not finite", h_ints[1]));
    i0v_used = ii != nullptr;
    // eq. 1.6: b = Phi^T d = Omega^T (H^T d)
    {
      Scope sc(this, WAMCT_K_OTHER, st);
      CHECKED(gather(kPlain, d, vox_segs, nullptr, nullptr, nullptr, nullptr, img, st));
      Geo3<T>::analysis(g, img, b, st);
    }
    LAUNCHED();
    has_data = true;
    return WAMCT_OK;
  }

  // ---------------------------------------------------------------- tree
  wamct_status enq_tree(hipStream_t s) override {
    {
      Scope sc(this, WAMCT_K_TREE, s);
      build_items3(g, mask, items, ints + 8, list_tmp, s);
      levmap3(g, mask, lev, levC, s);
      const int nbk = z0_partials3(g, rayf(), lev, levC, partd, part2, s);
      reduce_max(partd, nbk, scal + 0, s);
      reduce_sum(part2, nbk, scal + 1, s);
    }
    LAUNCHED();
    HIPCHK(hipMemcpyAsync(h_ints, ints, sizeof(int) * kInts, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(h_scal, scal, sizeof(double) * kScal, hipMemcpyDeviceToHost, s));
    tree_dirty = true;
    return WAMCT_OK;
  }
  wamct_status finish_tree(int32_t* n_split) override {
    build_segs();
    if (!(h_scal[0] > 0) || !std::isfinite(h_scal[0])) return fail(WAMCT_E_INVALID, "Z0 = 0: no ray crosses the volume");
    if (n_split) n_split[0] = h_ints[2];
    tree_dirty = false;
    return WAMCT_OK;
  }
  wamct_status rebuild_tree() {
    CHECKED(enq_tree(st));
    HIPCHK(hipStreamSynchronize(st));
    return finish_tree(nullptr);
  }
  wamct_status enq_reset(hipStream_t s) override {
    Launch<T>::fill(beta, N, T(0), s);
    approx_mask3(g, mask, s);
    fill_i32(ints + 0, 1, 0, s);
    fill_i32(ints + 2, 1, 0, s);
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
    HIPCHK(hipMemcpyAsync(mask_old, mk, N, hipMemcpyDeviceToDevice, st));
    fill_i32(ints + 1, 1, 0, st);
    check_mask3(g, mask_old, ints + 1, st);
    Launch<T>::check((const T*)bt, N, true, ints + 1, st);
    LAUNCHED();
    HIPCHK(hipMemcpyAsync(h_ints + 1, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h_ints[1]) return fail(WAMCT_E_INVALID, fmt("state rejected: %d invalid octree entries or non-finite coefficients", h_ints[1]));
    HIPCHK(hipMemcpyAsync(mask, mask_old, N, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(beta, bt, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
    Geo3<T>::apply_mask(g, beta, mask, st);
    fill_i32(ints + 0, 1, 0, st);
    LAUNCHED();
    iters = 0;
    return rebuild_tree();
  }
  wamct_status get_state(void* bt, uint8_t* mk, int32_t* it) override {
    if (bt) HIPCHK(hipMemcpyAsync(bt, beta, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
    if (mk) HIPCHK(hipMemcpyAsync(mk, mask, N, hipMemcpyDeviceToDevice, st));
    if (it) *it = iters;
    return WAMCT_OK;
  }

  // ---------------------------------------------------------------- iteration
  int forward_pass(hipStream_t s) {
    {
      Scope sc(this, WAMCT_K_SYNTH, s);
      Geo3<T>::synth_records(g, beta, lev, recR, recC, s);
    }
    Scope sc(this, WAMCT_K_FORWARD, s);
    return Geo3<T>::forward(g, rayf(), recR, recC, d, i0v_used ? i0v : nullptr, scal + 4, q, nullptr, partd, s);
  }
  void store_idiv(int nbk, double* out, bool counted, hipStream_t s) {
    Scope sc(this, WAMCT_K_OTHER, s);
    reduce_stack(false, partd, nbk, nbk, out ? out : scal + 3, 0, (out && counted) ? ints + 3 : nullptr, 1, s);
  }
  wamct_status enq_iteration(hipStream_t s, double* out, int64_t, bool counted) override {
    store_idiv(forward_pass(s), out, counted, s);
    {
      Scope sc(this, WAMCT_K_UPDATE, s);
      CHECKED(gather(kUpdate, q, segs, beta, ints + 0, nullptr, nullptr, nullptr, s));
    }
    ++iters;
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status enq_final(hipStream_t s, double* out, int64_t, bool counted) override {
    store_idiv(forward_pass(s), out, counted, s);
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status enq_begin(hipStream_t s) override {
    fill_i32(ints + 3, 1, 0, s);
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status iterate(int32_t n, double* idv) override {
    if (!has_data) return fail(WAMCT_E_STATE, "iterate before set_data");
    if (n < 0) return fail(WAMCT_E_INVALID, "n_iters must be >= 0");
    if (tree_dirty) CHECKED(rebuild_tree());
    for (int k = 0; k < n; ++k) CHECKED(enq_iteration(st, idv ? idv + k : nullptr, 0, false));
    return WAMCT_OK;
  }
  wamct_status enq_expand(hipStream_t s, double frac) override {
    if (g.L > 0 && rule == WAMCT_RULE_GRADIENT) {
      // q-hat of the current beta, residual d - q-hat (in q), c = Omega^T H^T (d - q-hat),
      // leaf scores (in mu64) and the split of every leaf above frac x the largest score
      forward_pass(s);
      {
        Scope sc(this, WAMCT_K_TREE, s);
        Launch<T>::residual_inplace(d, q, M, s);
        CHECKED(gather(kPlain, q, vox_segs, nullptr, nullptr, nullptr, nullptr, img, s));
        Geo3<T>::analysis(g, img, coefg, s);
        Launch<double>::fill(mu64, N, 0.0, s);
        HIPCHK(hipMemcpyAsync(mask_old, mask, N, hipMemcpyDeviceToDevice, s));
        Geo3<T>::grad_scores(g, mask_old, coefg, mu64, s);
        reduce_max(mu64, int(N), scal + 2, s);
        fill_i32(ints + 2, 1, 0, s);
        expand3(g, mask_old, mask, mu64, scal + 2, frac, ints + 2, s, WAMCT_RULE_GRADIENT);
      }
      LAUNCHED();
      return enq_tree(s);
    }
    if (g.L > 0 && g.wd == 2) {
      // Results: every slice synthesized (FP64), the images summed over the slices (in slice
      // order), and the tree every slice shares grown on the summed image
      {
        Scope sc(this, WAMCT_K_TREE, s);
        Geo3<T>::mu64(g, beta, mu64, partd, s);
        const DevGeom g2 = slice_geom();
        const int nbk = sum_slices(g2, mu64, partd, g.nz, s);
        reduce_max(partd, nbk, scal + 2, s);
        HIPCHK(hipMemcpyAsync(mask_old, mask, size_t(g.n) * g.n, hipMemcpyDeviceToDevice, s));
        fill_i32(ints + 2, 1, 0, s);
        expand(g2, mask_old, mask, mu64, scal + 2, frac, ints + 2, 1, s);
        broadcast_slice3(g, mask, s);
      }
      LAUNCHED();
    } else if (g.L > 0) {
      {
        Scope sc(this, WAMCT_K_TREE, s);
        const int nbk = Geo3<T>::mu64(g, beta, mu64, partd, s);
        reduce_max(partd, nbk, scal + 2, s);
        HIPCHK(hipMemcpyAsync(mask_old, mask, N, hipMemcpyDeviceToDevice, s));
        fill_i32(ints + 2, 1, 0, s);
        expand3(g, mask_old, mask, mu64, scal + 2, frac, ints + 2, s);
      }
      LAUNCHED();
    } else {
      fill_i32(ints + 2, 1, 0, s);
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
  // Explicit Z_s^(j): the octree masks are validated and copied into the context.
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
    const size_t bytes = size_t(n) * N;
    hipError_t er = hipMalloc((void**)&sched, bytes);
    if (er != hipSuccess) {
      (void)hipGetLastError();
      sched = nullptr;
      return fail(WAMCT_E_OOM, fmt("hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(er)));
    }
    HIPCHK(hipMemcpyAsync(sched, mk, bytes, hipMemcpyDeviceToDevice, st));
    fill_i32(ints + 1, 1, 0, st);
    for (int k = 0; k < n; ++k) check_mask3(g, sched + size_t(k) * N, ints + 1, st);
    LAUNCHED();
    HIPCHK(hipMemcpyAsync(h_ints + 1, ints + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h_ints[1]) {
      HIPCHK(hipFree(sched));
      sched = nullptr;
      return fail(WAMCT_E_INVALID, fmt("tree schedule rejected: %d invalid octree entries", h_ints[1]));
    }
    sched_at.assign(at, at + n);
    return WAMCT_OK;
  }
  wamct_status enq_schedule(hipStream_t s, int k) override {
    {
      Scope sc(this, WAMCT_K_TREE, s);
      HIPCHK(hipMemcpyAsync(mask, sched + size_t(k) * N, N, hipMemcpyDeviceToDevice, s));
      Geo3<T>::apply_mask(g, beta, mask, s);
      fill_i32(ints + 2, 1, 0, s);
    }
    LAUNCHED();
    return enq_tree(s);
  }
  wamct_status solve(int32_t n_iters, const int32_t* expand_at, int32_t n_expand, double frac,
                     double* idv) override {
    if (!has_data) return fail(WAMCT_E_STATE, "solve before set_data");
    if (!sched_at.empty() && n_expand > 0)
      return fail(WAMCT_E_INVALID, "a tree schedule is set: the expansion list must be empty");
    if (tree_dirty) CHECKED(rebuild_tree());
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
      CHECKED(enq_iteration(st, idv ? idv + j : nullptr, 0, false));
    }
    return enq_final(st, idv ? idv + n_iters : nullptr, 0, false);
  }
  wamct_status save_state(hipStream_t s) override {
    if (!beta_save) {
      CHECKED(alloc(beta_save, N));
      CHECKED(alloc(ints_save, kInts));
    }
    HIPCHK(hipMemcpyAsync(beta_save, beta, sizeof(T) * N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ints_save, ints, sizeof(int) * kInts, hipMemcpyDeviceToDevice, s));
    iters_save = iters;
    return WAMCT_OK;
  }
  wamct_status restore_state(hipStream_t s) override {
    if (!beta_save) return fail(WAMCT_E_STATE, "no saved state");
    HIPCHK(hipMemcpyAsync(beta, beta_save, sizeof(T) * N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(ints, ints_save, sizeof(int) * kInts, hipMemcpyDeviceToDevice, s));
    iters = iters_save;
    return WAMCT_OK;
  }
  void count_iters(int k) override { iters += k; }

  // ---------------------------------------------------------------- operators
  wamct_status synthesize(void* out) override {
    if (!out) return fail(WAMCT_E_INVALID, "mu must not be NULL");
    Geo3<T>::synth(g, beta, (T*)out, st);
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status project(const void* m, void* p) override {
    if (!m || !p) return fail(WAMCT_E_INVALID, "mu and p must not be NULL");
    Scope sc(this, WAMCT_K_OTHER, st);
    Geo3<T>::synth_records(g, (const T*)m, nullptr, recR, recC, st);   // the volume itself, one voxel per leaf
    Geo3<T>::forward(g, rayf(), recR, recC, nullptr, nullptr, nullptr, nullptr, (T*)p, nullptr, st);
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status backproject(const void* y, void* out) override {
    if (!y || !out) return fail(WAMCT_E_INVALID, "y and img must not be NULL");
    Scope sc(this, WAMCT_K_OTHER, st);
    CHECKED(gather(kPlain, (const T*)y, vox_segs, nullptr, nullptr, nullptr, nullptr, (T*)out, st));
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status backproject_split(const void* y, void* bp, void* bm) override {
    if (!y || !bp || !bm) return fail(WAMCT_E_INVALID, "y, bp and bm must not be NULL");
    if (tree_dirty) CHECKED(rebuild_tree());
    Launch<T>::fill((T*)bp, N, T(0), st);
    Launch<T>::fill((T*)bm, N, T(0), st);
    CHECKED(gather(kSplit, (const T*)y, segs, nullptr, nullptr, (T*)bp, (T*)bm, nullptr, st));
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status forward(void* qo, double* idv) override {
    if (!has_data) return fail(WAMCT_E_STATE, "forward before set_data");
    if (tree_dirty) CHECKED(rebuild_tree());
    const int nbk = forward_pass(st);
    if (idv) reduce_sum(partd, nbk, idv, st);
    if (qo) HIPCHK(hipMemcpyAsync(qo, q, sizeof(T) * M, hipMemcpyDeviceToDevice, st));
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status idiv(const void* qq, double* out) override {
    if (!has_data) return fail(WAMCT_E_STATE, "idiv before set_data");
    if (!qq || !out) return fail(WAMCT_E_INVALID, "q and out must not be NULL");
    if (M > (int64_t(1) << 31) - 1) return fail(WAMCT_E_UNSUPPORTED, "idiv of more than 2^31 rays");
    DevGeom flat{};
    flat.nv = 1; flat.nb = int(M);
    const int nbk = Launch<T>::idiv_terms(flat, (const T*)qq, d, partd, 1, st);
    reduce_sum(partd, nbk, out, st);
    LAUNCHED();
    return WAMCT_OK;
  }
  wamct_status get_b(void* out) override {
    if (!has_data) return fail(WAMCT_E_STATE, "get_b before set_data");
    if (!out) return fail(WAMCT_E_INVALID, "b must not be NULL");
    HIPCHK(hipMemcpyAsync(out, b, sizeof(T) * N, hipMemcpyDeviceToDevice, st));
    return WAMCT_OK;
  }
  wamct_status tree_stats(double* z0, int64_t* w, int64_t* n_active, int64_t* n_held) override {
    if (tree_dirty) CHECKED(rebuild_tree());
    double sc[2] = {0, 0};
    int held = 0;
    HIPCHK(hipMemcpyAsync(sc, scal, sizeof sc, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&held, ints, sizeof(int), hipMemcpyDeviceToHost, st));
    std::vector<uint8_t> hm;
    if (n_active) {
      hm.resize(size_t(N));
      HIPCHK(hipMemcpyAsync(hm.data(), mask, N, hipMemcpyDeviceToHost, st));
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
  wamct_status loss(int32_t, const void*, const void*, const void*, double, double*, void*) override {
    return fail(WAMCT_E_UNSUPPORTED, "the differentiable loss is implemented for 2-D scans only");
  }
  wamct_status loss_backward(int32_t, const void*, const void*, const double*, void*) override {
    return fail(WAMCT_E_UNSUPPORTED, "the differentiable loss is implemented for 2-D scans only");
  }
  wamct_status timing(int32_t on) override {
    if (on < 0 || on >= (1 << WAMCT_NK)) return fail(WAMCT_E_INVALID, fmt("timing mask %d outside [0, %d]", on, (1 << WAMCT_NK) - 1));
    HIPCHK(hipStreamSynchronize(st));
    harvest();
    for (int k = 0; k < WAMCT_NK; ++k) { tot_ms[k] = 0; tot_n[k] = 0; }
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
  wamct_status set_tiling(int32_t t) override {
    if (t < kMinTargetLanes || t > kMaxTargetLanes)
      return fail(WAMCT_E_INVALID, fmt("tiling %d outside [%d, %d]", t, kMinTargetLanes, kMaxTargetLanes));
    HIPCHK(hipStreamSynchronize(st));
    CHECKED(ensure_part(t));
    target_lanes = t;
    if (!tree_dirty) build_segs();
    else vox_segs = {make_segment(-1, 0, int(N), 0)};
    return WAMCT_OK;
  }
  int32_t tiling() const override { return target_lanes; }
  wamct_status set_subsets(int32_t ns) override {
    if (ns == 1) return WAMCT_OK;
    return fail(WAMCT_E_UNSUPPORTED, "ordered subsets are implemented for 2-D scans only");
  }
  int32_t subsets() const override { return 1; }
  wamct_status set_tree_sharing(int32_t on) override {
    if (on == 0) return WAMCT_OK;
    return fail(WAMCT_E_UNSUPPORTED, "tree sharing applies to stacks of 2-D slices");
  }
  int32_t tree_sharing() const override { return 0; }
  wamct_status set_tree_rule(int32_t r) override {
    if (r != WAMCT_RULE_VALUE && r != WAMCT_RULE_GRADIENT) return fail(WAMCT_E_INVALID, fmt("unknown tree rule %d", r));
    if (r == WAMCT_RULE_GRADIENT && g.wd == 2)
      return fail(WAMCT_E_UNSUPPORTED, "the residual-gradient rule is implemented for the octree (wavelet_dims 3)");
    HIPCHK(hipStreamSynchronize(st));
    if (r == WAMCT_RULE_GRADIENT && !coefg) CHECKED(alloc(coefg, N));   // gradient coefficients
    rule = r;
    return WAMCT_OK;
  }
  int32_t tree_rule() const override { return rule; }
  wamct_status set_penalty(double l) override {
    if (!(l >= 0.0) || !std::isfinite(l)) return fail(WAMCT_E_INVALID, "the penalty weight must be finite and >= 0");
    if (l > 0.0) return fail(WAMCT_E_UNSUPPORTED, "the roughness penalty is implemented for 2-D scans");
    return WAMCT_OK;
  }
  double penalty() const override { return 0.0; }
  int n_scans() const override { return 1; }
  hipStream_t stream() const override { return st; }
  double work() const override { return double(M) * double(g.n); }
  bool has_data_() const override { return has_data; }
  bool tree_dirty_() const override { return tree_dirty; }
};

}  // namespace

namespace wamct {
wamct_ctx* make_ctx3(const wamct_options& o) {
  if (o.dtype == WAMCT_F64) return new Ctx3<double>();
  return new Ctx3<float>();
}
}  // namespace wamct
