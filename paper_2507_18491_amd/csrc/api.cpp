// api.cpp -- C ABI of the layered-media dyadic FMM library (see include/lmfmm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "bessel_pq.h"
#include "../../include/lmfmm.h"
#include "gmres.h"
#include "kernels.h"
#include "plan.h"

#define TM_ROWS 64  // rows per M2L GEMM tile (32 per wave row, 2 wave rows)
#define TN_COLS 64

struct lm_ctx {
  int device = 0;
  std::string err;
  Medium med;
  bool layers_set = false;
  PlanParams prm;
  int m2l_variant = -1;       // M2L GEMM variant: -1 autotune per launch, else fixed
  int host_trees = 0;         // 1: octree records sorted on the host
  double tree_records = 0;    // records of every octree of the build
  float tree_sort_ms = 0;     // device time of their keys and sort
  Plan plan;
  bool built = false;
  DevPlan d;
  std::vector<void*> allocs;  // persistent device buffers of the current build
  double* d_src = nullptr;
  double* d_tgt = nullptr;
  // P2M work items (leaf, chunk, slot) of instances with p <= 12 ([0]) and
  // of higher orders ([1]), the sums of the leaves of several chunks (leaf,
  // first slot, chunks), and the scratch slots of those partials
  int* d_p2m[2] = {nullptr, nullptr};
  int* d_p2m_sum[2] = {nullptr, nullptr};
  int n_p2m[2] = {0, 0}, n_p2m_sum[2] = {0, 0}, p2m_p[2] = {0, 0};
  long long p2m_slots[2] = {0, 0};
  cd* p2m_part = nullptr;     // partial expansions [slot][rhs][3][(p+1)^2] of both groups
  long long p2m_part_cap = 0;
  std::vector<int*> d_m2m, d_l2l, d_l2p, d_p2p;
  std::vector<int> n_m2m, n_l2l, n_l2p, n_p2p;
  std::vector<int> l2p_inst;  // an instance of each L2P launch group (its kind and order)
  cd* ME = nullptr;
  cd* LE = nullptr;
  long long me_cap = 0, le_cap = 0;
  struct Chunk {
    int tile0, ntile, bt0, nbt;
    int variant = -1;                  // M2L GEMM variant chosen by the autotuner
    double ms[LM_M2L_VARIANTS] = {-1, -1, -1};  // its measurements (ms; < 0: none)
  };
  struct TileSet {            // M2L schedule for one right-hand-side count
    M2LTile* d_tiles = nullptr;
    long long* d_ybase = nullptr;
    std::vector<Chunk> chunks;
    int n_tiles = 0;
    long long y_need = 0;     // scratch elements
  };
  std::map<int, TileSet> tilesets;
  // lm_evaluate_noalloc: a single-right-hand-side M2L schedule whose work
  // buffers fit the static scratch (made with the build), their offsets in
  // the scratch (complex numbers: ME, LE, P2M partials, M2L outputs), and the
  // scratch bytes the build needs
  TileSet na_ts;
  bool na_ok = false;
  long long na_off[5] = {0, 0, 0, 0, 0};  // ME, LE, P2M partials, M2L outputs, direct-pair slots
  long long na_need = 0;
  cd* Y = nullptr;           // M2L scratch
  long long y_cap = 0;
  double t_plan_ms = 0, t_upload_ms = 0, t_tables_ms = 0;
  int pmax = 0;
  bool timing = false;
  struct EvSet {
    std::vector<hipEvent_t> ph;  // phase boundaries (LM_PHASES + 1)
    std::vector<int> kind;       // per timed launch: 0 M2L GEMM, 1 M2L reduction, 2 P2P, 3 S2T
    std::vector<hipEvent_t> sp;  // per timed launch: start and stop
  };
  std::vector<EvSet> evsets;  // per timed evaluation
  // adjoint and gradients
  bool p2p_red = false;                   // near-field arguments k r bounded: reduced-range sincos
  bool same_sets = false;                 // sources and targets are the same point array
  std::vector<double> host_src, host_tgt;  // kept when they differ (for the swapped build)
  std::vector<int64_t> host_soff, host_toff;
  lm_ctx* adj = nullptr;                   // swapped-role context (built on first use)
  MediumDev md;                            // medium as seen by the kernels
  struct S2TRange {
    int item0, n;  // work items of one component type (host grouping)
    bool smallz;   // |k_rho| rho <= 7.5 on Gamma_1: J0..J2 by their power series
  };
  std::vector<S2TRange> s2t_ranges;        // per reaction component with direct pairs
  // every component's work items in one launch per Bessel variant, longest
  // first, each target's totals in its own output slot, then one gather
  // that adds a point's slots in component order (forward, curl, gradient)
  int* d_s2t_items = nullptr;              // (target leaf, chunk, first slot, target order, source list, count)
  int* d_s2t_tlist = nullptr;              // per item: chunk positions of its targets in increasing t
  int* d_s2t_slist = nullptr;              // per item: its near source points in increasing u
  int s2t_launch[2][2] = {{0, 0}, {0, 0}}; // per variant (general, series): first item, count
  int* d_s2t_gpt = nullptr;                // points with slots
  int* d_s2t_gptr = nullptr;               // their slot ranges
  int* d_s2t_gslot = nullptr;              // slots in the points' fixed order
  int s2t_npts = 0;
  long long s2t_slots = 0;
  cd* S2TY = nullptr;                      // slot outputs [slot][rhs][3] (direct pairs, then the
  long long s2ty_cap = 0;                  // symmetric near field's partner sums: used one after the other)
  // symmetric free-space near field (targets are the sources): work items
  // (target leaf, chunk, first slot, partner range, own source box), the
  // partners (adjacent leaves of higher source-box id), and per point its
  // partner-sum slots in item order
  int* d_p2ps_items = nullptr;
  int p2ps_n = 0;
  int* d_p2ps_part = nullptr;
  int* d_p2ps_gpt = nullptr;
  int* d_p2ps_gptr = nullptr;
  int* d_p2ps_gslot = nullptr;
  int p2ps_npts = 0;
  long long p2ps_slots = 0;
  double p2ps_evals = 0;                   // kernel evaluations: own-leaf ordered pairs + partner pairs
  double contour_a = 0;
  cd* Jc = nullptr;                        // conjugated-input scratch
  long long jc_cap = 0;
  // iterative solve: Krylov basis and work vector, inner-product partials,
  // a small device block (vector table, sums, coefficients) and its pinned
  // host staging
  cd* kv_buf = nullptr;
  long long kv_cap = 0;
  cd* kv_part = nullptr;
  long long kv_part_cap = 0;
  void* kv_small = nullptr;
  void* kv_host = nullptr;
  size_t kv_small_cap = 0;
};

extern "C" int lm_destroy(lm_ctx* ctx);

static void clear_events(lm_ctx* ctx) {
  for (auto& v : ctx->evsets) {
    for (auto e : v.ph) hipEventDestroy(e);
    for (auto e : v.sp) hipEventDestroy(e);
  }
  ctx->evsets.clear();
}

static int fail(lm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPC(x)                                                                               \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess) return fail(ctx, LM_EHIP, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

static void free_build(lm_ctx* ctx) {
  clear_events(ctx);
  for (void* p : ctx->allocs) hipFree(p);
  ctx->allocs.clear();
  if (ctx->ME) hipFree(ctx->ME);
  if (ctx->LE) hipFree(ctx->LE);
  for (auto& kv : ctx->tilesets) {
    if (kv.second.d_tiles) hipFree(kv.second.d_tiles);
    if (kv.second.d_ybase) hipFree(kv.second.d_ybase);
  }
  ctx->tilesets.clear();
  if (ctx->na_ts.d_tiles) hipFree(ctx->na_ts.d_tiles);
  if (ctx->na_ts.d_ybase) hipFree(ctx->na_ts.d_ybase);
  ctx->na_ts = lm_ctx::TileSet();
  ctx->na_ok = false;
  ctx->na_need = 0;
  if (ctx->Y) hipFree(ctx->Y);
  ctx->Y = nullptr;
  ctx->y_cap = 0;
  ctx->ME = ctx->LE = nullptr;
  ctx->me_cap = ctx->le_cap = 0;
  if (ctx->p2m_part) hipFree(ctx->p2m_part);
  ctx->p2m_part = nullptr;
  ctx->p2m_part_cap = 0;
  for (int g = 0; g < 2; g++) {
    ctx->d_p2m[g] = ctx->d_p2m_sum[g] = nullptr;
    ctx->n_p2m[g] = ctx->n_p2m_sum[g] = ctx->p2m_p[g] = 0;
    ctx->p2m_slots[g] = 0;
  }
  ctx->d_m2m.clear();
  ctx->d_l2l.clear();
  ctx->d_l2p.clear();
  ctx->d_p2p.clear();
  ctx->n_m2m.clear();
  ctx->n_l2l.clear();
  ctx->n_l2p.clear();
  ctx->n_p2p.clear();
  ctx->l2p_inst.clear();
  memset(&ctx->d, 0, sizeof(ctx->d));
  ctx->built = false;
  if (ctx->adj) lm_destroy(ctx->adj);
  ctx->adj = nullptr;
  ctx->s2t_ranges.clear();
  ctx->d_s2t_items = ctx->d_s2t_gpt = ctx->d_s2t_gptr = ctx->d_s2t_gslot = nullptr;
  ctx->d_s2t_tlist = ctx->d_s2t_slist = nullptr;
  memset(ctx->s2t_launch, 0, sizeof(ctx->s2t_launch));
  ctx->s2t_npts = 0;
  ctx->s2t_slots = 0;
  ctx->d_p2ps_items = ctx->d_p2ps_part = ctx->d_p2ps_gpt = ctx->d_p2ps_gptr = ctx->d_p2ps_gslot = nullptr;
  ctx->p2ps_n = ctx->p2ps_npts = 0;
  ctx->p2ps_slots = 0;
  ctx->p2ps_evals = 0;
  if (ctx->S2TY) hipFree(ctx->S2TY);
  ctx->S2TY = nullptr;
  ctx->s2ty_cap = 0;
  if (ctx->Jc) hipFree(ctx->Jc);
  ctx->Jc = nullptr;
  ctx->jc_cap = 0;
  if (ctx->kv_buf) hipFree(ctx->kv_buf);
  if (ctx->kv_part) hipFree(ctx->kv_part);
  if (ctx->kv_small) hipFree(ctx->kv_small);
  if (ctx->kv_host) hipHostFree(ctx->kv_host);
  ctx->kv_buf = ctx->kv_part = nullptr;
  ctx->kv_small = ctx->kv_host = nullptr;
  ctx->kv_cap = ctx->kv_part_cap = 0;
  ctx->kv_small_cap = 0;
  ctx->same_sets = false;
  ctx->host_src.clear();
  ctx->host_tgt.clear();
  ctx->host_soff.clear();
  ctx->host_toff.clear();
}

// Host threads for the build's list construction: fn(i) for i < n, indices
// handed out one at a time; every fn writes only outputs of its own index,
// so the result does not depend on the thread count.
static unsigned host_threads() { return lm_host_thread_count(); }
static void par_for(size_t n, unsigned nth, const std::function<void(size_t)>& fn) {
  std::atomic<size_t> next_i{0};
  auto work = [&]() {
    for (size_t i = next_i++; i < n; i = next_i++) fn(i);
  };
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < nth && t < n; t++) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
}

template <class T>
static int upload(lm_ctx* ctx, T** out, const std::vector<T>& v) {
  *out = nullptr;
  if (v.empty()) return 0;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, v.size() * sizeof(T));
  if (e != hipSuccess) return fail(ctx, LM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  ctx->allocs.push_back(p);
  e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(ctx, LM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  *out = (T*)p;
  return 0;
}

static int dalloc(lm_ctx* ctx, void** out, size_t bytes) {
  *out = nullptr;
  if (bytes == 0) return 0;
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) return fail(ctx, LM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  ctx->allocs.push_back(*out);
  return 0;
}

// ---------------------------------------------------------------- static scratch
// Work buffers of lm_evaluate_noalloc, for callers that cannot allocate
// device memory: one array per GPU, held from the library's load until the
// process ends.  In host code `scratch` only names the array; its device
// address on each GPU comes from hipGetSymbolAddress (lm_create, once per
// device), and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[LM_NOALLOC_SCRATCH_BYTES];

#define LM_MAX_DEVICES 64
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[LM_MAX_DEVICES];   // device address of scratch per device
static int g_scratch_state[LM_MAX_DEVICES];   // 0: not looked up, 1: ok, -1: failed
static std::string g_scratch_err[LM_MAX_DEVICES];

// looks up the device address of `scratch` on device dev (with dev current);
// the caller's current device is restored
static void scratch_setup(int dev) {
  if (dev < 0 || dev >= LM_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_state[dev] != 0) return;
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e == hipSuccess) e = hipSetDevice(dev);
  void* ptr = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && !ptr) e = hipErrorInvalidSymbol;
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    g_scratch_state[dev] = -1;
    g_scratch_err[dev] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return;
  }
  g_scratch_ptr[dev] = ptr;
  g_scratch_state[dev] = 1;
}

// GEMM groups of one M2L block: runs of consecutive offsets that share one
// matrix (reaction: one table case, the offsets differing only in azimuth;
// free space: each offset alone).  f(o0, o1) gets the offsets [o0, o1).
template <class F>
static void m2l_groups(const Plan& pl, const M2LBlock& B, F&& f) {
  const M2LClass& C = pl.cls[B.cls];
  int o = 0;
  while (o < C.n_off) {
    int e = o + 1;
    if (C.nblk == 3)
      while (e < C.n_off && pl.offs[C.off0 + e].mat[0] == pl.offs[C.off0 + o].mat[0]) e++;
    f(o, e);
    o = e;
  }
}

static int make_schedule(lm_ctx* ctx, int n_rhs, long long budget, lm_ctx::TileSet& ts, long long* block_max);
static long long p2m_part_size(const lm_ctx* ctx, int n_rhs);

extern "C" {

int lm_default_params(lm_params* prm) {
  if (!prm) return LM_EINVAL;
  memset(prm, 0, sizeof(*prm));
  prm->p = 12;
  prm->p_free = 0;
  prm->free_depth = 0;
  prm->max_depth = 14;
  prm->gamma1_panels = 4;
  prm->contour_a = 0.0;
  prm->tail_digits = 60.0;
  prm->components = 3;
  prm->m2l_adapt = 1;
  prm->m2l_margin = 3.0;
  prm->react_s2t = 1;
  prm->m2l_variant = -1;
  prm->tol = 0.0;
  prm->host_trees = 0;
  return LM_OK;
}

int lm_create(lm_ctx** out, int hip_device) {
  if (!out) return LM_EINVAL;
  *out = nullptr;
  lm_ctx* ctx = new lm_ctx();
  ctx->device = hip_device;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || hip_device < 0 || hip_device >= n) {
    delete ctx;
    return LM_EHIP;
  }
  scratch_setup(hip_device);
  *out = ctx;
  return LM_OK;
}

int lm_destroy(lm_ctx* ctx) {
  if (!ctx) return LM_EINVAL;
  hipSetDevice(ctx->device);
  free_build(ctx);
  delete ctx;
  return LM_OK;
}

const char* lm_last_error(const lm_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int lm_set_layers(lm_ctx* ctx, int n_layers, const double* d_host, const double* k_host, const double* mu_host) {
  if (!ctx) return LM_EINVAL;
  if (n_layers < 1 || n_layers > LM_MAXL || !k_host || (n_layers > 1 && !d_host))
    return fail(ctx, LM_EINVAL, "n_layers out of range or null pointer");
  Medium m;
  m.n = n_layers;
  m.kmax = 0;
  for (int l = 0; l < n_layers; l++) {
    if (!(k_host[l] > 0) || !std::isfinite(k_host[l])) return fail(ctx, LM_EDOMAIN, "wavenumbers must be finite and > 0");
    const double mu = mu_host ? mu_host[l] : 1.0;
    if (!(mu > 0) || !std::isfinite(mu)) return fail(ctx, LM_EDOMAIN, "permeabilities must be finite and > 0");
    m.k[l] = k_host[l];
    m.mu[l] = mu;
    m.mu_one = m.mu_one && mu == 1.0;
    m.kmax = std::max(m.kmax, k_host[l]);
  }
  for (int l = 0; l < n_layers - 1; l++) {
    if (!std::isfinite(d_host[l])) return fail(ctx, LM_EDOMAIN, "interfaces must be finite");
    if (l > 0 && !(d_host[l] < d_host[l - 1])) return fail(ctx, LM_EDOMAIN, "interfaces must be strictly decreasing");
    m.d[l] = d_host[l];
  }
  ctx->med = m;
  ctx->layers_set = true;
  if (ctx->built) {
    hipSetDevice(ctx->device);
    free_build(ctx);
  }
  return LM_OK;
}

int lm_set_params(lm_ctx* ctx, const lm_params* p) {
  if (!ctx || !p) return LM_EINVAL;
  if (p->p < 1 || p->p > LM_PMAX_ORDER || p->p_free < 0 || p->p_free > LM_PMAX_ORDER)
    return fail(ctx, LM_EINVAL, "expansion order out of range (1..20)");
  if (p->max_depth < 1 || p->max_depth > 19) return fail(ctx, LM_EINVAL, "max_depth out of range (1..19)");
  if (p->components < 1 || p->components > 3) return fail(ctx, LM_EINVAL, "components must be 1, 2 or 3");
  if (p->m2l_adapt != 0 && p->m2l_adapt != 1) return fail(ctx, LM_EINVAL, "m2l_adapt must be 0 or 1");
  if (p->m2l_adapt && !(p->m2l_margin >= 0 && p->m2l_margin <= 30))
    return fail(ctx, LM_EINVAL, "m2l_margin out of range (0..30 decades)");
  if (p->react_s2t < 0 || p->react_s2t > 3) return fail(ctx, LM_EINVAL, "react_s2t must be 0, 1, 2 or 3");
  if (!(p->tol >= 0) || !std::isfinite(p->tol)) return fail(ctx, LM_EINVAL, "tol must be finite and >= 0");
  if (p->m2l_variant < -1 || p->m2l_variant >= LM_M2L_VARIANTS)
    return fail(ctx, LM_EINVAL, "m2l_variant must be -1 (autotune) or 0.." + std::to_string(LM_M2L_VARIANTS - 1));
  if (p->host_trees != 0 && p->host_trees != 1) return fail(ctx, LM_EINVAL, "host_trees must be 0 or 1");
  PlanParams q;
  q.p = p->p;
  q.p_free = p->p_free;
  q.free_depth = p->free_depth;
  q.max_depth = p->max_depth;
  q.gamma1_panels = p->gamma1_panels > 0 ? p->gamma1_panels : 4;
  q.contour_a = p->contour_a;
  q.tail_digits = p->tail_digits > 0 ? p->tail_digits : 60.0;
  q.components = p->components;
  q.m2l_adapt = p->m2l_adapt;
  q.m2l_margin = p->m2l_margin;
  q.react_s2t = p->react_s2t;
  q.tol = p->tol;
  ctx->prm = q;
  ctx->m2l_variant = p->m2l_variant;
  ctx->host_trees = p->host_trees;
  if (ctx->built) {
    hipSetDevice(ctx->device);
    free_build(ctx);
  }
  return LM_OK;
}

static bool finite_pts(const double* x, int64_t n) {
  for (int64_t i = 0; i < 3 * n; i++)
    if (!std::isfinite(x[i])) return false;
  return true;
}

static int build_common(lm_ctx* ctx, int n_geom, const int64_t* soff, const double* src_xyz, const int64_t* toff,
                        const double* tgt_xyz, void* stream);

int lm_build(lm_ctx* ctx, int64_t n_src, const double* src_xyz, int64_t n_tgt, const double* tgt_xyz,
             void* stream) {
  if (!ctx) return LM_EINVAL;
  if (!ctx->layers_set) return fail(ctx, LM_ESTATE, "lm_set_layers must be called before lm_build");
  if (n_src < 0 || n_tgt < 0 || (n_src > 0 && !src_xyz) || (n_tgt > 0 && !tgt_xyz))
    return fail(ctx, LM_EINVAL, "invalid point arrays");
  int64_t so[2] = {0, n_src}, to[2] = {0, n_tgt};
  return build_common(ctx, 1, so, src_xyz, to, tgt_xyz, stream);
}

int lm_build_batch(lm_ctx* ctx, int n_geom, const int64_t* src_off, const double* src_xyz, const int64_t* tgt_off,
                   const double* tgt_xyz, void* stream) {
  if (!ctx) return LM_EINVAL;
  if (!ctx->layers_set) return fail(ctx, LM_ESTATE, "lm_set_layers must be called before lm_build_batch");
  if (n_geom < 1 || n_geom > 65536 || !src_off || !tgt_off) return fail(ctx, LM_EINVAL, "invalid geometry count or offsets");
  if (src_off[0] != 0 || tgt_off[0] != 0) return fail(ctx, LM_EINVAL, "offsets must start at 0");
  for (int g = 0; g < n_geom; g++)
    if (src_off[g + 1] < src_off[g] || tgt_off[g + 1] < tgt_off[g])
      return fail(ctx, LM_EINVAL, "offsets must be non-decreasing");
  if ((src_off[n_geom] > 0 && !src_xyz) || (tgt_off[n_geom] > 0 && !tgt_xyz))
    return fail(ctx, LM_EINVAL, "invalid point arrays");
  return build_common(ctx, n_geom, src_off, src_xyz, tgt_off, tgt_xyz, stream);
}

static int build_common(lm_ctx* ctx, int n_geom, const int64_t* soff, const double* src_xyz, const int64_t* toff,
                        const double* tgt_xyz, void* stream) {
  const int64_t n_src = soff[n_geom], n_tgt = toff[n_geom];
  if (n_src > 2000000000LL || n_tgt > 2000000000LL) return fail(ctx, LM_EINVAL, "too many points");
  if (!finite_pts(src_xyz, n_src) || !finite_pts(tgt_xyz, n_tgt)) return fail(ctx, LM_EINVAL, "non-finite coordinates");
  const Medium& med = ctx->med;
  for (int pass = 0; pass < 2; pass++) {
    const double* x = pass ? tgt_xyz : src_xyz;
    int64_t n = pass ? n_tgt : n_src;
    for (int64_t i = 0; i < n; i++)
      for (int l = 0; l < med.n - 1; l++)
        if (fabs(x[3 * i + 2] - med.d[l]) <= 1e-12 * std::max(1.0, fabs(med.d[l])))
          return fail(ctx, LM_EDOMAIN, "a point lies on an interface");
  }
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  free_build(ctx);
  if (lm_upload_leg_tables()) return fail(ctx, LM_EHIP, "cannot upload the Legendre coefficient tables");
  auto t0 = std::chrono::steady_clock::now();
  // the points on the device first: the octrees' records are keyed and
  // sorted there
  int rc;
  {
    std::vector<double> sx(src_xyz, src_xyz + 3 * n_src), tx(tgt_xyz, tgt_xyz + 3 * n_tgt);
    if ((rc = upload(ctx, &ctx->d_src, sx))) return rc;
    if ((rc = upload(ctx, &ctx->d_tgt, tx))) return rc;
  }
  ctx->tree_records = 0;
  ctx->tree_sort_ms = 0;
  TreeSorter dev_sort = [&](const std::vector<TreeJob>& jobs, const std::vector<TreeSeg>& segs,
                            std::vector<uint64_t>& keys, std::vector<uint32_t>& pay,
                            std::vector<uint64_t>& boxes) -> std::string {
    std::string e =
        lm_device_tree_sort(jobs, segs, ctx->d_src, ctx->d_tgt, keys, pay, boxes, &ctx->tree_sort_ms, s);
    ctx->tree_records = (double)keys.size();
    return e;
  };
  std::string msg = lm_make_plan_multi(ctx->plan, med, ctx->prm, n_geom, soff, src_xyz, toff, tgt_xyz,
                                       ctx->host_trees || n_src == 0 || n_tgt == 0 ? nullptr : &dev_sort);
  if (!msg.empty()) {
    int code = LM_EDOMAIN;
    if (msg.compare(0, strlen(LM_PLAN_ACCURACY_PREFIX), LM_PLAN_ACCURACY_PREFIX) == 0)
      code = LM_EACCURACY;
    else if (msg.compare(0, 10, "tree sort:") == 0)
      code = msg.find("allocation") != std::string::npos ? LM_ENOMEM : LM_EHIP;
    return fail(ctx, code, msg);
  }
  auto t1 = std::chrono::steady_clock::now();
  Plan& pl = ctx->plan;
  ctx->pmax = std::max(pl.p, pl.pf);
  DevPlan& d = ctx->d;
  {
    // direct reaction near field: J0..J2 on Gamma_1 by their power series
    // where |k_rho| rho <= 7.5 for every pair of the component; the series
    // stops where the first omitted term (|z|/2)^{2n} / (n!)^2 falls below
    // 1e-19 at the largest |z| = a rho_max (at most LM_BPQ_NSERC terms,
    // enough for |z| = 7.5)
    const double a = ctx->prm.contour_a > 0 ? ctx->prm.contour_a : 1.5 * med.kmax;
    for (auto& ip : pl.inst) {
      ip.s2t_nser = 1;
      ip.s2t_smallz = 1;
      if (ip.kind != 1 || ip.s2t_rho < 0) continue;
      ip.s2t_smallz = a * ip.s2t_rho <= 7.5 ? 1 : 0;
      const double zh = 0.5 * a * ip.s2t_rho;
      double term = 1.0;
      while (ip.s2t_nser < LM_BPQ_NSERC) {
        term *= zh * zh / ((double)ip.s2t_nser * ip.s2t_nser);
        if (term < 1e-19) break;
        ip.s2t_nser++;
      }
    }
  }
  if ((rc = upload(ctx, &d.inst, pl.inst))) return rc;
  if ((rc = upload(ctx, &d.sbox, pl.sbox))) return rc;
  if ((rc = upload(ctx, &d.tbox, pl.tbox))) return rc;
  if ((rc = upload(ctx, &d.sbox_m2m, pl.sbox_m2m))) return rc;
  if ((rc = upload(ctx, &d.tbox_l2l, pl.tbox_l2l))) return rc;
  if ((rc = upload(ctx, &d.src_perm, pl.src_perm))) return rc;
  if ((rc = upload(ctx, &d.tgt_perm, pl.tgt_perm))) return rc;
  if ((rc = upload(ctx, &d.p2p_list, pl.p2p_list))) return rc;
  if ((rc = upload(ctx, &d.cls, pl.cls))) return rc;
  if ((rc = upload(ctx, &d.blocks, pl.blocks))) return rc;
  if ((rc = upload(ctx, &d.bt_tbox, pl.bt_tbox))) return rc;
  if ((rc = upload(ctx, &d.bt_ptr, pl.bt_ptr))) return rc;
  if ((rc = upload(ctx, &d.bt_pairs, pl.bt_pairs))) return rc;
  {
    std::vector<long long> pm(pl.pair_src.size());
    for (size_t q = 0; q < pm.size(); q++) pm[q] = pl.sbox[pl.pair_src[q]].me_off;
    if ((rc = upload(ctx, &d.pair_me, pm))) return rc;
  }
  if ((rc = upload(ctx, &d.bt_blk, pl.bt_blk))) return rc;
  if ((rc = upload(ctx, &d.pair_P, pl.pair_P))) return rc;
  if ((rc = upload(ctx, &d.pair_phi, pl.pair_phi))) return rc;
  if ((rc = upload(ctx, &d.gaunt, pl.gaunt))) return rc;
  d.gaunt_p = pl.gaunt_p;
  if ((rc = upload(ctx, &d.Bcoef, pl.Bcoef))) return rc;
  if ((rc = upload(ctx, &d.Ccoef, pl.Ccoef))) return rc;
  if ((rc = upload(ctx, &d.Ccoef0, pl.Ccoef0))) return rc;
  if ((rc = upload(ctx, &d.cases, pl.cases))) return rc;
  if ((rc = upload(ctx, &d.trans, pl.trans))) return rc;
  if ((rc = upload(ctx, &d.wq, std::vector<int>(LM_WQ_COUNT, 0)))) return rc;
  {
    // leaves of low-order instances (reaction components, typically few points
    // each) and of high-order ones are launched separately, each with LDS
    // sized for its own order
    // P2M work items: leaves of up to LM_P2M_CHUNK points write their
    // expansion; larger leaves are cut into chunks whose partials land in
    // scratch slots and are summed in chunk order (dense leaves spread over
    // many workgroups)
    std::vector<int> items[2], sums[2];
    for (int b : pl.p2m_leaves) {
      const int ip = pl.inst[pl.sbox[b].inst].p;
      const int g = ip <= 12 ? 0 : 1;
      ctx->p2m_p[g] = std::max(ctx->p2m_p[g], ip);
      const int n = pl.sbox[b].pt1 - pl.sbox[b].pt0;
      const int nch = (n + LM_P2M_CHUNK - 1) / LM_P2M_CHUNK;
      if (nch <= 1) {
        items[g].insert(items[g].end(), {b, 0, -1});
        continue;
      }
      const int slot0 = (int)ctx->p2m_slots[g];
      for (int c = 0; c < nch; c++) items[g].insert(items[g].end(), {b, c, slot0 + c});
      sums[g].insert(sums[g].end(), {b, slot0, nch});
      ctx->p2m_slots[g] += nch;
    }
    for (int g = 0; g < 2; g++) {
      if ((rc = upload(ctx, &ctx->d_p2m[g], items[g]))) return rc;
      if ((rc = upload(ctx, &ctx->d_p2m_sum[g], sums[g]))) return rc;
      ctx->n_p2m[g] = (int)items[g].size() / 3;
      ctx->n_p2m_sum[g] = (int)sums[g].size() / 3;
    }
  }
  for (auto& v : pl.m2m_parents) {
    int* p = nullptr;
    if ((rc = upload(ctx, &p, v))) return rc;
    ctx->d_m2m.push_back(p);
    ctx->n_m2m.push_back((int)v.size());
  }
  for (auto& v : pl.l2l_children) {
    int* p = nullptr;
    if ((rc = upload(ctx, &p, v))) return rc;
    ctx->d_l2l.push_back(p);
    ctx->n_l2l.push_back((int)v.size());
  }
  // Launch groups: instances that never share a target point run in one
  // launch: all free-space instances (a point lies in one layer), and the
  // instances of one reaction component type (lt, ls, up_t, up_s) across
  // geometries.  Groups launch in key order (free space first), so a point
  // receives its contributions in the same order in a batch of geometries
  // as in a build of its own geometry.
  auto group_of = [](const InstParams& ip) -> long long {
    if (ip.kind == 0) return -1;
    return (((long long)ip.lt * LM_MAXL + ip.ls) * 2 + ip.up_t) * 2 + ip.up_s;
  };
  {
    // L2P work items: (leaf, chunk of LM_L2P_CHUNK points), so that leaves
    // holding many points spread over many workgroups
    std::map<long long, std::vector<int>> items;
    std::map<long long, int> rep;
    for (size_t i = 0; i < pl.l2p_leaves.size(); i++) {
      const long long g = group_of(pl.inst[i]);
      int ch = LM_L2P_CHUNK(pl.inst[i].kind == 0 ? 0 : 1);
      std::vector<int>& v = items[g];
      rep.emplace(g, (int)i);
      for (int b : pl.l2p_leaves[i])
        for (int c = 0; c * ch < pl.tbox[b].pt1 - pl.tbox[b].pt0; c++) {
          v.push_back(b);
          v.push_back(c);
        }
    }
    for (auto& kv : items) {
      int* p = nullptr;
      if ((rc = upload(ctx, &p, kv.second))) return rc;
      ctx->d_l2p.push_back(p);
      ctx->n_l2p.push_back((int)kv.second.size() / 2);
      ctx->l2p_inst.push_back(rep[kv.first]);
    }
  }
  {
    // free-space near field: every free instance in one launch (each block
    // reads its wavenumber from its target box's instance)
    std::vector<int> v;
    for (auto& t : pl.p2p_tboxes) v.insert(v.end(), t.begin(), t.end());
    if (!v.empty()) {
      int* p = nullptr;
      if ((rc = upload(ctx, &p, v))) return rc;
      ctx->d_p2p.push_back(p);
      ctx->n_p2p.push_back((int)v.size() / 2);
    }
  }
  {
    // reaction near-field (S2T) work items: one launch per component type
    // and kernel variant (small or general complex arguments on Gamma_1)
    std::map<std::pair<long long, int>, std::vector<int>> items;
    const int n_items = (int)pl.s2t_items.size() / 2;
    for (int it = 0; it < n_items; it++) {
      const InstParams& ip = pl.inst[pl.tbox[pl.s2t_items[2 * it]].inst];
      std::vector<int>& v = items[std::make_pair(group_of(ip), ip.s2t_smallz)];
      v.push_back(pl.s2t_items[2 * it]);
      v.push_back(pl.s2t_items[2 * it + 1]);
    }
    std::vector<int> all;
    for (auto& kv : items) {
      lm_ctx::S2TRange r;
      r.item0 = (int)all.size() / 2;
      r.n = (int)kv.second.size() / 2;
      r.smallz = kv.first.second != 0;
      all.insert(all.end(), kv.second.begin(), kv.second.end());
      ctx->s2t_ranges.push_back(r);
    }
    // one launch per Bessel variant: slots are numbered in the fixed order
    // (component, leaf, chunk) of `all`; the launch order puts the longest
    // items first (rounds of 64 pairs times the component's node count), so
    // that the short ones fill the tail
    std::vector<int> slot0(n_items + 1, 0);
    long long slots = 0;
    for (int it = 0; it < (int)all.size() / 2; it++) {
      const TgtBox& tb = pl.tbox[all[2 * it]];
      const int t0 = tb.pt0 + all[2 * it + 1] * LM_S2T_CHUNK;
      slot0[it] = (int)slots;
      slots += std::min(LM_S2T_CHUNK, tb.pt1 - t0);
    }
    if (slots > 2000000000LL) return fail(ctx, LM_EINVAL, "too many direct reaction pair targets");
    ctx->s2t_slots = slots;
    std::vector<std::pair<double, int>> order[2];
    for (size_t r = 0; r < ctx->s2t_ranges.size(); r++) {
      const lm_ctx::S2TRange& R = ctx->s2t_ranges[r];
      for (int it = R.item0; it < R.item0 + R.n; it++) {
        const TgtBox& tb = pl.tbox[all[2 * it]];
        const int t0 = tb.pt0 + all[2 * it + 1] * LM_S2T_CHUNK;
        const long long nt = std::min(LM_S2T_CHUNK, tb.pt1 - t0);
        long long ns = 0;
        for (int li = tb.p2p0; li < tb.p2p1; li++) ns += pl.sbox[pl.p2p_list[li]].pt1 - pl.sbox[pl.p2p_list[li]].pt0;
        const double cost = (double)((nt * ns + LM_S2T_CHUNK - 1) / LM_S2T_CHUNK) * pl.inst[tb.inst].s2tn;
        order[R.smallz ? 1 : 0].push_back(std::make_pair(-cost, it));
      }
    }
    // per item: its targets ordered by t (distance of the effective location
    // from its interface plane) and its near sources by u (that of the
    // image), so that the pairs of one round of 64 have similar tail cuts
    // (the items and their list offsets in launch order here; the lists
    // themselves item by item on host threads, each into its own range)
    std::vector<int> items6, tlist, slist, seq;
    long long tl_n = 0, sl_n = 0;
    for (int v = 0; v < 2; v++) {
      std::stable_sort(order[v].begin(), order[v].end(),
                       [](const std::pair<double, int>& x, const std::pair<double, int>& y) { return x.first < y.first; });
      ctx->s2t_launch[v][0] = (int)items6.size() / 6;
      ctx->s2t_launch[v][1] = (int)order[v].size();
      for (auto& o : order[v]) {
        const int it = o.second;
        const TgtBox& tb = pl.tbox[all[2 * it]];
        const int t0 = tb.pt0 + all[2 * it + 1] * LM_S2T_CHUNK, nt = std::min(LM_S2T_CHUNK, tb.pt1 - t0);
        long long ns = 0;
        for (int li = tb.p2p0; li < tb.p2p1; li++) ns += pl.sbox[pl.p2p_list[li]].pt1 - pl.sbox[pl.p2p_list[li]].pt0;
        if (sl_n + ns > 2000000000LL) return fail(ctx, LM_EINVAL, "too many direct reaction pairs");
        items6.insert(items6.end(), {all[2 * it], all[2 * it + 1], slot0[it], (int)tl_n, (int)sl_n, (int)ns});
        seq.push_back(it);
        tl_n += nt;
        sl_n += ns;
      }
    }
    tlist.resize(tl_n);
    slist.resize(sl_n);
    par_for(seq.size(), host_threads(), [&](size_t k) {
      const int it = seq[k];
      const int* e = items6.data() + 6 * k;
      const TgtBox& tb = pl.tbox[all[2 * it]];
      const InstParams& ip = pl.inst[tb.inst];
      const int t0 = tb.pt0 + all[2 * it + 1] * LM_S2T_CHUNK, nt = std::min(LM_S2T_CHUNK, tb.pt1 - t0);
      const double dls = ip.up_s ? med.d[ip.ls - 1] : med.d[ip.ls];
      std::vector<std::pair<double, int>> tv, sv;
      tv.reserve(nt);
      sv.reserve(e[5]);
      for (int q = 0; q < nt; q++) {
        const double z = tgt_xyz[3 * pl.tgt_perm[t0 + q] + 2];
        tv.push_back(std::make_pair(ip.up_t ? z - med.d[ip.lt] : med.d[ip.lt - 1] - z, q));
      }
      for (int li = tb.p2p0; li < tb.p2p1; li++) {
        const SrcBox& sb = pl.sbox[pl.p2p_list[li]];
        for (int sp = sb.pt0; sp < sb.pt1; sp++) {
          const int sid = pl.src_perm[sp];
          const double z = src_xyz[3 * sid + 2];
          sv.push_back(std::make_pair(ip.up_s ? dls - z : z - dls, sid));
        }
      }
      auto by_first = [](const std::pair<double, int>& x, const std::pair<double, int>& y) { return x.first < y.first; };
      std::stable_sort(tv.begin(), tv.end(), by_first);
      std::stable_sort(sv.begin(), sv.end(), by_first);
      for (int q = 0; q < nt; q++) tlist[e[3] + q] = tv[q].second;
      for (int j = 0; j < e[5]; j++) slist[e[4] + j] = sv[j].second;
    });
    if ((rc = upload(ctx, &ctx->d_s2t_items, items6))) return rc;
    if ((rc = upload(ctx, &ctx->d_s2t_tlist, tlist))) return rc;
    if ((rc = upload(ctx, &ctx->d_s2t_slist, slist))) return rc;
    // gather lists: for each point with slots, its slots in `all` order
    std::vector<int> cnt(pl.n_tgt + 1, 0);
    for (int it = 0; it < (int)all.size() / 2; it++) {
      const TgtBox& tb = pl.tbox[all[2 * it]];
      const int t0 = tb.pt0 + all[2 * it + 1] * LM_S2T_CHUNK, t1 = std::min(tb.pt1, t0 + LM_S2T_CHUNK);
      for (int t = t0; t < t1; t++) cnt[pl.tgt_perm[t] + 1]++;
    }
    std::vector<int> gpt, gptr, start(pl.n_tgt, -1);
    int acc = 0;
    for (int64_t i = 0; i < pl.n_tgt; i++)
      if (cnt[i + 1] > 0) {
        start[i] = acc;
        gpt.push_back((int)i);
        gptr.push_back(acc);
        acc += cnt[i + 1];
      }
    gptr.push_back(acc);
    std::vector<int> gslot(acc), fill(pl.n_tgt, 0);
    for (int it = 0; it < (int)all.size() / 2; it++) {
      const TgtBox& tb = pl.tbox[all[2 * it]];
      const int t0 = tb.pt0 + all[2 * it + 1] * LM_S2T_CHUNK, t1 = std::min(tb.pt1, t0 + LM_S2T_CHUNK);
      for (int t = t0; t < t1; t++) {
        const int id = pl.tgt_perm[t];
        gslot[start[id] + fill[id]++] = slot0[it] + (t - t0);
      }
    }
    ctx->s2t_npts = (int)gpt.size();
    if ((rc = upload(ctx, &ctx->d_s2t_gpt, gpt))) return rc;
    if ((rc = upload(ctx, &ctx->d_s2t_gptr, gptr))) return rc;
    if ((rc = upload(ctx, &ctx->d_s2t_gslot, gslot))) return rc;
  }
  {
    // symmetric free-space near field, when the targets are the sources (the
    // same point of a free-space leaf is then a source and a target with the
    // same id): each unordered pair of adjacent leaves is evaluated once, in
    // the work items of the leaf with the lower source-box id
    const bool same = n_src == n_tgt && memcmp(soff, toff, (size_t)(n_geom + 1) * sizeof(int64_t)) == 0 &&
                      (src_xyz == tgt_xyz || n_src == 0 ||
                       memcmp(src_xyz, tgt_xyz, (size_t)n_src * 3 * sizeof(double)) == 0);
    std::vector<int> items6, part;
    long long slots = 0;
    double evals = 0;
    bool ok = same;
    for (size_t f = 0; ok && f < pl.p2p_tboxes.size(); f++)
      for (size_t i = 0; ok && i < pl.p2p_tboxes[f].size(); i += 2) {
        const int b = pl.p2p_tboxes[f][i], c = pl.p2p_tboxes[f][i + 1];
        const TgtBox& tb = pl.tbox[b];
        int self = -1;  // the source box of the same leaf
        for (int li = tb.p2p0; li < tb.p2p1; li++) {
          const SrcBox& sb = pl.sbox[pl.p2p_list[li]];
          if (sb.c[0] == tb.c[0] && sb.c[1] == tb.c[1] && sb.c[2] == tb.c[2] && sb.inst == tb.inst &&
              sb.pt1 - sb.pt0 == tb.pt1 - tb.pt0)
            self = pl.p2p_list[li];
        }
        if (self < 0) {
          ok = false;
          break;
        }
        const int p0 = (int)part.size();
        long long ns = 0;
        for (int li = tb.p2p0; li < tb.p2p1; li++)
          if (pl.p2p_list[li] > self) {
            part.push_back(pl.p2p_list[li]);
            ns += pl.sbox[pl.p2p_list[li]].pt1 - pl.sbox[pl.p2p_list[li]].pt0;
          }
        items6.insert(items6.end(), {b, c, (int)slots, p0, (int)part.size(), self});
        const int nt = std::min(LM_P2P_CHUNK, tb.pt1 - (tb.pt0 + c * LM_P2P_CHUNK));
        evals += (double)nt * ((pl.sbox[self].pt1 - pl.sbox[self].pt0) + ns);
        slots += ns;
        if (slots > 2000000000LL) ok = false;
      }
    if (ok && !items6.empty()) {
      // the items stay in box order (neighbouring items share partner
      // leaves in the cache; longest first measured no faster)
      // per point: its slots in item order.  The items are cut into nr
      // consecutive runs of about equal slot counts; each run counts its
      // slots per point, a point's slots from run r follow those of the
      // runs before it, and each run then fills its own positions (host
      // threads, the same lists as one pass over the items)
      const size_t n_it = items6.size() / 6;
      const int64_t nt_pts = pl.n_tgt;
      const unsigned nr = (unsigned)std::max<int64_t>(
          1, std::min<int64_t>(host_threads(), 250000000LL / std::max<int64_t>(1, nt_pts)));
      std::vector<size_t> run0(nr + 1, n_it);
      run0[0] = 0;
      for (unsigned r = 1, k = 0; r < nr; r++) {
        const long long target = slots * (long long)r / nr;
        while (k < n_it && items6[6 * k + 2] < target) k++;
        run0[r] = k;
      }
      std::vector<std::vector<int>> rcnt(nr);
      par_for(nr, nr, [&](size_t r) {
        rcnt[r].assign(nt_pts, 0);
        int* c = rcnt[r].data();
        for (size_t k = run0[r]; k < run0[r + 1]; k++)
          for (int pi = items6[6 * k + 3]; pi < items6[6 * k + 4]; pi++) {
            const SrcBox& sb = pl.sbox[part[pi]];
            for (int pt = sb.pt0; pt < sb.pt1; pt++) c[pl.src_perm[pt]]++;
          }
      });
      const int64_t blk = 1 << 16;
      const size_t nblk = (size_t)((nt_pts + blk - 1) / blk);
      std::vector<int> cnt(nt_pts, 0);
      par_for(nblk, host_threads(), [&](size_t bi) {
        for (int64_t i = bi * blk; i < std::min<int64_t>(nt_pts, (bi + 1) * blk); i++)
          for (unsigned r = 0; r < nr; r++) cnt[i] += rcnt[r][i];
      });
      std::vector<int> gpt, gptr, start(nt_pts, -1);
      int acc = 0;
      for (int64_t i = 0; i < nt_pts; i++)
        if (cnt[i] > 0) {
          start[i] = acc;
          gpt.push_back((int)i);
          gptr.push_back(acc);
          acc += cnt[i];
        }
      gptr.push_back(acc);
      // each run's counts become its first position per point
      par_for(nblk, host_threads(), [&](size_t bi) {
        for (int64_t i = bi * blk; i < std::min<int64_t>(nt_pts, (bi + 1) * blk); i++) {
          int off = start[i];
          for (unsigned r = 0; r < nr; r++) {
            const int c = rcnt[r][i];
            rcnt[r][i] = off;
            off += c;
          }
        }
      });
      std::vector<int> gslot(acc);
      par_for(nr, nr, [&](size_t r) {
        int* pos = rcnt[r].data();
        for (size_t k = run0[r]; k < run0[r + 1]; k++) {
          long long so = items6[6 * k + 2];
          for (int pi = items6[6 * k + 3]; pi < items6[6 * k + 4]; pi++) {
            const SrcBox& sb = pl.sbox[part[pi]];
            for (int pt = sb.pt0; pt < sb.pt1; pt++) gslot[pos[pl.src_perm[pt]]++] = (int)(so + (pt - sb.pt0));
            so += sb.pt1 - sb.pt0;
          }
        }
      });
      if ((rc = upload(ctx, &ctx->d_p2ps_items, items6))) return rc;
      if ((rc = upload(ctx, &ctx->d_p2ps_part, part))) return rc;
      if ((rc = upload(ctx, &ctx->d_p2ps_gpt, gpt))) return rc;
      if ((rc = upload(ctx, &ctx->d_p2ps_gptr, gptr))) return rc;
      if ((rc = upload(ctx, &ctx->d_p2ps_gslot, gslot))) return rc;
      ctx->p2ps_n = (int)(items6.size() / 6);
      ctx->p2ps_npts = (int)gpt.size();
      ctx->p2ps_slots = slots;
      ctx->p2ps_evals = evals;
    }
  }
  // matrices and table scratch
  void* vp = nullptr;
  if ((rc = dalloc(ctx, &vp, (size_t)pl.mat_size * sizeof(cd)))) return rc;
  d.mats = (cd*)vp;
  auto t2 = std::chrono::steady_clock::now();
  launch_trans(d, (int)pl.trans.size(), pl.gaunt_p, s);
  HIPC(hipGetLastError());
  MediumDev md;
  memset(&md, 0, sizeof(md));
  md.n = med.n;
  for (int l = 0; l < med.n; l++) {
    md.k[l] = med.k[l];
    md.mu[l] = med.mu[l];
  }
  for (int l = 0; l < med.n - 1; l++) md.d[l] = med.d[l];
  ctx->md = md;
  ctx->contour_a = ctx->prm.contour_a > 0 ? ctx->prm.contour_a : 1.5 * med.kmax;
  d.nodes = nullptr;
  if (!pl.node_kr.empty()) {
    // quadrature nodes with their densities: read by the table kernels
    // below and, for the direct reaction near field (S2T), by every
    // evaluation, so they live as long as the build
    void *pk = nullptr, *pw = nullptr, *pi = nullptr, *pn = nullptr;
    size_t nn = pl.node_kr.size();
    HIPC(hipMalloc(&pk, nn * sizeof(cd)));
    HIPC(hipMalloc(&pw, nn * sizeof(cd)));
    HIPC(hipMalloc(&pi, nn * sizeof(int)));
    if ((rc = dalloc(ctx, &pn, nn * sizeof(QNode)))) {
      hipFree(pk);
      hipFree(pw);
      hipFree(pi);
      return rc;
    }
    HIPC(hipMemcpy(pk, pl.node_kr.data(), nn * sizeof(cd), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(pw, pl.node_w.data(), nn * sizeof(cd), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(pi, pl.node_inst.data(), nn * sizeof(int), hipMemcpyHostToDevice));
    d.nodes = (QNode*)pn;
    launch_nodes(d, md, (int)nn, (int*)pi, (cd*)pk, (cd*)pw, s);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s));
    hipFree(pk);
    hipFree(pw);
    hipFree(pi);
  }
  if (!pl.cases.empty()) {
    void *pib = nullptr, *psc = nullptr;
    // integrals and assembly in batches of cases (bounded scratch)
    int maxnode = 0;
    for (auto& tc : pl.cases) maxnode = std::max(maxnode, tc.nnode);
    int NQ = 2 * pl.p + 3;
    long long per_case_scr = (long long)maxnode * (NQ + 1);
    long long per_case_ib = 5LL * 16 * (pl.p + 2) * NQ;
    int batch = (int)std::max(1LL, std::min((long long)pl.cases.size(), (long long)(256LL << 20) / (per_case_scr * 16)));
    HIPC(hipMalloc(&psc, (size_t)batch * per_case_scr * sizeof(cd)));
    HIPC(hipMalloc(&pib, (size_t)pl.cases.size() * per_case_ib * sizeof(cd)));
    d.ibuf = (cd*)pib;
    for (int c0 = 0; c0 < (int)pl.cases.size(); c0 += batch) {
      int nc = std::min(batch, (int)pl.cases.size() - c0);
      launch_tab_integrals(d, md, c0, nc, pl.p, (cd*)psc, maxnode, s);
      HIPC(hipGetLastError());
    }
    hipFree(psc);
    psc = nullptr;
    // the + and z output rows of a batch of cases into bounded scratch, then
    // the even and odd blocks of the mirror-adapted tensor into the tables
    long long stride = 0;
    for (auto& tc : pl.cases) stride = std::max(stride, 6LL * pl.inst[tc.inst].P * pl.inst[tc.inst].P);
    const int ncs = (int)pl.cases.size();
    const int bat = (int)std::max(1LL, std::min((long long)ncs, (512LL << 20) / (stride * 16)));
    HIPC(hipMalloc(&psc, (size_t)bat * stride * sizeof(cd)));
    for (int c0 = 0; c0 < ncs; c0 += bat) {
      const int nc = std::min(bat, ncs - c0);
      launch_tab_assemble(d, c0, nc, pl.p, pl.kmaxcheb, (ctx->pmax + 1) / 2 + 2, (cd*)psc, stride, s);
      launch_tab_sym(d, c0, nc, (cd*)psc, stride, s);
      HIPC(hipGetLastError());
    }
    HIPC(hipStreamSynchronize(s));
    hipFree(psc);
    hipFree(pib);
    d.ibuf = nullptr;
  }
  if (!ctx->s2t_ranges.empty() && !d.nodes)
    return fail(ctx, LM_EHIP, "internal: direct near field without quadrature nodes");
  HIPC(hipStreamSynchronize(s));
  auto t3 = std::chrono::steady_clock::now();
  ctx->t_plan_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  ctx->t_upload_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
  ctx->t_tables_ms = std::chrono::duration<double, std::milli>(t3 - t2).count();
  {
    // every near-field argument k r is below k_max times the diameter of
    // the point set (pairs only form within one geometry)
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int pass = 0; pass < 2; pass++) {
      const double* x = pass ? tgt_xyz : src_xyz;
      int64_t n = pass ? n_tgt : n_src;
      for (int64_t i = 0; i < n; i++)
        for (int c = 0; c < 3; c++) {
          lo[c] = std::min(lo[c], x[3 * i + c]);
          hi[c] = std::max(hi[c], x[3 * i + c]);
        }
    }
    double diam = 0;
    for (int c = 0; c < 3; c++) diam += hi[c] > lo[c] ? (hi[c] - lo[c]) * (hi[c] - lo[c]) : 0.0;
    ctx->p2p_red = med.kmax * sqrt(diam) < 0.5 * LM_SINCOS_RED_MAX;
  }
  ctx->same_sets = n_src == n_tgt && memcmp(soff, toff, (size_t)(n_geom + 1) * sizeof(int64_t)) == 0 &&
                   (src_xyz == tgt_xyz || n_src == 0 ||
                    memcmp(src_xyz, tgt_xyz, (size_t)n_src * 3 * sizeof(double)) == 0);
  if (!ctx->same_sets || ctx->prm.react_s2t) {
    // kept for the swapped-role builds (adjoint of distinct sets, gradients)
    ctx->host_src.assign(src_xyz, src_xyz + 3 * n_src);
    ctx->host_tgt.assign(tgt_xyz, tgt_xyz + 3 * n_tgt);
    ctx->host_soff.assign(soff, soff + n_geom + 1);
    ctx->host_toff.assign(toff, toff + n_geom + 1);
  }
  {
    // lm_evaluate_noalloc: work buffers of one right-hand side laid out in
    // the static scratch (256-byte aligned pieces), the M2L outputs chunked
    // to the room that is left
    auto up = [](long long n) { return (n + 15) / 16 * 16; };  // complex numbers, 256-byte multiples
    const long long cap = (long long)(LM_NOALLOC_SCRATCH_BYTES / sizeof(cd));
    ctx->na_off[0] = 0;
    ctx->na_off[1] = ctx->na_off[0] + up(pl.me_size);
    ctx->na_off[2] = ctx->na_off[1] + up(pl.le_size);
    ctx->na_off[4] = ctx->na_off[2] + up(p2m_part_size(ctx, 1));
    ctx->na_off[3] = ctx->na_off[4] + up(std::max(ctx->s2t_slots, ctx->p2ps_slots) * 3);
    long long bmax = 0;
    int rc2 = make_schedule(ctx, 1, std::max(0LL, cap - ctx->na_off[3]) * (long long)sizeof(cd), ctx->na_ts, &bmax);
    if (rc2) return rc2;
    ctx->na_need = (ctx->na_off[3] + std::max(up(ctx->na_ts.y_need), up(bmax / (long long)sizeof(cd)))) *
                   (long long)sizeof(cd);
    ctx->na_ok = ctx->na_need <= (long long)LM_NOALLOC_SCRATCH_BYTES;
  }
  ctx->built = true;
  return LM_OK;
}

// The M2L schedule for n_rhs right-hand sides: chunks of whole blocks whose
// M2L outputs fit `budget` bytes of scratch (each block gets its own scratch
// base, blocks differ in P), and the GEMM tiles of every chunk.  Host lists,
// uploaded into ts.  *block_max receives the scratch bytes of the largest
// block (a chunk holds at least one block, whatever the budget).
static int make_schedule(lm_ctx* ctx, int n_rhs, long long budget, lm_ctx::TileSet& ts, long long* block_max) {
  Plan& pl = ctx->plan;
  std::vector<M2LTile> tiles;
  std::vector<long long> ybase(std::max<size_t>(1, pl.blocks.size()), 0);
  long long need_max = 0;
  *block_max = 0;
  size_t bi = 0;
  while (bi < pl.blocks.size()) {
    lm_ctx::Chunk ch;
    ch.tile0 = (int)tiles.size();
    ch.bt0 = pl.blocks[bi].bt0;
    ch.nbt = 0;
    long long bytes = 0;
    while (bi < pl.blocks.size()) {
      const M2LBlock& B = pl.blocks[bi];
      const M2LClass& C = pl.cls[B.cls];
      long long bb = (long long)B.nq * 3 * n_rhs * C.P * (long long)sizeof(cd);
      *block_max = std::max(*block_max, bb);
      if (ch.nbt > 0 && bytes + bb > budget) break;
      ybase[bi] = bytes / (long long)sizeof(cd);
      bytes += bb;
      m2l_groups(pl, B, [&](int o0, int o1) {
        const int q0 = pl.offr[B.offr0 + o0], ncol = (pl.offr[B.offr0 + o1] - q0) * n_rhs;
        if (ncol == 0) return;
        // free space: three output types of Po rows; reaction: the even and
        // the odd block of the mirror-adapted tensor
        const M2LOffset& O = pl.offs[C.off0 + o0];
        const int po = O.pord, Po = (po + 1) * (po + 1);
        const bool sym = C.nblk == 3;
        // column tile outermost: the row tiles of both parts (or of the
        // three output types) of one column tile are consecutive, so they
        // run together on one XCD and read the tile's source vectors from
        // its L2 (with the row tile outermost, the source vectors of a
        // large group were read from HBM once per row tile)
        for (int c0 = 0; c0 < ncol; c0 += TN_COLS)
          for (int ot = 0; ot < (sym ? 2 : 3); ot++) {
            M2LTile t;
            t.mat = O.mat[sym ? ot : 0];
            t.ybase = ybase[bi];
            t.qo = q0;
            t.q0b = B.q0;
            t.P = C.P;
            t.p = pl.inst[C.inst].p;
            t.R = sym ? lm_sym_dim(po, ot) : Po;
            t.Pb = Po;
            t.Kf = sym ? lm_sym_dim(t.p, ot) : C.P;
            t.ot = ot;
            t.sym = sym ? 1 : 0;
            t.col0 = c0;
            t.ncol = std::min(TN_COLS, ncol - c0);
            for (int r0 = 0; r0 < t.R; r0 += TM_ROWS) {
              t.row0 = r0;
              tiles.push_back(t);
            }
          }
      });
      ch.nbt += B.nt;
      bi++;
    }
    ch.ntile = (int)tiles.size() - ch.tile0;
    need_max = std::max(need_max, bytes);
    ts.chunks.push_back(ch);
  }
  if (!tiles.empty()) {
    HIPC(hipMalloc((void**)&ts.d_tiles, tiles.size() * sizeof(M2LTile)));
    HIPC(hipMemcpy(ts.d_tiles, tiles.data(), tiles.size() * sizeof(M2LTile), hipMemcpyHostToDevice));
  }
  HIPC(hipMalloc((void**)&ts.d_ybase, ybase.size() * sizeof(long long)));
  HIPC(hipMemcpy(ts.d_ybase, ybase.data(), ybase.size() * sizeof(long long), hipMemcpyHostToDevice));
  ts.n_tiles = (int)tiles.size();
  ts.y_need = need_max / (long long)sizeof(cd);
  return LM_OK;
}

// complex numbers of the P2M partial expansions for n_rhs right-hand sides
static long long p2m_part_size(const lm_ctx* ctx, int n_rhs) {
  long long part = 0;
  for (int g = 0; g < 2; g++) part += ctx->p2m_slots[g] * n_rhs * 3LL * (ctx->p2m_p[g] + 1) * (ctx->p2m_p[g] + 1);
  return part;
}

// Work buffers and M2L schedule of one evaluation of n_rhs right-hand sides.
struct Work {
  cd* ME = nullptr;
  cd* LE = nullptr;
  cd* part = nullptr;
  cd* Y = nullptr;
  cd* S2TY = nullptr;  // direct-pair output slots
  lm_ctx::TileSet* ts = nullptr;
  bool tune = true;   // autotune untuned M2L launches (events, synchronisation)
  bool timed = true;  // record phase events when timing is on
};

// Work buffers and the M2L schedule for n_rhs right-hand sides.  Anything
// that must be (re)allocated is done after the stream has drained, so no
// buffer used by queued kernels is freed or overwritten.
static int ensure_rhs(lm_ctx* ctx, int n_rhs, hipStream_t s, Work* w) {
  Plan& pl = ctx->plan;
  long long me = pl.me_size * n_rhs, le = pl.le_size * n_rhs;
  long long part = p2m_part_size(ctx, n_rhs);
  bool have = ctx->tilesets.count(n_rhs) > 0;
  if (!(me <= ctx->me_cap && le <= ctx->le_cap && part <= ctx->p2m_part_cap && have &&
        ctx->tilesets[n_rhs].y_need <= ctx->y_cap)) {
    HIPC(hipStreamSynchronize(s));
    if (me > ctx->me_cap) {
      if (ctx->ME) hipFree(ctx->ME);
      ctx->ME = nullptr;
      HIPC(hipMalloc((void**)&ctx->ME, (size_t)std::max(1LL, me) * sizeof(cd)));
      ctx->me_cap = me;
    }
    if (le > ctx->le_cap) {
      if (ctx->LE) hipFree(ctx->LE);
      ctx->LE = nullptr;
      HIPC(hipMalloc((void**)&ctx->LE, (size_t)std::max(1LL, le) * sizeof(cd)));
      ctx->le_cap = le;
    }
    if (part > ctx->p2m_part_cap) {
      if (ctx->p2m_part) hipFree(ctx->p2m_part);
      ctx->p2m_part = nullptr;
      HIPC(hipMalloc((void**)&ctx->p2m_part, (size_t)part * sizeof(cd)));
      ctx->p2m_part_cap = part;
    }
    if (!have) {
      lm_ctx::TileSet ts;
      long long bmax = 0;
      // M2L scratch budget: fewer, larger launches for many right-hand
      // sides (each launch ends with a partial wave of tiles)
      int rc = make_schedule(ctx, n_rhs, 24LL << 30, ts, &bmax);
      if (rc) {
        if (ts.d_tiles) hipFree(ts.d_tiles);
        if (ts.d_ybase) hipFree(ts.d_ybase);
        return rc;
      }
      ctx->tilesets[n_rhs] = ts;
    }
    lm_ctx::TileSet& ts = ctx->tilesets[n_rhs];
    if (ts.y_need > ctx->y_cap) {
      if (ctx->Y) hipFree(ctx->Y);
      ctx->Y = nullptr;
      HIPC(hipMalloc((void**)&ctx->Y, (size_t)std::max(1LL, ts.y_need) * sizeof(cd)));
      ctx->y_cap = ts.y_need;
    }
  }
  const long long sy = std::max(ctx->s2t_slots, ctx->p2ps_slots) * n_rhs * 3;
  if (sy > ctx->s2ty_cap) {
    HIPC(hipStreamSynchronize(s));
    if (ctx->S2TY) hipFree(ctx->S2TY);
    ctx->S2TY = nullptr;
    ctx->s2ty_cap = 0;
    HIPC(hipMalloc((void**)&ctx->S2TY, (size_t)sy * sizeof(cd)));
    ctx->s2ty_cap = sy;
  }
  w->ME = ctx->ME;
  w->LE = ctx->LE;
  w->part = ctx->p2m_part;
  w->Y = ctx->Y;
  w->S2TY = ctx->S2TY;
  w->ts = &ctx->tilesets[n_rhs];
  return LM_OK;
}

static int evaluate_chunk(lm_ctx* ctx, int n_rhs, const void* J, void* A, void* stream, const cd* W = nullptr,
                          double* gX = nullptr, cd* Hc = nullptr, Work* wk = nullptr);

#define LM_RHS_CHUNK 16

int lm_evaluate(lm_ctx* ctx, int n_rhs, const void* J, void* A, void* stream) {
  if (!ctx) return LM_EINVAL;
  if (!ctx->built) return fail(ctx, LM_ESTATE, "lm_build must succeed before lm_evaluate");
  if (n_rhs < 1 || n_rhs > 4096) return fail(ctx, LM_EINVAL, "n_rhs out of range (1..4096)");
  Plan& pl = ctx->plan;
  if ((pl.n_src > 0 && !J) || (pl.n_tgt > 0 && !A)) return fail(ctx, LM_EINVAL, "null J or A");
  if (((uintptr_t)J % 16) || ((uintptr_t)A % 16)) return fail(ctx, LM_EINVAL, "J and A must be 16-byte aligned");
  for (int r0 = 0; r0 < n_rhs; r0 += LM_RHS_CHUNK) {
    int nr = std::min(LM_RHS_CHUNK, n_rhs - r0);
    const cd* Jc = J ? (const cd*)J + (long long)r0 * pl.n_src * 3 : nullptr;
    cd* Ac = A ? (cd*)A + (long long)r0 * pl.n_tgt * 3 : nullptr;
    int rc = evaluate_chunk(ctx, nr, Jc, Ac, stream);
    if (rc) return rc;
  }
  return LM_OK;
}

int lm_evaluate_noalloc(lm_ctx* ctx, int n_rhs, const void* J, void* A, void* stream) {
  if (!ctx) return LM_EINVAL;
  if (!ctx->built) return fail(ctx, LM_ESTATE, "lm_build must succeed before lm_evaluate_noalloc");
  if (n_rhs < 1 || n_rhs > 4096) return fail(ctx, LM_EINVAL, "n_rhs out of range (1..4096)");
  Plan& pl = ctx->plan;
  if ((pl.n_src > 0 && !J) || (pl.n_tgt > 0 && !A)) return fail(ctx, LM_EINVAL, "null J or A");
  if (((uintptr_t)J % 16) || ((uintptr_t)A % 16)) return fail(ctx, LM_EINVAL, "J and A must be 16-byte aligned");
  const int dev = ctx->device;
  if (dev < 0 || dev >= LM_MAX_DEVICES || g_scratch_state[dev] != 1)
    return fail(ctx, LM_EHIP, dev >= 0 && dev < LM_MAX_DEVICES && g_scratch_state[dev] < 0
                                  ? g_scratch_err[dev]
                                  : std::string("no static scratch on this device"));
  if (!ctx->na_ok)
    return fail(ctx, LM_ENOMEM,
                lm_fmt("lm_evaluate_noalloc: this build needs %lld bytes of scratch, the static scratch holds %lld",
                       ctx->na_need, (long long)LM_NOALLOC_SCRATCH_BYTES));
  cd* base = (cd*)g_scratch_ptr[dev];
  Work w;
  w.ME = base + ctx->na_off[0];
  w.LE = base + ctx->na_off[1];
  w.part = base + ctx->na_off[2];
  w.Y = base + ctx->na_off[3];
  w.S2TY = base + ctx->na_off[4];
  w.ts = &ctx->na_ts;
  w.tune = false;
  w.timed = false;
  // one right-hand side at a time (the work buffers hold one)
  for (int r = 0; r < n_rhs; r++) {
    const cd* Jr = J ? (const cd*)J + (long long)r * pl.n_src * 3 : nullptr;
    cd* Ar = A ? (cd*)A + (long long)r * pl.n_tgt * 3 : nullptr;
    int rc = evaluate_chunk(ctx, 1, Jr, Ar, stream, nullptr, nullptr, nullptr, &w);
    if (rc) return rc;
  }
  return LM_OK;
}

// One group of right-hand sides.  Normal mode (gX == nullptr, Hc == nullptr): A = G J.
// Curl mode (Hc != nullptr): the leaf passes and the direct reaction pairs
// add curl (G J) at every target into Hc; A is not touched.
// Gradient mode: the upward pass and M2L run on J as usual, then instead of
// writing A the leaf passes and the direct reaction pairs add, at every target
// point, Re sum_b W^b grad B_b
// (B the field of J) into gX [n_tgt][3]; A is not touched.
// The context that evaluates the transposed operator: by reciprocity
// (G(x, y) = G(y, x)^T when every mu is 1; with permeabilities the callers
// weight by mu, since G(x, y) mu(y) = G(y, x)^T mu(x)),
// sum_i G(x_i, x_j)^T v_i is the forward sum with the
// roles of sources and targets exchanged.  That is this context when the two
// point sets are the same array, otherwise a second context built (once, on
// the first call) with the sets swapped.
static int swapped_ctx(lm_ctx* ctx, hipStream_t s, lm_ctx** out) {
  *out = nullptr;
  if (ctx->same_sets) {
    *out = ctx;
    return LM_OK;
  }
  if (!ctx->adj) {
    lm_ctx* a = nullptr;
    int rc = lm_create(&a, ctx->device);
    if (rc) return fail(ctx, rc, "cannot create the swapped-role context");
    a->med = ctx->med;
    a->layers_set = true;
    a->prm = ctx->prm;
    a->m2l_variant = ctx->m2l_variant;
    int ng = (int)ctx->host_soff.size() - 1;
    rc = build_common(a, ng, ctx->host_toff.data(), ctx->host_tgt.data(), ctx->host_soff.data(),
                      ctx->host_src.data(), s);
    if (rc) {
      std::string m = a->err;
      lm_destroy(a);
      return fail(ctx, rc, "swapped-role build: " + m);
    }
    ctx->adj = a;
  }
  *out = ctx->adj;
  return LM_OK;
}

// Autotuner of the M2L GEMM (tile-shape variants of k_m2l, bitwise equal
// results): the first time a launch of the schedule runs outside graph
// capture, each variant is run twice on the real operands and timed with
// events on the evaluation stream (the second run counts, the first absorbs
// code loading); the fastest is kept for that launch.  Every run writes the
// same scratch vectors, so the evaluation continues with valid data.  Under
// capture nothing is timed and variant 0 is used until a later eager call.
static int tune_m2l(lm_ctx* ctx, const DevPlan& d, const Work& w, lm_ctx::Chunk& ch, int n_rhs, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPC(hipStreamIsCapturing(s, &cs));
  if (cs != hipStreamCaptureStatusNone) return LM_OK;
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return fail(ctx, LM_EHIP, "hipEventCreate failed");
  }
  int rc = LM_OK;
  int best = 0;
  for (int v = 0; v < LM_M2L_VARIANTS && rc == LM_OK; v++) {
    float ms = 0;
    for (int rep = 0; rep < 2 && rc == LM_OK; rep++) {
      if (hipEventRecord(e0, s) != hipSuccess) rc = LM_EHIP;
      launch_m2l(d, d.tiles + ch.tile0, ch.ntile, n_rhs, w.ME, w.Y, ctx->pmax, v, s);
      if (rc == LM_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                          hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = LM_EHIP;
    }
    ch.ms[v] = ms;
    if (rc == LM_OK && ch.ms[v] < ch.ms[best]) best = v;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return fail(ctx, rc, "M2L autotuning: a HIP call failed");
  ch.variant = best;
  return LM_OK;
}

static int ensure_jc(lm_ctx* ctx, long long n, hipStream_t s) {
  if (n <= ctx->jc_cap) return LM_OK;
  HIPC(hipStreamSynchronize(s));
  if (ctx->Jc) hipFree(ctx->Jc);
  ctx->Jc = nullptr;
  ctx->jc_cap = 0;
  HIPC(hipMalloc((void**)&ctx->Jc, (size_t)std::max(1LL, n) * sizeof(cd)));
  ctx->jc_cap = n;
  return LM_OK;
}

int lm_evaluate_h(lm_ctx* ctx, int n_rhs, const void* J, void* H, void* stream) {
  if (!ctx) return LM_EINVAL;
  if (!ctx->built) return fail(ctx, LM_ESTATE, "lm_build must succeed before lm_evaluate_h");
  if (n_rhs < 1 || n_rhs > 4096) return fail(ctx, LM_EINVAL, "n_rhs out of range (1..4096)");
  Plan& pl = ctx->plan;
  if ((pl.n_src > 0 && !J) || (pl.n_tgt > 0 && !H)) return fail(ctx, LM_EINVAL, "null J or H");
  if (((uintptr_t)J % 16) || ((uintptr_t)H % 16)) return fail(ctx, LM_EINVAL, "J and H must be 16-byte aligned");
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  for (int r0 = 0; r0 < n_rhs; r0 += LM_RHS_CHUNK) {
    int nr = std::min(LM_RHS_CHUNK, n_rhs - r0);
    const cd* Jc = (const cd*)J + (long long)r0 * pl.n_src * 3;
    cd* Hc = (cd*)H + (long long)r0 * pl.n_tgt * 3;
    int rc = evaluate_chunk(ctx, nr, Jc, nullptr, stream, nullptr, nullptr, Hc);
    if (rc) return rc;
  }
  // Faraday's law: H = curl E / mu of the target's layer
  if (!ctx->med.mu_one) launch_scale_mu((cd*)H, pl.n_tgt, n_rhs, ctx->d_tgt, ctx->md, -1, s);
  HIPC(hipGetLastError());
  return LM_OK;
}

int lm_evaluate_adjoint(lm_ctx* ctx, int n_rhs, const void* gA, void* gJ, void* stream) {
  if (!ctx) return LM_EINVAL;
  if (!ctx->built) return fail(ctx, LM_ESTATE, "lm_build must succeed before lm_evaluate_adjoint");
  if (n_rhs < 1 || n_rhs > 4096) return fail(ctx, LM_EINVAL, "n_rhs out of range (1..4096)");
  Plan& pl = ctx->plan;
  if ((pl.n_tgt > 0 && !gA) || (pl.n_src > 0 && !gJ)) return fail(ctx, LM_EINVAL, "null gA or gJ");
  if (((uintptr_t)gA % 16) || ((uintptr_t)gJ % 16)) return fail(ctx, LM_EINVAL, "gA and gJ must be 16-byte aligned");
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  lm_ctx* T = nullptr;
  int rc = swapped_ctx(ctx, s, &T);
  if (rc) return rc;
  int nr0 = std::min(LM_RHS_CHUNK, n_rhs);
  if ((rc = ensure_jc(ctx, (long long)nr0 * pl.n_tgt * 3, s))) return rc;
  for (int r0 = 0; r0 < n_rhs; r0 += LM_RHS_CHUNK) {
    int nr = std::min(LM_RHS_CHUNK, n_rhs - r0);
    const cd* g = (const cd*)gA + (long long)r0 * pl.n_tgt * 3;
    cd* o = (cd*)gJ + (long long)r0 * pl.n_src * 3;
    if (ctx->med.mu_one)
      launch_conj(ctx->Jc, g, (long long)nr * pl.n_tgt * 3, s);
    else  // reciprocity with permeabilities: G(x, y)^H = conj(G(y, x)) mu(x) / mu(y)
      launch_conj_mu(ctx->Jc, g, pl.n_tgt, nr, ctx->d_tgt, ctx->md, 1, s);
    rc = evaluate_chunk(T, nr, ctx->Jc, o, stream);
    if (rc) return T == ctx ? rc : fail(ctx, rc, "swapped-role evaluation: " + T->err);
    if (ctx->med.mu_one)
      launch_conj(o, o, (long long)nr * pl.n_src * 3, s);
    else
      launch_conj_mu(o, o, pl.n_src, nr, ctx->d_src, ctx->md, -1, s);
  }
  HIPC(hipGetLastError());
  return LM_OK;
}

int lm_grad_src_xyz(lm_ctx* ctx, int n_rhs, const void* J, const void* gA, double* gX, void* stream) {
  if (!ctx) return LM_EINVAL;
  if (!ctx->built) return fail(ctx, LM_ESTATE, "lm_build must succeed before lm_grad_src_xyz");
  if (n_rhs < 1 || n_rhs > 4096) return fail(ctx, LM_EINVAL, "n_rhs out of range (1..4096)");
  Plan& pl = ctx->plan;
  if ((pl.n_src > 0 && (!J || !gX)) || (pl.n_tgt > 0 && !gA)) return fail(ctx, LM_EINVAL, "null J, gA or gX");
  if (((uintptr_t)J % 16) || ((uintptr_t)gA % 16) || ((uintptr_t)gX % 8))
    return fail(ctx, LM_EINVAL, "J and gA must be 16-byte aligned, gX 8-byte aligned");
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  lm_ctx* T = nullptr;
  int rc = swapped_ctx(ctx, s, &T);
  if (rc) return rc;
  launch_fill_d(gX, 3 * pl.n_src, s);
  if (pl.n_src == 0 || pl.n_tgt == 0) {
    HIPC(hipGetLastError());
    return LM_OK;
  }
  int nr0 = std::min(LM_RHS_CHUNK, n_rhs);
  if ((rc = ensure_jc(ctx, (long long)nr0 * pl.n_tgt * 3, s))) return rc;
  for (int r0 = 0; r0 < n_rhs; r0 += LM_RHS_CHUNK) {
    int nr = std::min(LM_RHS_CHUNK, n_rhs - r0);
    const cd* g = (const cd*)gA + (long long)r0 * pl.n_tgt * 3;
    const cd* w = (const cd*)J + (long long)r0 * pl.n_src * 3;
    if (ctx->med.mu_one)
      launch_conj(ctx->Jc, g, (long long)nr * pl.n_tgt * 3, s);
    else
      launch_conj_mu(ctx->Jc, g, pl.n_tgt, nr, ctx->d_tgt, ctx->md, 1, s);
    rc = evaluate_chunk(T, nr, ctx->Jc, nullptr, stream, w, gX);
    if (rc) return T == ctx ? rc : fail(ctx, rc, "swapped-role evaluation: " + T->err);
  }
  if (!ctx->med.mu_one) launch_scale_mu_d(gX, pl.n_src, ctx->d_src, ctx->md, -1, s);
  HIPC(hipGetLastError());
  return LM_OK;
}

static int evaluate_chunk(lm_ctx* ctx, int n_rhs, const void* J, void* A, void* stream, const cd* W, double* gX,
                          cd* Hc, Work* wk) {
  if (!ctx) return LM_EINVAL;
  if (!ctx->built) return fail(ctx, LM_ESTATE, "lm_build must succeed before lm_evaluate");
  if (n_rhs < 1 || n_rhs > 4096) return fail(ctx, LM_EINVAL, "n_rhs out of range (1..4096)");
  Plan& pl = ctx->plan;
  const bool grad = gX != nullptr, curl = Hc != nullptr;
  if ((pl.n_src > 0 && !J) || (pl.n_tgt > 0 && !grad && !curl && !A)) return fail(ctx, LM_EINVAL, "null J or A");
  if (((uintptr_t)J % 16) || ((uintptr_t)A % 16)) return fail(ctx, LM_EINVAL, "J and A must be 16-byte aligned");
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  Work wl;
  int rc = LM_OK;
  if (!wk) {
    if ((rc = ensure_rhs(ctx, n_rhs, s, &wl))) return rc;
    wk = &wl;
  }
  const Work& w = *wk;
  const cd* Jc = (const cd*)J;
  cd* Ac = (cd*)A;
  DevPlan d = ctx->d;  // this evaluation's schedule
  d.tiles = w.ts->d_tiles;
  d.blk_ybase = w.ts->d_ybase;
  const int nch = (int)w.ts->chunks.size();
  lm_ctx::EvSet ev;
  const bool timed = w.timed && ctx->timing && ctx->evsets.size() < 4096;
  if (timed) {
    // phase boundaries, then a start/stop pair around every launch of the
    // M2L GEMM, the M2L reduction and the near-field kernels
    ev.ph.resize(LM_PHASES + 1);
    for (auto& e : ev.ph) HIPC(hipEventCreate(&e));
  }
  auto mark = [&](int i) {
    if (timed) (void)hipEventRecord(ev.ph[i], s);
  };
  auto span = [&](int kind, bool start) {
    if (!timed) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (start) ev.kind.push_back(kind);
    ev.sp.push_back(e);
    (void)hipEventRecord(e, s);
  };
  mark(0);
  if (curl)
    launch_fill(Hc, (long long)n_rhs * pl.n_tgt * 3, s);
  else if (!grad)
    launch_fill(Ac, (long long)n_rhs * pl.n_tgt * 3, s);
  if (pl.n_src > 0 && pl.n_tgt > 0) {
    // local expansions accumulate; multipole vectors of source boxes that
    // hold no sources (free-space leaves holding only targets) are read by
    // M2M but written by no pass, so they must hold zeros
    launch_fill(w.LE, pl.le_size * n_rhs, s);
    launch_fill(w.ME, pl.me_size * n_rhs, s);
  }
  mark(1);
  if (pl.n_src > 0 && pl.n_tgt > 0) {
    cd* part = w.part;
    for (int g = 0; g < 2; g++) {
      const int pg = ctx->p2m_p[g], Pg = (pg + 1) * (pg + 1);
      launch_p2m(d, ctx->d_p2m[g], ctx->n_p2m[g], ctx->d_src, Jc, pl.n_src, n_rhs, w.ME, part, pg, s);
      launch_p2m_sum(d, ctx->d_p2m_sum[g], ctx->n_p2m_sum[g], n_rhs, part, Pg, w.ME, s);
      part += ctx->p2m_slots[g] * n_rhs * 3 * Pg;
    }
    mark(2);
    for (int l = (int)ctx->d_m2m.size() - 1; l >= 0; l--)
      launch_m2m(d, ctx->d_m2m[l], ctx->n_m2m[l], n_rhs, w.ME, ctx->pmax, s);
    mark(3);
    for (int c = 0; c < nch; c++) {
      lm_ctx::Chunk& ch = w.ts->chunks[c];
      int v = ctx->m2l_variant >= 0 ? ctx->m2l_variant : ch.variant;
      if (v < 0 && w.tune) {
        if ((rc = tune_m2l(ctx, d, w, ch, n_rhs, s))) return rc;
        v = ch.variant;
      }
      if (v < 0) v = 0;
      span(0, true);
      launch_m2l(d, d.tiles + ch.tile0, ch.ntile, n_rhs, w.ME, w.Y, ctx->pmax, v, s);
      span(0, false);
      span(1, true);
      launch_m2l_reduce(d, ch.bt0, ch.nbt, n_rhs, w.Y, w.LE, ctx->pmax, s);
      span(1, false);
    }
    mark(4);
    for (int l = 1; l < (int)ctx->d_l2l.size(); l++)
      launch_l2l(d, ctx->d_l2l[l], ctx->n_l2l[l], n_rhs, w.LE, ctx->pmax, s);
    mark(5);
    for (size_t g = 0; g < ctx->d_l2p.size(); g++) {
      const int i = ctx->l2p_inst[g];
      int kind = pl.inst[i].kind == 0 ? 0 : 1;
      if (grad)
        launch_l2p_grad(d, ctx->d_l2p[g], ctx->n_l2p[g], kind, ctx->d_tgt, pl.n_tgt, n_rhs, w.LE, W, gX,
                        pl.inst[i].p, s);
      else if (curl)
        launch_l2p_curl(d, ctx->d_l2p[g], ctx->n_l2p[g], kind, ctx->d_tgt, pl.n_tgt, n_rhs, w.LE, Hc,
                        pl.inst[i].p, s);
      else
        launch_l2p(d, ctx->d_l2p[g], ctx->n_l2p[g], kind, ctx->d_tgt, pl.n_tgt, n_rhs, w.LE, Ac, pl.inst[i].p, s);
    }
    mark(6);
    if (!grad && !curl && ctx->p2ps_n > 0) {
      // targets are the sources: one kernel evaluation per unordered pair
      // (the partner sums through the slots, added in item order)
      span(2, true);
      launch_p2p_sym(d, ctx->d_p2ps_items, ctx->p2ps_n, ctx->d_p2ps_part, ctx->d_src, Jc, pl.n_src, n_rhs, Ac,
                     w.S2TY, ctx->p2p_red, s);
      launch_s2t_gather(ctx->d_p2ps_gpt, ctx->d_p2ps_gptr, ctx->d_p2ps_gslot, ctx->p2ps_npts, n_rhs, w.S2TY,
                        pl.n_tgt, Ac, s);
      span(2, false);
    }
    for (size_t f = 0; f < ctx->d_p2p.size() && (grad || curl || ctx->p2ps_n == 0); f++) {
      span(2, true);
      if (grad)
        launch_p2p_grad(d, ctx->d_p2p[f], ctx->n_p2p[f], ctx->d_src, Jc, pl.n_src, ctx->d_tgt, W, pl.n_tgt, n_rhs,
                        gX, ctx->p2p_red, s);
      else if (curl)
        launch_p2p_curl(d, ctx->d_p2p[f], ctx->n_p2p[f], ctx->d_src, Jc, pl.n_src, ctx->d_tgt, pl.n_tgt, n_rhs, Hc,
                        ctx->p2p_red, s);
      else
        launch_p2p(d, ctx->d_p2p[f], ctx->n_p2p[f], ctx->d_src, Jc, pl.n_src, ctx->d_tgt, pl.n_tgt, n_rhs, Ac,
                   ctx->p2p_red, s);
      span(2, false);
    }
    if (grad) {
      if (ctx->s2t_slots > 0) {
        // the slot buffer holds n_rhs complex triples per slot, at least the
        // one real triple per slot of the gradient
        double* Gs = (double*)w.S2TY;
        span(3, true);
        for (int v = 0; v < 2; v++)
          launch_s2t_grad(d, ctx->md, ctx->d_s2t_items + 6 * ctx->s2t_launch[v][0], ctx->d_s2t_tlist,
                          ctx->d_s2t_slist, ctx->s2t_launch[v][1], ctx->d_src, Jc, pl.n_src, ctx->d_tgt, W, pl.n_tgt,
                          n_rhs, ctx->contour_a, v == 1, Gs, s);
        launch_s2t_gather_grad(ctx->d_s2t_gpt, ctx->d_s2t_gptr, ctx->d_s2t_gslot, ctx->s2t_npts, Gs, gX, s);
        span(3, false);
      }
    } else if (ctx->s2t_slots > 0) {
      span(3, true);
      for (int v = 0; v < 2; v++)
        launch_s2t(d, ctx->md, ctx->d_s2t_items + 6 * ctx->s2t_launch[v][0], ctx->d_s2t_tlist, ctx->d_s2t_slist,
                   ctx->s2t_launch[v][1], ctx->d_src, Jc, pl.n_src, ctx->d_tgt, pl.n_tgt, n_rhs, ctx->contour_a, v == 1,
                   w.S2TY, s, curl);
      launch_s2t_gather(ctx->d_s2t_gpt, ctx->d_s2t_gptr, ctx->d_s2t_gslot, ctx->s2t_npts, n_rhs, w.S2TY, pl.n_tgt,
                        curl ? Hc : Ac, s);
      span(3, false);
    }
    mark(7);
  } else {
    for (int i = 2; i <= 7; i++) mark(i);
  }
  if (timed) ctx->evsets.push_back(ev);
  HIPC(hipGetLastError());
  return LM_OK;
}

int lm_set_timing(lm_ctx* ctx, int enable) {
  if (!ctx) return LM_EINVAL;
  HIPC(hipSetDevice(ctx->device));
  clear_events(ctx);
  ctx->timing = enable != 0;
  return LM_OK;
}

int lm_timings(lm_ctx* ctx, double* out, int n) {
  if (!ctx || !out || n < 1) return LM_EINVAL;
  HIPC(hipSetDevice(ctx->device));
  double acc[LM_TIMINGS_COUNT] = {0};
  for (auto& v : ctx->evsets) {
    HIPC(hipEventSynchronize(v.ph[LM_PHASES]));
    for (int i = 0; i < LM_PHASES; i++) {
      float ms = 0;
      HIPC(hipEventElapsedTime(&ms, v.ph[i], v.ph[i + 1]));
      acc[i] += ms;
    }
    for (size_t j = 0; j < v.kind.size() && 2 * j + 1 < v.sp.size(); j++) {
      float ms = 0;
      HIPC(hipEventElapsedTime(&ms, v.sp[2 * j], v.sp[2 * j + 1]));
      const int slot = LM_TIMING_M2L_GEMM_MS + 2 * v.kind[j];
      acc[slot] += ms;
      acc[slot + 1] += 1;
    }
  }
  acc[LM_PHASES] = (double)ctx->evsets.size();
  int m = n < LM_TIMINGS_COUNT ? n : LM_TIMINGS_COUNT;
  memcpy(out, acc, m * sizeof(double));
  return LM_OK;
}

int lm_m2l_variants(const lm_ctx* ctx, int n_rhs, int* variant_host, double* ms_host, int cap) {
  if (!ctx || cap < 0 || (cap > 0 && (!variant_host || !ms_host))) return LM_EINVAL;
  auto it = ctx->tilesets.find(n_rhs);
  if (it == ctx->tilesets.end()) return 0;
  const std::vector<lm_ctx::Chunk>& ch = it->second.chunks;
  for (int c = 0; c < (int)ch.size() && c < cap; c++) {
    variant_host[c] = ch[c].variant;
    for (int v = 0; v < LM_M2L_VARIANTS; v++) ms_host[(size_t)c * LM_M2L_VARIANTS + v] = ch[c].ms[v];
  }
  return (int)ch.size();
}

static uint64_t plan_digest(const Plan& pl);

int lm_stats(const lm_ctx* ctx, double* out, int n) {
  if (!ctx || !out || n < 1) return LM_EINVAL;
  const Plan& pl = ctx->plan;
  double v[LM_STATS_COUNT] = {0};
  v[LM_STAT_N_FREE_INST] = pl.n_free_inst;
  v[LM_STAT_N_REACT_INST] = pl.n_react_inst;
  v[LM_STAT_M2L_PAIRS_FREE] = (double)pl.n_m2l_pairs_free;
  v[LM_STAT_M2L_PAIRS_REACT] = (double)pl.n_m2l_pairs_react;
  v[LM_STAT_P2P_PAIRS] = (double)pl.n_p2p_pairs;
  v[LM_STAT_N_CASES] = (double)pl.cases.size();
  v[LM_STAT_N_NODES] = (double)pl.node_kr.size();
  v[LM_STAT_MAT_BYTES] = (double)pl.mat_size * 16.0;
  v[LM_STAT_ME_BYTES_PER_RHS] = (double)pl.me_size * 16.0;
  v[LM_STAT_LE_BYTES_PER_RHS] = (double)pl.le_size * 16.0;
  v[LM_STAT_T_PLAN_MS] = ctx->t_plan_ms;
  v[LM_STAT_T_UPLOAD_MS] = ctx->t_upload_ms;
  v[LM_STAT_T_TABLES_MS] = ctx->t_tables_ms;
  v[LM_STAT_N_SRC_BOXES] = (double)pl.sbox.size();
  v[LM_STAT_N_TGT_BOXES] = (double)pl.tbox.size();
  v[LM_STAT_N_M2L_CLASSES] = (double)pl.cls.size();
  v[LM_STAT_N_M2L_TILES_1RHS] = 0;
  {
    long long t = 0;
    for (auto& C : pl.cls) {
      const int p = pl.inst[C.inst].p;
      const long long rt = C.nblk == 3 ? (lm_sym_dim(p, 0) + TM_ROWS - 1) / TM_ROWS + (lm_sym_dim(p, 1) + TM_ROWS - 1) / TM_ROWS
                                       : 3LL * ((C.P + TM_ROWS - 1) / TM_ROWS);
      t += rt * ((C.n_tgt + TN_COLS - 1) / TN_COLS);
    }
    v[LM_STAT_N_M2L_TILES_1RHS] = (double)t;
  }
  {
    // M2L work (complex multiply-adds) per right-hand side: useful (free
    // space: a Po x Po product per pair and output type; reaction: the even
    // and the odd square block of the mirror-adapted tensor per pair) and as
    // executed by the 64 x 64 GEMM tiles (padding of partial tiles included)
    double cm = 0, ce = 0;
    for (const M2LBlock& B : pl.blocks) {
      const M2LClass& C = pl.cls[B.cls];
      m2l_groups(pl, B, [&](int o0, int o1) {
        const int np = pl.offr[B.offr0 + o1] - pl.offr[B.offr0 + o0];
        const int po = pl.offs[C.off0 + o0].pord, Po = (po + 1) * (po + 1);
        const double cols = (double)((np + TN_COLS - 1) / TN_COLS) * TN_COLS;
        for (int ot = 0; ot < (C.nblk == 3 ? 2 : 3); ot++) {
          const double R = C.nblk == 3 ? lm_sym_dim(po, ot) : Po;
          const double rows = (double)(((int)R + TM_ROWS - 1) / TM_ROWS) * TM_ROWS;
          cm += R * R * np;
          ce += rows * R * cols;
        }
      });
    }
    v[LM_STAT_M2L_CMAC_USEFUL] = cm;
    v[LM_STAT_M2L_CMAC_EXEC] = ce;
    double cd_ = 0;
    for (const M2LBlock& B : pl.blocks) {
      const M2LClass& C = pl.cls[B.cls];
      for (int o = 0; o < C.n_off; o++) {
        const int np = pl.offr[B.offr0 + o + 1] - pl.offr[B.offr0 + o];
        const int po = pl.offs[C.off0 + o].pord;
        const double Po = (po + 1) * (po + 1);
        cd_ += 3.0 * Po * C.nblk * Po * np;
      }
    }
    v[LM_STAT_M2L_CMAC_DENSE] = cd_;
    v[LM_STAT_P2P_KERNEL_EVALS] = ctx->p2ps_n > 0 ? ctx->p2ps_evals : (double)pl.n_p2p_pairs;
  }
  {
    // executed MFMA flops of the M2L GEMM per rhs (variant 0: 16 values of k
    // per chunk): a wave computes the 16 x 16 tiles that hold a row below
    // the offset's used rows and a column below the tile's pair count, over
    // k padded to whole chunks, with three real MFMAs per complex step
    double fe = 0;
    for (const M2LBlock& B : pl.blocks) {
      const M2LClass& C = pl.cls[B.cls];
      m2l_groups(pl, B, [&](int o0, int o1) {
        const long long np = pl.offr[B.offr0 + o1] - pl.offr[B.offr0 + o0];
        if (np == 0) return;
        const int po = pl.offs[C.off0 + o0].pord, Po = (po + 1) * (po + 1);
        // 64-column tiles: a wave computes the 16-column tiles below the tile's count
        const double cols = (double)(np / 64) * 64 + (double)(((np % 64) + 15) / 16) * 16;
        for (int ot = 0; ot < (C.nblk == 3 ? 2 : 3); ot++) {
          const int R = C.nblk == 3 ? lm_sym_dim(po, ot) : Po;
          const double rows = (double)((R / 64) * 64 + (((R % 64) + 15) / 16) * 16), kp = (double)((R + 15) / 16) * 16;
          fe += rows * cols * kp * 3.0 * 2.0;
        }
      });
    }
    v[LM_STAT_M2L_FLOP_EXEC] = fe;
  }
  {
    // algorithmic work of the other passes per rhs: 8 flops per complex
    // multiply-add of the expansion sums and translations; the M2L
    // reduction's bytes (outputs read once, local expansions read and
    // written once)
    double f_p2m = 0, f_m2m = 0, f_l2l = 0, f_l2p = 0, b_red = 0;
    for (int b : pl.p2m_leaves) {
      const SrcBox& sb = pl.sbox[b];
      f_p2m += (double)(sb.pt1 - sb.pt0) * 3.0 * pl.inst[sb.inst].P * 8.0;
    }
    for (size_t b = 0; b < pl.sbox.size(); b++)
      if (pl.sbox_m2m[b] >= 0) f_m2m += 3.0 * (double)pl.inst[pl.sbox[b].inst].P * pl.inst[pl.sbox[b].inst].P * 8.0;
    for (size_t b = 0; b < pl.tbox.size(); b++)
      if (pl.tbox_l2l[b] >= 0) f_l2l += 3.0 * (double)pl.inst[pl.tbox[b].inst].P * pl.inst[pl.tbox[b].inst].P * 8.0;
    for (size_t i = 0; i < pl.l2p_leaves.size(); i++) {
      const int p = pl.inst[i].p, pe = pl.inst[i].kind == 0 ? p + 2 : p;
      for (int b : pl.l2p_leaves[i])
        f_l2p += (double)(pl.tbox[b].pt1 - pl.tbox[b].pt0) * 3.0 * (pe + 1) * (pe + 1) * 8.0;
    }
    for (size_t q = 0; q < pl.pair_P.size(); q++) b_red += 3.0 * pl.pair_P[q] * 16.0;
    for (size_t bt = 0; bt < pl.bt_tbox.size(); bt++) b_red += 2.0 * 3.0 * pl.inst[pl.tbox[pl.bt_tbox[bt]].inst].P * 16.0;
    v[LM_STAT_P2M_FLOPS] = f_p2m;
    v[LM_STAT_M2M_FLOPS] = f_m2m;
    v[LM_STAT_L2L_FLOPS] = f_l2l;
    v[LM_STAT_L2P_FLOPS] = f_l2p;
    v[LM_STAT_REDUCE_BYTES] = b_red;
  }
  {
    // quadrature nodes summed over the direct reaction pairs: each pair runs
    // the first contour piece and the real tail up to its own cut
    // a + LM_S2T_DIGITS / (t + u) (needs the host copies of the points)
    double ne = 0;
    const bool have = !ctx->host_src.empty() && !ctx->host_tgt.empty();
    for (size_t it = 0; have && it < pl.s2t_items.size(); it += 2) {
      if (pl.s2t_items[it + 1] != 0) continue;  // one entry per leaf
      const TgtBox& tb = pl.tbox[pl.s2t_items[it]];
      const InstParams& ip = pl.inst[tb.inst];
      const cd* kr = pl.node_kr.data() + ip.s2t0;
      int n1 = 0;
      while (n1 < ip.s2tn && kr[n1].y != 0.0) n1++;  // first piece (complex nodes)
      const double dls = ip.up_s ? ctx->med.d[ip.ls - 1] : ctx->med.d[ip.ls];
      for (int t = tb.pt0; t < tb.pt1; t++) {
        const double zt = ctx->host_tgt[3 * pl.tgt_perm[t] + 2];
        const double tz = ip.up_t ? zt - ctx->med.d[ip.lt] : ctx->med.d[ip.lt - 1] - zt;
        for (int li = tb.p2p0; li < tb.p2p1; li++) {
          const SrcBox& sb = pl.sbox[pl.p2p_list[li]];
          for (int sp = sb.pt0; sp < sb.pt1; sp++) {
            const double zs = ctx->host_src[3 * pl.src_perm[sp] + 2];
            const double uz = ip.up_s ? dls - zs : zs - dls;
            const double kcut = ctx->contour_a + LM_S2T_DIGITS / (tz + uz);
            int lo = n1, hi = ip.s2tn;  // tail nodes <= kcut (increasing)
            while (lo < hi) {
              const int mid = (lo + hi) / 2;
              if (kr[mid].x <= kcut) lo = mid + 1; else hi = mid;
            }
            ne += (double)lo;
          }
        }
      }
    }
    v[LM_STAT_S2T_NODE_EVALS] = ne;
  }
  v[LM_STAT_N_LEAVES_P2M] = (double)pl.p2m_leaves.size();
  double fd = 0;
  for (int x : pl.free_depth_used) fd = std::max(fd, (double)x);
  v[LM_STAT_FREE_DEPTH] = fd;
  v[LM_STAT_S2T_PAIRS] = (double)pl.n_s2t_pairs;
  v[LM_STAT_TREE_RECORDS] = ctx->tree_records;
  v[LM_STAT_TREE_SORT_MS] = ctx->tree_sort_ms;
  if (n > LM_STAT_PLAN_DIGEST_HI) {
    const uint64_t h = plan_digest(pl);
    v[LM_STAT_PLAN_DIGEST_HI] = (double)(h >> 32);
    v[LM_STAT_PLAN_DIGEST_LO] = (double)(h & 0xffffffffull);
  }
  int m = n < LM_STATS_COUNT ? n : LM_STATS_COUNT;
  memcpy(out, v, m * sizeof(double));
  return LM_OK;
}

// FNV-style hash over 8-byte words of every array of a plan (trees, lists,
// M2L schedule, table cases, nodes, coefficient tables)
static uint64_t plan_digest(const Plan& pl) {
  {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t bytes) {
      const unsigned char* c = (const unsigned char*)p;
      h = (h ^ (uint64_t)bytes) * 1099511628211ull;
      size_t i = 0;
      for (; i + 8 <= bytes; i += 8) {
        uint64_t w;
        memcpy(&w, c + i, 8);
        h = (h ^ w) * 1099511628211ull;
      }
      for (; i < bytes; i++) h = (h ^ c[i]) * 1099511628211ull;
    };
    auto vec = [&](const auto& x) { mix(x.data(), x.size() * sizeof(x[0])); };
    auto vecs = [&](const auto& xs) {
      for (const auto& x : xs) vec(x);
    };
    vec(pl.inst), vec(pl.src_perm), vec(pl.tgt_perm), vec(pl.sbox), vec(pl.tbox), vec(pl.sbox_m2m), vec(pl.tbox_l2l);
    vecs(pl.m2m_parents), vecs(pl.l2l_children), vec(pl.p2m_leaves), vecs(pl.l2p_leaves), vecs(pl.p2p_tboxes);
    vec(pl.p2p_list), vec(pl.cls), vec(pl.offs), vec(pl.cls_tgt), vec(pl.cls_srcof), vec(pl.cls_srcof0);
    vec(pl.blocks), vec(pl.bt_tbox), vec(pl.bt_ptr), vec(pl.bt_pairs), vec(pl.pair_src), vec(pl.offr), vec(pl.bt_blk);
    vec(pl.pair_P), vec(pl.pair_phi), vec(pl.s2t_items), vec(pl.trans), vec(pl.cases), vec(pl.node_kr);
    vec(pl.node_w), vec(pl.node_inst), vec(pl.Bcoef), vec(pl.Ccoef), vec(pl.Ccoef0), vec(pl.free_depth_used);
    return h;
  }
}

int lm_selftest_math(int64_t n, const double* x_dev, double* out_dev, void* stream) {
  if (n < 0 || (n > 0 && (!x_dev || !out_dev))) return LM_EINVAL;
  launch_selftest_math(x_dev, n, out_dev, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? LM_OK : LM_EHIP;
}

// ---------------------------------------------------------------- host-only helpers
int lm_host_components(int n_layers, const double* d, const double* k, int* out, int cap) {
  if (n_layers < 1 || n_layers > LM_MAXL || !k || (n_layers > 1 && !d)) return LM_EINVAL;
  Medium m;
  m.n = n_layers;
  for (int l = 0; l < n_layers; l++) {
    m.k[l] = k[l];
    m.mu[l] = 1.0;
  }
  for (int l = 0; l < n_layers - 1; l++) m.d[l] = d[l];
  std::vector<InstParams> v;
  int n = lm_enumerate_components(m, v);
  for (int i = 0; i < n && i < cap; i++) {
    out[8 * i + 0] = v[i].lt;
    out[8 * i + 1] = v[i].ls;
    out[8 * i + 2] = v[i].up_t;
    out[8 * i + 3] = v[i].up_s;
    out[8 * i + 4] = v[i].sgn;
    out[8 * i + 5] = (int)v[i].at;
    out[8 * i + 6] = (int)v[i].as;
    out[8 * i + 7] = 0;
  }
  return n;
}

int lm_host_cheb_affine(int jmax, double a, double b, double* out) {
  if (jmax < 0 || jmax > 64 || !out) return LM_EINVAL;
  std::vector<double> C;
  lm_cheb_affine(jmax, a, b, C);
  memcpy(out, C.data(), C.size() * sizeof(double));
  return LM_OK;
}

int lm_host_legendre_cheb(int p, double* out, int* stride) {
  if (p < 0 || p > LM_PMAX_ORDER || !out || !stride) return LM_EINVAL;
  std::vector<double> B;
  lm_legendre_cheb(p, B);
  memcpy(out, B.data(), B.size() * sizeof(double));
  *stride = (p + 1) / 2 + 2;
  return LM_OK;
}

int lm_host_plan_stats(int n_layers, const double* d, const double* k, const lm_params* prm, int64_t n_src,
                       const double* src_xyz, int64_t n_tgt, const double* tgt_xyz, double* out, int n,
                       char* errbuf, int errlen) {
  lm_ctx tmp;
  int rc = lm_set_layers(&tmp, n_layers, d, k, nullptr);
  if (rc) {
    if (errbuf && errlen > 0) snprintf(errbuf, errlen, "%s", tmp.err.c_str());
    return rc;
  }
  if (prm && (rc = lm_set_params(&tmp, prm))) {
    if (errbuf && errlen > 0) snprintf(errbuf, errlen, "%s", tmp.err.c_str());
    return rc;
  }
  std::string msg = lm_make_plan(tmp.plan, tmp.med, tmp.prm, n_src, src_xyz, n_tgt, tgt_xyz);
  if (!msg.empty()) {
    if (errbuf && errlen > 0) snprintf(errbuf, errlen, "%s", msg.c_str());
    return msg.compare(0, strlen(LM_PLAN_ACCURACY_PREFIX), LM_PLAN_ACCURACY_PREFIX) == 0 ? LM_EACCURACY : LM_EDOMAIN;
  }
  return lm_stats(&tmp, out, n);
}

int lm_host_plan_digests(int n_layers, const double* d, const double* k, const lm_params* prm, int n_geom,
                         const int64_t* src_off, const double* src_xyz, const int64_t* tgt_off,
                         const double* tgt_xyz, uint64_t* digest, char* errbuf, int errlen) {
  if (n_geom < 1 || !src_off || !tgt_off || !digest || src_off[0] != 0 || tgt_off[0] != 0) return LM_EINVAL;
  for (int g = 0; g < n_geom; g++)
    if (src_off[g + 1] < src_off[g] || tgt_off[g + 1] < tgt_off[g]) return LM_EINVAL;
  if ((src_off[n_geom] > 0 && !src_xyz) || (tgt_off[n_geom] > 0 && !tgt_xyz)) return LM_EINVAL;
  lm_ctx tmp;
  int rc = lm_set_layers(&tmp, n_layers, d, k, nullptr);
  if (!rc && prm) rc = lm_set_params(&tmp, prm);
  if (rc) {
    if (errbuf && errlen > 0) snprintf(errbuf, errlen, "%s", tmp.err.c_str());
    return rc;
  }
  // the external route's contract, by plain loops: per tree, every
  // segment's records keyed by the bits of the three cell indices
  // interleaved one at a time, then a stable sort by key
  TreeSorter plain = [&](const std::vector<TreeJob>& jobs, const std::vector<TreeSeg>& segs,
                         std::vector<uint64_t>& keys, std::vector<uint32_t>& pay,
                         std::vector<uint64_t>& boxes) -> std::string {
    keys.clear();
    pay.clear();
    boxes.clear();
    for (const TreeJob& J : jobs) {
      std::vector<std::pair<uint64_t, uint32_t>> r;
      const double inv = (double)(1 << LM_TREE_DK) / J.S0;
      for (int q = 0; q < J.nseg; q++) {
        const TreeSeg& g = segs[J.seg0 + q];
        const double* xyz = g.tgt ? tgt_xyz : src_xyz;
        for (int i = 0; i < g.n; i++) {
          const double* x = xyz + 3 * (size_t)g.ids[i];
          const double z = g.za * x[2] + g.zb;
          const double c[3] = {x[0] - J.x0, x[1] - J.y0, z - J.z0};
          uint64_t key = 0;
          for (int a = 0; a < 3; a++) {
            long long u = (long long)floor(c[a] * inv);
            u = std::min(std::max(u, 0LL), (1LL << LM_TREE_DK) - 1);
            for (int b = 0; b < LM_TREE_DK; b++) key |= (uint64_t)((u >> b) & 1) << (3 * b + a);
          }
          r.push_back({key, (uint32_t)g.ids[i] | ((uint32_t)g.tag << 31)});
        }
      }
      std::stable_sort(r.begin(), r.end(), [](const std::pair<uint64_t, uint32_t>& a,
                                              const std::pair<uint64_t, uint32_t>& b) { return a.first < b.first; });
      // the boxes, level by level: a level-l box starts at every record whose
      // level-l cell differs from the previous record's, if every box above
      // it on the record's path is split (below the depth; with gap_only,
      // gap index 0)
      const size_t base = keys.size();
      for (size_t i = 0; i < r.size(); i++) {
        const uint64_t key = r[i].first;
        int depth = J.depth;
        if (J.gap_only)
          for (int l = 0; l < J.depth; l++) {
            long long iz = 0;
            for (int b = 0; b < l; b++) iz |= (long long)((key >> (3 * (LM_TREE_DK - l + b) + 2)) & 1) << b;
            const long long j = J.zflip ? (1LL << l) - 1 - iz : iz;
            if (j != 0) {
              depth = l;
              break;
            }
          }
        for (int l = 0; l <= depth; l++) {
          const int sh = 3 * (LM_TREE_DK - l);
          const bool starts = i == 0 || (l > 0 && (key >> sh) != (r[i - 1].first >> sh));
          if (starts) boxes.push_back(((uint64_t)l << 40) | (uint64_t)(base + i));
        }
      }
      for (const auto& e : r) {
        keys.push_back(e.first);
        pay.push_back(e.second);
      }
    }
    return "";
  };
  for (int route = 0; route < 2; route++) {
    Plan pl;
    std::string msg = lm_make_plan_multi(pl, tmp.med, tmp.prm, n_geom, src_off, src_xyz, tgt_off, tgt_xyz,
                                         route == 0 ? &plain : nullptr);
    if (!msg.empty()) {
      if (errbuf && errlen > 0) snprintf(errbuf, errlen, "%s", msg.c_str());
      return msg.compare(0, strlen(LM_PLAN_ACCURACY_PREFIX), LM_PLAN_ACCURACY_PREFIX) == 0 ? LM_EACCURACY
                                                                                           : LM_EDOMAIN;
    }
    digest[route] = plan_digest(pl);
  }
  return LM_OK;
}


// ---------------------------------------------------------------- iterative solve
// Device vectors of the GMRES iteration on a built context: the basis and the
// work vector live in ctx->kv_buf, the iterate X and the right-hand side B are
// the caller's arrays.  Inner products come back to the host through pinned
// memory (one stream synchronisation each); coefficient vectors go down the
// same way, each before the next synchronisation, so one staging block serves.
struct DevKrylov : KrylovSpace {
  lm_ctx* ctx = nullptr;
  hipStream_t s = nullptr;
  long long n3 = 0;
  const cd* diag = nullptr;
  cd* const* vt = nullptr;   // device vector table
  cd* dsum = nullptr;              // device inner products [(m+1) R]
  cd* dcoef = nullptr;             // device coefficients [(m+1) R]
  cd* hsum = nullptr;              // pinned host copies
  cd* hcoef = nullptr;
  double bytes = 0, ms_matvec = 0, ms_krylov = 0;
  struct Ev {
    hipEvent_t a, b;
    int kind;  // 0 matvec, 1 vector kernels
  };
  std::vector<hipEvent_t> owned;   // every event created here, destroyed with the object
  std::vector<hipEvent_t> pool;    // events free for reuse
  std::vector<Ev> pending;
  // the copy of hcoef to dcoef last enqueued: hcoef is not rewritten before
  // it has run (the copy reads the pinned buffer when the stream reaches it)
  hipEvent_t coef_ev = nullptr;
  bool coef_pending = false;
  int err = 0;

  ~DevKrylov() override {
    for (auto e : owned) hipEventDestroy(e);
  }
  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      err = 1;
      return nullptr;
    }
    owned.push_back(e);
    return e;
  }
  int tic(Ev& e, int kind) {
    e.a = ev();
    e.b = ev();
    e.kind = kind;
    if (err) return fail(ctx, LM_EHIP, "hipEventCreate failed");
    return hipEventRecord(e.a, s) == hipSuccess ? 0 : fail(ctx, LM_EHIP, "hipEventRecord failed");
  }
  int toc(Ev& e) {
    if (hipEventRecord(e.b, s) != hipSuccess) return fail(ctx, LM_EHIP, "hipEventRecord failed");
    pending.push_back(e);
    return 0;
  }
  // waits for the stream and books the elapsed times of the recorded spans
  int sync() {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(ctx, LM_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    for (auto& p : pending) {
      float ms = 0;
      hipEventElapsedTime(&ms, p.a, p.b);
      (p.kind ? ms_krylov : ms_matvec) += ms;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
    coef_pending = false;
    return 0;
  }
  int launched() {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : fail(ctx, LM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  }
  int put_coef(const cd* c, int count) {
    if (!coef_ev && !(coef_ev = ev())) return fail(ctx, LM_EHIP, "hipEventCreate failed");
    hipError_t e = coef_pending ? hipEventSynchronize(coef_ev) : hipSuccess;
    if (e != hipSuccess) return fail(ctx, LM_EHIP, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
    memcpy(hcoef, c, (size_t)count * n_rhs * sizeof(cd));
    e = hipMemcpyAsync(dcoef, hcoef, (size_t)count * n_rhs * sizeof(cd), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(coef_ev, s);
    if (e != hipSuccess) return fail(ctx, LM_EHIP, std::string("coefficient copy: ") + hipGetErrorString(e));
    coef_pending = true;
    return 0;
  }
  double vec_bytes() const { return (double)n_rhs * n3 * sizeof(cd); }

  int apply(int src, int dst) override {
    Ev e;
    int rc = tic(e, 0);
    if (rc) return rc;
    rc = lm_evaluate(ctx, n_rhs, host_ptr[src], host_ptr[dst], s);
    if (rc) return rc;
    if ((rc = toc(e))) return rc;
    if ((rc = tic(e, 1))) return rc;
    launch_kv_diag(vt, src, diag, dst, n3, n_rhs, s);
    if ((rc = launched())) return rc;
    bytes += 3 * vec_bytes() + (diag ? (double)n3 / 3 * sizeof(cd) : 0.0);
    return toc(e);
  }
  int dots(int first, int count, int w, cd* h) override {
    Ev e;
    int rc = tic(e, 1);
    if (rc) return rc;
    launch_kv_dots(vt, first, count, w, n3, n_rhs, kv_dots_nb(n3, n_rhs, count), ctx->kv_part, dsum, s);
    if ((rc = launched()) || (rc = toc(e))) return rc;
    bytes += (count + 1) * vec_bytes();
    hipError_t x = hipMemcpyAsync(hsum, dsum, (size_t)count * n_rhs * sizeof(cd), hipMemcpyDeviceToHost, s);
    if (x != hipSuccess) return fail(ctx, LM_EHIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(x));
    if ((rc = sync())) return rc;
    memcpy(h, hsum, (size_t)count * n_rhs * sizeof(cd));
    return 0;
  }
  int combine(int first, int count, const cd* c, int dst) override {
    int rc = put_coef(c, count);
    if (rc) return rc;
    Ev e;
    if ((rc = tic(e, 1))) return rc;
    launch_kv_combine(vt, first, count, dcoef, dst, n3, n_rhs, s);
    bytes += (count + 2) * vec_bytes();
    if ((rc = launched())) return rc;
    return toc(e);
  }
  int scale(int src, const cd* c, int dst) override {
    int rc = put_coef(c, 1);
    if (rc) return rc;
    Ev e;
    if ((rc = tic(e, 1))) return rc;
    launch_kv_scale(vt, src, dcoef, dst, n3, n_rhs, s);
    bytes += 2 * vec_bytes();
    if ((rc = launched())) return rc;
    return toc(e);
  }
  int rsub(int b, int w) override {
    Ev e;
    int rc = tic(e, 1);
    if (rc) return rc;
    launch_kv_rsub(vt, b, w, n3, n_rhs, s);
    bytes += 3 * vec_bytes();
    if ((rc = launched())) return rc;
    return toc(e);
  }
  std::vector<cd*> host_ptr;  // the same table on the host
};

int lm_solve(lm_ctx* ctx, int n_rhs, const void* diag, const void* B, void* X, double tol, int restart,
             int max_iter, double* relres_host, lm_solve_info* info, void* stream) {
  if (!ctx) return LM_EINVAL;
  if (!ctx->built) return fail(ctx, LM_ESTATE, "lm_build must succeed before lm_solve");
  if (!ctx->same_sets) return fail(ctx, LM_ESTATE, "lm_solve needs a build with the same source and target points");
  if (n_rhs < 1 || n_rhs > 4096) return fail(ctx, LM_EINVAL, "n_rhs out of range (1..4096)");
  if (restart < 1 || restart > LM_SOLVE_MAX_RESTART) return fail(ctx, LM_EINVAL, "restart out of range");
  if (max_iter < 1) return fail(ctx, LM_EINVAL, "max_iter must be >= 1");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, LM_EINVAL, "tol must be finite and > 0");
  const long long n = ctx->plan.n_src;
  if (n > 0 && (!B || !X)) return fail(ctx, LM_EINVAL, "null B or X");
  if (((uintptr_t)B % 16) || ((uintptr_t)X % 16) || ((uintptr_t)diag % 16))
    return fail(ctx, LM_EINVAL, "B, X and diag must be 16-byte aligned");
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) {
    for (int r = 0; r < n_rhs && relres_host; r++) relres_host[r] = 0.0;
    if (info) *info = lm_solve_info{0, 0, 0, 1, 0.0, 0.0, 0.0, 0.0};
    return LM_OK;
  }
  const int m = restart;
  const long long n3 = 3 * n;
  // buffers: basis 0..m and W; partials; small block = vector table + sums + coefficients
  const long long need = (long long)(m + 2) * n_rhs * n3;
  if (need > ctx->kv_cap) {
    if (ctx->kv_buf) hipFree(ctx->kv_buf);
    ctx->kv_buf = nullptr;
    ctx->kv_cap = 0;
    if (hipMalloc((void**)&ctx->kv_buf, (size_t)need * sizeof(cd)) != hipSuccess)
      return fail(ctx, LM_ENOMEM, "cannot allocate the Krylov basis");
    ctx->kv_cap = need;
  }
  long long pneed = 1;
  for (int c = 1; c <= m + 1; c++)
    pneed = std::max(pneed, (long long)c * n_rhs * kv_dots_nb(n3, n_rhs, c));
  if (pneed > ctx->kv_part_cap) {
    if (ctx->kv_part) hipFree(ctx->kv_part);
    ctx->kv_part = nullptr;
    ctx->kv_part_cap = 0;
    if (hipMalloc((void**)&ctx->kv_part, (size_t)pneed * sizeof(cd)) != hipSuccess)
      return fail(ctx, LM_ENOMEM, "cannot allocate the inner-product partials");
    ctx->kv_part_cap = pneed;
  }
  const size_t tab_bytes = 1024, vec_small = (size_t)(m + 1) * n_rhs * sizeof(cd);
  const size_t sneed = tab_bytes + 2 * vec_small;
  if (sneed > ctx->kv_small_cap) {
    if (ctx->kv_small) hipFree(ctx->kv_small);
    if (ctx->kv_host) hipHostFree(ctx->kv_host);
    ctx->kv_small = ctx->kv_host = nullptr;
    ctx->kv_small_cap = 0;
    if (hipMalloc(&ctx->kv_small, sneed) != hipSuccess || hipHostMalloc(&ctx->kv_host, sneed) != hipSuccess)
      return fail(ctx, LM_ENOMEM, "cannot allocate the solve's small buffers");
    ctx->kv_small_cap = sneed;
  }
  DevKrylov S;
  S.ctx = ctx;
  S.s = s;
  S.m = m;
  S.n_rhs = n_rhs;
  S.n3 = n3;
  S.diag = (const cd*)diag;
  S.host_ptr.resize(m + 4);
  for (int v = 0; v <= m + 1; v++) S.host_ptr[v] = ctx->kv_buf + (long long)v * n_rhs * n3;
  S.host_ptr[S.vX()] = (cd*)X;
  S.host_ptr[S.vB()] = (cd*)B;
  char* sm = (char*)ctx->kv_small;
  char* hm = (char*)ctx->kv_host;
  S.vt = (cd* const*)sm;
  S.dsum = (cd*)(sm + tab_bytes);
  S.dcoef = (cd*)(sm + tab_bytes + vec_small);
  S.hsum = (cd*)(hm + tab_bytes);
  S.hcoef = (cd*)(hm + tab_bytes + vec_small);
  memcpy(hm, S.host_ptr.data(), (m + 4) * sizeof(cd*));
  HIPC(hipMemcpyAsync(sm, hm, (m + 4) * sizeof(cd*), hipMemcpyHostToDevice, s));
  hipEvent_t e0 = S.ev(), e1 = S.ev();
  if (S.err) return fail(ctx, LM_EHIP, "hipEventCreate failed");
  HIPC(hipEventRecord(e0, s));
  std::vector<double> rr(n_rhs, 0.0);
  GmresResult gr;
  int rc = gmres_drive(S, tol, max_iter, rr.data(), &gr);
  if (rc) {
    hipStreamSynchronize(s);
    return rc;
  }
  HIPC(hipEventRecord(e1, s));
  if ((rc = S.sync())) return rc;
  float total = 0;
  hipEventElapsedTime(&total, e0, e1);
  if (relres_host) memcpy(relres_host, rr.data(), n_rhs * sizeof(double));
  if (info) {
    info->iters = gr.iters;
    info->matvecs = gr.matvecs;
    info->cycles = gr.cycles;
    info->converged = gr.converged;
    info->ms_total = total;
    info->ms_matvec = S.ms_matvec;
    info->ms_krylov = S.ms_krylov;
    info->krylov_bytes = S.bytes;
  }
  return LM_OK;
}

// The same driver on a dense host matrix (tests of the host logic), with the
// n_rhs columns of each vector stored one after the other (as on the device).
struct HostKrylov : KrylovSpace {
  int n = 0;
  const double* A = nullptr;          // complex128 [n][n]
  std::vector<std::vector<cd>> v;     // vectors 0..m+3, each [n_rhs][n]
  int apply(int src, int dst) override {
    const cd* a = (const cd*)A;
    for (int r = 0; r < n_rhs; r++)
      for (int i = 0; i < n; i++) {
        cd acc{0, 0};
        for (int j = 0; j < n; j++) acc = acc + a[(size_t)i * n + j] * v[src][(size_t)r * n + j];
        v[dst][(size_t)r * n + i] = acc;
      }
    return 0;
  }
  int dots(int first, int count, int w, cd* h) override {
    for (int k = 0; k < count; k++)
      for (int r = 0; r < n_rhs; r++) {
        cd acc{0, 0};
        for (int i = 0; i < n; i++) acc = acc + cconj(v[first + k][(size_t)r * n + i]) * v[w][(size_t)r * n + i];
        h[(size_t)k * n_rhs + r] = acc;
      }
    return 0;
  }
  int combine(int first, int count, const cd* c, int dst) override {
    for (int r = 0; r < n_rhs; r++)
      for (int i = 0; i < n; i++)
        for (int k = 0; k < count; k++)
          v[dst][(size_t)r * n + i] = v[dst][(size_t)r * n + i] + v[first + k][(size_t)r * n + i] * c[(size_t)k * n_rhs + r];
    return 0;
  }
  int scale(int src, const cd* c, int dst) override {
    for (int r = 0; r < n_rhs; r++)
      for (int i = 0; i < n; i++) v[dst][(size_t)r * n + i] = v[src][(size_t)r * n + i] * c[r];
    return 0;
  }
  int rsub(int b, int w) override {
    for (size_t i = 0; i < v[w].size(); i++) v[w][i] = v[b][i] - v[w][i];
    return 0;
  }
};

int lm_host_gmres_dense(int n, int n_rhs, const double* A, const double* b, double* x, double tol, int restart,
                        int max_iter, int* iters, double* relres) {
  if (n < 1 || n_rhs < 1 || n_rhs > 4096 || !A || !b || !x || restart < 1 || restart > LM_SOLVE_MAX_RESTART ||
      max_iter < 1 || !(tol > 0) || !std::isfinite(tol))
    return LM_EINVAL;
  HostKrylov S;
  S.n = n;
  S.m = restart;
  S.n_rhs = n_rhs;
  S.A = A;
  const size_t len = (size_t)n_rhs * n;
  S.v.assign(restart + 4, std::vector<cd>(len, cd{0, 0}));
  memcpy(S.v[S.vX()].data(), x, len * sizeof(cd));
  memcpy(S.v[S.vB()].data(), b, len * sizeof(cd));
  std::vector<double> rr(n_rhs, 0.0);
  GmresResult gr;
  gmres_drive(S, tol, max_iter, rr.data(), &gr);
  memcpy(x, S.v[S.vX()].data(), len * sizeof(cd));
  if (iters) *iters = gr.iters;
  if (relres) memcpy(relres, rr.data(), n_rhs * sizeof(double));
  return LM_OK;
}

}  // extern "C"
