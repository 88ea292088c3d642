// Host side of libpsfd: plan construction, operator pipelines, the BiCGSTAB
// driver and the C ABI declared in include/psfd.h.
//
// A plan holds a group of G >= 1 problems of one shape (same grid, optics,
// multilayer, PML, preconditioner and precision; angle, polarisation and
// permittivity may differ).  psfd_plan makes G = 1; psfd_solve_batch forms
// groups of compatible problems.  Every launch covers the whole group, the
// Krylov scalars are per problem on the device, and a converged problem is
// skipped by every kernel while the rest of its group iterates.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "psfd.h"
#include "psfd_internal.h"
#include "reduce.h"

using namespace psfd;

namespace {

thread_local std::string g_err;

psfd_status fail(psfd_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define CHK(...)                                                                         \
  do {                                                                                   \
    hipError_t e_ = (__VA_ARGS__);                                                       \
    if (e_ != hipSuccess)                                                                \
      return fail(PSFD_ERR_HIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CHKS(...)                           \
  do {                                      \
    psfd_status s_ = (__VA_ARGS__);         \
    if (s_ != PSFD_OK) return s_;           \
  } while (0)

// Device memory cache: blocks given back by a destroyed plan are kept per
// (device, size) and handed to the next plan asking for that size (plans of
// one shape are typically made and destroyed in a loop), at most kCacheMax
// bytes in all.  A failed allocation empties the cache and tries again;
// psfd_trim_cache() empties it on request, PSFD_CACHE=0 disables it.
std::mutex g_cache_mu;
std::multimap<std::pair<int, size_t>, void*> g_cache;
size_t g_cache_bytes = 0;
constexpr size_t kCacheMax = size_t(32) << 30;

bool cache_on() {
  static const bool on = [] {
    const char* e = std::getenv("PSFD_CACHE");
    return !(e && *e && std::atoi(e) == 0);
  }();
  return on;
}

void* cache_take(int dev, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find({dev, bytes});
  if (it == g_cache.end()) return nullptr;
  void* p = it->second;
  g_cache.erase(it);
  g_cache_bytes -= bytes;
  return p;
}

bool cache_put(int dev, size_t bytes, void* p) {
  if (!cache_on()) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (g_cache_bytes + bytes > kCacheMax) return false;
  g_cache.emplace(std::make_pair(dev, bytes), p);
  g_cache_bytes += bytes;
  return true;
}

void cache_trim() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& kv : g_cache) (void)hipFree(kv.second);
  g_cache.clear();
  g_cache_bytes = 0;
}

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kChunk = 16;         // BiCGSTAB iterations queued between convergence checks
constexpr int kMaxRestarts = 10;   // residual replacements (FP64) / refinement steps (mixed)

enum { OP_A = 0, OP_AM = 1, OP_AH = 2, OP_M = 3, OP_HF = 4 };  // OP_HF: F3^-1 w^2 F3
enum { V_R = 0, V_RH, V_P, V_V, V_S, V_T, V_Y, V_W, V_COUNT };

int fftfreq(int m, int n) { return (m < (n + 1) / 2) ? m : m - n; }

std::vector<cplx<double>> twiddles(int n) {
  std::vector<cplx<double>> w(n);
  for (int m = 0; m < n; ++m) {
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * m / n;
    w[m] = {(double)cosl(a), (double)sinl(a)};
  }
  return w;
}

}  // namespace


// A timed launch: events before and after it, its algorithmic bytes, and the
// Krylov iteration (within the chunk being launched) it belongs to, -1 outside.
struct ProfPair {
  hipEvent_t a = nullptr, b = nullptr;
  double bytes = 0.0;
  int iter = -1;
};

// Per-problem host data of a group.
struct ProbInfo {
  double theta = 0, phi = 0, kx0 = 0, ky0 = 0, kz0 = 0;
  int pol = 0;
};

struct psfd_plan {
  psfd_desc d{};  // problem 0's descriptor (shared fields for the whole group)
  std::vector<double> ml_eps_h, ml_d_h;
  int G = 1;
  std::vector<ProbInfo> prob;
  int nx = 0, ny = 0, nz = 0, nabs = 0, j0 = 0, jev = 0;
  double k0 = 0, kbg = 0;
  int64_t plane = 0, nfield = 0, nspec = 0;  // per problem
  hipStream_t st = nullptr;
  int prec = PSFD_C128;
  bool use_pc = true;
  std::vector<std::pair<void*, size_t>> allocs;  // device blocks and their sizes
  int alloc_dev = 0;

  OpTables<double> t64{};
  OpTables<float> t32{};
  cplx<double>* kd64 = nullptr;
  cplx<float>* kd32 = nullptr;
  cplx<double>* rte64 = nullptr;
  cplx<double>* rpe64 = nullptr;
  double* zabs64 = nullptr;

  cplx<double>* S64 = nullptr;
  cplx<double>* UW64 = nullptr;
  cplx<float>* S32 = nullptr;
  cplx<float>* UW32 = nullptr;

  cplx<double>* v64[V_COUNT] = {};
  cplx<float>* v32[V_COUNT] = {};
  cplx<double>* b64 = nullptr;
  cplx<double>* tmp64 = nullptr;
  cplx<double>* res64 = nullptr;
  cplx<double>* ebak64 = nullptr;  // the solution before a fold E += s M y (restored if it fails)
  double hf_w0 = 1.0, hf_eta = 0.0;  // weight of the physics loss's high-frequency penalty
  cplx<double>* E64 = nullptr;  // stacked solution of a batch group
  KState* ks = nullptr;
  KState* ks_host = nullptr;
  ProbParams* pp = nullptr;
  ProbParams* pp_host = nullptr;
  int* idle = nullptr;  // [G] 1: problem finished (skipped by operator kernels)
  int* idle_host = nullptr;
  double* part = nullptr;
  double* part2 = nullptr;  // ||s||^2 partials of the forward x pass (read with omega's)

  // batch handle (psfd_plan_batch): the recorded problems
  bool is_batch = false;
  std::vector<psfd_desc> bdesc;
  std::vector<std::vector<double>> b_ml_eps, b_ml_d;
  std::vector<const void*> beps;

  // solves run on a private non-blocking stream (capturable), joined to the caller's
  hipStream_t own_st = nullptr;
  hipEvent_t join_ev = nullptr;
  hipGraphExec_t gexec[2][2] = {};  // captured iteration chunk [complex64?][adjoint?]
  bool use_graphs = true;
  int cur_iter = -1;  // iteration (within the chunk being launched) of the next launches

  // kernel timing (psfd_profile_enable)
  int prof_kernel = 0;
  int prof_elem = 16;  // element size of the timed launches (the working precision)
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfPair> ev_open;
  double prof_ms = 0.0, prof_bytes = 0.0;
  int64_t prof_launches = 0;

  ~psfd_plan() {
    // nothing may still run on the blocks that go back to the cache
    if (!allocs.empty()) {
      if (st) (void)hipStreamSynchronize(st);
      else (void)hipDeviceSynchronize();
      if (own_st) (void)hipStreamSynchronize(own_st);
    }
    for (auto& row : gexec)
      for (auto& g : row)
        if (g) (void)hipGraphExecDestroy(g);
    if (own_st) (void)hipStreamDestroy(own_st);
    if (join_ev) (void)hipEventDestroy(join_ev);
    for (auto& pr : ev_open) { ev_pool.push_back(pr.a); ev_pool.push_back(pr.b); }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (auto& a : allocs)
      if (!cache_put(alloc_dev, a.second, a.first)) (void)hipFree(a.first);
    if (ks_host) (void)hipHostFree(ks_host);
    if (pp_host) (void)hipHostFree(pp_host);
    if (idle_host) (void)hipHostFree(idle_host);
  }
};

namespace {

template <typename T>
psfd_status dalloc(struct psfd_plan* P, T** out, size_t count) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  int dev = 0;
  CHK(hipGetDevice(&dev));
  void* q = cache_take(dev, bytes);
  if (!q) {
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {  // the cache may hold the memory: give it back and try again
      (void)hipGetLastError();
      cache_trim();
      e = hipMalloc(&q, bytes);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(PSFD_ERR_ALLOC, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                      hipGetErrorString(e));
    }
  }
  P->alloc_dev = dev;
  P->allocs.push_back({q, bytes});
  *out = static_cast<T*>(q);
  return PSFD_OK;
}

template <typename T>
psfd_status upload(struct psfd_plan* P, T** out, const std::vector<T>& h) {
  CHKS(dalloc(P, out, h.size()));
  CHK(hipMemcpyAsync(*out, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, P->st));
  return PSFD_OK;
}

template <typename T>
std::vector<T> to_t(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}
template <typename T>
std::vector<cplx<T>> to_tc(const std::vector<cplx<double>>& v) {
  std::vector<cplx<T>> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = {(T)v[i].re, (T)v[i].im};
  return o;
}

psfd_status validate(const psfd_desc* d) {
  if (!d) return fail(PSFD_ERR_ARG, "desc is NULL");
  if (!lateral_size_ok(d->nx) || !lateral_size_ok(d->ny))
    return fail(PSFD_ERR_ARG, "nx, ny must be one of 16, 32, 64, 128, 192, 256, 512, 1024");
  if (d->nz_abs < 1 || d->nz_gap_bot < 1 || d->nz_gap_top < 0 || d->nz_pml < 0)
    return fail(PSFD_ERR_ARG, "need nz_abs >= 1, nz_gap_bot >= 1, nz_gap_top >= 0, nz_pml >= 0");
  const int nz = d->nz_abs + d->nz_gap_bot + d->nz_gap_top + 2 * d->nz_pml;
  if (!axial_size_ok(nz)) return fail(PSFD_ERR_ARG, "Nz must be one of 24, 32, 48, 64, 96, 128, 192, 256, 324, 384, 576, 648, 768");
  if (!(d->dx > 0) || !(d->dy > 0) || !(d->dz > 0) || !(d->lambda > 0))
    return fail(PSFD_ERR_ARG, "dx, dy, dz, lambda must be positive");
  if (!(d->eps_bg > 0)) return fail(PSFD_ERR_ARG, "eps_bg must be positive");
  if (d->pol != 0 && d->pol != 1) return fail(PSFD_ERR_ARG, "pol must be 0 (TE) or 1 (TM)");
  if (d->n_ml < 0 || (d->n_ml > 0 && (!d->ml_eps || !d->ml_thick)))
    return fail(PSFD_ERR_ARG, "multilayer tables missing");
  if (d->prec < PSFD_C128 || d->prec > PSFD_C64_BF16PC_REFINE64)
    return fail(PSFD_ERR_ARG, "unknown precision");
  if (d->pml_order < 0 || !(d->pml_sigma0 >= 0)) return fail(PSFD_ERR_ARG, "bad PML parameters");
  if (!(d->pc_mmin >= 0 && d->pc_mmin <= 1) || !(d->pc_gamma > 0) || !(d->pc_reg >= 0))
    return fail(PSFD_ERR_ARG, "bad preconditioner parameters");
  if (!std::isfinite(d->theta) || !std::isfinite(d->phi)) return fail(PSFD_ERR_ARG, "bad angles");
  if (!(d->ml_kz_min >= 0.0 && d->ml_kz_min <= 1.0)) return fail(PSFD_ERR_ARG, "bad ml_kz_min");
  return PSFD_OK;
}

// Problems that may share a plan: everything but angle, polarisation and
// permittivity must agree.
bool same_group(const psfd_desc& a, const psfd_desc& b) {
  if (a.nx != b.nx || a.ny != b.ny || a.nz_abs != b.nz_abs || a.nz_gap_bot != b.nz_gap_bot ||
      a.nz_gap_top != b.nz_gap_top || a.nz_pml != b.nz_pml)
    return false;
  if (a.dx != b.dx || a.dy != b.dy || a.dz != b.dz || a.lambda != b.lambda || a.eps_bg != b.eps_bg)
    return false;
  if (a.n_ml != b.n_ml || a.eps_sub[0] != b.eps_sub[0] || a.eps_sub[1] != b.eps_sub[1]) return false;
  for (int i = 0; i < a.n_ml; ++i)
    if (a.ml_eps[2 * i] != b.ml_eps[2 * i] || a.ml_eps[2 * i + 1] != b.ml_eps[2 * i + 1] ||
        a.ml_thick[i] != b.ml_thick[i])
      return false;
  if (a.pml_sigma0 != b.pml_sigma0 || a.pml_order != b.pml_order || a.precond != b.precond)
    return false;
  if (a.pc_mmin != b.pc_mmin || a.pc_kref != b.pc_kref || a.pc_gamma != b.pc_gamma ||
      a.pc_reg != b.pc_reg || a.prec != b.prec || a.ml_kz_min != b.ml_kz_min)
    return false;
  return true;
}

template <typename T>
OpTables<T>& tab(struct psfd_plan* P);
template <>
OpTables<double>& tab<double>(struct psfd_plan* P) { return P->t64; }
template <>
OpTables<float>& tab<float>(struct psfd_plan* P) { return P->t32; }

template <typename T>
cplx<T>* wsS(struct psfd_plan* P);
template <>
cplx<double>* wsS<double>(struct psfd_plan* P) { return P->S64; }
template <>
cplx<float>* wsS<float>(struct psfd_plan* P) { return P->S32; }
template <typename T>
cplx<T>* wsUW(struct psfd_plan* P);
template <>
cplx<double>* wsUW<double>(struct psfd_plan* P) { return P->UW64; }
template <>
cplx<float>* wsUW<float>(struct psfd_plan* P) { return P->UW32; }
template <typename T>
cplx<T>** vecs(struct psfd_plan* P);
template <>
cplx<double>** vecs<double>(struct psfd_plan* P) { return P->v64; }
template <>
cplx<float>** vecs<float>(struct psfd_plan* P) { return P->v32; }

enum { PROF_OFF = 0, PROF_AXIAL = 1, PROF_YFFT = 2, PROF_XFWD = 3, PROF_XINV = 4 };

hipEvent_t take_event(struct psfd_plan* P) {
  if (!P->ev_pool.empty()) {
    hipEvent_t e = P->ev_pool.back();
    P->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// When kernel `which` is being timed (psfd_profile_enable), give the tables a
// pair of events for the next launch: the launch packet records them at the
// kernel's start and end, so the pair brackets the kernel alone.  (Event-
// record nodes captured into a graph do not update the events' timestamps on
// replay with this HIP runtime, so timing runs the chunks without graphs.)
template <typename T>
hipError_t arm_events(struct psfd_plan* P, OpTables<T>& t, int which, double bytes) {
  t.prof_start = t.prof_stop = nullptr;
  if (P->prof_kernel != which || P->prof_elem != (int)sizeof(cplx<T>)) return hipSuccess;
  hipEvent_t a = take_event(P), b = take_event(P);
  if (!a || !b) return hipErrorOutOfMemory;
  t.prof_start = a;
  t.prof_stop = b;
  P->ev_open.push_back(ProfPair{a, b, bytes, P->cur_iter});
  return hipSuccess;
}

// Fold completed timed launches into the totals (after a stream sync).  A
// chunk launches its iterations whether or not the problem is still running
// (the kernels of a finished problem return at once): only launches of the
// first `executed` iterations of the chunk count.
void fold_pair(struct psfd_plan* P, const ProfPair& pr, int executed) {
  if (pr.iter >= executed) return;
  float ms = 0.f;
  const hipError_t e = hipEventElapsedTime(&ms, pr.a, pr.b);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // the failed query must not surface at the next launch
    return;
  }
  P->prof_ms += ms;
  P->prof_bytes += pr.bytes;
  P->prof_launches += 1;
}

void collect_events(struct psfd_plan* P, int executed = 1 << 30) {
  for (auto& pr : P->ev_open) {
    fold_pair(P, pr, executed);
    P->ev_pool.push_back(pr.a);
    P->ev_pool.push_back(pr.b);
  }
  P->ev_open.clear();
}

// Destroy the captured chunks (they hold the old schedules).
void drop_graphs(struct psfd_plan* P) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      if (P->gexec[i][j]) (void)hipGraphExecDestroy(P->gexec[i][j]);
      P->gexec[i][j] = nullptr;
    }
}

// Fusion hooks of one operator application: a vector update folded into the
// first x pass and inner products folded into the last x pass.
template <typename T>
struct Fuse {
  PreOp<T> pre;
  PostOp<T> post;
  int* nblk_post = nullptr;  // receives the number of partials per problem written by post
  int* nblk_pre = nullptr;   // receives the number of partials per problem written by pre
};

constexpr int kKsStride = (int)(sizeof(KState) / sizeof(int));
static_assert(sizeof(KState) % sizeof(int) == 0, "KState must hold whole ints");

// One operator application over the group (see the kernel files for the
// math).  skip/skip_stride: per-problem flags that make the kernels return.
// The algorithmic bytes of each launch count every complex element it must
// read or write once.
template <typename T>
hipError_t op_apply(struct psfd_plan* P, const cplx<T>* x, cplx<T>* y, int op, const int* skip,
                    int skip_stride, const Fuse<T>& fz = Fuse<T>()) {
  OpTables<T> t = tab<T>(P);
  t.skip = skip;
  t.skip_stride = skip_stride;
  if (op == OP_HF) {
    t.hf_mode = 1;
    t.hf_w0 = (T)P->hf_w0;
    t.hf_eta = (T)P->hf_eta;
  }
  cplx<T>* S = wsS<T>(P);
  cplx<T>* UW = wsUW<T>(P);
  hipStream_t st = P->st;
  const int p3 = 3 * P->nz, pa = 3 * P->nabs;
  const double pl = (double)P->plane * P->G * sizeof(cplx<T>);  // bytes of one plane, whole group
  hipError_t e;
  const bool adj = op == OP_AH;
  const int nin = adj ? p3 + pa : p3;  // planes through the forward lateral transform
  const int ax_mode = op == OP_A ? AX_A : (op == OP_AM ? AX_AM : (adj ? AX_AH : AX_M));
  const int nout = (op == OP_A || op == OP_AM) ? p3 + pa : p3;  // planes out of the axial kernel
  const int cmode = (op == OP_A || op == OP_AM) ? CB_FWD : (adj ? CB_ADJ : CB_PLAIN);
  const int npre = fz.pre.mode == PRE_P ? 3 + 1 : (fz.pre.mode == PRE_S ? 2 + 1 : 1);
  int nb_first = 0;
  // x pass (forward): read the field (+ conj(kd) and absorber rows for the adjoint), write nin planes
  e = arm_events(P, t, PROF_XFWD, pl * (p3 * npre + nin + (adj ? pa + P->nabs : 0)));
  if (e == hipSuccess) e = launch_xfft_fwd<T>(t, x, S, adj, fz.pre, &nb_first, st);
  if (e != hipSuccess) return e;
  if (fz.nblk_pre) *fz.nblk_pre = nb_first;
  t.prof_start = t.prof_stop = nullptr;
  e = arm_events(P, t, PROF_YFFT, 2.0 * pl * nin);
  if (e == hipSuccess) e = launch_yfft<T>(t, S, nin, false, st);
  if (e != hipSuccess) return e;
  e = arm_events(P, t, PROF_AXIAL, pl * (nin + nout));
  if (e == hipSuccess) e = launch_axial<T>(t, S, UW, ax_mode, st);
  if (e != hipSuccess) return e;
  e = arm_events(P, t, PROF_YFFT, 2.0 * pl * nout);
  if (e == hipSuccess) e = launch_yfft<T>(t, UW, nout, true, st);
  if (e != hipSuccess) return e;
  double comb = cmode == CB_FWD ? pl * (nout + P->nabs + p3)
                                : (cmode == CB_ADJ ? pl * (p3 + pa + P->nabs + p3) : 2.0 * pl * p3);
  if (fz.post.mode == POST_DOT) comb += pl * p3;
  e = arm_events(P, t, PROF_XINV, comb);
  if (e != hipSuccess) return e;
  return launch_xfft_inv<T>(t, UW, y, cmode, adj ? x : nullptr, fz.post, fz.nblk_post, st);
}

psfd_status ensure_fp32(struct psfd_plan* P) {
  if (P->S32) return PSFD_OK;
  CHKS(dalloc(P, &P->S32, (size_t)(P->nspec * P->G)));
  CHKS(dalloc(P, &P->UW32, (size_t)(P->nspec * P->G)));
  return PSFD_OK;
}

template <typename T>
psfd_status ensure_krylov(struct psfd_plan* P) {
  cplx<T>** v = vecs<T>(P);
  if (v[0]) return PSFD_OK;
  for (int i = 0; i < V_COUNT; ++i) CHKS(dalloc(P, &v[i], (size_t)(P->nfield * P->G)));
  return PSFD_OK;
}

psfd_status ensure_solver_common(struct psfd_plan* P) {
  if (P->ks) return PSFD_OK;
  const int G = P->G;
  CHKS(dalloc(P, &P->ks, (size_t)G));
  CHKS(dalloc(P, &P->pp, (size_t)G));
  CHKS(dalloc(P, &P->idle, (size_t)G));
  // per problem: one partial set per block of the largest reducing grid
  // (x pass rows, or the streaming kernels' blocks)
  const int64_t per = (int64_t)(3 * P->nz + 3 * P->nabs) * P->ny + 8192;
  CHKS(dalloc(P, &P->part, (size_t)(per * KPART * G)));
  CHKS(dalloc(P, &P->part2, (size_t)(per * KPART * G)));
  CHKS(dalloc(P, &P->b64, (size_t)(P->nfield * G)));
  CHKS(dalloc(P, &P->tmp64, (size_t)(P->nfield * G)));
  CHKS(dalloc(P, &P->res64, (size_t)(P->nfield * G)));
  CHKS(dalloc(P, &P->ebak64, (size_t)(P->nfield * G)));
  CHK(hipMemsetAsync(P->ks, 0, sizeof(KState) * G, P->st));
  CHK(hipMemsetAsync(P->idle, 0, sizeof(int) * G, P->st));
  CHK(hipHostMalloc((void**)&P->ks_host, sizeof(KState) * G, hipHostMallocDefault));
  CHK(hipHostMalloc((void**)&P->pp_host, sizeof(ProbParams) * G, hipHostMallocDefault));
  CHK(hipHostMalloc((void**)&P->idle_host, sizeof(int) * G, hipHostMallocDefault));
  std::memset(P->pp_host, 0, sizeof(ProbParams) * G);
  std::memset(P->idle_host, 0, sizeof(int) * G);
  return PSFD_OK;
}

psfd_status read_state(struct psfd_plan* P) {
  CHK(hipMemcpyAsync(P->ks_host, P->ks, sizeof(KState) * P->G, hipMemcpyDeviceToHost, P->st));
  CHK(hipStreamSynchronize(P->st));
  return PSFD_OK;
}

// pp_host and idle_host are pinned: an asynchronous copy reads them when it
// runs, not when it is queued, so the copy is waited for before the host may
// change them again (without the wait, a group's reliable update could send
// the parameters written after it, and every member's residual was rescaled).
psfd_status push_params(struct psfd_plan* P) {
  CHK(hipMemcpyAsync(P->pp, P->pp_host, sizeof(ProbParams) * P->G, hipMemcpyHostToDevice, P->st));
  CHK(hipMemcpyAsync(P->idle, P->idle_host, sizeof(int) * P->G, hipMemcpyHostToDevice, P->st));
  CHK(hipStreamSynchronize(P->st));
  return PSFD_OK;
}

// ||a_b||^2 per problem into ks_host[b].red[0]
psfd_status norm2_group(struct psfd_plan* P, const cplx<double>* a) {
  CHK(launch_k_norm2<double>(a, P->nfield, P->G, P->part, P->st));
  CHK(launch_finalize(FIN_RED0, P->ks, P->part, red_blocks(P->nfield, P->G), P->G, P->pp, P->st));
  return read_state(P);
}

// Right-preconditioned BiCGSTAB on op(prec(y)) = r (r in vecs[V_R]); y in
// vecs[V_Y]; per-problem ||b||^2, tolerance and budget from P->pp (pushed by
// the caller).  One iteration, with the vector updates and inner products
// fused into the operator's x passes:
//   [p = r + beta(p - omega v) -> x-FFT] ... [x-IFFT -> v, <rh, v>]  fin: alpha
//   [s = r - alpha v, ||s|| -> x-FFT]  fin: half-step test
//   ... [x-IFFT -> t, <t, s>, ||t||]  fin: omega
//   [y += alpha p + omega s, r = s - omega t, ||r||, <rh, r>]  fin: rho, beta, stop test
// Returns when every problem of the group has stopped (converged, budget
// used, breakdown or idle) or after `maxit` launched iterations.  Problems
// that request a reliable update (KS_UPDATE) are served by `on_update`
// between chunks while the others keep iterating.
// shadow (optional, complex128 [G] fields): the shadow residual of this run
// in place of r (the recurrence then starts with rho = <shadow, r>).
template <typename T, typename U>
psfd_status run_bicgstab(struct psfd_plan* P, bool adjoint, int maxit, U&& on_update,
                         const cplx<double>* shadow = nullptr) {
  cplx<T>** V = vecs<T>(P);
  const int64_t n = P->nfield;
  const int G = P->G;
  hipStream_t st = P->st;
  KState* ks = P->ks;
  double* part = P->part;
  const int* skip = &ks->done;
  const bool pc = P->use_pc;
  CHK(launch_k_init<T>(V[V_RH], V[V_R], V[V_P], V[V_V], V[V_Y], n, G, part, st));
  CHK(launch_finalize(FIN_INIT, ks, part, red_blocks(n, G), G, P->pp, st));
  if (shadow) {
    CHK(launch_k_scale_copy<T, double>(V[V_RH], shadow, nullptr, n, G, st));
    CHK(launch_k_norm2<T>(V[V_RH], n, G, part, st));
    CHK(launch_finalize(FIN_RED0, ks, part, red_blocks(n, G), G, P->pp, st));
    CHK(launch_k_dot_rr<T>(V[V_RH], V[V_R], n, G, part, st));
    CHK(launch_finalize(FIN_SHADOW, ks, part, red_blocks(n, G), G, P->pp, st));
  }

  // The first operator of a composite (M then A^H) carries the update; the last carries the dot.
  auto apply = [&](const cplx<T>* in, cplx<T>* out, Fuse<T>& fz) -> hipError_t {
    if (!adjoint) return op_apply<T>(P, in, out, pc ? OP_AM : OP_A, skip, kKsStride, fz);
    if (!pc) return op_apply<T>(P, in, out, OP_AH, skip, kKsStride, fz);
    Fuse<T> f1, f2;
    f1.pre = fz.pre;
    f1.nblk_pre = fz.nblk_pre;
    f2.post = fz.post;
    f2.nblk_post = fz.nblk_post;
    hipError_t e = op_apply<T>(P, in, V[V_W], OP_M, skip, kKsStride, f1);
    if (e != hipSuccess) return e;
    return op_apply<T>(P, V[V_W], out, OP_AH, skip, kKsStride, f2);
  };
  // the unpreconditioned adjoint transforms extra rows of the input: update p separately
  const bool fuse_p = !(adjoint && !pc);
  int nb_v = 0, nb_t = 0, nb_s = 0;
  auto launch_iters = [&](int count) -> psfd_status {
    for (int i = 0; i < count; ++i) {
      P->cur_iter = i;
      Fuse<T> fa;
      if (fuse_p) {
        fa.pre.mode = PRE_P;
        fa.pre.r = V[V_R];
        fa.pre.pv = V[V_P];
        fa.pre.v = V[V_V];
        fa.pre.ks = ks;
      } else {
        CHK(launch_k_p_update<T>(V[V_P], V[V_R], V[V_V], n, G, ks, st));
      }
      fa.post.mode = POST_DOT;
      fa.post.d = V[V_RH];
      fa.post.part = part;
      fa.nblk_post = &nb_v;
      CHK(apply(V[V_P], V[V_V], fa));
      CHK(launch_finalize(FIN_ALPHA, ks, part, nb_v, G, P->pp, st));

      Fuse<T> fb;
      fb.pre.mode = PRE_S;
      fb.pre.r = V[V_R];
      fb.pre.pv = V[V_S];
      fb.pre.v = V[V_V];
      fb.pre.ks = ks;
      fb.pre.part = P->part2;
      fb.nblk_pre = &nb_s;
      fb.post.mode = POST_DOT;
      fb.post.d = V[V_S];
      fb.post.part = part;
      fb.nblk_post = &nb_t;
      CHK(apply(V[V_S], V[V_T], fb));
      // omega, with the half-step test on ||s|| from the forward pass's partials
      CHK(launch_finalize(FIN_OMEGA, ks, part, nb_t, G, P->pp, st, P->part2, nb_s));

      CHK(launch_k_xr_update<T>(V[V_Y], V[V_R], V[V_P], V[V_S], V[V_T], V[V_RH], n, G, ks, part,
                                st));
      CHK(launch_finalize(FIN_RHO, ks, part, red_blocks(n, G), G, P->pp, st));
    }
    P->cur_iter = -1;
    return PSFD_OK;
  };
  // A full chunk is captured once per plan into a HIP graph and replayed:
  // every launch argument is fixed per plan, per-problem budgets and
  // convergence are tested on the device, so the same graph serves every
  // chunk of every solve.
  hipGraphExec_t& gx = P->gexec[sizeof(T) == 4 ? 1 : 0][adjoint ? 1 : 0];
  const bool graphs = P->use_graphs && P->prof_kernel == PROF_OFF;
  int launched = 0;
  int iter_seen = 0;  // iterations of this run (FIN_INIT set the counter to 0)
  while (launched < maxit) {
    if (graphs) {
      if (!gx) {
        hipGraph_t g = nullptr;
        CHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        psfd_status cs = launch_iters(kChunk);
        hipError_t ce = hipStreamEndCapture(st, &g);
        if (cs != PSFD_OK) {
          if (g) (void)hipGraphDestroy(g);
          return cs;
        }
        CHK(ce);
        hipError_t ie = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        CHK(ie);
      }
      CHK(hipGraphLaunch(gx, st));
      launched += kChunk;
    } else {
      const int chunk = std::min(kChunk, maxit - launched);
      CHKS(launch_iters(chunk));
      launched += chunk;
    }
    CHKS(read_state(P));
    {
      // PSFD_TRACE=2: the recursive residual of each problem every 512 iterations
      static const bool trace2 = [] {
        const char* e = std::getenv("PSFD_TRACE");
        return e && std::atoi(e) >= 2;
      }();
      if (trace2)
        for (int b = 0; b < G; ++b) {
          const KState& k = P->ks_host[b];
          if (k.iter / 512 != (k.iter - kChunk) / 512 && k.iter >= 512 && k.bnorm2 > 0)
            fprintf(stderr, "psfd trace: p%d %s iteration %d of this run: recursive r/r_run0 %.3e\n", b,
                    sizeof(T) == 4 ? "c64" : "fp64", k.iter, std::sqrt(k.rnorm2 / k.bnorm2));
        }
    }
    if (P->prof_kernel != PROF_OFF) {
      // timed launches: single-problem plans count the chunk's executed iterations
      collect_events(P, G == 1 ? P->ks_host[0].iter - iter_seen : (1 << 30));
    }
    if (G == 1) iter_seen = P->ks_host[0].iter;
    bool upd = false;
    for (int b = 0; b < G; ++b) upd = upd || P->ks_host[b].done == KS_UPDATE;
    if (upd) CHKS(on_update());
    bool all = true;
    for (int b = 0; b < G && all; ++b) all = P->ks_host[b].done != 0 && P->ks_host[b].done != KS_UPDATE;
    if (all) break;
  }
  return PSFD_OK;
}

psfd_status no_update() { return PSFD_OK; }

// r = b - op(E) in FP64 (op = A or A^H, no preconditioner) for every problem
// not marked idle; ||r_b||^2 lands in ks_host[b].red[0].  An idle problem's r
// is left as it was and its red[0] means nothing.
psfd_status true_residual(struct psfd_plan* P, const cplx<double>* b, const cplx<double>* E,
                          cplx<double>* r, bool adjoint) {
  CHK(op_apply<double>(P, E, P->tmp64, adjoint ? OP_AH : OP_A, P->idle, 1));
  CHK(launch_k_residual<double>(r, b, P->tmp64, P->nfield, P->G, P->idle, P->part, P->st));
  CHK(launch_finalize(FIN_RED0, P->ks, P->part, red_blocks(P->nfield, P->G), P->G, P->pp, P->st));
  return read_state(P);
}

double inner_tolerance(double tol, double rrel) {
  static const double floor_tol = [] {
    const char* s = std::getenv("PSFD_INNER_TOL");
    return s ? std::atof(s) : 3e-5;
  }();
  double t = 0.3 * tol / rrel;
  if (t < floor_tol) t = floor_tol;
  if (t > 0.1) t = 0.1;
  return t;
}

RhsArgs rhs_args(const struct psfd_plan* P, int b) {
  const ProbInfo& q = P->prob[b];
  return RhsArgs{P->nx, P->ny, P->nz, P->nabs, P->j0, q.pol, P->k0, q.kz0, q.theta, q.phi,
                 P->zabs64, P->rte64 + (int64_t)b * P->plane, P->rpe64 + (int64_t)b * P->plane,
                 P->kd64 + (int64_t)b * P->nabs * P->plane};
}

psfd_status rhs_group(struct psfd_plan* P, cplx<double>* b) {
  for (int i = 0; i < P->G; ++i) CHK(launch_rhs<double>(rhs_args(P, i), b + i * P->nfield, P->st));
  return PSFD_OK;
}


// ---------------------------------------------------------------- autotuner
// Kernel schedules (radix schedule and rows per block of the x passes, radix
// schedule and tile width of the y pass, axial kernel variant) are chosen per
// (precision, nx, ny, Nz, N_abs, group size rounded up to a power of two) by
// timing the working-precision operator of the solve on the plan itself,
// one knob at a time; the result is kept for the life of the process.  A
// table of earlier choices (tune_table.txt next to the library, or the file
// PSFD_TUNE_FILE names; written by psfd_tune_save) is read once per process:
// shapes it lists take its schedules without timing.
struct TuneKey {
  int elem, nx, ny, nz, nabs, gb;
  bool operator<(const TuneKey& o) const {
    return std::tie(elem, nx, ny, nz, nabs, gb) < std::tie(o.elem, o.nx, o.ny, o.nz, o.nabs, o.gb);
  }
};
struct TuneVal {
  int v[4] = {0, 0, 0, 0};  // sched_xf, sched_xi, sched_y, sched_ax
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
std::once_flag g_tune_load_once;

std::string tune_file_path() {
  if (const char* e = std::getenv("PSFD_TUNE_FILE")) return e;  // "" disables the table
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&tune_file_path), &info) && info.dli_fname) {
    std::string so(info.dli_fname);
    const size_t slash = so.rfind('/');
    return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tune_table.txt";
  }
  return "";
}

// Lines "elem nx ny nz nabs group : xf xi y ax" ('#' starts a comment; elem is
// 4 for complex64 plans, 8 for complex128); entries out of range are ignored.
void load_tune_table() {
  std::call_once(g_tune_load_once, [] {
    const std::string path = tune_file_path();
    if (path.empty()) return;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[256];
    std::lock_guard<std::mutex> lk(g_tune_mu);
    while (std::fgets(line, sizeof line, f)) {
      if (line[0] == '#') continue;
      TuneKey k{};
      TuneVal v;
      if (std::sscanf(line, "%d %d %d %d %d %d : %d %d %d %d", &k.elem, &k.nx, &k.ny, &k.nz, &k.nabs,
                      &k.gb, &v.v[0], &v.v[1], &v.v[2], &v.v[3]) != 10)
        continue;
      bool ok = k.elem == 4 || k.elem == 8;  // bytes of the real type
      for (int i = 0; i < 4; ++i) ok = ok && v.v[i] >= 0 && v.v[i] <= 3;
      if (ok) g_tune[k] = v;
    }
    std::fclose(f);
  });
}

template <typename T>
void set_sched(OpTables<T>& t, const TuneVal& v) {
  t.sched_xf = v.v[0];
  t.sched_xi = v.v[1];
  t.sched_y = v.v[2];
  t.sched_ax = v.v[3];
}

// Schedules from the table (or from an earlier tuning in this process); with
// `timing`, a shape not yet known is tuned now, else it keeps the defaults.
template <typename T>
psfd_status autotune(struct psfd_plan* P, bool timing) {
  load_tune_table();
  int gb = 1;
  while (gb < P->G) gb *= 2;
  const TuneKey key{(int)sizeof(T), P->nx, P->ny, P->nz, P->nabs, gb};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      set_sched(tab<T>(P), it->second);
      return PSFD_OK;
    }
  }
  if (!timing) return PSFD_OK;
  CHKS(ensure_solver_common(P));
  if (sizeof(T) == 4) CHKS(ensure_fp32(P));
  CHKS(ensure_krylov<T>(P));
  hipStream_t st = P->st;
  // The iteration's own kernel variants are timed: p update fused into the
  // forward x pass, inner products fused into the inverse x pass (on the
  // Krylov work vectors; their contents do not matter for the timing).
  cplx<T>** V = vecs<T>(P);
  Fuse<T> fz;
  fz.pre.mode = PRE_P;
  fz.pre.r = V[V_R];
  fz.pre.pv = V[V_P];
  fz.pre.v = V[V_V];
  fz.pre.ks = P->ks;
  fz.post.mode = POST_DOT;
  fz.post.d = V[V_RH];
  fz.post.part = P->part;
  cplx<T>* x = V[V_P];
  cplx<T>* y = V[V_T];
  const int op = P->use_pc ? OP_AM : OP_A;
  // Each knob is judged by the duration of the kernel it controls, taken
  // from the launch packets' own timestamps (the profiling events).
  const int saved_kernel = P->prof_kernel, saved_elem = P->prof_elem;
  auto measure = [&](const TuneVal& v, int which, float* us) -> psfd_status {
    set_sched(tab<T>(P), v);
    P->prof_kernel = PROF_OFF;
    CHK(op_apply<T>(P, x, y, op, nullptr, 0, fz));  // first launch of new code objects
    float best = 1e30f;
    for (int rep = 0; rep < 5; ++rep) {
      P->prof_kernel = which;
      P->prof_elem = (int)sizeof(cplx<T>);
      P->prof_ms = 0.0;
      P->prof_launches = 0;
      P->prof_bytes = 0.0;
      for (int i = 0; i < 3; ++i) CHK(op_apply<T>(P, x, y, op, nullptr, 0, fz));
      CHK(hipStreamSynchronize(st));
      collect_events(P);
      if (P->prof_launches > 0) best = std::min(best, (float)(1e3 * P->prof_ms / P->prof_launches));
    }
    P->prof_kernel = PROF_OFF;
    *us = best;
    return PSFD_OK;
  };
  TuneVal cur;
  const int order[4] = {3, 0, 1, 2};
  const int nval[4] = {4, 4, 4, 4};
  const int kern[4] = {PROF_XFWD, PROF_XINV, PROF_YFFT, PROF_AXIAL};
  for (int k : order) {
    float cur_us = 0.f;
    CHKS(measure(cur, kern[k], &cur_us));
    for (int val = 0; val < nval[k]; ++val) {
      if (val == cur.v[k]) continue;
      TuneVal cand = cur;
      cand.v[k] = val;
      float us = 0.f;
      CHKS(measure(cand, kern[k], &us));
      if (us < 0.97f * cur_us) {  // keep the default unless clearly faster
        cur = cand;
        cur_us = us;
      }
    }
  }
  P->prof_kernel = saved_kernel;
  P->prof_elem = saved_elem;
  P->prof_ms = 0.0;
  P->prof_launches = 0;
  P->prof_bytes = 0.0;
  set_sched(tab<T>(P), cur);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = cur;
  return PSFD_OK;
}

bool tune_forced_off() {
  const char* s = std::getenv("PSFD_TUNE");
  return s && *s && std::atoi(s) == 0;
}

// Schedules of a new plan; PSFD_TUNE=0 keeps the defaults (no table, no timing).
psfd_status tune_plan(struct psfd_plan* P, bool timing) {
  if (tune_forced_off()) return PSFD_OK;
  if (P->prec == PSFD_C128) return autotune<double>(P, timing);
  return autotune<float>(P, timing);
}

// PSFD_TUNE=1 / 0 forces tuning on / off; otherwise `dflt`.
bool tune_wanted(bool dflt) {
  const char* s = std::getenv("PSFD_TUNE");
  if (!s || !*s) return dflt;
  return std::atoi(s) != 0;
}

psfd_status solve_body(struct psfd_plan* P, const cplx<double>* b_in, const cplx<double>* x0,
                       cplx<double>* E, double tol, int maxit, bool adjoint, psfd_info* infos,
                       const cplx<double>* shadow);

// The solve runs on the plan's private stream, after the work already queued on
// the caller's stream; it returns with that private stream drained.  b_in, x0,
// E: stacked [G] fields; infos: [G].
psfd_status solve_impl(struct psfd_plan* P, const void* b_in, const void* x0, void* E_out,
                       double tol, int maxit, bool adjoint, psfd_info* infos,
                       const void* shadow = nullptr) {
  CHK(hipEventRecord(P->join_ev, P->st));
  CHK(hipStreamWaitEvent(P->own_st, P->join_ev, 0));
  hipStream_t user = P->st;
  P->st = P->own_st;
  psfd_status s = solve_body(P, static_cast<const cplx<double>*>(b_in),
                             static_cast<const cplx<double>*>(x0), static_cast<cplx<double>*>(E_out),
                             tol, maxit, adjoint, infos, static_cast<const cplx<double>*>(shadow));
  hipError_t e = hipStreamSynchronize(P->own_st);
  P->st = user;
  if (s == PSFD_OK && e != hipSuccess) return fail(PSFD_ERR_HIP, hipGetErrorString(e));
  return s;
}

// Every problem of the group is solved to FP64 true r_rel <= tol:
//   FP64 plans: BiCGSTAB with residual replacement (restart from the current
//   field) when the recursive residual drifts from the true one;
//   mixed plans: iterative refinement, each step a complex64 BiCGSTAB on the
//   normalised FP64 residual to a relative tolerance of about 0.3 tol / r_rel.
// A problem that has finished is idle in the group's later runs.
// shadow: optional shadow residual of the first Krylov run (later runs take
// their starting residual).
psfd_status solve_body(struct psfd_plan* P, const cplx<double>* b_in, const cplx<double>* x0,
                       cplx<double>* E, double tol, int maxit, bool adjoint, psfd_info* infos,
                       const cplx<double>* shadow) {
  bool mixed = P->prec != PSFD_C128;
  const int G = P->G;
  CHKS(ensure_solver_common(P));
  if (mixed) {
    CHKS(ensure_fp32(P));
    CHKS(ensure_krylov<float>(P));
  } else {
    CHKS(ensure_krylov<double>(P));
  }
  const int64_t n = P->nfield;
  hipStream_t st = P->st;
  const cplx<double>* b = b_in;
  if (!b) {
    if (adjoint) return fail(PSFD_ERR_ARG, "the adjoint solve needs an explicit right-hand side");
    CHKS(rhs_group(P, P->b64));
    b = P->b64;
  }
  CHKS(norm2_group(P, b));
  std::vector<double> bn2(G), rrel(G, 0.0), rn(G, 0.0);
  std::vector<int> fin(G, 0), outer(G, 0), total(G, 0);
  std::vector<psfd_status> status(G, PSFD_NOT_CONVERGED);
  std::vector<psfd_info> loc(G);
  for (int i = 0; i < G; ++i) {
    bn2[i] = P->ks_host[i].red[0];
    if (!std::isfinite(bn2[i])) return fail(PSFD_ERR_ARG, "right-hand side is not finite");
  }
  for (int i = 0; i < G; ++i) {
    P->idle_host[i] = 0;
    if (bn2[i] == 0.0) {  // zero right-hand side: E = 0
      fin[i] = 1;
      status[i] = PSFD_OK;
      P->idle_host[i] = 1;
    }
  }
  CHKS(push_params(P));  // idle flags before the first operator apply

  cplx<double>* r64 = mixed ? P->res64 : P->v64[V_R];
  if (x0) {  // the initial residual from x0 itself, so that a bad x0 leaves E untouched
    CHKS(true_residual(P, b, x0, r64, adjoint));
    for (int i = 0; i < G; ++i)
      if (!fin[i] && !std::isfinite(P->ks_host[i].red[0]))
        return fail(PSFD_ERR_ARG, "initial guess gives a non-finite residual");
  }
  if (x0 && x0 != E)
    CHK(hipMemcpyAsync(E, x0, sizeof(cplx<double>) * n * G, hipMemcpyDeviceToDevice, st));
  if (!x0) CHK(hipMemsetAsync(E, 0, sizeof(cplx<double>) * n * G, st));
  for (int i = 0; i < G; ++i)
    if (bn2[i] == 0.0) CHK(hipMemsetAsync(E + i * n, 0, sizeof(cplx<double>) * n, st));

  if (x0) {
    for (int i = 0; i < G; ++i) {
      if (fin[i]) continue;
      loc[i].applies += 1;
      const double rr2 = P->ks_host[i].red[0];
      rrel[i] = std::sqrt(rr2 / bn2[i]);
      rn[i] = std::sqrt(rr2);
    }
  } else {
    CHK(hipMemcpyAsync(r64, b, sizeof(cplx<double>) * n * G, hipMemcpyDeviceToDevice, st));
    for (int i = 0; i < G; ++i)
      if (!fin[i]) {
        rrel[i] = 1.0;
        rn[i] = std::sqrt(bn2[i]);
      }
  }
  // Reliable updates (mixed single-problem plans): the complex64 residual is
  // replaced by the true FP64 residual each time it has fallen by kDelta
  // since the last replacement, so one run reaches the final tolerance with
  // the Krylov recurrence intact.  Group plans use the plain restart form
  // (inner runs to a loose relative tolerance, then a fresh start): there
  // every member's update stops the whole group's chunk for a host round
  // trip (160 batched uneven solves: 83 s with updates, 79 s with restarts).
  // PSFD_RELIABLE=0 / 1 selects the restart form / reliable updates for
  // every plan.
  static const double kDelta = [] {  // PSFD_RELIABLE_DELTA overrides (measurement aid)
    const char* e = std::getenv("PSFD_RELIABLE_DELTA");
    return (e && *e) ? std::atof(e) : 0.01;
  }();
  // PSFD_TRACE=1: one line per Krylov run end and per reliable update on stderr
  // (2: also the recursive residual every 512 iterations)
  static const bool trace = [] {
    const char* e = std::getenv("PSFD_TRACE");
    return e && *e && *e != '0';
  }();
  const bool reliable = mixed && [G] {
    const char* e = std::getenv("PSFD_RELIABLE");
    return (e && *e) ? std::atoi(e) != 0 : G == 1;
  }();
  std::vector<double> rn0(G, 0.0);  // normalisation of the current complex64 run
  // Every fold E += s M y is checked against the FP64 true residual: a
  // problem whose residual does not drop below the one at its last accepted
  // point gets its previous E back (a diverged or drifted Krylov run never
  // worsens the returned field), and a mixed plan continues in FP64.
  // rr_acc: ||b - A E||^2 of the current field; rr_best: of the field kept in
  // ebak64, the best accepted so far (copied there before a fold whenever the
  // current field is the best).
  std::vector<double> rr_acc(G, 0.0), rr_best(G, 0.0);
  for (int i = 0; i < G; ++i) rr_acc[i] = rr_best[i] = rn[i] * rn[i];
  std::vector<int> rejected(G, 0);
  std::vector<int> stall(G, 0);  // complex64 runs in a row without progress
  const size_t fbytes = sizeof(cplx<double>) * (size_t)n;
  auto save_E = [&]() -> psfd_status {
    for (int i = 0; i < G; ++i) {
      if (!(rr_acc[i] <= rr_best[i])) continue;
      CHK(hipMemcpyAsync(P->ebak64 + i * n, E + i * n, fbytes, hipMemcpyDeviceToDevice, st));
      rr_best[i] = rr_acc[i];
    }
    return PSFD_OK;
  };
  // After a fold E += s M y: the end of a Krylov run keeps the new field only if
  // its residual fell below the current one; a reliable update inside a running
  // Krylov process (relaxed) keeps it unless the residual is not finite or has
  // grown 100-fold over the best (BiCGSTAB residuals are not monotone: an update
  // on the way down from a spike may sit above the last one, and ending the run
  // there would throw its Krylov space away).  A rejected fold gets the best field
  // back.
  constexpr double kGrow2 = 1e4;
  auto keep_or_restore = [&](const std::vector<int>& mask, std::vector<int>& rej,
                             bool relaxed) -> psfd_status {
    bool any = false;
    for (int i = 0; i < G; ++i) {
      rej[i] = 0;
      if (!mask[i]) continue;
      const double rr2 = P->ks_host[i].red[0];
      if (relaxed ? (rr2 < kGrow2 * rr_best[i]) : (rr2 < rr_acc[i])) continue;
      CHK(hipMemcpyAsync(E + i * n, P->ebak64 + i * n, fbytes, hipMemcpyDeviceToDevice, st));
      rej[i] = 1;
      any = true;
    }
    if (any) CHKS(true_residual(P, b, E, r64, adjoint));
    for (int i = 0; i < G; ++i)
      if (mask[i]) {
        rr_acc[i] = P->ks_host[i].red[0];
        if (rej[i]) {
          rejected[i] = 1;
          loc[i].applies += 1;
        }
      }
    return PSFD_OK;
  };
  auto on_update = [&]() -> psfd_status {
    std::vector<int> upd(G, 0);
    for (int i = 0; i < G; ++i) upd[i] = P->ks_host[i].done == KS_UPDATE;
    for (int i = 0; i < G; ++i) {
      ProbParams& q = P->pp_host[i];
      q.mask = upd[i];
      q.scale = upd[i] ? rn0[i] : 0.0;  // E += rn0 M y
      q.iscale = 0.0;                   // then y = 0
      P->idle_host[i] = !upd[i];
    }
    CHKS(push_params(P));
    cplx<float>* y = P->v32[V_Y];
    CHKS(save_E());
    if (P->use_pc) {
      CHK(op_apply<float>(P, y, P->v32[V_W], OP_M, P->idle, 1));
      CHK(launch_k_axpy<double, float>(E, P->v32[V_W], P->pp, n, G, st));
    } else {
      CHK(launch_k_axpy<double, float>(E, y, P->pp, n, G, st));
    }
    CHK(launch_k_scale_copy<float, float>(y, y, P->pp, n, G, st));
    CHKS(true_residual(P, b, E, r64, adjoint));
    std::vector<int> rej(G, 0);
    CHKS(keep_or_restore(upd, rej, true));
    for (int i = 0; i < G; ++i) {
      if (!upd[i]) continue;
      loc[i].applies += 2;
      const double rr2 = P->ks_host[i].red[0];
      if (trace)
        fprintf(stderr, "psfd trace: p%d update at run iter %d: recursive %.3e true %.3e %s\n", i,
                P->ks_host[i].iter, std::sqrt(P->ks_host[i].rnorm2 / P->ks_host[i].bnorm2) * rn0[i] /
                std::sqrt(bn2[i]), std::sqrt(rr2 / bn2[i]), rej[i] ? "REJECTED" : "ok");
      rrel[i] = std::sqrt(rr2 / bn2[i]);
      P->pp_host[i].iscale = std::isfinite(rr2) ? 1.0 / rn0[i] : 0.0;  // r = r_true / rn0
    }
    CHKS(push_params(P));
    CHK(launch_k_scale_copy<float, double>(P->v32[V_R], r64, P->pp, n, G, st));
    CHK(launch_k_dot_rr<float>(P->v32[V_RH], P->v32[V_R], n, G, P->part, st));
    CHK(launch_finalize(FIN_REPLACE, P->ks, P->part, red_blocks(n, G), G, P->pp, st));
    bool stop = false;
    for (int i = 0; i < G; ++i) stop = stop || rej[i];
    if (stop) {  // a rejected update ends that problem's complex64 run
      CHKS(read_state(P));
      for (int i = 0; i < G; ++i) {
        if (!rej[i]) continue;
        P->ks_host[i].done = KS_BREAK;
        P->ks_host[i].status = 3;
        CHK(hipMemcpyAsync(P->ks + i, P->ks_host + i, sizeof(KState), hipMemcpyHostToDevice, st));
      }
    }
    for (int i = 0; i < G; ++i) {  // back to the run's parameters (the final fold uses them)
      ProbParams& q = P->pp_host[i];
      P->idle_host[i] = fin[i];
      q.mask = 1.0;
      q.scale = fin[i] ? 0.0 : rn0[i];
      q.iscale = fin[i] ? 0.0 : 1.0 / rn0[i];
    }
    CHKS(push_params(P));
    return read_state(P);
  };
  for (;;) {
    int active = 0, budget = 0;
    for (int i = 0; i < G; ++i) {
      if (fin[i]) continue;
      if (rrel[i] <= tol) {
        status[i] = PSFD_OK;
        fin[i] = 1;
      } else if (total[i] >= maxit || outer[i] > kMaxRestarts) {
        fin[i] = 1;  // status stays NOT_CONVERGED or BREAKDOWN
      } else {
        ++active;
        budget = std::max(budget, maxit - total[i]);
      }
    }
    if (!active) break;
    for (int i = 0; i < G; ++i) {
      ProbParams& q = P->pp_host[i];
      q = ProbParams{};
      P->idle_host[i] = fin[i];
      if (fin[i]) {
        q.tol2 = -1.0;
        continue;
      }
      q.itmax = (double)(maxit - total[i]);
      q.mask = 1.0;
      if (mixed) {
        // the run solves for the normalised residual r / rn (norm 1 at its start)
        const double it = reliable ? 0.5 * tol / rrel[i] : inner_tolerance(tol, rrel[i]);
        q.bnorm2 = 1.0;
        q.tol2 = it * it;
        q.iscale = 1.0 / rn[i];
        q.scale = rn[i];
        q.delta2 = reliable ? kDelta * kDelta : 0.0;
        rn0[i] = rn[i];
      } else {
        q.bnorm2 = bn2[i];
        q.tol2 = tol * tol;
        q.scale = 1.0;
      }
    }
    CHKS(push_params(P));
    std::vector<double> rr_start(rr_acc);
    for (int i = 0; i < G; ++i) rejected[i] = 0;
    if (mixed) {
      CHK(launch_k_scale_copy<float, double>(P->v32[V_R], r64, P->pp, n, G, st));
      CHKS(run_bicgstab<float>(P, adjoint, budget, on_update, shadow));
      cplx<float>* y = P->v32[V_Y];
      CHKS(save_E());
      if (P->use_pc) {
        CHK(op_apply<float>(P, y, P->v32[V_W], OP_M, P->idle, 1));
        CHK(launch_k_axpy<double, float>(E, P->v32[V_W], P->pp, n, G, st));
      } else {
        CHK(launch_k_axpy<double, float>(E, y, P->pp, n, G, st));
      }
    } else {
      CHKS(run_bicgstab<double>(P, adjoint, budget, no_update, shadow));
      cplx<double>* y = P->v64[V_Y];
      CHKS(save_E());
      if (P->use_pc) {
        CHK(op_apply<double>(P, y, P->tmp64, OP_M, P->idle, 1));
        CHK(launch_k_axpy<double, double>(E, P->tmp64, P->pp, n, G, st));
      } else {
        CHK(launch_k_axpy<double, double>(E, y, P->pp, n, G, st));
      }
    }
    shadow = nullptr;  // only the first run takes the caller's shadow residual
    std::vector<int> run_done(G, 0);
    for (int i = 0; i < G; ++i) {
      if (fin[i]) continue;
      const KState& k = P->ks_host[i];
      total[i] += k.iter;
      loc[i].applies += 2 * k.iter + 1;
      loc[i].rrel_hist_last = k.bnorm2 > 0 ? std::sqrt(k.rnorm2 / k.bnorm2) : 0.0;
      loc[i].restarts = outer[i] + 1;
      run_done[i] = k.done;
    }
    CHKS(true_residual(P, b, E, r64, adjoint));
    {
      std::vector<int> act(G, 0), rej(G, 0);
      for (int i = 0; i < G; ++i) act[i] = !fin[i];
      CHKS(keep_or_restore(act, rej, false));
    }
    bool escalate = false;
    for (int i = 0; i < G; ++i) {
      if (fin[i]) continue;
      const double rr2 = P->ks_host[i].red[0];
      if (!std::isfinite(rr2)) {
        status[i] = PSFD_BREAKDOWN;
        rrel[i] = rr2;
        fin[i] = 1;
        continue;
      }
      rrel[i] = std::sqrt(rr2 / bn2[i]);
      rn[i] = std::sqrt(rr2);
      if (run_done[i] == KS_BREAK && rrel[i] > tol && outer[i] >= kMaxRestarts)
        status[i] = PSFD_BREAKDOWN;
      outer[i] += 1;
      // A complex64 run that ended in a rejected fold or a breakdown without
      // its residual falling fourfold is a stall; after two stalls in a row
      // the rest of the solve runs on FP64 Krylov vectors.  A run that made
      // progress and then met its precision floor (a rejected update) is
      // followed by a fresh complex64 run normalised to the new residual.
      const bool progressed = rr2 < 0.0625 * rr_start[i];
      const bool failed = rejected[i] || run_done[i] == KS_BREAK;
      stall[i] = (failed && !progressed) ? stall[i] + 1 : 0;
      if (trace)
        fprintf(stderr, "psfd trace: p%d run %d (%s) ended: %d iters, done %d status %d, true rrel %.3e%s, "
                "stall %d\n", i, outer[i], mixed ? "c64" : "fp64", P->ks_host[i].iter, run_done[i],
                P->ks_host[i].status, rrel[i], rejected[i] ? " (fold rejected)" : "", stall[i]);
      if (mixed && rrel[i] > tol && stall[i] >= 2) escalate = true;
    }
    if (escalate) {
      mixed = false;
      CHKS(ensure_krylov<double>(P));
      CHK(hipMemcpyAsync(P->v64[V_R], r64, fbytes * G, hipMemcpyDeviceToDevice, st));
      r64 = P->v64[V_R];
    }
  }
  for (int i = 0; i < G; ++i) {
    // an unconverged problem returns its best field
    if (status[i] != PSFD_OK && rr_best[i] < rr_acc[i] && std::isfinite(rr_best[i])) {
      CHK(hipMemcpyAsync(E + i * n, P->ebak64 + i * n, fbytes, hipMemcpyDeviceToDevice, st));
      rrel[i] = std::sqrt(rr_best[i] / bn2[i]);
    }
    loc[i].iters = total[i];
    loc[i].rrel_true = rrel[i];
    loc[i].status = status[i];
    if (infos) infos[i] = loc[i];
  }
  if (G == 1 && status[0] != PSFD_OK)
    return fail(status[0], "solve stopped at relative residual " + std::to_string(rrel[0]));
  return PSFD_OK;
}

psfd_status set_eps_impl(struct psfd_plan* P, const void* const* eps) {
  const int64_t n = (int64_t)P->nabs * P->nx * P->ny;
  for (int i = 0; i < P->G; ++i)
    CHK(launch_eps_contrast(static_cast<const cplx<double>*>(eps[i]), (int)n, P->k0, P->d.eps_bg,
                            P->kd64 + i * n, P->kd32 ? P->kd32 + i * n : nullptr, P->st));
  CHK(hipStreamSynchronize(P->st));
  return PSFD_OK;
}

psfd_status plan_group_impl(int G, const psfd_desc* descs, const void* const* eps, void* stream,
                            struct psfd_plan** out) {
  if (G < 1 || !descs || !eps || !out) return fail(PSFD_ERR_ARG, "NULL argument");
  for (int i = 0; i < G; ++i) {
    CHKS(validate(&descs[i]));
    if (!eps[i]) return fail(PSFD_ERR_ARG, "eps must not be NULL");
    if (i > 0 && !same_group(descs[0], descs[i]))
      return fail(PSFD_ERR_ARG, "problems of a group must share everything but angle, "
                                "polarisation and permittivity");
  }
  const psfd_desc* d = &descs[0];
  struct psfd_plan* P = new (std::nothrow) struct psfd_plan();
  if (!P) return fail(PSFD_ERR_ALLOC, "host allocation failed");
  struct Guard {
    struct psfd_plan* p;
    ~Guard() { delete p; }
  } guard{P};
  P->d = *d;
  P->G = G;
  P->st = static_cast<hipStream_t>(stream);
  P->prec = d->prec;
  P->use_pc = d->precond != 0;
  P->ml_eps_h.assign(d->ml_eps, d->ml_eps + 2 * d->n_ml);
  P->ml_d_h.assign(d->ml_thick, d->ml_thick + d->n_ml);
  P->d.ml_eps = nullptr;
  P->d.ml_thick = nullptr;
  P->nx = d->nx;
  P->ny = d->ny;
  P->nabs = d->nz_abs;
  P->nz = d->nz_abs + d->nz_gap_bot + d->nz_gap_top + 2 * d->nz_pml;
  P->j0 = d->nz_pml + d->nz_gap_bot;
  P->jev = P->j0 - 1;
  P->plane = (int64_t)d->nx * d->ny;
  P->nfield = 3 * (int64_t)P->nz * P->plane;
  P->nspec = (int64_t)(3 * P->nz + 3 * P->nabs) * P->plane;
  P->k0 = kTwoPi / d->lambda;
  P->kbg = P->k0 * std::sqrt(d->eps_bg);
  P->prob.resize(G);
  for (int i = 0; i < G; ++i) {
    ProbInfo& q = P->prob[i];
    q.theta = descs[i].theta;
    q.phi = descs[i].phi;
    q.pol = descs[i].pol;
    q.kx0 = P->kbg * std::sin(q.theta) * std::cos(q.phi);
    q.ky0 = P->kbg * std::sin(q.theta) * std::sin(q.phi);
    q.kz0 = P->kbg * std::cos(q.theta);
  }

  std::vector<double> kx((size_t)G * P->nx), ky((size_t)G * P->ny), kz(P->nz), zabs(P->nabs);
  std::vector<double> cphi(G), sphi(G);
  for (int i = 0; i < G; ++i) {
    for (int m = 0; m < P->nx; ++m)
      kx[(size_t)i * P->nx + m] = P->prob[i].kx0 + kTwoPi * (fftfreq(m, P->nx) / (P->nx * d->dx));
    for (int m = 0; m < P->ny; ++m)
      ky[(size_t)i * P->ny + m] = P->prob[i].ky0 + kTwoPi * (fftfreq(m, P->ny) / (P->ny * d->dy));
    cphi[i] = std::cos(P->prob[i].phi);
    sphi[i] = std::sin(P->prob[i].phi);
  }
  for (int m = 0; m < P->nz; ++m) kz[m] = kTwoPi * (fftfreq(m, P->nz) / (P->nz * d->dz));
  for (int j = 0; j < P->nabs; ++j) zabs[j] = (j + 0.5) * d->dz;
  std::vector<cplx<double>> inv_s(P->nz);
  const int np = d->nz_pml;
  for (int j = 0; j < P->nz; ++j) {
    double dist = -1.0;
    if (j < np) dist = (np - j - 0.5) * d->dz;
    else if (j >= P->nz - np) dist = (j - (P->nz - np) + 0.5) * d->dz;
    cplx<double> s = {1.0, 0.0};
    if (dist >= 0.0) s.im = d->pml_sigma0 * std::pow(dist / (np * d->dz), (double)d->pml_order);
    inv_s[j] = cdiv(cplx<double>{1.0, 0.0}, s);
  }
  const auto twx = twiddles(P->nx), twy = twiddles(P->ny), twz = twiddles(P->nz);

  OpTables<double>& t = P->t64;
  t.nx = P->nx; t.ny = P->ny; t.nz = P->nz; t.nabs = P->nabs; t.j0 = P->j0; t.jev = P->jev;
  t.nprob = G; t.pfield = P->nfield; t.pspec = P->nspec;
  double *kx_d, *ky_d, *kz_d, *cphi_d, *sphi_d;
  cplx<double>*is_d, *twx_d, *twy_d, *twz_d;
  CHKS(upload(P, &kx_d, kx));
  CHKS(upload(P, &ky_d, ky));
  CHKS(upload(P, &kz_d, kz));
  CHKS(upload(P, &P->zabs64, zabs));
  CHKS(upload(P, &is_d, inv_s));
  CHKS(upload(P, &twx_d, twx));
  CHKS(upload(P, &twy_d, twy));
  CHKS(upload(P, &twz_d, twz));
  CHKS(upload(P, &cphi_d, cphi));
  CHKS(upload(P, &sphi_d, sphi));
  t.kx = kx_d; t.ky = ky_d; t.kz = kz_d; t.inv_s = is_d; t.zabs = P->zabs64;
  t.tw_x = twx_d; t.tw_y = twy_d; t.tw_z = twz_d;
  t.cphi = cphi_d; t.sphi = sphi_d;
  t.kbg2 = P->kbg * P->kbg;
  t.k0 = P->k0;
  t.kz_live = std::max(d->ml_kz_min, 1e-9) * P->k0;
  t.dz = d->dz;
  const double kref = d->pc_kref > 0 ? d->pc_kref : P->kbg;
  t.pc_mmin = d->pc_mmin;
  t.pc_kref2 = kref * kref;
  t.pc_gamma = d->pc_gamma;
  t.pc_reg = d->pc_reg;
  t.pc_bf16 = d->prec == PSFD_C64_BF16PC_REFINE64;
  t.ax_lds = std::getenv("PSFD_AXIAL_LDS") != nullptr;

  // multilayer reflections per lateral mode, per problem
  CHKS(dalloc(P, &P->rte64, (size_t)(P->plane * G)));
  CHKS(dalloc(P, &P->rpe64, (size_t)(P->plane * G)));
  cplx<double>* ml_eps_d = nullptr;
  double* ml_d_d = nullptr;
  std::vector<cplx<double>> mle(d->n_ml);
  for (int i = 0; i < d->n_ml; ++i) mle[i] = {P->ml_eps_h[2 * i], P->ml_eps_h[2 * i + 1]};
  CHKS(upload(P, &ml_eps_d, mle));
  CHKS(upload(P, &ml_d_d, P->ml_d_h));
  for (int i = 0; i < G; ++i) {
    TmmArgs ta{P->nx, P->ny, kx_d + (int64_t)i * P->nx, ky_d + (int64_t)i * P->ny, P->k0,
               d->eps_bg, d->n_ml, ml_eps_d, ml_d_d, cplx<double>{d->eps_sub[0], d->eps_sub[1]}};
    CHK(launch_tmm(ta, P->rte64 + i * P->plane, P->rpe64 + i * P->plane, P->st));
  }
  t.r_te = P->rte64;
  t.r_pe = P->rpe64;

  CHKS(dalloc(P, &P->kd64, (size_t)((int64_t)P->nabs * P->plane * G)));
  t.kd = P->kd64;
  CHKS(dalloc(P, &P->S64, (size_t)(P->nspec * G)));
  CHKS(dalloc(P, &P->UW64, (size_t)(P->nspec * G)));

  if (P->prec != PSFD_C128) {
    OpTables<float>& f = P->t32;
    f.nx = t.nx; f.ny = t.ny; f.nz = t.nz; f.nabs = t.nabs; f.j0 = t.j0; f.jev = t.jev;
    f.nprob = G; f.pfield = t.pfield; f.pspec = t.pspec;
    float *fkx, *fky, *fkz, *fza, *fcp, *fsp;
    cplx<float>*fis, *ftx, *fty, *ftz, *frte, *frpe;
    CHKS(upload(P, &fkx, to_t<float>(kx)));
    CHKS(upload(P, &fky, to_t<float>(ky)));
    CHKS(upload(P, &fkz, to_t<float>(kz)));
    CHKS(upload(P, &fza, to_t<float>(zabs)));
    CHKS(upload(P, &fcp, to_t<float>(cphi)));
    CHKS(upload(P, &fsp, to_t<float>(sphi)));
    CHKS(upload(P, &fis, to_tc<float>(inv_s)));
    CHKS(upload(P, &ftx, to_tc<float>(twx)));
    CHKS(upload(P, &fty, to_tc<float>(twy)));
    CHKS(upload(P, &ftz, to_tc<float>(twz)));
    CHKS(dalloc(P, &frte, (size_t)(P->plane * G)));
    CHKS(dalloc(P, &frpe, (size_t)(P->plane * G)));
    CHK(launch_k_scale_copy<float, double>(frte, P->rte64, nullptr, P->plane, G, P->st));
    CHK(launch_k_scale_copy<float, double>(frpe, P->rpe64, nullptr, P->plane, G, P->st));
    CHKS(dalloc(P, &P->kd32, (size_t)((int64_t)P->nabs * P->plane * G)));
    f.kx = fkx; f.ky = fky; f.kz = fkz; f.zabs = fza; f.inv_s = fis;
    f.tw_x = ftx; f.tw_y = fty; f.tw_z = ftz; f.r_te = frte; f.r_pe = frpe; f.kd = P->kd32;
    f.cphi = fcp; f.sphi = fsp;
    f.kbg2 = (float)t.kbg2; f.k0 = (float)t.k0; f.dz = (float)t.dz; f.kz_live = (float)t.kz_live;
    f.pc_mmin = (float)t.pc_mmin; f.pc_kref2 = (float)t.pc_kref2;
    f.pc_gamma = (float)t.pc_gamma; f.pc_reg = (float)t.pc_reg; f.pc_bf16 = t.pc_bf16;
    f.ax_lds = t.ax_lds;
    CHKS(ensure_fp32(P));
  }
  CHK(hipStreamCreateWithFlags(&P->own_st, hipStreamNonBlocking));
  CHK(hipEventCreateWithFlags(&P->join_ev, hipEventDisableTiming));
  P->use_graphs = std::getenv("PSFD_NO_GRAPH") == nullptr;
  CHKS(set_eps_impl(P, eps));
  CHKS(tune_plan(P, tune_wanted(G > 1)));
  CHK(hipStreamSynchronize(P->st));
  guard.p = nullptr;
  *out = P;
  return PSFD_OK;
}

// ---- allocation-free layout smoothing
// The workspace of psfd_layout_eps_noalloc: two lateral planes (the complex
// layout and its spectrum) and the x and y twiddle tables, in one file-scope
// device array.  Every GPU the library runs on holds its own copy for the
// life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (kept per device).
constexpr int64_t kNoAllocPlane = 512 * 512;  // largest nx * ny
constexpr int kNoAllocTw = 1024;               // largest nx, ny
constexpr int64_t kNoAllocElems = 2 * kNoAllocPlane + 2 * kNoAllocTw;
static __device__ __align__(256) cplx<double> scratch[kNoAllocElems];

constexpr int kNoAllocMaxDev = 64;
std::mutex g_scratch_mu;
cplx<double>* g_scratch_ptr[kNoAllocMaxDev] = {};

psfd_status scratch_of_current_device(cplx<double>** out) {
  int dev = -1;
  CHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDev) return fail(PSFD_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(PSFD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<cplx<double>*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return PSFD_OK;
}

// Same arithmetic as layout_impl; the twiddles are generated on the device
// into the workspace instead of uploaded, and nothing is allocated, freed or
// synchronised (the launches are queued on the caller's stream).
psfd_status layout_noalloc_impl(const psfd_desc* d, const double* a_bin, const double eps_abs[2],
                                double sigma, void* eps_out, void* stream) {
  if (!d || !a_bin || !eps_abs || !eps_out) return fail(PSFD_ERR_ARG, "NULL argument");
  if (!lateral_size_ok(d->nx) || !lateral_size_ok(d->ny) || d->nz_abs < 1)
    return fail(PSFD_ERR_ARG, "unsupported lateral size or nz_abs < 1");
  if ((int64_t)d->nx * d->ny > kNoAllocPlane || d->nx > kNoAllocTw || d->ny > kNoAllocTw)
    return fail(PSFD_ERR_ARG, "psfd_layout_eps_noalloc takes nx * ny <= 512 * 512 (its fixed "
                              "workspace); use psfd_layout_eps for larger layouts");
  if (!(sigma >= 0) || !(d->dx > 0) || !(d->dy > 0)) return fail(PSFD_ERR_ARG, "bad sigma/dx/dy");
  hipStream_t st = static_cast<hipStream_t>(stream);
  cplx<double>* ws = nullptr;
  CHKS(scratch_of_current_device(&ws));
  const int nx = d->nx, ny = d->ny;
  cplx<double>* A = ws;
  cplx<double>* B = ws + kNoAllocPlane;
  cplx<double>* twx = ws + 2 * kNoAllocPlane;
  cplx<double>* twy = twx + kNoAllocTw;
  CHK(launch_twiddles(twx, nx, st));
  CHK(launch_twiddles(twy, ny, st));
  OpTables<double> t{};
  t.nx = nx; t.ny = ny; t.nz = 1; t.nabs = 1; t.j0 = 0;
  t.tw_x = twx;
  t.tw_y = twy;
  CHK(launch_real_to_cplx(a_bin, nx * ny, A, st));
  CHK(launch_plane_fft<double>(t, A, B, false, st));
  CHK(launch_smooth_mult(B, nx, ny, d->dx, d->dy, sigma, st));
  CHK(launch_plane_fft<double>(t, B, A, true, st));
  CHK(launch_fill_eps(A, nx, ny, d->nz_abs, 1.0 / ((double)nx * ny), d->eps_bg,
                      cplx<double>{eps_abs[0], eps_abs[1]}, static_cast<cplx<double>*>(eps_out),
                      st));
  return PSFD_OK;
}

psfd_status plan_impl(const psfd_desc* d, const void* eps, void* stream, struct psfd_plan** out) {
  const void* e[1] = {eps};
  return plan_group_impl(1, d, e, stream, out);
}

psfd_status layout_impl(const psfd_desc* d, const double* a_bin, const double eps_abs[2],
                        double sigma, void* eps_out, void* stream) {
  if (!d || !a_bin || !eps_abs || !eps_out) return fail(PSFD_ERR_ARG, "NULL argument");
  if (!lateral_size_ok(d->nx) || !lateral_size_ok(d->ny) || d->nz_abs < 1)
    return fail(PSFD_ERR_ARG, "unsupported lateral size or nz_abs < 1");
  if (!(sigma >= 0) || !(d->dx > 0) || !(d->dy > 0)) return fail(PSFD_ERR_ARG, "bad sigma/dx/dy");
  hipStream_t st = static_cast<hipStream_t>(stream);
  struct psfd_plan tmp;  // owns the temporaries
  tmp.st = st;
  const int nx = d->nx, ny = d->ny;
  OpTables<double> t{};
  t.nx = nx; t.ny = ny; t.nz = 1; t.nabs = 1; t.j0 = 0;
  cplx<double>*twx, *twy, *A, *B;
  CHKS(upload(&tmp, &twx, twiddles(nx)));
  CHKS(upload(&tmp, &twy, twiddles(ny)));
  t.tw_x = twx;
  t.tw_y = twy;
  CHKS(dalloc(&tmp, &A, (size_t)nx * ny));
  CHKS(dalloc(&tmp, &B, (size_t)nx * ny));
  CHK(launch_real_to_cplx(a_bin, nx * ny, A, st));
  CHK(launch_plane_fft<double>(t, A, B, false, st));
  CHK(launch_smooth_mult(B, nx, ny, d->dx, d->dy, sigma, st));
  CHK(launch_plane_fft<double>(t, B, A, true, st));
  CHK(launch_fill_eps(A, nx, ny, d->nz_abs, 1.0 / ((double)nx * ny), d->eps_bg,
                      cplx<double>{eps_abs[0], eps_abs[1]}, static_cast<cplx<double>*>(eps_out),
                      st));
  CHK(hipStreamSynchronize(st));
  return PSFD_OK;
}

// The physics loss of the paper's PINO (equation loss) at a field E:
//   J = (1/N) ||r||^2 + (lambda/N) sum_alpha ||w(nu) F3 r_alpha||^2,  r = A E - b,
// with F3 unnormalised, so the penalty equals lambda <r, H r>, H = F3^-1 w^2 F3
// (Parseval).  H is the M-mode spectral pass with w(nu)^2 as its multiplier;
// <r, H r> rides on its inverse x pass.  The gradient field
//   g = (1/N) r' + lambda H r',  r' = b - A E = -r,
// gives dJ/dE = -2 A^H g and dJ/d eps = 2 k0^2 sum_alpha g_alpha conj(Psi_alpha)
// (PyTorch's convention grad = dJ/dRe + i dJ/dIm).
psfd_status pino_loss_impl(struct psfd_plan* P, const void* E_in, double w0, double eta,
                           double lam, double* out, void* g_out) {
  if (!P || !E_in || !out) return fail(PSFD_ERR_ARG, "NULL argument");
  if (P->is_batch || P->G != 1) return fail(PSFD_ERR_ARG, "psfd_pino_loss takes a single-problem plan");
  if (!std::isfinite(w0) || !std::isfinite(eta) || !(lam >= 0) || !std::isfinite(lam))
    return fail(PSFD_ERR_ARG, "need finite w0, eta and lambda >= 0");
  if (g_out == E_in) return fail(PSFD_ERR_ARG, "g must not overlap E");
  CHKS(ensure_solver_common(P));
  const auto* E = static_cast<const cplx<double>*>(E_in);
  const int64_t n = P->nfield;
  hipStream_t st = P->st;
  P->idle_host[0] = 0;
  P->pp_host[0] = ProbParams{};
  P->pp_host[0].mask = 1.0;
  CHKS(push_params(P));
  CHKS(rhs_group(P, P->b64));
  CHKS(true_residual(P, P->b64, E, P->res64, false));  // r' = b - A E
  const double rr = P->ks_host[0].red[0];
  P->hf_w0 = w0;
  P->hf_eta = eta;
  Fuse<double> fz;
  int nb = 0;
  fz.post.mode = POST_DOT;
  fz.post.d = P->res64;
  fz.post.part = P->part;
  fz.nblk_post = &nb;
  CHK(op_apply<double>(P, P->res64, P->tmp64, OP_HF, P->idle, 1, fz));  // H r'
  CHK(launch_finalize(FIN_RED3, P->ks, P->part, nb, 1, P->pp, st));
  CHKS(read_state(P));
  const double rh = P->ks_host[0].red[0];  // Re <r', H r'>
  const double N = (double)P->nx * P->ny * P->nz;
  out[0] = rr / N + lam * rh;
  out[1] = rr / N;
  out[2] = lam * rh;
  if (g_out) {
    auto* g = static_cast<cplx<double>*>(g_out);
    P->pp_host[0].iscale = 1.0 / N;
    P->pp_host[0].scale = lam;
    CHKS(push_params(P));
    CHK(launch_k_scale_copy<double, double>(g, P->res64, P->pp, n, 1, st));
    CHK(launch_k_axpy<double, double>(g, P->tmp64, P->pp, n, 1, st));
  }
  return PSFD_OK;
}

// Row means of a planar stack over the absorber rows, walked once from the
// top face z = nz_abs dz downwards: each row [j dz, (j+1) dz) collects the
// overlap-weighted permittivity of the layers it meets and the background
// for the part no layer covers.
psfd_status layered_impl(const psfd_desc* d, int32_t n, const double* leps, const double* ld,
                         void* eps_out, void* stream) {
  if (!d || !eps_out || n < 0 || (n > 0 && (!leps || !ld))) return fail(PSFD_ERR_ARG, "NULL argument");
  if (!lateral_size_ok(d->nx) || !lateral_size_ok(d->ny) || d->nz_abs < 1 || !(d->dz > 0))
    return fail(PSFD_ERR_ARG, "unsupported lateral size, nz_abs < 1 or dz <= 0");
  for (int i = 0; i < n; ++i)
    if (!(ld[i] >= 0) || !std::isfinite(ld[i]) || !std::isfinite(leps[2 * i]) ||
        !std::isfinite(leps[2 * i + 1]))
      return fail(PSFD_ERR_ARG, "layer thicknesses must be finite and >= 0");
  const int na = d->nz_abs;
  const double dz = d->dz;
  std::vector<cplx<double>> rows(na);
  int i = 0;                     // current layer
  double ltop = na * dz;         // its top face
  for (int j = na - 1; j >= 0; --j) {
    const double lo = j * dz, hi = (j + 1) * dz;
    double re = 0.0, im = 0.0, cov = 0.0;
    while (i < n) {
      const double lbot = ltop - ld[i];
      const double ov = std::min(hi, ltop) - std::max(lo, lbot);
      if (ov > 0) {
        re += leps[2 * i] * ov;
        im += leps[2 * i + 1] * ov;
        cov += ov;
      }
      if (lbot < lo) break;  // the layer continues into the row below
      ltop = lbot;
      ++i;
    }
    rows[j] = {(re + d->eps_bg * (dz - cov)) / dz, im / dz};
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  struct psfd_plan tmp;  // owns the temporary
  tmp.st = st;
  cplx<double>* rows_d = nullptr;
  CHKS(upload(&tmp, &rows_d, rows));
  CHK(launch_fill_rows(rows_d, (int64_t)d->nx * d->ny, na, static_cast<cplx<double>*>(eps_out), st));
  CHK(hipStreamSynchronize(st));
  return PSFD_OK;
}

// Specular (0, 0)-order reflection coefficient referred to the top face of
// the absorber region.  The plane means of E_x, E_y at the observation row
// and at the evaluation row come from the device; the rest is scalar:
// the upgoing (0, 0) amplitude at the observation row is the scattered
// field plus the multilayer response to the scattered field (evaluation
// row amplitude carried to z_ml, split into TE / TM as the operator does,
// times r_TE / r_pE, carried up) plus the multilayer reflection of the
// incident wave.
psfd_status specular_impl(struct psfd_plan* P, const void* E, double* r_out) {
  if (!P || !E || !r_out) return fail(PSFD_ERR_ARG, "NULL argument");
  if (P->is_batch || P->G != 1) return fail(PSFD_ERR_ARG, "psfd_specular takes a single-problem plan");
  const int64_t plane = P->plane;
  const int jobs = P->j0 + P->nabs, jev = P->jev;
  PlaneSet ps;
  ps.off[0] = (int64_t)jobs * plane;
  ps.off[1] = (int64_t)(P->nz + jobs) * plane;
  ps.off[2] = (int64_t)jev * plane;
  ps.off[3] = (int64_t)(P->nz + jev) * plane;
  ps.off[4] = (int64_t)(2 * P->nz + jev) * plane;
  const int nblk = (int)std::min<int64_t>(64, (plane + 255) / 256);
  cplx<double>* part = nullptr;
  struct psfd_plan tmp;  // owns the temporary
  tmp.st = P->st;
  CHKS(dalloc(&tmp, &part, (size_t)5 * nblk));
  CHK(launch_plane_sums(static_cast<const cplx<double>*>(E), ps, plane, nblk, part, P->st));
  std::vector<cplx<double>> h((size_t)5 * nblk + 2);
  CHK(hipMemcpyAsync(h.data(), part, sizeof(cplx<double>) * 5 * nblk, hipMemcpyDeviceToHost, P->st));
  CHK(hipMemcpyAsync(h.data() + 5 * nblk, P->rte64, sizeof(cplx<double>), hipMemcpyDeviceToHost, P->st));
  CHK(hipMemcpyAsync(h.data() + 5 * nblk + 1, P->rpe64, sizeof(cplx<double>), hipMemcpyDeviceToHost,
                     P->st));
  CHK(hipStreamSynchronize(P->st));
  std::complex<double> m[5];
  for (int q = 0; q < 5; ++q) {
    std::complex<double> acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += std::complex<double>(h[q * nblk + b].re, h[q * nblk + b].im);
    m[q] = acc / (double)plane;
  }
  const std::complex<double> rte(h[5 * nblk].re, h[5 * nblk].im);
  const std::complex<double> rpe(h[5 * nblk + 1].re, h[5 * nblk + 1].im);
  const ProbInfo& q = P->prob[0];
  const double kt = std::hypot(q.kx0, q.ky0);
  double sx, sy, tx, ty;
  if (kt == 0.0) {
    sx = -std::sin(q.phi); sy = std::cos(q.phi); tx = std::cos(q.phi); ty = std::sin(q.phi);
  } else {
    sx = -q.ky0 / kt; sy = q.kx0 / kt; tx = q.kx0 / kt; ty = q.ky0 / kt;
  }
  const double dz = P->d.dz;
  const double z_t = P->nabs * dz, z_obs = z_t + 0.5 * dz;
  const std::complex<double> I(0.0, 1.0);
  const double kz = q.kz0;
  const bool live = std::abs(kz) >= P->t64.kz_live;
  const std::complex<double> down = std::exp(-I * kz * (0.5 * dz));
  const std::complex<double> us = live ? rte * (sx * m[2] + sy * m[3]) * down : 0.0;
  // TM amplitude: least-squares fit of the downgoing TM polarisation (1, kt/kz)
  const double q_tz = live ? kt / kz : 0.0;
  const double w_t = 1.0 / (1.0 + q_tz * q_tz), w_z = q_tz * w_t;
  const std::complex<double> up = live ? rpe * (w_t * (tx * m[2] + ty * m[3]) + w_z * m[4]) * down : 0.0;
  const std::complex<double> ph = std::exp(I * kz * z_obs);
  std::complex<double> ux = m[0] + (us * sx + up * tx) * ph;
  std::complex<double> uy = m[1] + (us * sy + up * ty) * ph;
  // incident wave reflected by the multilayer, tangential part
  const double ct = std::cos(q.theta);
  if (q.pol == 0) {
    ux += rte * (-std::sin(q.phi)) * ph;
    uy += rte * std::cos(q.phi) * ph;
  } else {
    ux += rpe * (ct * std::cos(q.phi)) * ph;
    uy += rpe * (ct * std::sin(q.phi)) * ph;
  }
  const std::complex<double> val = q.pol == 0 ? sx * ux + sy * uy : -(tx * ux + ty * uy) / ct;
  const std::complex<double> r = val * std::exp(-I * kz * z_obs) * std::exp(2.0 * I * kz * z_t);
  r_out[0] = r.real();
  r_out[1] = r.imag();
  return PSFD_OK;
}

template <typename T>
psfd_status apply_entry(struct psfd_plan* P, const void* x, void* y, int op) {
  if (!P || !x || !y) return fail(PSFD_ERR_ARG, "NULL argument");
  if (P->is_batch) return fail(PSFD_ERR_ARG, "a batch handle only serves psfd_solve_batch");
  if (x == y) return fail(PSFD_ERR_ARG, "x and y must not overlap");
  if (sizeof(T) == 4 && !P->t32.kx)
    return fail(PSFD_ERR_ARG, "complex64 entry points need a PSFD_C64_* plan");
  if (sizeof(T) == 4) CHKS(ensure_fp32(P));
  CHK(op_apply<T>(P, static_cast<const cplx<T>*>(x), static_cast<cplx<T>*>(y), op, nullptr, 0));
  return PSFD_OK;
}

template <typename F>
psfd_status guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const std::bad_alloc&) {
    return fail(PSFD_ERR_ALLOC, "host allocation failed");
  } catch (...) {
    return fail(PSFD_ERR_HIP, "unexpected exception");
  }
}

psfd_status plan_batch_impl(int n, const psfd_desc* descs, const void* const* eps, void* stream,
                            struct psfd_plan** out) {
  if (n < 1 || !descs || !eps || !out) return fail(PSFD_ERR_ARG, "bad batch arguments");
  for (int i = 0; i < n; ++i) {
    psfd_status st = validate(&descs[i]);
    if (st != PSFD_OK) return fail(st, "problem " + std::to_string(i) + ": " + g_err);
    if (!eps[i]) return fail(PSFD_ERR_ARG, "problem " + std::to_string(i) + ": eps is NULL");
  }
  struct psfd_plan* B = new (std::nothrow) struct psfd_plan();
  if (!B) return fail(PSFD_ERR_ALLOC, "host allocation failed");
  B->is_batch = true;
  B->st = static_cast<hipStream_t>(stream);
  for (int i = 0; i < n; ++i) {
    psfd_desc d = descs[i];
    B->b_ml_eps.emplace_back(d.ml_eps, d.ml_eps + 2 * d.n_ml);
    B->b_ml_d.emplace_back(d.ml_thick, d.ml_thick + d.n_ml);
    B->bdesc.push_back(d);
    B->beps.push_back(eps[i]);
  }
  for (int i = 0; i < n; ++i) {  // point the copies at the owned tables
    B->bdesc[i].ml_eps = B->b_ml_eps[i].data();
    B->bdesc[i].ml_thick = B->b_ml_d[i].data();
  }
  *out = B;
  return PSFD_OK;
}

// Problems are grouped (same shape and shared parameters, at most
// kGroupVoxels voxels and kGroupMax problems per group, largest first); each
// group is one plan whose launches cover all its members.  Groups run on
// PSFD_BATCH_WORKERS host threads (default 2), each with its own stream.
psfd_status solve_batch_impl(struct psfd_plan* B, const void* const* x0, void* const* E, double tol,
                             int maxit, psfd_info* infos) {
  if (!B || !B->is_batch || !E || !infos) return fail(PSFD_ERR_ARG, "bad batch arguments");
  const int n = (int)B->bdesc.size();
  for (int i = 0; i < n; ++i)
    if (!E[i]) return fail(PSFD_ERR_ARG, "E[" + std::to_string(i) + "] is NULL");
  CHK(B->st ? hipStreamSynchronize(B->st) : hipDeviceSynchronize());
  int dev = 0;
  CHK(hipGetDevice(&dev));
  auto voxels = [&](int i) {
    const psfd_desc& d = B->bdesc[i];
    return (int64_t)d.nx * d.ny * (d.nz_abs + d.nz_gap_bot + d.nz_gap_top + 2 * d.nz_pml);
  };
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return voxels(a) > voxels(b); });
  int64_t max_vox = (int64_t)1 << 26;
  if (const char* v = std::getenv("PSFD_GROUP_VOXELS")) max_vox = std::max<int64_t>(1, std::atoll(v));
  int max_g = 256;
  if (const char* v = std::getenv("PSFD_GROUP_MAX")) max_g = std::max(1, std::atoi(v));
  std::vector<std::vector<int>> groups;
  std::vector<int64_t> gvox;
  for (int i : order) {
    int at = -1;
    for (size_t g = 0; g < groups.size(); ++g) {
      if ((int)groups[g].size() < max_g && gvox[g] + voxels(i) <= max_vox &&
          same_group(B->bdesc[groups[g][0]], B->bdesc[i])) {
        at = (int)g;
        break;
      }
    }
    if (at < 0) {
      groups.emplace_back();
      gvox.push_back(0);
      at = (int)groups.size() - 1;
    }
    groups[at].push_back(i);
    gvox[at] += voxels(i);
  }
  int workers = 2;
  if (const char* w = std::getenv("PSFD_BATCH_WORKERS")) workers = std::max(1, std::atoi(w));
  workers = std::min<int>(workers, (int)groups.size());
  std::vector<psfd_status> status(n, PSFD_OK);
  std::vector<std::string> errs(n);
  std::atomic<int> next(0);
  auto work = [&]() {
    if (hipSetDevice(dev) != hipSuccess) return;
    hipStream_t ws = nullptr;
    if (hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess) ws = nullptr;
    for (int k = next++; k < (int)groups.size(); k = next++) {
      const std::vector<int>& mem = groups[k];
      const int G = (int)mem.size();
      std::vector<psfd_desc> ds(G);
      std::vector<const void*> es(G);
      for (int j = 0; j < G; ++j) {
        ds[j] = B->bdesc[mem[j]];
        es[j] = B->beps[mem[j]];
      }
      std::vector<psfd_info> inf(G);
      struct psfd_plan* p = nullptr;
      psfd_status st = guarded([&] { return plan_group_impl(G, ds.data(), es.data(), ws, &p); });
      if (st == PSFD_OK && G == 1) st = guarded([&] { return tune_plan(p, tune_wanted(true)); });
      if (st == PSFD_OK) {
        st = guarded([&]() -> psfd_status {
          CHKS(dalloc(p, &p->E64, (size_t)(p->nfield * G)));
          const size_t fb = sizeof(cplx<double>) * (size_t)p->nfield;
          if (x0) {
            for (int j = 0; j < G; ++j) {
              if (x0[mem[j]]) CHK(hipMemcpyAsync(p->E64 + j * p->nfield, x0[mem[j]], fb,
                                                 hipMemcpyDeviceToDevice, ws));
              else CHK(hipMemsetAsync(p->E64 + j * p->nfield, 0, fb, ws));
            }
          }
          CHKS(solve_impl(p, nullptr, x0 ? p->E64 : nullptr, p->E64, tol, maxit, false, inf.data()));
          for (int j = 0; j < G; ++j)
            CHK(hipMemcpyAsync(E[mem[j]], p->E64 + j * p->nfield, fb, hipMemcpyDeviceToDevice, ws));
          CHK(hipStreamSynchronize(ws));
          return PSFD_OK;
        });
      }
      for (int j = 0; j < G; ++j) {
        const int i = mem[j];
        infos[i] = inf[j];
        if (st != PSFD_OK) {
          errs[i] = g_err;
          infos[i].status = st;
          status[i] = st;
        } else if (inf[j].status != PSFD_OK) {
          status[i] = (psfd_status)inf[j].status;
          errs[i] = "stopped at relative residual " + std::to_string(inf[j].rrel_true);
        }
      }
      delete p;
    }
    if (ws) (void)hipStreamDestroy(ws);
  };
  std::vector<std::thread> pool;
  for (int w = 0; w < workers; ++w) pool.emplace_back(work);
  for (auto& t : pool) t.join();
  for (int i = 0; i < n; ++i)
    if (status[i] != PSFD_OK) return fail(status[i], "problem " + std::to_string(i) + ": " + errs[i]);
  return PSFD_OK;
}

}  // namespace

extern "C" {

psfd_status psfd_layout_eps(const psfd_desc* d, const double* a_bin_dev, const double eps_abs[2],
                            double sigma, void* eps_out, void* hip_stream) {
  return guarded([&] { return layout_impl(d, a_bin_dev, eps_abs, sigma, eps_out, hip_stream); });
}

psfd_status psfd_layout_eps_noalloc(const psfd_desc* d, const double* a_bin_dev,
                                    const double eps_abs[2], double sigma, void* eps_out,
                                    void* hip_stream) {
  return guarded([&] { return layout_noalloc_impl(d, a_bin_dev, eps_abs, sigma, eps_out, hip_stream); });
}

psfd_status psfd_plan(const psfd_desc* d, const void* eps_abs_dev, void* hip_stream,
                      psfd_plan_t* out) {
  return guarded([&] { return plan_impl(d, eps_abs_dev, hip_stream, out); });
}

psfd_status psfd_set_eps(psfd_plan_t p, const void* eps_abs_dev) {
  if (!p || !eps_abs_dev || p->is_batch) return fail(PSFD_ERR_ARG, "NULL argument");
  const void* e[1] = {eps_abs_dev};
  return guarded([&] { return set_eps_impl(p, e); });
}

psfd_status psfd_rhs(psfd_plan_t p, void* b) {
  if (!p || !b || p->is_batch) return fail(PSFD_ERR_ARG, "NULL argument");
  return guarded([&] { return rhs_group(p, static_cast<cplx<double>*>(b)); });
}

psfd_status psfd_apply(psfd_plan_t p, const void* x, void* y) {
  return guarded([&] { return apply_entry<double>(p, x, y, OP_A); });
}
psfd_status psfd_adjoint(psfd_plan_t p, const void* x, void* y) {
  return guarded([&] { return apply_entry<double>(p, x, y, OP_AH); });
}
psfd_status psfd_precond(psfd_plan_t p, const void* x, void* y) {
  return guarded([&] { return apply_entry<double>(p, x, y, OP_M); });
}
psfd_status psfd_apply_c64(psfd_plan_t p, const void* x, void* y) {
  return guarded([&] { return apply_entry<float>(p, x, y, OP_A); });
}
psfd_status psfd_adjoint_c64(psfd_plan_t p, const void* x, void* y) {
  return guarded([&] { return apply_entry<float>(p, x, y, OP_AH); });
}
psfd_status psfd_precond_c64(psfd_plan_t p, const void* x, void* y) {
  return guarded([&] { return apply_entry<float>(p, x, y, OP_M); });
}

psfd_status psfd_solve(psfd_plan_t p, const void* b, const void* x0, void* E, double tol,
                       int32_t maxit, int32_t adjoint, psfd_info* info) {
  if (!p || !E || p->is_batch) return fail(PSFD_ERR_ARG, "NULL argument or batch handle");
  if (!(tol > 0) || maxit < 0) return fail(PSFD_ERR_ARG, "need tol > 0 and maxit >= 0");
  if (b && b == E) return fail(PSFD_ERR_ARG, "b and E must not overlap");
  return guarded([&] { return solve_impl(p, b, x0, E, tol, maxit, adjoint != 0, info); });
}

psfd_status psfd_solve_shadow(psfd_plan_t p, const void* b, const void* x0, void* E, double tol,
                              int32_t maxit, int32_t adjoint, const void* shadow,
                              psfd_info* info) {
  if (!p || !E || !shadow || p->is_batch)
    return fail(PSFD_ERR_ARG, "NULL argument or batch handle");
  if (!(tol > 0) || maxit < 0) return fail(PSFD_ERR_ARG, "need tol > 0 and maxit >= 0");
  if (b && b == E) return fail(PSFD_ERR_ARG, "b and E must not overlap");
  if (shadow == E) return fail(PSFD_ERR_ARG, "shadow and E must not overlap");
  return guarded([&] { return solve_impl(p, b, x0, E, tol, maxit, adjoint != 0, info, shadow); });
}

psfd_status psfd_residual(psfd_plan_t p, const void* b, const void* E, void* r, double* norm2) {
  if (!p || !E || !r || p->is_batch) return fail(PSFD_ERR_ARG, "NULL argument or batch handle");
  if (r == E || (b && r == b)) return fail(PSFD_ERR_ARG, "r must not overlap E or b");
  return guarded([&]() -> psfd_status {
    CHKS(ensure_solver_common(p));
    const cplx<double>* bb = static_cast<const cplx<double>*>(b);
    if (!bb) {
      CHKS(rhs_group(p, p->b64));
      bb = p->b64;
    }
    p->idle_host[0] = 0;
    CHKS(push_params(p));
    CHKS(true_residual(p, bb, static_cast<const cplx<double>*>(E), static_cast<cplx<double>*>(r),
                       false));
    if (norm2) *norm2 = p->ks_host[0].red[0];
    return PSFD_OK;
  });
}

psfd_status psfd_eps_grad(psfd_plan_t p, const void* E, const void* u, double scale, void* grad) {
  if (!p || !E || !u || !grad || p->is_batch) return fail(PSFD_ERR_ARG, "NULL argument or batch handle");
  return guarded([&]() -> psfd_status {
    // E + E_ML[E] on absorber rows: forward lateral transform, axial kernel (W planes),
    // inverse lateral transform of the W planes only
    OpTables<double> t = p->t64;
    const int p3 = 3 * p->nz, pa = 3 * p->nabs;
    cplx<double>* S = p->S64;
    cplx<double>* UW = p->UW64;
    cplx<double>* Wr = S;  // reuse: the spectrum is no longer needed once UW is formed
    CHK(launch_xfft_fwd<double>(t, static_cast<const cplx<double>*>(E), S, false,
                                PreOp<double>{}, nullptr, p->st));
    CHK(launch_yfft<double>(t, S, p3, false, p->st));
    CHK(launch_axial<double>(t, S, UW, AX_A, p->st));
    cplx<double>* Wp = UW + (int64_t)p3 * p->plane;
    CHK(launch_yfft<double>(t, Wp, pa, true, p->st));
    CHK(launch_xfft_inv_rows<double>(t, Wp, Wr, (int64_t)pa * p->ny, p->st));
    CHK(launch_eps_grad(rhs_args(p, 0), Wr, static_cast<const cplx<double>*>(u), scale,
                        static_cast<cplx<double>*>(grad), p->st));
    return PSFD_OK;
  });
}

psfd_status psfd_plan_batch(int32_t n, const psfd_desc* descs, const void* const* eps_abs_dev,
                            void* hip_stream, psfd_plan_t* out) {
  return guarded([&] { return plan_batch_impl(n, descs, eps_abs_dev, hip_stream, out); });
}

psfd_status psfd_solve_batch(psfd_plan_t batch, const void* const* x0, void* const* E, double tol,
                             int32_t maxit, psfd_info* infos) {
  if (!(tol > 0) || maxit < 0) return fail(PSFD_ERR_ARG, "need tol > 0 and maxit >= 0");
  return guarded([&] { return solve_batch_impl(batch, x0, E, tol, maxit, infos); });
}

psfd_status psfd_ml_reflection(psfd_plan_t p, void* r_te, void* r_pe) {
  if (!p || !r_te || !r_pe || p->is_batch) return fail(PSFD_ERR_ARG, "NULL argument");
  return guarded([&]() -> psfd_status {
    const size_t bytes = sizeof(cplx<double>) * (size_t)p->plane;
    CHK(hipMemcpyAsync(r_te, p->rte64, bytes, hipMemcpyDeviceToDevice, p->st));
    CHK(hipMemcpyAsync(r_pe, p->rpe64, bytes, hipMemcpyDeviceToDevice, p->st));
    return PSFD_OK;
  });
}

}  // extern "C"

namespace {

struct FfnoLayout {
  FfnoArgs a{};
  int64_t n_weights = 0;
  size_t off_v = 0, off_u = 0, off_T = 0, off_G = 0, off_U = 0, off_tx = 0, off_ty = 0, off_tz = 0;
  size_t off_w2t = 0, off_kzt = 0, off_pz = 0, off_qx = 0, off_q4 = 0, off_W = 0, off_Z = 0;
  size_t bytes = 0;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

psfd_status ffno_layout(const psfd_ffno_desc* d, FfnoLayout* L) {
  if (!d) return fail(PSFD_ERR_ARG, "desc is NULL");
  const bool dims = (d->d_v == 32 && d->d_h == 64) || (d->d_v == 16 && d->d_h == 32) ||
                    (d->d_v == 8 && d->d_h == 16);
  if (!dims) return fail(PSFD_ERR_ARG, "(d_v, d_h) must be (32, 64), (16, 32) or (8, 16)");
  if (d->nx < 4 || d->ny < 4 || d->nz < 4 || d->nx > 8192 || d->ny > 8192 || d->nz > 4096)
    return fail(PSFD_ERR_ARG, "need 4 <= nx, ny <= 8192 and 4 <= nz <= 4096");
  if (d->n_layers < 1 || d->n_layers > kFfnoMaxLayers) return fail(PSFD_ERR_ARG, "1 <= n_layers <= 16");
  if (d->kx_max < 0 || d->ky_max < 0 || d->kz_max < 0 || 2 * d->kx_max >= d->nx ||
      2 * d->ky_max >= d->ny || 2 * d->kz_max >= d->nz || d->kz_max > 15 || d->kx_max > 31)
    return fail(PSFD_ERR_ARG, "need 0 <= 2 k_max < n for every axis, kx_max <= 31, kz_max <= 15");
  FfnoArgs& a = L->a;
  a.nx = d->nx; a.ny = d->ny; a.nz = d->nz; a.dv = d->d_v; a.dh = d->d_h; a.nl = d->n_layers;
  a.mx = d->kx_max + 1; a.my = 2 * d->ky_max + 1; a.mz = d->kz_max + 1; a.ky_max = d->ky_max;
  const int64_t dv = a.dv, dh = a.dh;
  L->n_weights = dv * 4 + dv + a.nl * (dv * dv * a.my * a.mx * 2 + dv * dv * a.mz * 2 + dh * dv +
                                       dh + dv * dh + dv) + 6 * dv + 6;
  const size_t vox = (size_t)a.nz * a.ny * a.nx;
  size_t o = 0;
  L->off_v = o; o = align256(o + sizeof(float) * dv * vox);
  L->off_u = o; o = align256(o + sizeof(float) * dv * vox);
  L->off_T = o; o = align256(o + sizeof(float2) * dv * a.nz * a.ny * a.mx);
  L->off_G = o; o = align256(o + sizeof(float2) * dv * a.nz * a.my * a.mx);
  L->off_U = o; o = align256(o + sizeof(float2) * dv * a.nz * a.my * a.mx);
  L->off_tx = o; o = align256(o + sizeof(float2) * a.nx);
  L->off_ty = o; o = align256(o + sizeof(float2) * a.ny);
  L->off_tz = o; o = align256(o + sizeof(float2) * a.nz);
  L->off_w2t = o; o = align256(o + sizeof(float) * a.nl * dv * dh);
  L->off_kzt = o; o = align256(o + sizeof(float2) * a.nl * a.mz * dv * dv);
  L->off_pz = o; o = align256(o + sizeof(float2) * 16 * (size_t)(a.nz + 3));
  L->off_qx = o; o = align256(o + sizeof(float2) * 32 * (size_t)((a.nx + 15) / 16 + 7));
  L->off_q4 = o; o = align256(o + sizeof(float2) * 32 * (size_t)(4 * ((a.nx + 63) / 64) + 4));
  L->off_W = o; o = align256(o + sizeof(float2) * dv * a.mz * (size_t)a.ny * a.nx);
  L->off_Z = o; o = align256(o + sizeof(float2) * dv * a.mz * (size_t)a.ny * a.nx);
  L->bytes = o;
  return PSFD_OK;
}

}  // namespace

extern "C" {

psfd_status psfd_ffno_sizes(const psfd_ffno_desc* d, int64_t* n_weights, int64_t* workspace_bytes) {
  FfnoLayout L;
  CHKS(ffno_layout(d, &L));
  if (n_weights) *n_weights = L.n_weights;
  if (workspace_bytes) *workspace_bytes = (int64_t)L.bytes;
  return PSFD_OK;
}

psfd_status psfd_ffno_forward(const psfd_ffno_desc* d, const float* weights, const float* a_in,
                              void* E, void* workspace, void* hip_stream) {
  FfnoLayout L;
  CHKS(ffno_layout(d, &L));
  if (!weights || !a_in || !E || !workspace) return fail(PSFD_ERR_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 || reinterpret_cast<uintptr_t>(weights) % 8 ||
      reinterpret_cast<uintptr_t>(a_in) % 4 || reinterpret_cast<uintptr_t>(E) % 16)
    return fail(PSFD_ERR_ARG, "workspace must be 256-byte, weights 8-byte, a_in 4-byte and E "
                              "16-byte aligned");
  return guarded([&]() -> psfd_status {
    const FfnoArgs& a = L.a;
    FfnoPtrs w{};
    const float* q = weights;
    const int64_t dv = a.dv, dh = a.dh;
    w.P = q; q += dv * 4;
    w.p = q; q += dv;
    for (int l = 0; l < a.nl; ++l) {
      w.Kxy[l] = reinterpret_cast<const float2*>(q); q += dv * dv * a.my * a.mx * 2;
      w.Kz[l] = reinterpret_cast<const float2*>(q); q += dv * dv * a.mz * 2;
      w.W1[l] = q; q += dh * dv;
      w.b1[l] = q; q += dh;
      w.W2[l] = q; q += dv * dh;
      w.b2[l] = q; q += dv;
    }
    w.Q = q; q += 6 * dv;
    w.q = q;
    char* ws = static_cast<char*>(workspace);
    w.v = reinterpret_cast<float*>(ws + L.off_v);
    w.u = reinterpret_cast<float*>(ws + L.off_u);
    w.T = reinterpret_cast<float2*>(ws + L.off_T);
    w.G = reinterpret_cast<float2*>(ws + L.off_G);
    w.U = reinterpret_cast<float2*>(ws + L.off_U);
    w.twx = reinterpret_cast<float2*>(ws + L.off_tx);
    w.twy = reinterpret_cast<float2*>(ws + L.off_ty);
    w.twz = reinterpret_cast<float2*>(ws + L.off_tz);
    w.W2T = reinterpret_cast<float*>(ws + L.off_w2t);
    w.KzT = reinterpret_cast<float2*>(ws + L.off_kzt);
    w.pz = reinterpret_cast<float2*>(ws + L.off_pz);
    w.qx = reinterpret_cast<float2*>(ws + L.off_qx);
    w.q4 = reinterpret_cast<float2*>(ws + L.off_q4);
    w.W = reinterpret_cast<float2*>(ws + L.off_W);
    w.Z = reinterpret_cast<float2*>(ws + L.off_Z);
    CHK(ffno_forward(a, w, a_in, static_cast<cplx<double>*>(E), static_cast<hipStream_t>(hip_stream)));
    return PSFD_OK;
  });
}

psfd_status psfd_pino_loss(psfd_plan_t p, const void* E, double w0, double eta_hf,
                           double lambda_hf, double loss[3], void* g) {
  return guarded([&] { return pino_loss_impl(p, E, w0, eta_hf, lambda_hf, loss, g); });
}

psfd_status psfd_layered_eps(const psfd_desc* d, int32_t n_layers, const double* layers_eps,
                             const double* layers_thick, void* eps_abs_dev, void* hip_stream) {
  return guarded([&] { return layered_impl(d, n_layers, layers_eps, layers_thick, eps_abs_dev, hip_stream); });
}

psfd_status psfd_specular(psfd_plan_t p, const void* E, double r[2]) {
  return guarded([&] { return specular_impl(p, E, r); });
}

psfd_status psfd_contour_segments(const void* planes, int32_t nx, int32_t ny, int32_t nplanes,
                                  int64_t plane_stride, double dx, double dy, int32_t nlines,
                                  double i_th, double w, int32_t max_seg, double* seg,
                                  int32_t* nseg, void* hip_stream) {
  if (!planes || !seg || !nseg) return fail(PSFD_ERR_ARG, "NULL argument");
  if (nx < 2 || ny < 2 || nx > kContourLineMax || ny > kContourLineMax || nplanes < 1 ||
      nplanes > 65535 || nlines < 1 || 2 * nlines > 65535 || max_seg < 1 ||
      plane_stride < (int64_t)nx * ny)
    return fail(PSFD_ERR_ARG, "bad sizes (2 <= nx, ny <= 1024, nplanes >= 1, nlines >= 1, max_seg >= 1)");
  if (!(dx > 0) || !(dy > 0) || !(w > 0) || !std::isfinite(i_th))
    return fail(PSFD_ERR_ARG, "need dx, dy, w > 0 and a finite threshold");
  return guarded([&]() -> psfd_status {
    ContourArgs a{static_cast<const cplx<double>*>(planes), plane_stride, nx, ny, nlines, max_seg,
                  dx, dy, i_th, w, seg, nseg};
    CHK(launch_contour_segments(a, nplanes, static_cast<hipStream_t>(hip_stream)));
    return PSFD_OK;
  });
}

psfd_status psfd_contour_deviation(const double* seg_ref, const int32_t* nseg_ref,
                                   const double* seg, const int32_t* nseg, int32_t nx, int32_t ny,
                                   int32_t nplanes, double dx, double dy, int32_t nlines,
                                   int32_t max_seg, double demag, double thr, double* delta,
                                   double* stats, void* hip_stream) {
  if (!seg_ref || !nseg_ref || !seg || !nseg || !delta || !stats)
    return fail(PSFD_ERR_ARG, "NULL argument");
  if (nx < 2 || ny < 2 || nplanes < 1 || nlines < 1 || max_seg < 1)
    return fail(PSFD_ERR_ARG, "bad sizes");
  if (!(dx > 0) || !(dy > 0) || !(demag > 0) || !std::isfinite(thr))
    return fail(PSFD_ERR_ARG, "need dx, dy, demag > 0");
  return guarded([&]() -> psfd_status {
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t items = (int64_t)nplanes * 2 * nlines * max_seg;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (items + 255) / 256));
    struct psfd_plan tmp;  // owns the temporary
    tmp.st = st;
    double* part = nullptr;
    CHKS(dalloc(&tmp, &part, (size_t)nb * 5));
    DeviationArgs a{seg_ref, nseg_ref, seg, nseg, nplanes, nlines, max_seg, nx * dx, ny * dy,
                    demag, thr, delta, part};
    CHK(launch_contour_deviation(a, nb, st));
    std::vector<double> h((size_t)nb * 5);
    CHK(hipMemcpyAsync(h.data(), part, sizeof(double) * nb * 5, hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    for (int k = 0; k < 5; ++k) {
      double s = 0.0;
      for (int b = 0; b < nb; ++b) s += h[(size_t)b * 5 + k];
      stats[k] = s;
    }
    return PSFD_OK;
  });
}

psfd_status psfd_profile_enable(psfd_plan_t p, int32_t kernel) {
  if (!p || p->is_batch || kernel < PROF_OFF || kernel > PROF_XINV) return fail(PSFD_ERR_ARG, "bad argument");
  return guarded([&]() -> psfd_status {
    CHK(p->st ? hipStreamSynchronize(p->st) : hipDeviceSynchronize());
    collect_events(p);
    p->prof_kernel = kernel;
    p->prof_elem = p->prec == PSFD_C128 ? 16 : 8;
    p->prof_ms = 0.0;
    p->prof_bytes = 0.0;
    p->prof_launches = 0;
    return PSFD_OK;
  });
}

psfd_status psfd_profile_read(psfd_plan_t p, double* total_ms, int64_t* launches, double* bytes) {
  if (!p || p->is_batch || !total_ms || !launches || !bytes) return fail(PSFD_ERR_ARG, "NULL argument");
  return guarded([&]() -> psfd_status {
    CHK(p->st ? hipStreamSynchronize(p->st) : hipDeviceSynchronize());
    collect_events(p);
    *total_ms = p->prof_ms;
    *launches = p->prof_launches;
    *bytes = p->prof_bytes;
    return PSFD_OK;
  });
}

psfd_status psfd_tune(psfd_plan_t p) {
  if (!p || p->is_batch) return fail(PSFD_ERR_ARG, "NULL argument or batch handle");
  return guarded([&]() -> psfd_status {
    drop_graphs(p);  // captured chunks hold the old schedules
    CHKS(p->prec == PSFD_C128 ? autotune<double>(p, true) : autotune<float>(p, true));
    CHK(hipStreamSynchronize(p->st));
    return PSFD_OK;
  });
}

psfd_status psfd_tune_save(const char* path) {
  if (!path || !*path) return fail(PSFD_ERR_ARG, "NULL or empty path");
  return guarded([&]() -> psfd_status {
    load_tune_table();
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(PSFD_ERR_ARG, std::string("cannot write ") + path);
    std::fprintf(f, "# libpsfd kernel schedules (elem: 4 complex64 plans, 8 complex128): "
                    "elem nx ny nz nabs group : xf xi y ax\n");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune)
      std::fprintf(f, "%d %d %d %d %d %d : %d %d %d %d\n", kv.first.elem, kv.first.nx, kv.first.ny,
                   kv.first.nz, kv.first.nabs, kv.first.gb, kv.second.v[0], kv.second.v[1],
                   kv.second.v[2], kv.second.v[3]);
    const bool ok = std::fclose(f) == 0;
    return ok ? PSFD_OK : fail(PSFD_ERR_ARG, std::string("cannot write ") + path);
  });
}

psfd_status psfd_set_schedule(psfd_plan_t p, const int32_t* sched) {
  if (!p || p->is_batch || !sched) return fail(PSFD_ERR_ARG, "NULL argument or batch handle");
  for (int k = 0; k < 4; ++k)
    if (sched[k] < 0 || sched[k] > 3) return fail(PSFD_ERR_ARG, "schedule out of range");
  return guarded([&]() -> psfd_status {
    CHK(p->st ? hipStreamSynchronize(p->st) : hipDeviceSynchronize());
    drop_graphs(p);
    TuneVal v;
    for (int k = 0; k < 4; ++k) v.v[k] = sched[k];
    set_sched(p->t64, v);
    set_sched(p->t32, v);
    return PSFD_OK;
  });
}

psfd_status psfd_schedule(psfd_plan_t p, int32_t* sched) {
  if (!p || p->is_batch || !sched) return fail(PSFD_ERR_ARG, "NULL argument or batch handle");
  const bool f = p->prec != PSFD_C128;
  sched[0] = f ? p->t32.sched_xf : p->t64.sched_xf;
  sched[1] = f ? p->t32.sched_xi : p->t64.sched_xi;
  sched[2] = f ? p->t32.sched_y : p->t64.sched_y;
  sched[3] = f ? p->t32.sched_ax : p->t64.sched_ax;
  return PSFD_OK;
}

int64_t psfd_field_size(psfd_plan_t p) { return p ? p->nfield : 0; }

void psfd_destroy(psfd_plan_t p) {
  if (!p) return;
  if (p->st) (void)hipStreamSynchronize(p->st);
  else (void)hipDeviceSynchronize();
  delete p;
}

void psfd_trim_cache(void) { cache_trim(); }

const char* psfd_last_error(void) { return g_err.c_str(); }

}  // extern "C"
