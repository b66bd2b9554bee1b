// Host side of the F-statistic search library: plans, admission, launch
// orchestration, candidate drain, per-kernel timing.  C ABI in include/fstat.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/fstat.h"
#include "fstat_kernels.hpp"
#include "fstat_launch.hpp"
#include "fstat_drain.hpp"
#include "fstat_tmpl.hpp"
#include "fstat_vet.hpp"

using namespace fstat;

namespace {

thread_local std::string g_last_error;

constexpr int LOG_MIN = 10, LOG_MAX = 20;  // supported FFT lengths 2^10 .. 2^20

struct SegInfo {
  fstat_segment s;
  int nfft, M;                 // interpolated transform length and upsampling FFT length nfft/2
  int logL, P, Q;              // nfft = P * Q
  int PM, QM;                  // M = PM * QM
  int kmin, kmax;
  // the template FFTs: tL = nfft, or nfft/2 with interbinning; tL = tP * tQ
  int tlog, tP, tQ, tL;
  double ibw = 0.0;            // interbinning weight (0 without interbinning)
};

// The templates of one search call: nsky sky positions times nfdot spindowns, given
// either as an explicit spindown list or as the spindown integers of a lattice grid.
struct Grid {
  const double *alpha = nullptr, *delta = nullptr;
  int nsky = 0, nfdot = 0;
  const double* fdot = nullptr;                        // explicit list, or NULL on a lattice
  const double *w_freq = nullptr, *w_spin = nullptr;   // lattice: per-sky w0, w1 components
  int s_lo = 0;                                        // lattice: spindown integer of index 0
  double m10 = 0.0, m11 = 0.0;                         // lattice: w0, w1 of the spindown row
  bool operator==(const Grid& o) const {
    return alpha == o.alpha && delta == o.delta && nsky == o.nsky && nfdot == o.nfdot && fdot == o.fdot &&
           w_freq == o.w_freq && w_spin == o.w_spin && s_lo == o.s_lo && m10 == o.m10 && m11 == o.m11;
  }
};

struct SearchRecord {
  int nsky = 0, nfdot = 0;
  // pinned: alpha[nsky], delta[nsky], then fdot[nfdot] (explicit list) or
  // w_freq[nsky], w_spin[nsky] (lattice grid)
  double* host = nullptr;
  bool lattice = false;
  int s_lo = 0;
  double m10 = 0.0, m11 = 0.0;
};

struct ProfRec {
  int cls;
  hipEvent_t a, b;
  bool borrowed = false;   // owned by a graph entry, not by the event pool
};

// A captured search call, replayed while the call's arguments stay the same.
struct GraphEntry {
  int segment = 0, mode = 0;
  Grid grid;
  void* spectrum = nullptr;
  void* ws = nullptr;
  bool profiled = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<ProfRec> events;   // event pairs recorded by the graph's own nodes
};

struct Tables {
  void* dev = nullptr;         // one allocation for both precisions
  size_t off_tw1024[2] = {0, 0};
  size_t off_lo[2][LOG_MAX + 1] = {};
  size_t off_hi[2][LOG_MAX + 1] = {};
  size_t off_g[2] = {0, 0};
  size_t off_stage[2] = {0, 0};
  size_t bytes = 0;
};

}  // namespace

struct fstat_vet_s {
  int max_batch = 0;
  int n_cu = 256;                // compute units of the device (the convolution grid)
  int steps = 0;                 // Adam steps taken
  void* mem = nullptr;           // one allocation for everything below
  float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  uint16_t *wf2, *wt2, *wf3, *wt3, *w4b, *w5b;
  uint16_t *wq2, *wq3;           // convolution weights in matrix-core fragment order (inference)
  float *u, *z1, *z2, *z3, *z4, *z5, *a5, *logit, *dlogit, *lterm, *dz5, *dh4, *dx, *da, *dwm, *loss;
  float* scratch = nullptr;      // split-K partial tiles and reduction partials
  uint16_t *a1b, *a2b, *a3b, *a4b, *colA, *colB, *colC, *dz5b, *dz4b, *dzb;
  std::string last_error;
};

struct fstat_plan_s {
  std::vector<SegInfo> segs;
  fstat_options opt;
  bool fp64 = false;
  int device = 0;
  int Sb = 1, B = 1;           // skies per batch, templates per launch
  bool scale_B = true;         // B chosen by the library: shorter transforms take more per launch
  int variant_a = 1;           // pass A kernel variant (0 sequential series, 1 paired; the autotuner may pick 0)
  int variant_b = 1;           // pass B kernel variant (0 row tiles, 1 streaming wavefronts)
  int n_cu = 256;              // compute units of the device
  size_t cx_bytes = 8;
  // workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  // per-sky parameters and resampled series twice (the sky batch being prepared and the
  // one being searched), per-sky scratch, template intermediate
  size_t off_sp[2] = {0, 0}, off_part = 0, off_zt[2] = {0, 0}, off_sky = 0, off_tmpl = 0;
  size_t off_xs = 0;   // FP64 with interbinning: the second pass's transforms [B][tL][2]
  int nblk_max = 0;
  long n_max = 0, L_max = 0, M_max = 0;
  long TL_max = 0;             // longest template FFT
  // tables and candidates
  Tables tab;
  CandEntry* d_cand = nullptr;
  unsigned long long* d_count = nullptr;
  int* d_search_next = nullptr;   // device copy of the search index (advanced by the search itself)
  double* d_sky_pos = nullptr;    // (alpha, delta) of fstat_sky_stages
  int search_count = 0;
  // graph replay: a plan-owned stream joined to the caller's stream by events
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // the per-sky stage of the next sky batch runs on its own stream (default priority)
  // while the current batch's templates run; events order the two and the buffers
  hipStream_t sstream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_sky[2] = {nullptr, nullptr}, ev_tmpl[2] = {nullptr, nullptr};
  std::vector<GraphEntry> graphs;
  // candidate vetting: patch capture after the F kernel
  fstat_vet_t vet = nullptr;
  long long patch_capacity = 0;
  float* d_patches = nullptr;    // [patch_capacity][256]
  float* d_spec = nullptr;       // the current launch's 2F rows [B][k_max - k_min]
  unsigned long long* d_first = nullptr;
  bool scored = false;
  std::vector<SearchRecord> searches;
  // device memory of the key-ordering drain (grown on demand, kept until destroy)
  void* drain_ws = nullptr;
  size_t drain_bytes = 0;
  void* drain_out = nullptr;     // records, keys and lists formed on the device
  size_t drain_out_bytes = 0;
  hipStream_t last_stream = nullptr;
  bool used_stream = false;
  // profiling
  bool profiling = false;
  // every launch on the caller's stream (no sky stream, no events): the static-scratch call
  bool single_stream = false;
  // this device's copy of the static scratch (address taken when the plan was made)
  void* static_ws = nullptr;
  std::string static_err;
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfRec> prof;
  std::string last_error;
};

// ------------------------------------------------------------------ helpers
static fstat_status fail(fstat_plan_t plan, fstat_status st, const std::string& msg) {
  if (plan) plan->last_error = msg;
  else g_last_error = msg;
  return st;
}

// ------------------------------------------------------------- launch checks
// Every launch goes through FSTAT_LAUNCH: its grid, workgroup and LDS are checked on the
// host (launch_problem) against the device's limits and the kernel's compiled maximum
// workgroup size and static LDS, read once per kernel and device.  A launch outside them
// is not dispatched: it is refused, later launches on this thread are refused too until
// launch_status() reports the refusal (as hipErrorInvalidConfiguration; the text names the
// kernel and the limit), so that no kernel runs on the results of one that did not.
constexpr int MAX_DEVICES = 64;
static thread_local bool g_refused = false;
static thread_local std::string g_refusal, g_last_refusal;
static thread_local bool g_dlim_ok[MAX_DEVICES] = {};
static thread_local DeviceLaunchLimits g_dlim[MAX_DEVICES];
static thread_local std::unordered_map<const void*, KernelLaunchLimits> g_klim[MAX_DEVICES];

static bool read_launch_limits(const void* fn, DeviceLaunchLimits* d, KernelLaunchLimits* k) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return false;
  if (!g_dlim_ok[dev]) {
    DeviceLaunchLimits lim;
    auto get = [&](hipDeviceAttribute_t a, int64_t* out) {
      int v = 0;
      if (hipDeviceGetAttribute(&v, a, dev) == hipSuccess && v > 0) *out = v;
    };
    get(hipDeviceAttributeMaxThreadsPerBlock, &lim.max_threads_per_block);
    get(hipDeviceAttributeMaxBlockDimX, &lim.max_block[0]);
    get(hipDeviceAttributeMaxBlockDimY, &lim.max_block[1]);
    get(hipDeviceAttributeMaxBlockDimZ, &lim.max_block[2]);
    get(hipDeviceAttributeMaxGridDimX, &lim.max_grid[0]);
    get(hipDeviceAttributeMaxGridDimY, &lim.max_grid[1]);
    get(hipDeviceAttributeMaxGridDimZ, &lim.max_grid[2]);
    get(hipDeviceAttributeMaxSharedMemoryPerBlock, &lim.max_lds_per_block);
    g_dlim[dev] = lim;
    g_dlim_ok[dev] = true;
  }
  *d = g_dlim[dev];
  auto it = g_klim[dev].find(fn);
  if (it == g_klim[dev].end()) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, fn) != hipSuccess) return false;
    KernelLaunchLimits kl;
    if (a.maxThreadsPerBlock > 0) kl.max_threads_per_block = a.maxThreadsPerBlock;
    kl.static_lds = (int64_t)a.sharedSizeBytes;
    it = g_klim[dev].emplace(fn, kl).first;
  }
  *k = it->second;
  return true;
}

static bool launch_allowed(const void* fn, const char* name, dim3 g, dim3 b, long long dyn_lds) {
  if (g_refused) return false;
  DeviceLaunchLimits d;
  KernelLaunchLimits k;
  if (!read_launch_limits(fn, &d, &k)) return true;   // limits unknown: the runtime decides
  const int64_t grid[3] = {g.x, g.y, g.z}, block[3] = {b.x, b.y, b.z};
  const std::string why = launch_problem(d, k, grid, block, dyn_lds);
  if (why.empty()) return true;
  g_refused = true;
  g_refusal = std::string(name) + ": " + why;
  return false;
}

// The status of the launches since the last call: a refusal, else the runtime's last error.
static hipError_t launch_status() {
  if (g_refused) {
    g_refused = false;
    g_last_refusal = g_refusal;
    return hipErrorInvalidConfiguration;
  }
  return hipGetLastError();
}

// Text of a HIP error, with the refused launch when the error is a refusal.
static std::string hip_error_text(hipError_t e) {
  std::string t = hipGetErrorString(e);
  if (e == hipErrorInvalidConfiguration && !g_last_refusal.empty()) {
    t += " (launch refused before dispatch, " + g_last_refusal + ")";
    g_last_refusal.clear();
  }
  return t;
}

#define FSTAT_LAUNCH(kernel, grid, block, lds, stream, ...)                                                    \
  do {                                                                                                          \
    if (launch_allowed(reinterpret_cast<const void*>(&kernel), #kernel, dim3(grid), dim3(block), (long long)(lds))) \
      hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);                                        \
  } while (0)

static fstat_status hip_fail(fstat_plan_t plan, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hip_error_text(e);
  return fail(plan, e == hipErrorOutOfMemory ? FSTAT_E_NOMEM : FSTAT_E_DEVICE, msg);
}

#define HIP_TRY(plan, expr, what)                  \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(plan, e_, what); \
  } while (0)

static int ilog2_exact(long v) {
  int e = 0;
  while ((1L << e) < v) ++e;
  return ((1L << e) == v) ? e : -1;
}

static long next_pow2(long v) {
  long m = 1;
  while (m < v) m <<= 1;
  return m;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

template <typename F>
static void with_len(int len, F&& f) {
  switch (len) {
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    case 1024: f(std::integral_constant<int, 1024>{}); break;
    default: break;
  }
}

template <typename T>
static int tw_of(int len) {
  int tw = 0;
  with_len(len, [&](auto c) { tw = tile_width<T, decltype(c)::value>(); });
  return tw;
}

// Interbinning whose second pass is the tiled kernel plus a separate 2F pass: FP64, and
// mixed precision for template transforms with P > 512 rows' length (nfft = 2^20).
static bool tiled_interbinning(fstat_plan_t p) {
  if (!p->opt.interbinning) return false;
  if (p->fp64) return true;
  for (const SegInfo& si : p->segs)
    if (si.tP > 512) return true;
  return false;
}

// Workspace layout for Sb skies and B templates (bytes).
static size_t layout(fstat_plan_t p, int Sb, int B, bool commit) {
  const size_t cx = p->cx_bytes;
  size_t off = 0;
  size_t o_sp[2], o_zt[2];
  for (int k = 0; k < 2; ++k) {
    o_sp[k] = off;
    off = align256(off + (size_t)Sb * sizeof(SkyParams));
  }
  const size_t o_part = off;
  off = align256(off + (size_t)Sb * p->nblk_max * 3 * sizeof(double));
  for (int k = 0; k < 2; ++k) {
    o_zt[k] = off;
    off = align256(off + (size_t)Sb * 2 * p->n_max * cx);
  }
  // per-sky scratch: za [2][M], Z [2][M], tmp [2][L], u [2][L] per sky
  const size_t o_sky = off;
  off = align256(off + (size_t)Sb * (4 * p->M_max + 4 * p->L_max) * cx);
  // template intermediate [B][tL][2]
  const size_t o_tmpl = off;
  off = align256(off + (size_t)B * 2 * p->TL_max * cx);
  // interbinning through the tiled second pass (FP64, or P > 512): the transforms
  // themselves, for the interbinning epilogue
  const size_t o_xs = off;
  if (tiled_interbinning(p)) off = align256(off + (size_t)B * 2 * p->TL_max * cx);
  if (commit) {
    for (int k = 0; k < 2; ++k) {
      p->off_sp[k] = o_sp[k];
      p->off_zt[k] = o_zt[k];
    }
    p->off_part = o_part;
    p->off_sky = o_sky;
    p->off_tmpl = o_tmpl;
    p->off_xs = o_xs;
  }
  return off;
}

template <typename T>
static void fill_tables(std::vector<unsigned char>& buf, Tables& tb, int which, int kt) {
  auto put = [&](size_t count) {
    size_t off = align256(buf.size());
    buf.resize(off + count * sizeof(cx<T>));
    return off;
  };
  auto wexp = [](long m, long L) {
    // exp(-2 pi i m / L) evaluated in double precision, then rounded to T
    const double a = 2.0 * M_PI * (double)m / (double)L;
    cx<T> w;
    w.re = (T)std::cos(a);
    w.im = (T)(-std::sin(a));
    return w;
  };
  size_t o = put(1024);
  tb.off_tw1024[which] = o;
  for (int m = 0; m < 1024; ++m) reinterpret_cast<cx<T>*>(buf.data() + o)[m] = wexp(m, 1024);
  for (int e = LOG_MIN; e <= LOG_MAX; ++e) {
    const long L = 1L << e;
    size_t lo = put(1024);
    tb.off_lo[which][e] = lo;
    for (int m = 0; m < 1024; ++m) reinterpret_cast<cx<T>*>(buf.data() + lo)[m] = wexp(m, L);
    const long nh = std::max(1L, L / 1024);
    size_t hi = put(nh);
    tb.off_hi[which][e] = hi;
    for (long m = 0; m < nh; ++m) reinterpret_cast<cx<T>*>(buf.data() + hi)[m] = wexp((1024 * m) % L, L);
  }
  // per-stage twiddles [k][r-1] of the template kernels (layout of stage_tw_offset)
  size_t os = put(STAGE_TW_ENTRIES);
  tb.off_stage[which] = os;
  for (int ns = 8; ns <= 512; ns *= 8)
    for (int rr = 2; rr <= 8; rr *= 2)
      for (int k = 0; k < ns; ++k)
        for (int r = 1; r < rr; ++r)
          reinterpret_cast<cx<T>*>(buf.data() + os)[stage_tw_offset(ns, rr) + k * (rr - 1) + (r - 1)] =
              wexp((long)k * r, (long)ns * rr);
  size_t og = align256(buf.size());
  buf.resize(og + (kt + 1) * sizeof(T));
  tb.off_g[which] = og;
  const double z = std::sqrt(3.0) - 2.0;
  for (int k = 0; k <= kt; ++k)
    reinterpret_cast<T*>(buf.data() + og)[k] = (T)(std::pow(z, k) / (2.0 * std::sqrt(3.0)));
}

constexpr int KT_F32 = 16, KT_F64 = 32;

static SegConst seg_const(const SegInfo& si) {
  SegConst sc;
  sc.n = (int)si.s.n;
  sc.nfft = si.nfft;
  sc.dt = si.s.dt;
  sc.f_off = si.s.f_off;
  sc.sigma2 = si.s.sigma2;
  sc.lat = si.s.lat;
  sc.gamma = si.s.gamma;
  sc.phi_r = si.s.phi_r;
  sc.x = si.s.x;
  sc.r = si.s.r_ssb;
  return sc;
}

// ------------------------------------------------------------- static scratch
// Device memory of the entry point that allocates nothing (fstat_twoF_spectrum_static):
// the search workspace of one call, in a static array of which each GPU the library runs
// on holds its own copy until the process ends.  Host code never uses the array's name
// as an address: the address of this device's copy comes from hipGetSymbolAddress, once
// per device with that device current (static_scratch_address), and is kept per device.
static __device__ __align__(256) unsigned char scratch[FSTAT_STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES] = {};

static hipError_t static_scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// ------------------------------------------------------------- profiling
static hipEvent_t take_event(fstat_plan_t p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  fstat_plan_t p;
  int cls;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(fstat_plan_t p_, int cls_, hipStream_t st_) : p(p_), cls(cls_), st(st_) {
    if (p->profiling) {
      a = take_event(p);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (p->profiling && a) {
      hipEvent_t b = take_event(p);
      if (b) {
        (void)hipEventRecord(b, st);
        p->prof.push_back({cls, a, b, false});
      } else {
        p->ev_pool.push_back(a);
      }
    }
  }
};

// ------------------------------------------------------------- launches
template <typename T>
struct Dev {
  fstat_plan_t p;
  const cx<T>* tw1024;
  const cx<T>* twst;
  const T* g;
  const cx<T>* lo(int e) const {
    return (const cx<T>*)((const char*)p->tab.dev + p->tab.off_lo[sizeof(T) == 8][e]);
  }
  const cx<T>* hi(int e) const {
    return (const cx<T>*)((const char*)p->tab.dev + p->tab.off_hi[sizeof(T) == 8][e]);
  }
  explicit Dev(fstat_plan_t p_) : p(p_) {
    const int w = sizeof(T) == 8;
    tw1024 = (const cx<T>*)((const char*)p->tab.dev + p->tab.off_tw1024[w]);
    g = (const T*)((const char*)p->tab.dev + p->tab.off_g[w]);
    twst = (const cx<T>*)((const char*)p->tab.dev + p->tab.off_stage[w]);
  }
  int buf = 0;   // which of the two per-sky buffers
  SkyParams* sp() const { return (SkyParams*)((char*)p->ws + p->off_sp[buf]); }
  double* part() const { return (double*)((char*)p->ws + p->off_part); }
  cx<T>* zt() const { return (cx<T>*)((char*)p->ws + p->off_zt[buf]); }
  cx<T>* sky() const { return (cx<T>*)((char*)p->ws + p->off_sky); }
  cx<T>* tmpl() const { return (cx<T>*)((char*)p->ws + p->off_tmpl); }
  cx<T>* xs() const { return (cx<T>*)((char*)p->ws + p->off_xs); }
};

// forward or inverse L-point FFT of `items` pairs of series, two passes
template <typename T, bool INV, int SRC>
static hipError_t fft_two_pass(const Dev<T>& d, int logL, int P, int Q, const cx<T>* in, long ld_in,
                               int nvalid, cx<T>* tmp, cx<T>* out, long ld_out, int items, T scale,
                               hipStream_t st, const cx<T>* shlo = nullptr, const cx<T>* shhi = nullptr) {
  const int L = 1 << logL;
  hipError_t err = hipSuccess;
  with_len(Q, [&](auto c) {
    constexpr int QQ = decltype(c)::value;
    const int ntiles = P / tile_width<T, QQ>();
    FSTAT_LAUNCH((k_fft_pass_a<T, QQ, INV, SRC>), dim3(ntiles * items), dim3(NT), 0, st, in, ld_in,
                       nvalid, tmp, P, L, d.tw1024, d.lo(logL), d.hi(logL), shlo, shhi);
    err = launch_status();
  });
  if (err != hipSuccess) return err;
  with_len(P, [&](auto c) {
    constexpr int PP = decltype(c)::value;
    const int ntiles = Q / tile_width<T, PP>();
    FSTAT_LAUNCH((k_fft_pass_b<T, PP, INV>), dim3(ntiles * items), dim3(NT), 0, st, tmp, out, ld_out, Q,
                       L, scale, d.tw1024);
    err = launch_status();
  });
  return err;
}

// Per-sky stage for skies [sky0, sky0 + nb) of segment si; leaves zt and SkyParams.
template <typename T>
static fstat_status run_sky_batch(fstat_plan_t p, const Dev<T>& d, const SegInfo& si, const double* alpha,
                                  const double* delta, int sky0, int nb, hipStream_t st) {
  const SegConst sc = seg_const(si);
  const int n = sc.n, L = si.nfft, M = si.M;
  const int nblk = (n + NT - 1) / NT;
  cx<T>* za = d.sky();                             // [nb][2][M]
  cx<T>* Z = za + (size_t)nb * 2 * M;              // [nb][2][M]
  cx<T>* tmp = Z + (size_t)nb * 2 * M;             // [nb][2][L] (M used)
  cx<T>* o = tmp + (size_t)nb * 2 * L;             // [nb][2][M]: odd samples of the 2x upsampling
  {
    ProfScope ps(p, FSTAT_KERNEL_SKY_PREP, st);
    FSTAT_LAUNCH(k_sky_setup, dim3((nb + 63) / 64), dim3(64), 0, st, alpha, delta, sky0, nb, sc, d.sp());
    FSTAT_LAUNCH((k_sky_demod<T>), dim3(nblk, nb), dim3(NT), 0, st, sc, d.sp(), za, (long)M, d.part());
    FSTAT_LAUNCH(k_sky_finalize, dim3(nb), dim3(NT), 0, st, sc, d.sp(), d.part(), nblk,
                       p->opt.form == FSTAT_FORM_FULL ? 1 : 0);
    HIP_TRY(p, launch_status(), "sky stage launch");
  }
  {
    ProfScope ps(p, FSTAT_KERNEL_RESAMPLE, st);
    HIP_TRY(p, (fft_two_pass<T, false, SRC_PLAIN>(d, si.logL - 1, si.PM, si.QM, za, M, n, tmp, Z, M, nb, (T)1, st)),
            "upsampling forward FFT");
    // 2x band-limited upsampling: the even samples are za itself, the odd ones the inverse
    // M-point transform of the spectrum shifted by half a sample
    HIP_TRY(p, (fft_two_pass<T, true, SRC_HALFSHIFT>(d, si.logL - 1, si.PM, si.QM, Z, M, 0, tmp, o, M, nb,
                                                      (T)(1.0 / M), st, d.lo(si.logL), d.hi(si.logL))),
            "upsampling inverse FFT");
    constexpr int KT = sizeof(T) == 8 ? KT_F64 : KT_F32;
    FSTAT_LAUNCH((k_spline<T, KT>), dim3(nblk, nb), dim3(NT), 0, st, sc, d.sp(), za, o, (long)M, d.zt(),
                       (long)n, d.g);
    HIP_TRY(p, launch_status(), "spline launch");
  }
  return FSTAT_OK;
}

// Template stage for the nb skies of the current batch: nb * nfdot templates in launches of B.
// workgroups per compute unit of the streaming second pass.  Its LDS and registers allow
// four; three wavefronts per SIMD read the interleaved intermediate faster on MI355X
// (0.70 against 0.75 us per 2^18-point template), and grids between three and four per
// CU are slower still (uneven CUs).
constexpr int STREAM_WG_PER_CU = 3;
// the interbinning second pass holds two units' outputs per lane: with the bins [0, nfft/2)
// (half the outputs) it needs 135-165 VGPRs and three workgroups per CU are resident, with
// other bin ranges 190-225 and two
constexpr int IB_WG_PER_CU_HALF = 3, IB_WG_PER_CU_FULL = 2;
// the streaming second pass for rows of 1024 points: one row (two wavefronts) per
// workgroup, and six workgroups per compute unit (its 141-155 VGPRs leave three wavefronts
// per SIMD; two rows per 256-thread workgroup ran 1% slower)
constexpr int STREAM2_NT = 128;
constexpr int STREAM2_WG_PER_CU = 3 * 256 / STREAM2_NT;

template <typename T>
static fstat_status run_templates(fstat_plan_t p, const Dev<T>& d, const SegInfo& si, int sky0, int nb,
                                  const Grid& g, int mode, OutArgs oa, hipStream_t st) {
  const int nfdot = g.nfdot;
  TmplArgs ta;
  ta.n = (int)si.s.n;
  ta.P = si.tP;
  ta.Q = si.tQ;
  ta.L = si.tL;
  ta.ibw = (float)si.ibw;
  ta.nfdot = nfdot;
  ta.sky0 = sky0;
  ta.dt = si.s.dt;
  ta.fdot = g.fdot;
  ta.ldzt = si.s.n;
  ta.w_freq = g.w_freq;
  ta.w_spin = g.w_spin;
  ta.m10 = g.m10;
  ta.m11 = g.m11;
  ta.bins_per_rad = (double)si.nfft / (2.0 * M_PI);
  ta.s_lo = g.s_lo;
  ta.nfft = si.nfft;
  const int total = nb * nfdot;
  cx<T>* tbuf = d.tmpl();
  // the plan's B templates per launch are sized for its longest transform; when the
  // library chose B, a segment with a shorter transform fits proportionally more templates
  // in the same intermediate memory (and in the launch-sized 2F rows of the patch capture),
  // so it takes fewer, fuller launches
  const int Bs = p->scale_B ? (int)std::min<long>((long)p->B * (p->TL_max / si.tL), 4096L) : p->B;
  for (int t0 = 0; t0 < total; t0 += Bs) {
    const int nt = std::min(Bs, total - t0);
    ta.t0 = t0;
    hipError_t err = hipSuccess;
    {
      ProfScope ps(p, FSTAT_KERNEL_TEMPLATE_A, st);
      with_len(si.tQ, [&](auto c) {
        constexpr int QQ = decltype(c)::value;
        if constexpr (QQ >= 64) {
          const int ntiles = si.tP / tw_a<T, QQ>();
          // first-stage inputs r >= rnz are zero for every column when n <= rnz tL / 8
          int rnz = 8;
          for (int r = 7; r >= 3; --r)
            if (8L * si.s.n <= (long)r * si.tL) rnz = r;
          auto go = [&](auto rnz_c) {
            constexpr int RZ = decltype(rnz_c)::value;
            if (p->variant_a == 1)
              FSTAT_LAUNCH((k_tmpl_a_pair<T, QQ, RZ>), dim3(ntiles * nt), dim3(tmpl_nt_a<T, QQ>()), 0, st, ta,
                                 d.zt(), tbuf, d.twst, d.lo(si.tlog), d.hi(si.tlog));
            else
              FSTAT_LAUNCH((k_tmpl_a<T, QQ, RZ>), dim3(ntiles * nt), dim3(tmpl_nt_a<T, QQ>()), 0, st, ta, d.zt(),
                                 tbuf, d.twst, d.lo(si.tlog), d.hi(si.tlog));
          };
          switch (rnz) {
            case 3: go(std::integral_constant<int, 3>{}); break;
            case 4: go(std::integral_constant<int, 4>{}); break;
            case 5: go(std::integral_constant<int, 5>{}); break;
            case 6: go(std::integral_constant<int, 6>{}); break;
            case 7: go(std::integral_constant<int, 7>{}); break;
            default: go(std::integral_constant<int, 8>{}); break;
          }
          err = launch_status();
        } else {
          err = hipErrorInvalidValue;
        }
      });
    }
    HIP_TRY(p, err, "template pass A launch");
    const bool capture = (mode == 0 && p->vet != nullptr);
    if (capture) {
      FSTAT_LAUNCH(k_record_count, dim3(1), dim3(1), 0, st, p->d_count, p->d_first);
      oa.spectrum = p->d_spec;
    }
    {
      ProfScope ps(p, FSTAT_KERNEL_TEMPLATE_B, st);
      with_len(si.tP, [&](auto c) {
        constexpr int PP = decltype(c)::value;
        if constexpr (sizeof(T) == 4 && PP >= 64 && PP <= 512) {
          if (si.ibw != 0.0) {
            // interbinning: about one resident round of wavefronts walking chunks of row units
            const long units = si.tQ / stream_rpw<PP>();
            const long chunks = (long)nt * (units / std::min<long>(units, IB_CHUNK));
            const bool half = (oa.k_min == 0 && oa.k_max == si.nfft / 2);
            const long wgs = std::min((chunks + 3) / 4, (long)p->n_cu * (half ? IB_WG_PER_CU_HALF : IB_WG_PER_CU_FULL));
            auto go = [&](auto mode_c, auto half_c) {
              constexpr int MD = decltype(mode_c)::value;
              constexpr bool HF = decltype(half_c)::value;
              FSTAT_LAUNCH((k_tmpl_b_ib<PP, MD, HF>), dim3((unsigned)wgs), dim3(256), 0, st, ta, nt, d.sp(),
                                 (const cx<float>*)tbuf, oa, (const cx<float>*)d.twst);
            };
            using BT = std::true_type;
            using BF = std::false_type;
            if (capture) half ? go(std::integral_constant<int, 2>{}, BT{}) : go(std::integral_constant<int, 2>{}, BF{});
            else if (mode == 0) half ? go(std::integral_constant<int, 0>{}, BT{}) : go(std::integral_constant<int, 0>{}, BF{});
            else half ? go(std::integral_constant<int, 1>{}, BT{}) : go(std::integral_constant<int, 1>{}, BF{});
            err = launch_status();
            return;
          }
          if (p->variant_b == 1) {
          // streaming kernel: about one resident round of wavefronts walks the launch's row units
          const long waves = (long)nt * (si.tQ / stream_rpw<PP>());
          const long wgs = std::min((waves + 3) / 4, (long)p->n_cu * STREAM_WG_PER_CU);
          const dim3 grid((unsigned)wgs);
          const bool half = (oa.k_min == 0 && oa.k_max == si.nfft / 2);
          auto go = [&](auto mode_c, auto half_c) {
            constexpr int MD = decltype(mode_c)::value;
            constexpr bool HF = decltype(half_c)::value;
            FSTAT_LAUNCH((k_tmpl_b_stream<T, PP, MD, HF>), grid, dim3(256), 0, st, ta, nt, d.sp(), tbuf, oa,
                               d.twst);
          };
          using I0 = std::integral_constant<int, 0>;
          using I1 = std::integral_constant<int, 1>;
          using I2 = std::integral_constant<int, 2>;
          using BT = std::true_type;
          using BF = std::false_type;
          if (capture) half ? go(I2{}, BT{}) : go(I2{}, BF{});
          else if (mode == 0) half ? go(I0{}, BT{}) : go(I0{}, BF{});
          else half ? go(I1{}, BT{}) : go(I1{}, BF{});
          err = launch_status();
          return;
          }
        }
        if constexpr (sizeof(T) == 4 && PP == 1024) {
          if (si.ibw == 0.0 && p->variant_b == 1 && !capture) {
            // rows of 1024 points, two wavefronts each: about one resident round of
            // workgroups walks the launch's units of two rows
            constexpr int NT2 = STREAM2_NT;
            const long units = (long)nt * (si.tQ / (NT2 / groups_per_col<PP>()));
            const long wgs = std::min(units, (long)p->n_cu * STREAM2_WG_PER_CU);
            const bool half = (oa.k_min == 0 && oa.k_max == si.nfft / 2);
            auto go = [&](auto mode_c, auto half_c) {
              constexpr int MD = decltype(mode_c)::value;
              constexpr bool HF = decltype(half_c)::value;
              FSTAT_LAUNCH((k_tmpl_b_stream2<MD, HF, NT2>), dim3((unsigned)wgs), dim3(NT2), 0, st, ta, nt, d.sp(),
                           tbuf, oa, d.twst);
            };
            using I0 = std::integral_constant<int, 0>;
            using I1 = std::integral_constant<int, 1>;
            using BT = std::true_type;
            using BF = std::false_type;
            if (mode == 0) half ? go(I0{}, BT{}) : go(I0{}, BF{});
            else half ? go(I1{}, BT{}) : go(I1{}, BF{});
            err = launch_status();
            return;
          }
        }
        if constexpr (PP >= 64) {
          const int ntiles = si.tQ / tw_b<T, PP>();
          if (si.ibw != 0.0) {
            // interbinning through the tiled pass (FP64, or P > 512): it stores the
            // transforms, then an epilogue forms the interbinned 2F of the launch's templates
            OutArgs ox = oa;
            ox.spectrum = d.xs();
            FSTAT_LAUNCH((k_tmpl_b<T, PP, 3>), dim3(ntiles * nt), dim3(tmpl_nt_b<T, PP>()), 0, st, ta, d.sp(),
                               tbuf, ox, d.twst);
            err = launch_status();
            if (err != hipSuccess) return;
            const int kc0 = oa.k_min / 2, nkc = (oa.k_max + 1) / 2 - kc0;
            const dim3 grid((unsigned)((nkc + 255) / 256), (unsigned)nt);
            const cx<T>* xs = d.xs();
            if (capture)
              FSTAT_LAUNCH((k_interbin_2f<T, 2>), grid, dim3(256), 0, st, ta, d.sp(), xs, oa, si.ibw, kc0, nkc);
            else if (mode == 0)
              FSTAT_LAUNCH((k_interbin_2f<T, 0>), grid, dim3(256), 0, st, ta, d.sp(), xs, oa, si.ibw, kc0, nkc);
            else
              FSTAT_LAUNCH((k_interbin_2f<T, 1>), grid, dim3(256), 0, st, ta, d.sp(), xs, oa, si.ibw, kc0, nkc);
            err = launch_status();
            return;
          }
          if (capture)
            FSTAT_LAUNCH((k_tmpl_b<T, PP, 2>), dim3(ntiles * nt), dim3(tmpl_nt_b<T, PP>()), 0, st, ta, d.sp(),
                               tbuf, oa, d.twst);
          else if (mode == 0)
            FSTAT_LAUNCH((k_tmpl_b<T, PP, 0>), dim3(ntiles * nt), dim3(tmpl_nt_b<T, PP>()), 0, st, ta, d.sp(),
                               tbuf, oa, d.twst);
          else
            FSTAT_LAUNCH((k_tmpl_b<T, PP, 1>), dim3(ntiles * nt), dim3(tmpl_nt_b<T, PP>()), 0, st, ta, d.sp(),
                               tbuf, oa, d.twst);
          err = launch_status();
        } else {
          err = hipErrorInvalidValue;
        }
      });
    }
    HIP_TRY(p, err, "template pass B launch");
    if (capture) {
      // the streaming second pass stores its rows transposed (k_tmpl_b_stream)
      const bool transposed = !p->fp64 && si.ibw == 0.0 && p->variant_b == 1 && si.tP >= 64 && si.tP <= 512;
      const bool half = (oa.k_min == 0 && oa.k_max == si.nfft / 2);
      const int tq = transposed ? si.tQ : 0, trow = transposed ? (half ? si.tP / 2 : si.tP) : 0;
      FSTAT_LAUNCH(k_capture_patches, dim3(2048), dim3(256), 0, st, p->d_cand, p->d_spec, p->d_patches,
                   (unsigned long long)p->patch_capacity, p->d_count, p->d_first, oa.k_min, oa.k_max, t0, nfdot, sky0,
                   tq, trow);
      HIP_TRY(p, launch_status(), "patch capture launch");
    }
  }
  return FSTAT_OK;
}

static fstat_status ensure_workspace(fstat_plan_t p) {
  if (p->ws) return FSTAT_OK;
  const size_t need = layout(p, p->Sb, p->B, true);
  void* w = nullptr;
  HIP_TRY(p, hipMalloc(&w, need), "workspace allocation");
  p->ws = w;
  p->ws_bytes = need;
  p->ws_owned = true;
  return FSTAT_OK;
}

template <typename T>
static fstat_status search_impl(fstat_plan_t p, int segment, const Grid& g, int mode, void* spectrum,
                                hipStream_t st) {
  const int nsky = g.nsky;
  Dev<T> d(p);
  OutArgs oa;
  oa.threshold = p->opt.threshold_2F;
  oa.search_next = p->d_search_next;
  oa.cand = p->d_cand;
  oa.count = p->d_count;
  oa.capacity = p->opt.candidate_capacity;
  oa.spectrum = spectrum;
  const int s0 = segment < 0 ? 0 : segment;
  const int s1 = segment < 0 ? (int)p->segs.size() : segment + 1;
  for (int s = s0; s < s1; ++s) {
    const SegInfo& si = p->segs[s];
    oa.segment = s;
    oa.k_min = si.kmin;
    oa.k_max = si.kmax;
    // Sky batch b is prepared on the plan's sky stream into buffer b % 2 while batch b - 1
    // is searched on `st`: the sky stream waits for the templates of batch b - 2 (the last
    // reader of that buffer), the templates of batch b for its sky stage.  With per-launch
    // profiling on, the sky stage stays on `st`, so that each timed kernel runs alone.
    const int nbatch = (nsky + p->Sb - 1) / p->Sb;
    hipStream_t sst = (p->profiling || p->single_stream) ? st : p->sstream;
    if (sst != st) {
      HIP_TRY(p, hipEventRecord(p->ev_fork, st), "sky stream fork");
      HIP_TRY(p, hipStreamWaitEvent(sst, p->ev_fork, 0), "sky stream fork");
    }
    auto sky_stage = [&](int b) -> fstat_status {
      Dev<T> db = d;
      db.buf = b & 1;
      if (b >= 2 && sst != st) HIP_TRY(p, hipStreamWaitEvent(sst, p->ev_tmpl[b & 1], 0), "sky stream order");
      const int sky0 = b * p->Sb;
      fstat_status r = run_sky_batch<T>(p, db, si, g.alpha, g.delta, sky0, std::min(p->Sb, nsky - sky0), sst);
      if (r != FSTAT_OK) return r;
      if (sst != st) HIP_TRY(p, hipEventRecord(p->ev_sky[b & 1], sst), "sky stream order");
      return FSTAT_OK;
    };
    fstat_status r = sky_stage(0);
    if (r != FSTAT_OK) return r;
    for (int b = 0; b < nbatch; ++b) {
      if (sst != st) {
        if (b + 1 < nbatch && (r = sky_stage(b + 1)) != FSTAT_OK) return r;
        HIP_TRY(p, hipStreamWaitEvent(st, p->ev_sky[b & 1], 0), "sky stream join");
      } else if (b > 0 && (r = sky_stage(b)) != FSTAT_OK) {
        return r;
      }
      Dev<T> db = d;
      db.buf = b & 1;
      const int sky0 = b * p->Sb;
      r = run_templates<T>(p, db, si, sky0, std::min(p->Sb, nsky - sky0), g, mode, oa, st);
      if (r != FSTAT_OK) return r;
      if (sst != st) HIP_TRY(p, hipEventRecord(p->ev_tmpl[b & 1], st), "sky stream order");
    }
  }
  return FSTAT_OK;
}

// All launches of one search call (begin-search marker first).
static fstat_status enqueue_search(fstat_plan_t p, int segment, const Grid& g, int mode, void* spectrum,
                                   hipStream_t st) {
  if (!p->sstream && !p->single_stream) {
    HIP_TRY(p, hipStreamCreateWithFlags(&p->sstream, hipStreamNonBlocking), "sky stream");
    HIP_TRY(p, hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming), "sky stream event");
    for (int k = 0; k < 2; ++k) {
      HIP_TRY(p, hipEventCreateWithFlags(&p->ev_sky[k], hipEventDisableTiming), "sky stream event");
      HIP_TRY(p, hipEventCreateWithFlags(&p->ev_tmpl[k], hipEventDisableTiming), "sky stream event");
    }
  }
  if (mode == 0) {
    FSTAT_LAUNCH(k_begin_search, dim3(1), dim3(1), 0, st, p->d_search_next);
    HIP_TRY(p, launch_status(), "search marker launch");
  }
  return p->fp64 ? search_impl<double>(p, segment, g, mode, spectrum, st)
                 : search_impl<float>(p, segment, g, mode, spectrum, st);
}

// Eagerly, or as a captured HIP graph that is replayed while the call's arguments are
// unchanged.  Graphs run on a plan-owned stream (default priority) that waits for the
// caller's stream and that the caller's stream then waits for, so the call stays
// asynchronous and ordered on the caller's stream.
static fstat_status run_search(fstat_plan_t p, int segment, const Grid& grid, int mode, void* spectrum,
                               hipStream_t st) {
  // per-launch event timing needs eager launches (events recorded by graph nodes do not
  // report elapsed times)
  if (!p->opt.use_graph || p->profiling)
    return enqueue_search(p, segment, grid, mode, spectrum, st);
  if (!p->gstream) {
    HIP_TRY(p, hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking), "graph stream");
    HIP_TRY(p, hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming), "graph event");
    HIP_TRY(p, hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming), "graph event");
  }
  GraphEntry* ge = nullptr;
  for (auto& g : p->graphs)
    if (g.segment == segment && g.grid == grid && g.mode == mode && g.spectrum == spectrum && g.ws == p->ws &&
        g.profiled == p->profiling)
      ge = &g;
  HIP_TRY(p, hipEventRecord(p->ev_in, st), "graph join");
  HIP_TRY(p, hipStreamWaitEvent(p->gstream, p->ev_in, 0), "graph join");
  if (!ge) {
    GraphEntry g;
    g.segment = segment;
    g.grid = grid;
    g.mode = mode;
    g.spectrum = spectrum;
    g.ws = p->ws;
    g.profiled = p->profiling;
    const size_t nprof = p->prof.size();
    HIP_TRY(p, hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal), "graph capture");
    fstat_status r = enqueue_search(p, segment, grid, mode, spectrum, p->gstream);
    hipError_t ec = hipStreamEndCapture(p->gstream, &g.graph);
    // the event pairs recorded during capture belong to the graph's nodes
    g.events.assign(p->prof.begin() + nprof, p->prof.end());
    p->prof.resize(nprof);
    if (r != FSTAT_OK) {
      if (g.graph) (void)hipGraphDestroy(g.graph);
      return r;
    }
    if (ec != hipSuccess) return hip_fail(p, ec, "graph capture");
    hipError_t ei = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g.graph);
      return hip_fail(p, ei, "graph instantiate");
    }
    if (p->graphs.size() >= 4) {
      GraphEntry& old = p->graphs.front();
      (void)hipStreamSynchronize(p->gstream);
      (void)hipGraphExecDestroy(old.exec);
      (void)hipGraphDestroy(old.graph);
      for (auto& pr : old.events) {
        (void)hipEventDestroy(pr.a);
        (void)hipEventDestroy(pr.b);
      }
      p->graphs.erase(p->graphs.begin());
    }
    p->graphs.push_back(std::move(g));
    ge = &p->graphs.back();
  }
  HIP_TRY(p, hipGraphLaunch(ge->exec, p->gstream), "graph launch");
  // the graph re-records its own event pairs on every replay: report this replay's
  // durations (copies of the handles, which the graph entry owns)
  for (const auto& pr : ge->events) p->prof.push_back({pr.cls, pr.a, pr.b, true});
  HIP_TRY(p, hipEventRecord(p->ev_out, p->gstream), "graph join");
  HIP_TRY(p, hipStreamWaitEvent(st, p->ev_out, 0), "graph join");
  return FSTAT_OK;
}

static std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  return arch + "-cu" + std::to_string(prop.multiProcessorCount);
}

// Tuned (B, Sb, variant) for this device, largest FFT length and precision from the cache file.
// precision field of a tuning-cache line: the precision, plus 2 with interbinning
static int cache_precision(const fstat_options& o) { return o.precision + 2 * (o.interbinning ? 1 : 0); }

// Interbinning weight c for a transform of L points over the n nonzero samples: a
// sinusoid midway between bins k and k + 1 has transform values whose difference has
// modulus 2 sin(pi n / 2L) sin(pi (n - 1) / 2L) / sin(pi / 2L), and its exact value
// midway is n; c makes c |X_k - X_{k+1}| equal to it (about pi/4 when n = L).
static double interbin_weight(long n, long L) {
  const double h = M_PI / (2.0 * (double)L);
  return (double)n * std::sin(h) / (2.0 * std::sin(h * (double)n) * std::sin(h * (double)(n - 1)));
}

static bool cache_lookup(const char* path, const std::string& tag, long nfft, int prec, int* B, int* Sb, int* var) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char dtag[128];
  long nf;
  int pr, b, sb, v;
  bool found = false;
  while (std::fscanf(f, "%127s %ld %d %d %d %d", dtag, &nf, &pr, &b, &sb, &v) == 6) {
    if (tag == dtag && nf == nfft && pr == prec && b > 0 && sb > 0 && v >= 0 && v <= 3) {
      *B = b;
      *Sb = sb;
      *var = v;
      found = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

// ------------------------------------------------------------------ vetting network
namespace {
inline dim3 blocks_for(long count, int per = 256) { return dim3((unsigned)((count + per - 1) / per)); }

fstat_status vet_fail(fstat_vet_t v, fstat_status st, const std::string& msg) {
  if (v) v->last_error = msg;
  else g_last_error = msg;
  return st;
}

#define VET_TRY(v, expr, what)                                                        \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return vet_fail(v, e_ == hipErrorOutOfMemory ? FSTAT_E_NOMEM : FSTAT_E_DEVICE,  \
                      std::string(what) + ": " + hip_error_text(e_));                 \
  } while (0)

// C[m][n] = sum_k A(m, k) B(k, n) on the matrix cores.  Products with a long K and a small
// output split K over workgroups into partial tiles (in `scratch`) summed in a fixed order.
constexpr long VET_SCRATCH = 8L << 20;  // floats of split-K and reduction scratch
void gemm(hipStream_t st, int M, int N, int K, const uint16_t* A, long sam, long sak, const uint16_t* B, long sbk,
          long sbn, float* Cm, long ldc, float* scratch = nullptr) {
  const int tiles = ((N + 63) / 64) * ((M + 63) / 64);
  int splits = 1;
  if (scratch && tiles < 256 && K >= 4096) {
    splits = std::min(K / 1024, 1024 / tiles);
    while (splits > 1 && (long)splits * M * N > VET_SCRATCH) --splits;
    splits = std::max(splits, 1);
  }
  const int kchunk = ((K + splits - 1) / splits + 15) / 16 * 16;
  dim3 grid((N + 63) / 64, (M + 63) / 64, splits);
  if (splits == 1) {
    FSTAT_LAUNCH(vet::k_gemm_bf16, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, Cm, ldc, 0L,
                       kchunk);
  } else {
    const long count = (long)M * N;
    FSTAT_LAUNCH(vet::k_gemm_bf16, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbk, sbn, scratch, (long)N,
                       count, kchunk);
    FSTAT_LAUNCH(vet::k_vet_sum_splits, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, scratch, splits,
                       count, N, ldc, Cm);
  }
}

// out[j] = sum_r m[r][j] (rows x cols, FP32), two fixed-order stages
void colsum(hipStream_t st, const float* m, long rows, int cols, float* out, float* scratch) {
  const long per = 4096;
  const int chunks = (int)((rows + per - 1) / per);
  FSTAT_LAUNCH(vet::k_vet_colsum_part, dim3(cols, chunks), dim3(256), 0, st, m, rows, cols, per, scratch);
  FSTAT_LAUNCH(vet::k_vet_colsum_final, dim3((cols + 255) / 256), dim3(256), 0, st, scratch, chunks, cols, out);
}

void vet_prepare(fstat_vet_t v, hipStream_t st) {
  FSTAT_LAUNCH(vet::k_vet_prepare, blocks_for((long)vet::H * vet::X), dim3(256), 0, st, v->theta, v->wf2,
                     v->wt2, v->wf3, v->wt3, v->w4b, v->w5b);
  FSTAT_LAUNCH(vet::k_vet_prepare_frag, blocks_for(vet::WQ_ELEMS), dim3(256), 0, st, v->theta, v->wq2, v->wq3);
}

// Scoring of n <= max_batch patches in two parts: the three convolutions into x (one
// kernel, four 64-position items per patch spread over one workgroup per compute unit),
// then the dense layers from x (the 8192 -> 128 product reads x from HBM, split four ways
// along K).
constexpr int INFER_SPLITS = 4;
static_assert((long)INFER_SPLITS * 8192 * vet::H <= VET_SCRATCH, "split-K partials of a full batch fit the scratch");
static_assert(vet::X % (INFER_SPLITS * vet::GW_K) == 0, "K splits of whole stages");
void vet_conv_stage(fstat_vet_t v, const float* patches, int n, uint16_t* x, hipStream_t st) {
  using namespace vet;
  const long items = (long)n * CV_ITEMS;
  const unsigned grid = (unsigned)std::max(1L, std::min<long>(v->n_cu, (items + CV_WAVES - 1) / CV_WAVES));
  FSTAT_LAUNCH(k_vet_conv_infer, dim3(grid), dim3(CV_NT), 0, st, patches, n, v->theta, v->wq2, v->wq3, x);
}

void vet_dense_stage(fstat_vet_t v, const uint16_t* x, int n, float* out, hipStream_t st, CandEntry* cand) {
  using namespace vet;
  const int nbp = (n + GW_M - 1) / GW_M * GW_M;
  FSTAT_LAUNCH(k_gemm_nt_wide, dim3(1, nbp / GW_M, INFER_SPLITS), dim3(GW_NT), 0, st, nbp, X, x, v->w4b, v->scratch,
               X / INFER_SPLITS);
  const long count = (long)nbp * H;
  // the split-K sum, the two small layers and the score in one launch
  FSTAT_LAUNCH(k_vet_head_infer<INFER_SPLITS>, dim3((unsigned)((n + HD_NP - 1) / HD_NP)), dim3(256), 0, st,
               v->scratch, count, n, v->theta, v->w5b, out, cand);
}

// All n patches in batches of max_batch on the caller's stream: each batch's convolutions,
// then its dense layers (logits to out_of(i)).  The convolution kernel holds every compute
// unit's LDS, so a second stream for the next batch's convolutions cannot run beside the
// product: measured, it made scoring slower, not faster.
template <typename OutOf>
static fstat_status vet_score_all(fstat_vet_t v, const float* patches, long long n, hipStream_t st, OutOf out_of,
                                  CandEntry* cand) {
  for (long long i = 0; i < n; i += v->max_batch) {
    const int b = (int)std::min<long long>(v->max_batch, n - i);
    vet_conv_stage(v, patches + i * vet::L, b, v->a3b, st);
    VET_TRY(v, launch_status(), "scoring launch");
    vet_dense_stage(v, v->a3b, b, out_of(i), st, cand ? cand + i : nullptr);
    VET_TRY(v, launch_status(), "scoring launch");
  }
  return FSTAT_OK;
}

// forward of n <= max_batch patches; logits to `out`
void vet_forward_batch(fstat_vet_t v, const float* patches, int n, float* out, hipStream_t st) {
  using namespace vet;
  const long NL = (long)n * L;
  FSTAT_LAUNCH(k_vet_input, blocks_for(NL), dim3(256), 0, st, patches, NL, v->u);
  FSTAT_LAUNCH(k_vet_conv1, blocks_for(NL * C), dim3(256), 0, st, v->u, n, v->theta, v->z1, v->a1b);
  FSTAT_LAUNCH(k_vet_im2col, blocks_for(NL * KC), dim3(256), 0, st, v->a1b, n, 1, v->colA);
  gemm(st, (int)NL, C, KC, v->colA, KC, 1, v->wf2, C, 1, v->z2, C);
  FSTAT_LAUNCH(k_vet_bias_relu, blocks_for(NL * C), dim3(256), 0, st, v->z2, NL, C, v->theta + O_B2, v->a2b,
                     (float*)nullptr);
  FSTAT_LAUNCH(k_vet_im2col, blocks_for(NL * KC), dim3(256), 0, st, v->a2b, n, 1, v->colB);
  gemm(st, (int)NL, C, KC, v->colB, KC, 1, v->wf3, C, 1, v->z3, C);
  FSTAT_LAUNCH(k_vet_bias_relu, blocks_for(NL * C), dim3(256), 0, st, v->z3, NL, C, v->theta + O_B3, v->a3b,
                     (float*)nullptr);
  {
    // the 8192 -> 128 layer: LDS-tiled product, K split so that the grid fills the chip
    const int nbp = (n + GT - 1) / GT * GT;
    const int tiles = (H / GT) * (nbp / GT);
    int splits = 1;
    while (splits < 32 && tiles * splits < 256) splits <<= 1;
    FSTAT_LAUNCH(k_gemm_nt_lds, dim3(H / GT, nbp / GT, splits), dim3(256), 0, st, nbp, H, X, v->a3b, v->w4b,
                       v->scratch, X / splits);
    const long count = (long)nbp * H;
    FSTAT_LAUNCH(k_vet_sum_splits, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, v->scratch, splits,
                       count, H, (long)H, v->z4);
  }
  FSTAT_LAUNCH(k_vet_bias_relu, blocks_for((long)n * H), dim3(256), 0, st, v->z4, (long)n, H, v->theta + O_B4,
                     v->a4b, (float*)nullptr);
  gemm(st, n, H, H, v->a4b, H, 1, v->w5b, 1, H, v->z5, H);
  FSTAT_LAUNCH(k_vet_bias_relu, blocks_for((long)n * H), dim3(256), 0, st, v->z5, (long)n, H, v->theta + O_B5,
                     (uint16_t*)nullptr, v->a5);
  FSTAT_LAUNCH(k_vet_fc3, blocks_for(n), dim3(256), 0, st, v->a5, n, v->theta, out);
}

void vet_backward(fstat_vet_t v, const float* labels, int n, hipStream_t st) {
  using namespace vet;
  const long NL = (long)n * L;
  float* g = v->grad;
  float* sc = v->scratch;
  FSTAT_LAUNCH(k_vet_head_backward, blocks_for((long)n * H), dim3(256), 0, st, v->logit, labels, n, v->theta,
                     v->z5, v->dz5, v->dz5b, v->dlogit, v->lterm);
  FSTAT_LAUNCH(k_vet_head_reduce, dim3(1), dim3(1024), 0, st, v->dlogit, v->a5, v->lterm, n, g, v->loss);
  gemm(st, H, H, n, v->dz5b, 1, H, v->a4b, H, 1, g + O_W5, H, sc);             // dW5 = dz5^T a4
  colsum(st, v->dz5, (long)n, H, g + O_B5, sc);
  gemm(st, n, H, H, v->dz5b, H, 1, v->w5b, H, 1, v->dh4, H);                   // dh4 = dz5 W5
  FSTAT_LAUNCH(k_vet_relu_mask, blocks_for((long)n * H), dim3(256), 0, st, v->dh4, v->z4, (long)n * H, v->dz4b);
  gemm(st, H, X, n, v->dz4b, 1, H, v->a3b, X, 1, g + O_W4, X, sc);             // dW4 = dz4^T x
  colsum(st, v->dh4, (long)n, H, g + O_B4, sc);
  gemm(st, n, X, H, v->dz4b, H, 1, v->w4b, X, 1, v->dx, X);                    // dx = dz4 W4
  FSTAT_LAUNCH(k_vet_relu_mask, blocks_for(NL * C), dim3(256), 0, st, v->dx, v->z3, NL * C, v->dzb);
  gemm(st, KC, C, (int)NL, v->colB, 1, KC, v->dzb, C, 1, v->dwm, C, sc);        // dW3 (im2col layout)
  FSTAT_LAUNCH(k_vet_scatter_conv_grad, blocks_for(C * C * KW), dim3(256), 0, st, v->dwm, g + O_W3);
  colsum(st, v->dx, NL, C, g + O_B3, sc);
  FSTAT_LAUNCH(k_vet_im2col, blocks_for(NL * KC), dim3(256), 0, st, v->dzb, n, -1, v->colC);
  gemm(st, (int)NL, C, KC, v->colC, KC, 1, v->wt3, C, 1, v->da, C);             // da2
  FSTAT_LAUNCH(k_vet_relu_mask, blocks_for(NL * C), dim3(256), 0, st, v->da, v->z2, NL * C, v->dzb);
  gemm(st, KC, C, (int)NL, v->colA, 1, KC, v->dzb, C, 1, v->dwm, C, sc);        // dW2
  FSTAT_LAUNCH(k_vet_scatter_conv_grad, blocks_for(C * C * KW), dim3(256), 0, st, v->dwm, g + O_W2);
  colsum(st, v->da, NL, C, g + O_B2, sc);
  FSTAT_LAUNCH(k_vet_im2col, blocks_for(NL * KC), dim3(256), 0, st, v->dzb, n, -1, v->colC);
  gemm(st, (int)NL, C, KC, v->colC, KC, 1, v->wt2, C, 1, v->da, C);             // da1
  FSTAT_LAUNCH(k_vet_relu_mask, blocks_for(NL * C), dim3(256), 0, st, v->da, v->z1, NL * C, v->dzb);
  {
    const long per = 256;
    const int chunks = (int)((NL + per - 1) / per);
    const int ncols = C * (KW + 1);
    FSTAT_LAUNCH(k_vet_conv1_backward_part, dim3(chunks), dim3(256), 0, st, v->da, v->u, NL, per, sc);
    FSTAT_LAUNCH(k_vet_colsum_final, dim3((ncols + 255) / 256), dim3(256), 0, st, sc, chunks, ncols,
                       sc + (long)chunks * ncols);
    FSTAT_LAUNCH(k_vet_conv1_scatter, dim3(1), dim3(256), 0, st, sc + (long)chunks * ncols, g);
  }
}
}  // namespace

int64_t fstat_vet_param_count(void) { return vet::N_PARAMS; }

fstat_status fstat_vet_create(int32_t max_batch, fstat_vet_t* out) {
  using namespace vet;
  if (!out) return vet_fail(nullptr, FSTAT_E_INVAL, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > 8192) return vet_fail(nullptr, FSTAT_E_INVAL, "max_batch outside [1, 8192]");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return vet_fail(nullptr, FSTAT_E_DEVICE, "no HIP device");
  auto v = new (std::nothrow) fstat_vet_s();
  if (!v) return vet_fail(nullptr, FSTAT_E_NOMEM, "vetter allocation");
  v->max_batch = max_batch;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      v->n_cu = ncu;
  }
  const size_t nb = (size_t)max_batch, NL = nb * L;
  // rows of the 8192 -> 128 products (training tiles of 64 rows, scoring tiles of 128)
  const size_t nbp = (nb + vet::GW_M - 1) / vet::GW_M * vet::GW_M;
  struct Part { void** p; size_t bytes; };
  std::vector<Part> parts = {
      {(void**)&v->theta, N_PARAMS * 4}, {(void**)&v->grad, N_PARAMS * 4}, {(void**)&v->m1, N_PARAMS * 4},
      {(void**)&v->m2, N_PARAMS * 4}, {(void**)&v->wf2, KC * C * 2}, {(void**)&v->wt2, KC * C * 2},
      {(void**)&v->wf3, KC * C * 2}, {(void**)&v->wt3, KC * C * 2}, {(void**)&v->w4b, (size_t)H * X * 2},
      {(void**)&v->w5b, H * H * 2}, {(void**)&v->wq2, WQ_ELEMS * 2}, {(void**)&v->wq3, WQ_ELEMS * 2}, {(void**)&v->u, NL * 4}, {(void**)&v->z1, NL * C * 4},
      {(void**)&v->z2, NL * C * 4}, {(void**)&v->z3, NL * C * 4}, {(void**)&v->z4, nbp * H * 4},
      {(void**)&v->z5, nb * H * 4}, {(void**)&v->a5, nb * H * 4}, {(void**)&v->logit, nb * 4},
      {(void**)&v->dlogit, nb * 4}, {(void**)&v->lterm, nb * 4}, {(void**)&v->dz5, nb * H * 4},
      {(void**)&v->dh4, nb * H * 4}, {(void**)&v->dx, NL * C * 4}, {(void**)&v->da, NL * C * 4},
      {(void**)&v->dwm, KC * C * 4}, {(void**)&v->loss, 4}, {(void**)&v->scratch, (size_t)VET_SCRATCH * 4},
      {(void**)&v->a1b, NL * C * 2},
      {(void**)&v->a2b, NL * C * 2}, {(void**)&v->a3b, nbp * X * 2},
      {(void**)&v->a4b, nb * H * 2},
      {(void**)&v->colA, NL * KC * 2}, {(void**)&v->colB, NL * KC * 2}, {(void**)&v->colC, NL * KC * 2},
      {(void**)&v->dz5b, nb * H * 2}, {(void**)&v->dz4b, nb * H * 2}, {(void**)&v->dzb, NL * C * 2}};
  size_t total = 0;
  for (auto& pt : parts) total = align256(total + pt.bytes);
  hipError_t e = hipMalloc(&v->mem, total);
  if (e != hipSuccess) {
    delete v;
    return vet_fail(nullptr, e == hipErrorOutOfMemory ? FSTAT_E_NOMEM : FSTAT_E_DEVICE, "vetter device memory");
  }
  size_t off = 0;
  for (auto& pt : parts) {
    *pt.p = (char*)v->mem + off;
    off = align256(off + pt.bytes);
  }
  if ((e = hipMemset(v->mem, 0, total)) != hipSuccess) {
    (void)hipFree(v->mem);
    delete v;
    return vet_fail(nullptr, FSTAT_E_DEVICE, "vetter memset");
  }
  *out = v;
  return FSTAT_OK;
}

fstat_status fstat_vet_set_params(fstat_vet_t v, const float* params, int64_t n) {
  if (!v || !params || n != vet::N_PARAMS) return vet_fail(v, FSTAT_E_INVAL, "bad arguments");
  VET_TRY(v, hipMemcpy(v->theta, params, n * 4, hipMemcpyHostToDevice), "parameter copy");
  VET_TRY(v, hipMemset(v->m1, 0, n * 4), "optimiser reset");
  VET_TRY(v, hipMemset(v->m2, 0, n * 4), "optimiser reset");
  v->steps = 0;
  vet_prepare(v, nullptr);
  VET_TRY(v, launch_status(), "weight preparation");
  VET_TRY(v, hipDeviceSynchronize(), "weight preparation");
  return FSTAT_OK;
}

fstat_status fstat_vet_get_params(fstat_vet_t v, float* params, int64_t n) {
  if (!v || !params || n != vet::N_PARAMS) return vet_fail(v, FSTAT_E_INVAL, "bad arguments");
  VET_TRY(v, hipDeviceSynchronize(), "synchronize");
  VET_TRY(v, hipMemcpy(params, v->theta, n * 4, hipMemcpyDeviceToHost), "parameter copy");
  return FSTAT_OK;
}

fstat_status fstat_vet_forward(fstat_vet_t v, const float* patches, int64_t n, float* logits, void* stream) {
  if (!v || n < 0 || (n > 0 && (!patches || !logits))) return vet_fail(v, FSTAT_E_INVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  return vet_score_all(v, patches, n, st, [&](long long i) { return logits + i; }, (CandEntry*)nullptr);
}

fstat_status fstat_vet_gradient(fstat_vet_t v, const float* patches, const float* labels, int64_t n, float* loss,
                                float* grad, void* stream) {
  if (!v || !patches || !labels || n < 1 || n > v->max_batch) return vet_fail(v, FSTAT_E_INVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  vet_forward_batch(v, patches, (int)n, v->logit, st);
  vet_backward(v, labels, (int)n, st);
  VET_TRY(v, launch_status(), "gradient launch");
  if (loss) VET_TRY(v, hipMemcpyAsync(loss, v->loss, 4, hipMemcpyDeviceToDevice, st), "loss copy");
  if (grad) VET_TRY(v, hipMemcpyAsync(grad, v->grad, vet::N_PARAMS * 4, hipMemcpyDeviceToDevice, st), "grad copy");
  return FSTAT_OK;
}

fstat_status fstat_vet_adam_step(fstat_vet_t v, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!v || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return vet_fail(v, FSTAT_E_INVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  v->steps += 1;
  const double step = lr * std::sqrt(1.0 - std::pow((double)beta2, v->steps)) / (1.0 - std::pow((double)beta1, v->steps));
  FSTAT_LAUNCH(vet::k_vet_adam, blocks_for(vet::N_PARAMS), dim3(256), 0, st, v->theta, v->grad, v->m1, v->m2,
                     (long)vet::N_PARAMS, (float)step, beta1, beta2, eps);
  vet_prepare(v, st);
  VET_TRY(v, launch_status(), "optimiser launch");
  return FSTAT_OK;
}

fstat_status fstat_vet_destroy(fstat_vet_t v) {
  if (!v) return FSTAT_OK;
  (void)hipDeviceSynchronize();
  if (v->mem) (void)hipFree(v->mem);
  delete v;
  return FSTAT_OK;
}

static void drop_graphs(fstat_plan_t plan) {
  if (plan->gstream) (void)hipStreamSynchronize(plan->gstream);
  for (auto& ge : plan->graphs) {
    if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    if (ge.graph) (void)hipGraphDestroy(ge.graph);
  }
  plan->graphs.clear();
}

fstat_status fstat_plan_attach_vetter(fstat_plan_t plan, fstat_vet_t vet, int64_t patch_capacity) {
  if (!plan) return fail(plan, FSTAT_E_INVAL, "NULL plan");
  drop_graphs(plan);  // captured searches do not contain the patch capture
  (void)hipDeviceSynchronize();
  if (plan->d_patches) (void)hipFree(plan->d_patches);
  if (plan->d_spec) (void)hipFree(plan->d_spec);
  if (plan->d_first) (void)hipFree(plan->d_first);
  plan->d_patches = nullptr;
  plan->d_spec = nullptr;
  plan->d_first = nullptr;
  plan->vet = nullptr;
  plan->patch_capacity = 0;
  if (!vet) return FSTAT_OK;
  if (patch_capacity < 1 || patch_capacity > plan->opt.candidate_capacity)
    return fail(plan, FSTAT_E_INVAL, "patch_capacity outside [1, candidate_capacity]");
  // a launch's 2F rows: bins [k_min, k_max) per template, or the streaming second pass's
  // transposed rows (all tP outputs of each of the tQ rows)
  long nbins = 0;
  for (auto& si : plan->segs) nbins = std::max({nbins, (long)(si.kmax - si.kmin), (long)si.tP * si.tQ});
  HIP_TRY(plan, hipMalloc((void**)&plan->d_patches, (size_t)patch_capacity * 256 * sizeof(float)), "patch store");
  HIP_TRY(plan, hipMalloc((void**)&plan->d_spec, (size_t)plan->B * nbins * sizeof(float)), "launch spectrum buffer");
  HIP_TRY(plan, hipMalloc((void**)&plan->d_first, sizeof(unsigned long long)), "count copy");
  plan->vet = vet;
  plan->patch_capacity = patch_capacity;
  return FSTAT_OK;
}

fstat_status fstat_plan_vet_candidates(fstat_plan_t plan, void* stream) {
  if (!plan) return fail(plan, FSTAT_E_INVAL, "NULL plan");
  if (!plan->vet) return fail(plan, FSTAT_E_STATE, "no vetting network attached");
  hipStream_t st = (hipStream_t)stream;
  if (plan->used_stream) HIP_TRY(plan, hipStreamSynchronize(plan->last_stream), "stream synchronize");
  HIP_TRY(plan, hipDeviceSynchronize(), "device synchronize");
  unsigned long long count = 0;
  HIP_TRY(plan, hipMemcpy(&count, plan->d_count, sizeof count, hipMemcpyDeviceToHost), "count copy");
  const long long n = std::min<long long>({(long long)count, plan->opt.candidate_capacity, plan->patch_capacity});
  // batches of the vetter's size: logits into its own buffer, scores into the entries
  fstat_vet_t v = plan->vet;
  const fstat_status rs = vet_score_all(v, plan->d_patches, n, st, [&](long long) { return v->logit; }, plan->d_cand);
  if (rs != FSTAT_OK) return fail(plan, rs, v->last_error);
  HIP_TRY(plan, launch_status(), "scoring launch");
  HIP_TRY(plan, hipStreamSynchronize(st), "scoring");
  plan->scored = true;
  plan->last_stream = st;
  plan->used_stream = true;
  return FSTAT_OK;
}

// ------------------------------------------------------------------ C ABI
// (C linkage comes from the declarations in fstat.h)

void fstat_options_default(fstat_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->nfft = 0;
  opt->k_min = 0;
  opt->k_max = 0;
  opt->threshold_2F = 20.0;
  opt->precision = FSTAT_PREC_MIXED;
  opt->form = FSTAT_FORM_SIMPLIFIED;
  opt->candidate_capacity = 1LL << 24;
  opt->workspace_budget_bytes = 0;
  opt->templates_per_launch = 0;
  opt->skies_per_batch = 0;
  opt->use_graph = 1;
  opt->tuning_cache_path = nullptr;
  opt->interbinning = 0;
}

const char* fstat_strerror(fstat_status st) {
  switch (st) {
    case FSTAT_OK: return "success";
    case FSTAT_E_INVAL: return "invalid argument";
    case FSTAT_E_NOMEM: return "out of memory";
    case FSTAT_E_ADMISSION: return "segment does not fit the workspace budget";
    case FSTAT_E_OVERFLOW: return "candidate buffer overflow";
    case FSTAT_E_DEVICE: return "HIP device error";
    case FSTAT_E_STATE: return "invalid plan state";
    case FSTAT_E_NOT_IMPLEMENTED: return "not implemented";
  }
  return "unknown status";
}

const char* fstat_last_error(fstat_plan_t plan) {
  return plan ? plan->last_error.c_str() : g_last_error.c_str();
}

fstat_status fstat_plan(const fstat_segment* segs, int32_t nseg, const fstat_options* opt_in,
                        fstat_plan_t* out_plan) {
  if (!out_plan) return fail(nullptr, FSTAT_E_INVAL, "out_plan is NULL");
  *out_plan = nullptr;
  if (!segs || nseg <= 0) return fail(nullptr, FSTAT_E_INVAL, "need at least one segment");
  fstat_options opt;
  if (opt_in) opt = *opt_in;
  else fstat_options_default(&opt);
  if (opt.precision != FSTAT_PREC_FP64 && opt.precision != FSTAT_PREC_MIXED)
    return fail(nullptr, FSTAT_E_INVAL, "unknown precision");
  if (opt.form != FSTAT_FORM_SIMPLIFIED && opt.form != FSTAT_FORM_FULL)
    return fail(nullptr, FSTAT_E_INVAL, "unknown form");
  if (opt.candidate_capacity < 1) return fail(nullptr, FSTAT_E_INVAL, "candidate_capacity must be >= 1");
  if (opt.templates_per_launch < 0 || opt.skies_per_batch < 0)
    return fail(nullptr, FSTAT_E_INVAL, "batch sizes must be >= 0");
  if (!(std::isfinite(opt.threshold_2F))) return fail(nullptr, FSTAT_E_INVAL, "threshold must be finite");
  if (opt.k_min < 0 || opt.k_max < 0 || (opt.k_max != 0 && opt.k_max <= opt.k_min))
    return fail(nullptr, FSTAT_E_INVAL, "bad bin range");
  if (opt.interbinning != 0 && opt.interbinning != 1) return fail(nullptr, FSTAT_E_INVAL, "interbinning must be 0 or 1");

  auto p = new (std::nothrow) fstat_plan_s();
  if (!p) return fail(nullptr, FSTAT_E_NOMEM, "plan allocation");
  p->opt = opt;
  p->fp64 = opt.precision == FSTAT_PREC_FP64;
  p->cx_bytes = p->fp64 ? 16 : 8;
  for (int i = 0; i < nseg; ++i) {
    const fstat_segment& s = segs[i];
    char msg[160];
    if (s.n < 2048 || s.n > (1L << (LOG_MAX - 1))) {
      std::snprintf(msg, sizeof msg, "segment %d: n=%lld outside [2048, %ld]", i, (long long)s.n, 1L << (LOG_MAX - 1));
      delete p;
      return fail(nullptr, FSTAT_E_INVAL, msg);
    }
    if (!(s.dt > 0) || !std::isfinite(s.dt) || !(s.sigma2 > 0) || !std::isfinite(s.sigma2) ||
        !std::isfinite(s.f_off) || !std::isfinite(s.lat) || !std::isfinite(s.gamma) || !std::isfinite(s.phi_r)) {
      std::snprintf(msg, sizeof msg, "segment %d: dt and sigma2 must be > 0 and all parameters finite", i);
      delete p;
      return fail(nullptr, FSTAT_E_INVAL, msg);
    }
    if (!s.x || !s.r_ssb) {
      std::snprintf(msg, sizeof msg, "segment %d: x and r_ssb must be device pointers", i);
      delete p;
      return fail(nullptr, FSTAT_E_INVAL, msg);
    }
    SegInfo si;
    si.s = s;
    const long nf = opt.nfft ? opt.nfft : next_pow2(2 * s.n);
    const int e = ilog2_exact(nf);
    if (e < 0 || nf < 2 * s.n || e < 12 || e > LOG_MAX) {
      std::snprintf(msg, sizeof msg, "segment %d: nfft=%ld must be a power of two in [2n, 2^%d]", i, nf, LOG_MAX);
      delete p;
      return fail(nullptr, FSTAT_E_INVAL, msg);
    }
    si.nfft = (int)nf;
    si.M = (int)(nf / 2);
    si.logL = e;
    si.P = 1 << ((e + 1) / 2);
    si.Q = 1 << (e / 2);
    si.PM = 1 << (e / 2);
    si.QM = 1 << ((e - 1) / 2);
    si.kmin = opt.k_min;
    si.kmax = opt.k_max ? opt.k_max : si.nfft / 2;
    si.tlog = e;
    si.tP = si.P;
    si.tQ = si.Q;
    si.tL = si.nfft;
    if (opt.interbinning) {
      if (e < 13) {
        std::snprintf(msg, sizeof msg, "segment %d: interbinning needs nfft >= 2^13 (nfft=%ld)", i, nf);
        delete p;
        return fail(nullptr, FSTAT_E_INVAL, msg);
      }
      si.tlog = e - 1;
      si.tP = 1 << (e / 2);
      si.tQ = 1 << ((e - 1) / 2);
      si.tL = si.tP * si.tQ;
      si.ibw = interbin_weight(s.n, si.tL);
    }
    if (si.kmax > si.nfft) {
      std::snprintf(msg, sizeof msg, "segment %d: k_max=%d beyond nfft=%d", i, si.kmax, si.nfft);
      delete p;
      return fail(nullptr, FSTAT_E_INVAL, msg);
    }
    p->segs.push_back(si);
    p->n_max = std::max(p->n_max, (long)s.n);
    p->L_max = std::max(p->L_max, (long)si.nfft);
    p->TL_max = std::max(p->TL_max, (long)si.tL);
    p->M_max = std::max(p->M_max, (long)si.M);
  }
  p->nblk_max = (int)((p->n_max + NT - 1) / NT);

  // batch sizes: requested or defaults, shrunk to the budget (admission)
  int Sb = opt.skies_per_batch ? opt.skies_per_batch : (p->fp64 ? 4 : 8);
  int B = opt.templates_per_launch ? opt.templates_per_launch : (p->fp64 ? 16 : 256);
  bool tuned = false;
  if (!opt.skies_per_batch && !opt.templates_per_launch && opt.tuning_cache_path) {
    int tb = 0, ts = 0, tv = 0;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0 &&
        cache_lookup(opt.tuning_cache_path, device_tag(), p->L_max, cache_precision(opt), &tb, &ts, &tv)) {
      B = tb;
      Sb = ts;
      p->variant_a = tv & 1;
      p->variant_b = tv >> 1;
      tuned = true;
    }
  }
  (void)tuned;
  const size_t budget = opt.workspace_budget_bytes;
  if (budget) {
    if (layout(p, 1, 1, false) > budget) {
      char msg[200];
      std::snprintf(msg, sizeof msg, "largest segment needs %zu workspace bytes with one sky and one template; budget %zu",
                    layout(p, 1, 1, false), budget);
      delete p;
      return fail(nullptr, FSTAT_E_ADMISSION, msg);
    }
    while (layout(p, Sb, B, false) > budget && (Sb > 1 || B > 1)) {
      if (B > 1 && (B >= 2 * Sb || Sb == 1)) B = (B + 1) / 2;
      else Sb = (Sb + 1) / 2;
    }
  }
  p->Sb = Sb;
  p->B = B;
  p->scale_B = (opt.templates_per_launch == 0);
  layout(p, Sb, B, true);

  // device resources
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    delete p;
    return fail(nullptr, FSTAT_E_DEVICE, "no HIP device available");
  }
  (void)hipGetDevice(&p->device);
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && ncu > 0)
      p->n_cu = ncu;
  }
  {
    // the static scratch of this device, for fstat_twoF_spectrum_static
    const hipError_t es = static_scratch_address(p->device, &p->static_ws);
    if (es != hipSuccess) p->static_err = std::string("static scratch address: ") + hipGetErrorString(es);
  }
  std::vector<unsigned char> tb;
  fill_tables<float>(tb, p->tab, 0, KT_F32);
  fill_tables<double>(tb, p->tab, 1, KT_F64);
  p->tab.bytes = tb.size();
  if ((e = hipMalloc(&p->tab.dev, tb.size())) != hipSuccess ||
      (e = hipMemcpy(p->tab.dev, tb.data(), tb.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMalloc((void**)&p->d_cand, (size_t)opt.candidate_capacity * sizeof(CandEntry))) != hipSuccess ||
      (e = hipMalloc((void**)&p->d_count, sizeof(unsigned long long))) != hipSuccess ||
      (e = hipMemset(p->d_count, 0, sizeof(unsigned long long))) != hipSuccess ||
      (e = hipMalloc((void**)&p->d_search_next, sizeof(int))) != hipSuccess ||
      (e = hipMalloc((void**)&p->d_sky_pos, 2 * sizeof(double))) != hipSuccess ||
      (e = hipMemset(p->d_search_next, 0, sizeof(int))) != hipSuccess) {
    std::string msg = std::string("plan device allocation: ") + hipGetErrorString(e);
    fstat_destroy(p);
    return fail(nullptr, e == hipErrorOutOfMemory ? FSTAT_E_NOMEM : FSTAT_E_DEVICE, msg);
  }
  *out_plan = p;
  return FSTAT_OK;
}

fstat_status fstat_plan_workspace_size(fstat_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(plan, FSTAT_E_INVAL, "NULL argument");
  *bytes = layout(plan, plan->Sb, plan->B, false);
  return FSTAT_OK;
}

fstat_status fstat_plan_set_workspace(fstat_plan_t plan, void* dev_ptr, size_t bytes) {
  if (!plan) return fail(plan, FSTAT_E_INVAL, "NULL plan");
  const size_t need = layout(plan, plan->Sb, plan->B, false);
  if (!dev_ptr || bytes < need || ((uintptr_t)dev_ptr & 255))
    return fail(plan, FSTAT_E_INVAL, "workspace NULL, too small or not 256-byte aligned");
  if (plan->ws_owned && plan->ws) {
    (void)hipDeviceSynchronize();
    (void)hipFree(plan->ws);
  }
  plan->ws = dev_ptr;
  plan->ws_bytes = bytes;
  plan->ws_owned = false;
  layout(plan, plan->Sb, plan->B, true);
  return FSTAT_OK;
}

static fstat_status check_lists(fstat_plan_t plan, int32_t segment, const double* alpha, const double* delta,
                                int32_t nsky, const double* fdot, int32_t nfdot) {
  if (!plan) return fail(plan, FSTAT_E_INVAL, "NULL plan");
  if (segment < -1 || segment >= (int32_t)plan->segs.size()) return fail(plan, FSTAT_E_INVAL, "segment out of range");
  if (nsky <= 0 || nfdot <= 0) return fail(plan, FSTAT_E_INVAL, "nsky and nfdot must be > 0");
  if (!alpha || !delta || !fdot) return fail(plan, FSTAT_E_INVAL, "template lists must be device pointers");
  if ((long long)nsky * nfdot > (1LL << 30)) return fail(plan, FSTAT_E_INVAL, "too many templates in one call");
  return FSTAT_OK;
}

// Pinned host copies of a search call's lists, for the candidate records.
static fstat_status record_search(fstat_plan_t plan, const Grid& g, hipStream_t st) {
  SearchRecord rec;
  rec.nsky = g.nsky;
  rec.nfdot = g.nfdot;
  rec.lattice = g.fdot == nullptr;
  rec.s_lo = g.s_lo;
  rec.m10 = g.m10;
  rec.m11 = g.m11;
  const size_t nd = rec.lattice ? 4 * (size_t)g.nsky : 2 * (size_t)g.nsky + g.nfdot;
  HIP_TRY(plan, hipHostMalloc((void**)&rec.host, nd * sizeof(double), hipHostMallocDefault), "pinned list copy");
  plan->searches.push_back(rec);
  const size_t ns = (size_t)g.nsky * sizeof(double);
  HIP_TRY(plan, hipMemcpyAsync(rec.host, g.alpha, ns, hipMemcpyDeviceToHost, st), "list copy");
  HIP_TRY(plan, hipMemcpyAsync(rec.host + g.nsky, g.delta, ns, hipMemcpyDeviceToHost, st), "list copy");
  if (rec.lattice) {
    HIP_TRY(plan, hipMemcpyAsync(rec.host + 2 * g.nsky, g.w_freq, ns, hipMemcpyDeviceToHost, st), "list copy");
    HIP_TRY(plan, hipMemcpyAsync(rec.host + 3 * g.nsky, g.w_spin, ns, hipMemcpyDeviceToHost, st), "list copy");
  } else {
    HIP_TRY(plan, hipMemcpyAsync(rec.host + 2 * g.nsky, g.fdot, g.nfdot * sizeof(double), hipMemcpyDeviceToHost, st),
            "list copy");
  }
  return FSTAT_OK;
}

static Grid explicit_grid(const double* alpha, const double* delta, int nsky, const double* fdot, int nfdot) {
  Grid g;
  g.alpha = alpha;
  g.delta = delta;
  g.nsky = nsky;
  g.fdot = fdot;
  g.nfdot = nfdot;
  return g;
}

fstat_status fstat_search_batch(fstat_plan_t plan, int32_t segment, const double* alpha, const double* delta,
                                int32_t nsky, const double* fdot, int32_t nfdot, void* stream) {
  fstat_status r = check_lists(plan, segment, alpha, delta, nsky, fdot, nfdot);
  if (r != FSTAT_OK) return r;
  r = ensure_workspace(plan);
  if (r != FSTAT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  const Grid g = explicit_grid(alpha, delta, nsky, fdot, nfdot);
  if ((r = record_search(plan, g, st)) != FSTAT_OK) return r;
  plan->last_stream = st;
  plan->used_stream = true;
  r = run_search(plan, segment, g, 0, nullptr, st);
  plan->search_count++;
  return r;
}

fstat_status fstat_twoF_spectrum(fstat_plan_t plan, int32_t segment, const double* alpha, const double* delta,
                                 int32_t nsky, const double* fdot, int32_t nfdot, void* out, void* stream) {
  fstat_status r = check_lists(plan, segment, alpha, delta, nsky, fdot, nfdot);
  if (r != FSTAT_OK) return r;
  if (segment < 0) return fail(plan, FSTAT_E_INVAL, "spectrum needs one segment");
  if (!out) return fail(plan, FSTAT_E_INVAL, "out is NULL");
  r = ensure_workspace(plan);
  if (r != FSTAT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  plan->last_stream = st;
  plan->used_stream = true;
  return run_search(plan, segment, explicit_grid(alpha, delta, nsky, fdot, nfdot), 1, out, st);
}

fstat_status fstat_twoF_spectrum_static(fstat_plan_t plan, int32_t segment, const double* alpha,
                                        const double* delta, int32_t nsky, const double* fdot, int32_t nfdot,
                                        void* out, void* stream) {
  fstat_status r = check_lists(plan, segment, alpha, delta, nsky, fdot, nfdot);
  if (r != FSTAT_OK) return r;
  if (segment < 0) return fail(plan, FSTAT_E_INVAL, "spectrum needs one segment");
  if (!out) return fail(plan, FSTAT_E_INVAL, "out is NULL");
  if (!plan->static_ws) return fail(plan, FSTAT_E_DEVICE, plan->static_err);
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != plan->device)
    return fail(plan, FSTAT_E_STATE, "the plan's device is not the current device");
  const size_t cap = FSTAT_STATIC_SCRATCH_BYTES;
  if (layout(plan, 1, 1, false) > cap) {
    char msg[200];
    std::snprintf(msg, sizeof msg, "the plan's largest segment needs %zu workspace bytes with one sky and one "
                  "template; the static scratch holds %zu", layout(plan, 1, 1, false), cap);
    return fail(plan, FSTAT_E_INVAL, msg);
  }
  // the plan's batch sizes, shrunk as by admission until the workspace fits the scratch
  int Sb = std::min(plan->Sb, (int)nsky), B = plan->B;
  while (layout(plan, Sb, B, false) > cap && (Sb > 1 || B > 1)) {
    if (B > 1 && (B >= 2 * Sb || Sb == 1)) B = (B + 1) / 2;
    else Sb = (Sb + 1) / 2;
  }
  // run on the scratch, every launch on `stream`, then restore the plan's own workspace,
  // batch sizes and layout (the enqueued kernels hold their arguments by value)
  void* const ws0 = plan->ws;
  const int Sb0 = plan->Sb, B0 = plan->B;
  const bool prof0 = plan->profiling;
  plan->ws = plan->static_ws;
  plan->Sb = Sb;
  plan->B = B;
  layout(plan, Sb, B, true);
  plan->single_stream = true;
  plan->profiling = false;
  hipStream_t st = (hipStream_t)stream;
  r = enqueue_search(plan, segment, explicit_grid(alpha, delta, nsky, fdot, nfdot), 1, out, st);
  plan->single_stream = false;
  plan->profiling = prof0;
  plan->ws = ws0;
  plan->Sb = Sb0;
  plan->B = B0;
  layout(plan, Sb0, B0, true);
  plan->last_stream = st;
  plan->used_stream = true;
  return r;
}

// ------------------------------------------------------------------ lattice grid
static constexpr double AU_SECONDS = 149597870700.0 / 299792458.0;  // light time over 1 AU

static bool finite_lattice(const fstat_lattice* lat) {
  for (double v : lat->M)
    if (!std::isfinite(v)) return false;
  return std::isfinite(lat->epsilon) && std::isfinite(lat->f_ref) && lat->f_ref > 0.0;
}

// sky components of the two sky rows and the box bound of |n|, |m| on the sky's disk
static bool sky_rows(const fstat_lattice* lat, double* n_max, double* m_max) {
  const double* M = lat->M;
  const double det = M[10] * M[15] - M[11] * M[14];
  const double w = 2.0 * M_PI * lat->f_ref * AU_SECONDS;
  if (!(std::fabs(det) > 0.0)) return false;
  *n_max = w * std::hypot(M[14], M[15]) / std::fabs(det);
  *m_max = w * std::hypot(M[10], M[11]) / std::fabs(det);
  return std::isfinite(*n_max) && std::isfinite(*m_max);
}

fstat_status fstat_lattice_sky_range(const fstat_lattice* lat, int32_t box[4]) {
  if (!lat || !box) return fail(nullptr, FSTAT_E_INVAL, "NULL argument");
  if (!finite_lattice(lat)) return fail(nullptr, FSTAT_E_INVAL, "lattice values must be finite, f_ref > 0");
  double nm, mm;
  if (!sky_rows(lat, &nm, &mm)) return fail(nullptr, FSTAT_E_INVAL, "the sky rows are parallel");
  if (nm >= 1e9 || mm >= 1e9) return fail(nullptr, FSTAT_E_INVAL, "sky range beyond int32");
  const int32_t n_hi = (int32_t)std::floor(nm), m_hi = (int32_t)std::floor(mm);
  box[0] = -n_hi;
  box[1] = n_hi;
  box[2] = -m_hi;
  box[3] = m_hi;
  return FSTAT_OK;
}

fstat_status fstat_lattice_sky(const fstat_lattice* lat, int32_t hemisphere, const int32_t box[4],
                               int64_t capacity, double* alpha, double* delta, double* w_freq, double* w_spin,
                               int32_t* nm, int64_t* count, void* stream) {
  if (!lat || !box || !count) return fail(nullptr, FSTAT_E_INVAL, "NULL argument");
  if (!finite_lattice(lat)) return fail(nullptr, FSTAT_E_INVAL, "lattice values must be finite, f_ref > 0");
  if (hemisphere != 1 && hemisphere != -1) return fail(nullptr, FSTAT_E_INVAL, "hemisphere must be +1 or -1");
  if (box[1] < box[0] || box[3] < box[2]) return fail(nullptr, FSTAT_E_INVAL, "empty box");
  const long long nspan = (long long)box[1] - box[0] + 1, mspan = (long long)box[3] - box[2] + 1;
  if (nspan > (1LL << 26) || mspan > (1LL << 26) || nspan * mspan > (1LL << 26))
    return fail(nullptr, FSTAT_E_INVAL, "box holds more than 2^26 points");
  if (capacity < 0) return fail(nullptr, FSTAT_E_INVAL, "capacity < 0");
  if (capacity > 0 && (!alpha || !delta || !w_freq || !w_spin))
    return fail(nullptr, FSTAT_E_INVAL, "output arrays must be device pointers");
  const double* M = lat->M;
  LatSkyArgs a;
  a.r2x = M[10];
  a.r2y = M[11];
  a.r3x = M[14];
  a.r3y = M[15];
  a.r2f = M[8];
  a.r2s = M[9];
  a.r3f = M[12];
  a.r3s = M[13];
  a.w = 2.0 * M_PI * lat->f_ref * AU_SECONDS;
  a.ce = std::cos(lat->epsilon);
  a.se = std::sin(lat->epsilon);
  a.hemi = (double)hemisphere;
  a.n_lo = box[0];
  a.m_lo = box[2];
  a.mspan = (int)mspan;
  a.total = nspan * mspan;
  a.capacity = capacity;
  a.alpha = alpha;
  a.delta = delta;
  a.w_freq = w_freq;
  a.w_spin = w_spin;
  a.nm = capacity > 0 ? nm : nullptr;
  a.count = (long long*)count;
  FSTAT_LAUNCH(k_lattice_sky, dim3(1), dim3(256), 0, (hipStream_t)stream, a);
  hipError_t e = launch_status();
  if (e != hipSuccess) return hip_fail(nullptr, e, "lattice sky launch");
  return FSTAT_OK;
}

// The constraints that let the FFT and one resampling per sky serve the grid.
static fstat_status check_lattice_search(fstat_plan_t plan, int32_t segment, const fstat_lattice* lat) {
  const double* M = lat->M;
  for (double v : lat->M)
    if (!std::isfinite(v)) return fail(plan, FSTAT_E_INVAL, "lattice values must be finite");
  if (!(M[0] > 0.0) || M[1] != 0.0 || M[2] != 0.0 || M[3] != 0.0)
    return fail(plan, FSTAT_E_INVAL, "row 0 of the lattice must be (w_F > 0, 0, 0, 0)");
  if (M[6] != 0.0 || M[7] != 0.0) return fail(plan, FSTAT_E_INVAL, "row 1 of the lattice must have no sky components");
  const int s0 = segment < 0 ? 0 : segment, s1 = segment < 0 ? (int)plan->segs.size() : segment + 1;
  for (int i = s0; i < s1; ++i) {
    const double q = M[0] * (double)plan->segs[i].nfft / (2.0 * M_PI);
    if (q < 0.5 || std::fabs(q - std::round(q)) > 1e-6 * std::max(1.0, q)) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "segment %d: row 0 is %.9g bins of nfft=%d, not a whole number", i, q,
                    plan->segs[i].nfft);
      return fail(plan, FSTAT_E_INVAL, msg);
    }
  }
  return FSTAT_OK;
}

fstat_status fstat_search_lattice(fstat_plan_t plan, int32_t segment, const fstat_lattice* lat,
                                  const double* alpha, const double* delta, const double* w_freq,
                                  const double* w_spin, int32_t nsky, int32_t s_lo, int32_t s_hi,
                                  void* spectrum, void* stream) {
  if (!plan) return fail(plan, FSTAT_E_INVAL, "NULL plan");
  if (!lat) return fail(plan, FSTAT_E_INVAL, "NULL lattice");
  if (s_hi < s_lo) return fail(plan, FSTAT_E_INVAL, "s_hi < s_lo");
  if ((long long)s_hi - s_lo + 1 > (1LL << 30)) return fail(plan, FSTAT_E_INVAL, "too many spindowns");
  const int nfdot = s_hi - s_lo + 1;
  // the explicit-list checks, with w_freq standing in for the spindown list
  fstat_status r = check_lists(plan, segment, alpha, delta, nsky, w_freq, nfdot);
  if (r != FSTAT_OK) return r;
  if (!w_spin) return fail(plan, FSTAT_E_INVAL, "template lists must be device pointers");
  if ((r = check_lattice_search(plan, segment, lat)) != FSTAT_OK) return r;
  if (spectrum && segment < 0) return fail(plan, FSTAT_E_INVAL, "spectrum needs one segment");
  r = ensure_workspace(plan);
  if (r != FSTAT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  Grid g;
  g.alpha = alpha;
  g.delta = delta;
  g.nsky = nsky;
  g.nfdot = nfdot;
  g.w_freq = w_freq;
  g.w_spin = w_spin;
  g.s_lo = s_lo;
  g.m10 = lat->M[4];
  g.m11 = lat->M[5];
  plan->last_stream = st;
  plan->used_stream = true;
  if (spectrum) return run_search(plan, segment, g, 1, spectrum, st);
  if ((r = record_search(plan, g, st)) != FSTAT_OK) return r;
  r = run_search(plan, segment, g, 0, nullptr, st);
  plan->search_count++;
  return r;
}

template <typename T>
static fstat_status sky_stages_impl(fstat_plan_t plan, const SegInfo& si, const double* ad, double* abc, void* za,
                                    void* zb, void* ua, void* ub, void* zta, void* ztb, hipStream_t st) {
  Dev<T> d(plan);
  fstat_status r = run_sky_batch<T>(plan, d, si, ad, ad + 1, 0, 1, st);
  if (r != FSTAT_OK) return r;
  const size_t n = si.s.n, M = si.M, L = si.nfft, cb = sizeof(cx<T>);
  cx<T>* zab = d.sky();
  cx<T>* o = zab + 4 * M + 2 * L;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    return dst ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) : hipSuccess;
  };
  HIP_TRY(plan, cp(za, zab, n * cb), "stage copy");
  HIP_TRY(plan, cp(zb, zab + M, n * cb), "stage copy");
  // the 2x upsampled series, assembled from the series and its half-sample shift
  cx<T>* u = zab + 2 * M;   // the spectrum's space, no longer needed
  FSTAT_LAUNCH((k_upsampled<T>), dim3((unsigned)((L + NT - 1) / NT), 2), dim3(NT), 0, st, zab, o, (long)M,
                     (int)n, (int)L, u);
  HIP_TRY(plan, launch_status(), "upsampled series launch");
  HIP_TRY(plan, cp(ua, u, L * cb), "stage copy");
  HIP_TRY(plan, cp(ub, u + L, L * cb), "stage copy");
  HIP_TRY(plan, cp(zta, d.zt(), n * cb), "stage copy");
  HIP_TRY(plan, cp(ztb, d.zt() + n, n * cb), "stage copy");
  if (abc) {
    SkyParams* sp = d.sp();
    HIP_TRY(plan, hipMemcpyAsync(abc, &sp->A, 3 * sizeof(double), hipMemcpyDeviceToDevice, st), "stage copy");
  }
  return FSTAT_OK;
}

fstat_status fstat_sky_stages(fstat_plan_t plan, int32_t segment, double alpha, double delta, double* abc, void* za,
                              void* zb, void* ua, void* ub, void* zta, void* ztb, void* stream) {
  if (!plan) return fail(plan, FSTAT_E_INVAL, "NULL plan");
  if (segment < 0 || segment >= (int32_t)plan->segs.size()) return fail(plan, FSTAT_E_INVAL, "segment out of range");
  fstat_status r = ensure_workspace(plan);
  if (r != FSTAT_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  // the sky position goes through the plan's small device array, as a search's lists do
  double* ad = plan->d_sky_pos;
  double h[2] = {alpha, delta};
  HIP_TRY(plan, hipStreamSynchronize(st), "sky position copy");
  HIP_TRY(plan, hipMemcpy(ad, h, sizeof h, hipMemcpyHostToDevice), "sky position copy");
  const SegInfo& si = plan->segs[segment];
  r = plan->fp64 ? sky_stages_impl<double>(plan, si, ad, abc, za, zb, ua, ub, zta, ztb, st)
                 : sky_stages_impl<float>(plan, si, ad, abc, za, zb, ua, ub, zta, ztb, st);
  (void)hipStreamSynchronize(st);
  plan->last_stream = st;
  plan->used_stream = true;
  return r;
}

// Key order on the device (fstat_drain.hpp: count -> offsets -> write, then each
// template's range by bin), leaving d_cand[0, stored) ordered.
static fstat_status order_on_device(fstat_plan_t p, long long stored) {
  const int nsearch = (int)p->searches.size();
  const int search0 = p->search_count - nsearch;
  const int nseg = (int)p->segs.size();
  if (nsearch == 0) return fail(p, FSTAT_E_STATE, "candidates without a search to drain");
  std::vector<DrainSearch> hs((size_t)nsearch);
  long long ntpl = 0;
  for (int i = 0; i < nsearch; ++i) {
    hs[(size_t)i].base = ntpl;
    hs[(size_t)i].nsky = p->searches[(size_t)i].nsky;
    hs[(size_t)i].nfdot = p->searches[(size_t)i].nfdot;
    ntpl += (long long)nseg * p->searches[(size_t)i].nsky * p->searches[(size_t)i].nfdot;
  }
  if (ntpl > (1LL << 31))
    return fail(p, FSTAT_E_STATE, "more than 2^31 templates searched since the last drain: drain more often");
  const long long ntiles = (ntpl + SCAN_TILE - 1) / SCAN_TILE;
  size_t o = 0;
  auto put = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  const size_t o_grp = put((size_t)stored * sizeof(CandEntry)), o_rank = put((size_t)stored * 4),
               o_cnt = put((size_t)ntpl * 4), o_off = put((size_t)(ntpl + 1) * 8), o_sums = put((size_t)ntiles * 8),
               o_srch = put((size_t)nsearch * sizeof(DrainSearch)), o_flag = put(2 * 4);
  if (o > p->drain_bytes) {
    if (p->drain_ws) (void)hipFree(p->drain_ws);
    p->drain_ws = nullptr;
    p->drain_bytes = 0;
    HIP_TRY(p, hipMalloc(&p->drain_ws, o), "drain ordering memory");
    p->drain_bytes = o;
  }
  char* w = (char*)p->drain_ws;
  CandEntry* grouped = (CandEntry*)(w + o_grp);
  unsigned* rank = (unsigned*)(w + o_rank);
  unsigned* counts = (unsigned*)(w + o_cnt);
  unsigned long long* off = (unsigned long long*)(w + o_off);
  unsigned long long* sums = (unsigned long long*)(w + o_sums);
  DrainSearch* ds = (DrainSearch*)(w + o_srch);
  unsigned* flags = (unsigned*)(w + o_flag);   // [0] key outside its search, [1] repeated bin of a template
  HIP_TRY(p, hipMemcpy(ds, hs.data(), hs.size() * sizeof(DrainSearch), hipMemcpyHostToDevice), "drain tables");
  const hipStream_t st = nullptr;
  const unsigned gblk = (unsigned)std::min<long long>((stored + DRAIN_NT - 1) / DRAIN_NT, 1LL << 20);
  FSTAT_LAUNCH(k_drain_zero, dim3((unsigned)std::min<long long>((ntpl + DRAIN_NT - 1) / DRAIN_NT, 1LL << 20)),
               dim3(DRAIN_NT), 0, st, counts, ntpl);
  FSTAT_LAUNCH(k_drain_zero, dim3(1), dim3(DRAIN_NT), 0, st, flags, 2LL);
  FSTAT_LAUNCH(k_drain_count, dim3(gblk), dim3(DRAIN_NT), 0, st, p->d_cand, stored, ds, nsearch, search0, nseg, counts,
               rank, flags);
  HIP_TRY(p, launch_status(), "drain count launch");
  unsigned hf[2] = {0, 0};
  HIP_TRY(p, hipMemcpy(hf, flags, sizeof hf, hipMemcpyDeviceToHost), "drain flags");
  if (hf[0]) return fail(p, FSTAT_E_STATE, "a stored candidate's key lies outside its search");
  FSTAT_LAUNCH(k_scan_tile_sums, dim3((unsigned)ntiles), dim3(DRAIN_NT), 0, st, counts, ntpl, sums);
  FSTAT_LAUNCH(k_scan_sums, dim3(1), dim3(DRAIN_NT), 0, st, sums, ntiles);
  FSTAT_LAUNCH(k_scan_apply, dim3((unsigned)ntiles), dim3(DRAIN_NT), 0, st, counts, ntpl, sums, off);
  FSTAT_LAUNCH(k_drain_scatter, dim3(gblk), dim3(DRAIN_NT), 0, st, p->d_cand, stored, ds, nsearch, search0, nseg, off,
               rank, grouped, flags);
  FSTAT_LAUNCH(k_drain_order, dim3((unsigned)std::min<long long>(ntpl, 1LL << 18)), dim3(DRAIN_NT), 0, st, grouped, off,
               ntpl, p->d_cand);
  FSTAT_LAUNCH(k_drain_order_long, dim3((unsigned)std::min<long long>(ntpl, 2LL * p->n_cu)), dim3(DRAIN_LONG_NT), 0,
               st, grouped, off, ntpl, p->d_cand, flags + 1);
  HIP_TRY(p, launch_status(), "drain ordering launch");
  HIP_TRY(p, hipMemcpy(hf, flags, sizeof hf, hipMemcpyDeviceToHost), "drain flags");
  if (hf[0] || hf[1]) return fail(p, FSTAT_E_STATE, "a template's candidates repeat a bin");
  return FSTAT_OK;
}

// Records and keys of the first `nout` entries of d_cand (in key order) formed on the device
// and copied straight into the caller's arrays (either may be NULL).
static fstat_status form_on_device(fstat_plan_t p, long long nout, fstat_candidate* out, fstat_candidate_key* keys) {
  const int nsearch = (int)p->searches.size();
  const int search0 = p->search_count - nsearch;
  std::vector<size_t> nd((size_t)nsearch);
  size_t ndouble = 0;
  for (int i = 0; i < nsearch; ++i) {
    const SearchRecord& sr = p->searches[(size_t)i];
    nd[(size_t)i] = sr.lattice ? 4 * (size_t)sr.nsky : 2 * (size_t)sr.nsky + sr.nfdot;
    ndouble += nd[(size_t)i];
  }
  size_t o = 0;
  auto put = [&](size_t bytes) { const size_t at = o; o = align256(o + bytes); return at; };
  const size_t o_rec = put(out ? (size_t)nout * sizeof(fstat_candidate) : 0),
               o_key = put(keys ? (size_t)nout * sizeof(fstat_candidate_key) : 0), o_val = put(ndouble * 8),
               o_list = put((size_t)nsearch * sizeof(DrainList)), o_seg = put(p->segs.size() * sizeof(DrainSeg));
  if (o > p->drain_out_bytes) {
    if (p->drain_out) (void)hipFree(p->drain_out);
    p->drain_out = nullptr;
    p->drain_out_bytes = 0;
    HIP_TRY(p, hipMalloc(&p->drain_out, o), "drain record memory");
    p->drain_out_bytes = o;
  }
  char* w = (char*)p->drain_out;
  double* vals = (double*)(w + o_val);
  std::vector<DrainList> hl((size_t)nsearch);
  size_t at = 0;
  for (int i = 0; i < nsearch; ++i) {
    const SearchRecord& sr = p->searches[(size_t)i];
    HIP_TRY(p, hipMemcpy(vals + at, sr.host, nd[(size_t)i] * 8, hipMemcpyHostToDevice), "drain lists");
    DrainList& L = hl[(size_t)i];
    L.v = vals + at;
    L.nsky = sr.nsky;
    L.lattice = sr.lattice ? 1 : 0;
    L.s_lo = sr.s_lo;
    L.m10 = sr.m10;
    L.m11 = sr.m11;
    at += nd[(size_t)i];
  }
  std::vector<DrainSeg> hg(p->segs.size());
  for (size_t i = 0; i < p->segs.size(); ++i) {
    hg[i].f_off = p->segs[i].s.f_off;
    hg[i].dt = p->segs[i].s.dt;
    hg[i].nfft = p->segs[i].nfft;
  }
  DrainList* dl = (DrainList*)(w + o_list);
  DrainSeg* dg = (DrainSeg*)(w + o_seg);
  HIP_TRY(p, hipMemcpy(dl, hl.data(), hl.size() * sizeof(DrainList), hipMemcpyHostToDevice), "drain lists");
  HIP_TRY(p, hipMemcpy(dg, hg.data(), hg.size() * sizeof(DrainSeg), hipMemcpyHostToDevice), "drain segments");
  fstat_candidate* drec = out ? (fstat_candidate*)(w + o_rec) : nullptr;
  fstat_candidate_key* dkey = keys ? (fstat_candidate_key*)(w + o_key) : nullptr;
  const unsigned blk = (unsigned)std::min<long long>((nout + DRAIN_NT - 1) / DRAIN_NT, 1LL << 20);
  FSTAT_LAUNCH(k_drain_records, dim3(blk), dim3(DRAIN_NT), 0, (hipStream_t)nullptr, p->d_cand, nout, dl, search0, dg,
               p->scored ? 1 : 0, drec, dkey);
  HIP_TRY(p, launch_status(), "drain records launch");
  if (out) HIP_TRY(p, hipMemcpy(out, drec, (size_t)nout * sizeof(fstat_candidate), hipMemcpyDeviceToHost), "record copy");
  if (keys)
    HIP_TRY(p, hipMemcpy(keys, dkey, (size_t)nout * sizeof(fstat_candidate_key), hipMemcpyDeviceToHost), "key copy");
  return FSTAT_OK;
}

fstat_status fstat_candidates(fstat_plan_t plan, fstat_candidate* out, fstat_candidate_key* keys, int64_t capacity,
                              int64_t* n_found) {
  if (!plan || !n_found) return fail(plan, FSTAT_E_INVAL, "NULL argument");
  if (capacity < 0) return fail(plan, FSTAT_E_INVAL, "capacity < 0");
  *n_found = 0;
  if (plan->used_stream) HIP_TRY(plan, hipStreamSynchronize(plan->last_stream), "stream synchronize");
  HIP_TRY(plan, hipDeviceSynchronize(), "device synchronize");
  unsigned long long count = 0;
  HIP_TRY(plan, hipMemcpy(&count, plan->d_count, sizeof count, hipMemcpyDeviceToHost), "count copy");
  const long long stored = std::min<long long>((long long)count, plan->opt.candidate_capacity);
  if (!out && !keys) {
    // count-only drain: nothing is copied or sorted
    plan->scored = false;
    HIP_TRY(plan, hipMemset(plan->d_count, 0, sizeof(unsigned long long)), "count reset");
    for (auto& sr : plan->searches) (void)hipHostFree(sr.host);
    plan->searches.clear();
    *n_found = (int64_t)count;
    if ((long long)count > plan->opt.candidate_capacity)
      return fail(plan, FSTAT_E_OVERFLOW, "more candidates than the device buffer holds");
    return FSTAT_OK;
  }
  // key order, records and keys on the device; the first min(stored, capacity) copied out
  const long long nout = std::min<long long>(stored, capacity);
  if (stored > 0 && nout > 0) {
    fstat_status r = order_on_device(plan, stored);
    if (r == FSTAT_OK) r = form_on_device(plan, nout, out, keys);
    if (r != FSTAT_OK) return r;
  }
  HIP_TRY(plan, hipMemset(plan->d_count, 0, sizeof(unsigned long long)), "count reset");
  for (auto& sr : plan->searches) (void)hipHostFree(sr.host);
  plan->searches.clear();
  plan->scored = false;
  *n_found = (int64_t)count;
  if ((long long)count > plan->opt.candidate_capacity || (long long)count > capacity)
    return fail(plan, FSTAT_E_OVERFLOW, "more candidates than buffer capacity");
  return FSTAT_OK;
}

fstat_status fstat_profile_enable(fstat_plan_t plan, int32_t on) {
  if (!plan) return fail(plan, FSTAT_E_INVAL, "NULL plan");
  plan->profiling = on != 0;
  return FSTAT_OK;
}

fstat_status fstat_profile_read(fstat_plan_t plan, int32_t kernel_class, int64_t* launches, double* total_ms,
                                int32_t reset) {
  if (!plan || kernel_class < 0 || kernel_class >= FSTAT_KERNEL_COUNT)
    return fail(plan, FSTAT_E_INVAL, "bad arguments");
  int64_t cnt = 0;
  double tot = 0.0;
  for (auto& pr : plan->prof) {
    if (pr.cls != kernel_class) continue;
    HIP_TRY(plan, hipEventSynchronize(pr.b), "event synchronize");
    float ms = 0.f;
    HIP_TRY(plan, hipEventElapsedTime(&ms, pr.a, pr.b), "event elapsed");
    tot += ms;
    ++cnt;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = tot;
  if (reset) {
    std::vector<ProfRec> keep;
    for (auto& pr : plan->prof) {
      if (pr.cls == kernel_class) {
        if (!pr.borrowed) {
          plan->ev_pool.push_back(pr.a);
          plan->ev_pool.push_back(pr.b);
        }
      } else {
        keep.push_back(pr);
      }
    }
    plan->prof.swap(keep);
  }
  return FSTAT_OK;
}

fstat_status fstat_plan_info(fstat_plan_t plan, int32_t segment, int32_t* nfft, int32_t* p, int32_t* q,
                             int32_t* templates_per_launch, int32_t* skies_per_batch, int32_t* pass_a_variant,
                             int32_t* pass_b_variant) {
  if (!plan || segment < 0 || segment >= (int32_t)plan->segs.size())
    return fail(plan, FSTAT_E_INVAL, "bad arguments");
  const SegInfo& si = plan->segs[segment];
  if (nfft) *nfft = si.nfft;
  if (p) *p = si.tP;
  if (q) *q = si.tQ;
  if (templates_per_launch) *templates_per_launch = plan->B;
  if (skies_per_batch) *skies_per_batch = plan->Sb;
  if (pass_a_variant) *pass_a_variant = plan->variant_a;
  if (pass_b_variant) *pass_b_variant = plan->variant_b;
  return FSTAT_OK;
}

// ------------------------------------------------------------------ autotuner
fstat_status fstat_autotune(fstat_plan_t plan, int32_t segment, double budget_ms, void* stream) {
  if (!plan || segment < 0 || segment >= (int32_t)plan->segs.size() || !(budget_ms > 0))
    return fail(plan, FSTAT_E_INVAL, "bad arguments");
  if (plan->ws && !plan->ws_owned) return fail(plan, FSTAT_E_STATE, "autotune must precede fstat_plan_set_workspace");
  if (plan->vet) return fail(plan, FSTAT_E_STATE, "autotune must precede fstat_plan_attach_vetter");
  hipStream_t st = (hipStream_t)stream;
  const SegInfo& si = plan->segs[segment];
  // trial template lists: 128 sky positions spread over the sphere (several batches of
  // every candidate batch size, so that the first batch's sky stage, which no template
  // work hides, weighs little), 256 spindowns
  const int nsky = 128, nfdot = 256;
  std::vector<double> h(2 * nsky + nfdot);
  for (int i = 0; i < nsky; ++i) {
    h[i] = std::fmod(2.0 * M_PI * i * 0.6180339887498949, 2.0 * M_PI);
    h[nsky + i] = std::asin(1.0 - (2.0 * i + 1.0) / nsky);
  }
  for (int i = 0; i < nfdot; ++i) h[2 * nsky + i] = -1e-9 * i / (nfdot - 1);
  double* dl = nullptr;
  HIP_TRY(plan, hipMalloc(&dl, h.size() * sizeof(double)), "autotune lists");
  struct Cand { int B, Sb, v; };
  std::vector<Cand> cands;
  for (int v = 0; v < 2; ++v)
    for (int b : {64, 128, 256, 512})
      for (int sb : {16, 32})
        if (!plan->opt.workspace_budget_bytes || layout(plan, sb, b, false) <= plan->opt.workspace_budget_bytes)
          cands.push_back({b, sb, v});
  const int B0 = plan->B, Sb0 = plan->Sb, V0 = plan->variant_a;
  const int graph0 = plan->opt.use_graph;
  const bool prof0 = plan->profiling;
  plan->opt.use_graph = 0;
  plan->profiling = false;
  double best = 1e300;
  Cand bestc{B0, Sb0, V0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fstat_status r = FSTAT_OK;
  hipError_t e = hipMemcpy(dl, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) r = hip_fail(plan, e, "autotune setup");
  const double per_cand_ms = budget_ms / std::max<size_t>(1, cands.size());
  for (size_t ci = 0; r == FSTAT_OK && ci < cands.size(); ++ci) {
    const Cand c = cands[ci];
    plan->B = c.B;
    plan->Sb = c.Sb;
    plan->variant_a = c.v;
    if (plan->ws_owned && plan->ws) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(plan->ws);
      plan->ws = nullptr;
    }
    if ((r = ensure_workspace(plan)) != FSTAT_OK) break;
    // warm-up on one sky batch, then time whole batches until the share of the budget is used
    const int ns = std::min(nsky, c.Sb);
    if ((r = run_search(plan, segment, explicit_grid(dl, dl + nsky, ns, dl + 2 * nsky, nfdot), 0, nullptr, st)) !=
        FSTAT_OK)
      break;
    double ms_sum = 0.0;
    long tmpl = 0;
    int reps = 0;
    while (reps < 8 && (reps < 1 || ms_sum < per_cand_ms)) {
      (void)hipEventRecord(e0, st);
      if ((r = run_search(plan, segment, explicit_grid(dl, dl + nsky, nsky, dl + 2 * nsky, nfdot), 0, nullptr, st)) !=
          FSTAT_OK)
        break;
      (void)hipEventRecord(e1, st);
      if ((e = hipEventSynchronize(e1)) != hipSuccess) {
        r = hip_fail(plan, e, "autotune timing");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_sum += ms;
      tmpl += (long)nsky * nfdot;
      ++reps;
    }
    if (r != FSTAT_OK) break;
    const double per_tmpl = ms_sum / (double)tmpl;
    if (per_tmpl < best) {
      best = per_tmpl;
      bestc = c;
    }
  }
  (void)hipStreamSynchronize(st);
  // discard the trial candidates and searches
  (void)hipMemset(plan->d_count, 0, sizeof(unsigned long long));
  (void)hipMemset(plan->d_search_next, 0, sizeof(int));
  plan->search_count = 0;
  for (auto& sr : plan->searches) (void)hipHostFree(sr.host);
  plan->searches.clear();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(dl);
  plan->opt.use_graph = graph0;
  plan->profiling = prof0;
  plan->B = bestc.B;
  plan->Sb = bestc.Sb;
  plan->variant_a = bestc.v;
  if (plan->ws_owned && plan->ws) {
    (void)hipFree(plan->ws);
    plan->ws = nullptr;
    plan->ws_owned = false;
  }
  layout(plan, plan->Sb, plan->B, true);
  if (r != FSTAT_OK) return r;
  if (plan->opt.tuning_cache_path) {
    FILE* f = std::fopen(plan->opt.tuning_cache_path, "a");
    if (f) {
      std::fprintf(f, "%s %ld %d %d %d %d\n", device_tag().c_str(), plan->L_max, cache_precision(plan->opt), plan->B,
                   plan->Sb, plan->variant_a | (plan->variant_b << 1));
      std::fclose(f);
    }
  }
  return FSTAT_OK;
}

fstat_status fstat_destroy(fstat_plan_t plan) {
  if (!plan) return FSTAT_OK;
  if (plan->tab.dev || plan->ws || plan->d_cand) (void)hipDeviceSynchronize();
  for (auto& pr : plan->prof) {
    if (pr.borrowed) continue;
    (void)hipEventDestroy(pr.a);
    (void)hipEventDestroy(pr.b);
  }
  for (auto e : plan->ev_pool) (void)hipEventDestroy(e);
  for (auto& sr : plan->searches) (void)hipHostFree(sr.host);
  if (plan->ws_owned && plan->ws) (void)hipFree(plan->ws);
  if (plan->tab.dev) (void)hipFree(plan->tab.dev);
  if (plan->d_cand) (void)hipFree(plan->d_cand);
  if (plan->d_count) (void)hipFree(plan->d_count);
  if (plan->d_search_next) (void)hipFree(plan->d_search_next);
  if (plan->d_sky_pos) (void)hipFree(plan->d_sky_pos);
  if (plan->d_patches) (void)hipFree(plan->d_patches);
  if (plan->d_spec) (void)hipFree(plan->d_spec);
  if (plan->d_first) (void)hipFree(plan->d_first);
  if (plan->drain_ws) (void)hipFree(plan->drain_ws);
  if (plan->drain_out) (void)hipFree(plan->drain_out);
  for (auto& ge : plan->graphs) {
    if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    if (ge.graph) (void)hipGraphDestroy(ge.graph);
    for (auto& pr : ge.events) {
      (void)hipEventDestroy(pr.a);
      (void)hipEventDestroy(pr.b);
    }
  }
  if (plan->sstream) (void)hipStreamSynchronize(plan->sstream);
  for (int k = 0; k < 2; ++k) {
    if (plan->ev_sky[k]) (void)hipEventDestroy(plan->ev_sky[k]);
    if (plan->ev_tmpl[k]) (void)hipEventDestroy(plan->ev_tmpl[k]);
  }
  if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
  if (plan->sstream) (void)hipStreamDestroy(plan->sstream);
  if (plan->ev_in) (void)hipEventDestroy(plan->ev_in);
  if (plan->ev_out) (void)hipEventDestroy(plan->ev_out);
  if (plan->gstream) (void)hipStreamDestroy(plan->gstream);
  delete plan;
  return FSTAT_OK;
}

