// Host runtime of the C ABI declared in include/lsh.h: validation, workspace
// carving, tables, and the solver loops (conjugate gradients, basic scheme,
// FP32/FP64 iterative refinement) driving the transform kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include <sys/mman.h>
#include <ucontext.h>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "dispatch.hpp"
#include "solver_kernels.hpp"
#include "tiny.hpp"
#include "lsh.h"

// Named host ranges for profilers (rocprofv3 --marker-trace): setup, solves,
// the inner solves and refinement residuals of the mixed path, tuning and
// ensembles.  Started and stopped by id (not a per-thread stack), since the
// members of an ensemble interleave on one thread as fibers.
struct TraceRange {
  roctx_range_id_t id;
  explicit TraceRange(const char* name) : id(roctxRangeStartA(name)) {}
  ~TraceRange() { roctxRangeStop(id); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

using namespace lsh;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }
// axis lengths with compiled transform instances: powers of two up to 1024,
// and 48, 96, 192 (3 * 2^m), 80, 160 (5 * 2^m)
bool supported_axis(long long v) {
  if (is_pow2(v)) return v <= 1024;
  return v == 48 || v == 96 || v == 192 || v == 80 || v == 160;
}

// ---------------------------------------------------------------------------
// small dense linear algebra on the host (c <= 6)
// ---------------------------------------------------------------------------
// Inverse by Gauss-Jordan with partial pivoting; false when singular.
bool invert(int n, const double* a, double* inv) {
  double m[6][12];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) m[i][j] = j < n ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
  double scale = 0.0;
  for (int i = 0; i < n * n; ++i) scale = std::max(scale, std::fabs(a[i]));
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(m[r][col]) > std::fabs(m[piv][col])) piv = r;
    if (!(std::fabs(m[piv][col]) > 1e-13 * scale)) return false;
    if (piv != col)
      for (int j = 0; j < 2 * n; ++j) std::swap(m[col][j], m[piv][j]);
    const double d = m[col][col];
    for (int j = 0; j < 2 * n; ++j) m[col][j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = m[r][col];
      if (f != 0.0)
        for (int j = 0; j < 2 * n; ++j) m[r][j] -= f * m[col][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) inv[i * n + j] = m[i][n + j];
  return true;
}

// Eigenvalues of a symmetric matrix (cyclic Jacobi).
void sym_eigvals(int n, const double* a, double* ev) {
  double m[6][6];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) m[i][j] = 0.5 * (a[i * n + j] + a[j * n + i]);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += m[i][j] * m[i][j];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (std::fabs(m[p][q]) < 1e-300) continue;
        const double th = 0.5 * (m[q][q] - m[p][p]) / m[p][q];
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double mkp = m[k][p], mkq = m[k][q];
          m[k][p] = c * mkp - s * mkq;
          m[k][q] = s * mkp + c * mkq;
        }
        for (int k = 0; k < n; ++k) {
          const double mpk = m[p][k], mqk = m[q][k];
          m[p][k] = c * mpk - s * mqk;
          m[q][k] = s * mpk + c * mqk;
        }
      }
  }
  for (int i = 0; i < n; ++i) ev[i] = m[i][i];
}

bool symmetric(int n, const double* a) {
  double scale = 0.0;
  for (int i = 0; i < n * n; ++i) scale = std::max(scale, std::fabs(a[i]));
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (std::fabs(a[i * n + j] - a[j * n + i]) > 1e-12 * scale) return false;
  return true;
}

struct KTimer {
  int cls;
  double bytes;
  hipEvent_t a, b;
};

// Kernel classes for the timing facility; the transform and update kernels
// are split by element type (FP32 / FP64).
const char* kClassNames[] = {"xfwd_f32",   "xfwd_f64",   "y_f32",   "y_f64",   "zgamma_f32",
                             "zgamma_f64", "xinv_f32",   "xinv_f64", "cg_update_f32", "cg_update_f64",
                             "scalars",    "init",       "mean",     "copy",          "gradient",
                             "persistent_cg"};
enum KClass {
  K_XFWD = 0, K_Y = 2, K_ZG = 4, K_XINV = 6, K_CGUPD = 8,  // + 1 for FP64
  K_SCAL = 10, K_INIT, K_MEAN, K_COPY, K_GRAD, K_TINY, K_NCLASS
};
template <typename T> constexpr int kcls(int base) { return base + (sizeof(T) == 8 ? 1 : 0); }

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct lsh_ctx {
  int dim = 0, physics = 0, precision = 0, max_loads = 0, c = 0;
  int n[3] = {1, 1, 1};
  hipStream_t stream = nullptr;
  Geo geo{};
  long long F = 0;  // reals per load field

  // host-side problem definition
  bool have_ref = false, have_phase = false;
  std::vector<double> A0;
  int green = LSH_GREEN_FILTERED;
  int nphase = 0;
  std::vector<double> moduli;
  std::vector<uint8_t> phase_host;
  const uint8_t* phase_dev_src = nullptr;
  bool tables_dirty = true, phase_dirty = true, consts_ready = false;
  GreenParams gp{};
  char* gtab = nullptr;   // bound consistent-operator table (FP64 entries, then FP32)
  size_t gtab_size = 0;
  int series = 8;
  int iso = 0;  // every phase matrix has the short form (see phase_row)
  bool mat_voxel = false;  // material given per voxel (lsh_set_voxel_moduli) instead of per phase
  bool cg_fused = true;    // CG with p.Lp from the x and z passes and r updated in the x-inverse pass
  bool persistent = true;  // small grids: the whole CG loop of a load in one workgroup
  bool tab_em = false;     // second table matrix: (A-A0)(A+A0)^{-1} (Eyre--Milton) instead of A-A0
  // stored operator of the z pass (filtered operator, 3D, three or six
  // components; FP32 entries in a mixed context, FP64 in an FP64 one): formed
  // once per reference medium instead of at every application.  LSH_GSTORE=0
  // keeps the operator formed on the fly.
  bool gstore = true;
  bool gst_dirty = true;
  char* sbuf = nullptr;    // bound solver buffer (MINRES fields)
  size_t sbuf_size = 0;
  int tune[2][NPASS] = {{0, 0, 0, 0}, {0, 0, 0, 0}};  // kernel-shape variant per (FP32/FP64, pass)
  // CG breakdown threshold g (|p.Lp| <= g r.r) for FP32 and FP64 fields:
  // eps times a bound of ||L||_2 (max ||(A - A0)^{-1}|| over the phases plus
  // ||A0^{-1}||, which bounds every Green operator)
  double bd_guard[2] = {0.0, 0.0};

  // workspace
  char* ws = nullptr;
  size_t ws_need = 0, ws_size = 0;
  int ws_device = -1;   // device holding the workspace (-1: unknown)
  // pinned host staging of the state and result reads (the solver scalars
  // and sums come back through it without blocking the host thread), and the
  // event a wait records
  void* hpin = nullptr;
  hipEvent_t wait_ev = nullptr;
  // spectrum buffers used instead of the workspace's while set (the
  // allocation-free operator: main spectrum in the caller's output, Nyquist
  // plane in the per-device scratch array)
  void* ovr_sm = nullptr;
  void* ovr_sn = nullptr;
  int hist_loads = 0;   // loads of the last solve (their residual histories are valid)
  struct {
    size_t x64, r64, p64, p64b, d32, r32, p32, p32b, s64m, s64n, s32m, s32n, phase, i0, ptab64, ptab32, vc64, vc32, tw64, tw32,
        wt64, wt32, loads, wgrad, st_out, st_in, mstate, guess, partials, sums, gst, hist, hcnt, end;
  } off{};
  long long pstride = 0, nsums = 0;
  int twoff[3] = {0, 0, 0};
  int wstride = 0;

  // initial guesses for the next solve (per load; the guess itself is in x64),
  // and the flags of the solve in progress (staging of their upload)
  std::vector<uint8_t> h_guess, h_guess_up;

  // host staging kept alive across asynchronous copies
  std::vector<double> h_ptab64, h_loads;
  std::vector<float> h_ptab32;
  std::vector<uint8_t> h_i0;
  std::vector<double> h_tw64, h_wt64;
  std::vector<float> h_tw32, h_wt32;

  // last solve
  int last_nload = 0;
  bool have_solution = false;
  std::vector<double> last_loads, sigma;

  // graphs: one solver iteration captured once and replayed
  bool use_graphs = true;
  hipStream_t cap_stream = nullptr;
  struct IterGraph {
    hipGraphExec_t exec = nullptr;
    long long key = -1;
  } graphs[5];   // CG FP64, CG FP32, fixed point; CG FP64 and FP32 of odd iterations (fused step)
  long long graph_epoch = 0;  // bumped whenever captured kernel arguments may change

  // timing
  bool timing = false;
  int nact = 1 << 30;  // host's count of loads still iterating (bounds the bytes of a launch)
  bool xf_first = false;  // the CG x pass being queued is the first of its solve
  std::vector<KTimer> pending;
  std::vector<hipEvent_t> pool;
  double tsum[K_NCLASS] = {0};
  double tbytes[K_NCLASS] = {0};
  long long tcount[K_NCLASS] = {0};

  std::string err;

  template <typename T> T* ptr(size_t o) const { return reinterpret_cast<T*>(ws + o); }
};

namespace {

lsh_status fail(lsh_ctx* ctx, lsh_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(ctx, LSH_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

#define STCHK(expr)                       \
  do {                                    \
    lsh_status s_ = (expr);               \
    if (s_ != LSH_OK) return s_;          \
  } while (0)

lsh_status check_launch(lsh_ctx* ctx, int r, const char* what) {
  if (r < 0) return fail(ctx, LSH_EINVAL, std::string("unsupported grid size for ") + what);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, LSH_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return LSH_OK;
}

// ------------------------- kernel timing ---------------------------------
hipEvent_t take_event(lsh_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events when timing is on; `bytes` is the
// launch's algorithmic HBM traffic (what the pass must read and write).
struct Scope {
  lsh_ctx* ctx;
  int cls;
  double bytes;
  hipEvent_t a = nullptr;
  Scope(lsh_ctx* c, int k, double b = 0.0) : ctx(c), cls(k), bytes(b) {
    if (ctx->timing) {
      a = take_event(ctx);
      if (a) (void)hipEventRecord(a, ctx->stream);
    }
  }
  ~Scope() {
    if (ctx->timing && a) {
      hipEvent_t b = take_event(ctx);
      if (b) {
        (void)hipEventRecord(b, ctx->stream);
        ctx->pending.push_back({cls, bytes, a, b});
      }
    }
  }
};

void drain_timers(lsh_ctx* ctx) {
  if (ctx->pending.empty()) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& t : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      ctx->tsum[t.cls] += ms;
      ctx->tbytes[t.cls] += t.bytes;
      ctx->tcount[t.cls] += 1;
    }
    ctx->pool.push_back(t.a);
    ctx->pool.push_back(t.b);
  }
  ctx->pending.clear();
}

// ------------------------- waits and the ensemble fibers ----------------
// lsh_solve_many runs the solves of an ensemble as fibers (user-level
// contexts) on the calling thread.  Every wait for the GPU inside a solve
// (wait_stream) records an event on the context's stream and, inside a
// fiber, hands the thread to the next fiber until the event has passed; so
// the members' kernels overlap on their own streams while every HIP call
// comes from one host thread, one member at a time.
struct Fiber {
  ucontext_t uc{};
  void* stack = nullptr;
  size_t stack_bytes = 0;
  bool done = false;
  std::function<void()> body;
};

struct FiberSched {
  ucontext_t main{};
  Fiber* cur = nullptr;
};
thread_local FiberSched t_fibers;

void fiber_yield() {
  Fiber* f = t_fibers.cur;
  if (f) swapcontext(&f->uc, &t_fibers.main);
}

void fiber_entry() {
  Fiber* f = t_fibers.cur;
  f->body();
  f->done = true;
  swapcontext(&f->uc, &t_fibers.main);
}

// Wait until the work queued on the context's stream has finished.
lsh_status wait_stream(lsh_ctx* ctx) {
  if (t_fibers.cur == nullptr) {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return LSH_OK;
  }
  if (!ctx->wait_ev) HIPCHK(hipEventCreateWithFlags(&ctx->wait_ev, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ctx->wait_ev, ctx->stream));
  while (true) {
    const hipError_t q = hipEventQuery(ctx->wait_ev);
    if (q == hipSuccess) break;
    if (q != hipErrorNotReady) return fail(ctx, LSH_EHIP, std::string("event query: ") + hipGetErrorString(q));
    fiber_yield();
    if (ctx->ws_device >= 0) {
      int cur = -1;
      if (hipGetDevice(&cur) == hipSuccess && cur != ctx->ws_device) HIPCHK(hipSetDevice(ctx->ws_device));
    }
  }
  return LSH_OK;
}

// Pinned staging: the LoadState records of max_loads loads, then max_loads c doubles.
lsh_status pinned(lsh_ctx* ctx, void** out) {
  if (!ctx->hpin) {
    const size_t bytes = sizeof(LoadState) * ctx->max_loads + sizeof(double) * ctx->max_loads * ctx->c;
    HIPCHK(hipHostMalloc(&ctx->hpin, bytes, hipHostMallocDefault));
  }
  *out = ctx->hpin;
  return LSH_OK;
}

// Copy n bytes from the device into host memory h through the pinned staging
// (at byte offset `at` of it), waiting with wait_stream.
lsh_status read_back(lsh_ctx* ctx, void* h, const void* dev, size_t n, size_t at) {
  void* p = nullptr;
  STCHK(pinned(ctx, &p));
  char* stage = static_cast<char*>(p) + at;
  HIPCHK(hipMemcpyAsync(stage, dev, n, hipMemcpyDeviceToHost, ctx->stream));
  STCHK(wait_stream(ctx));
  std::memcpy(h, stage, n);
  return LSH_OK;
}

// ------------------------- layout ----------------------------------------
// grids whose z pass has a stored-operator instance
bool gst_shape(const lsh_ctx* ctx) { return ctx->dim == 3 && ctx->n[2] > 1 && (ctx->c == 3 || ctx->c == 6); }

void compute_layout(lsh_ctx* ctx) {
  const long long L = ctx->max_loads, F = ctx->F, c = ctx->c;
  const long long V = ctx->geo.nvox;
  const long long nyq = (long long)c * ctx->n[2] * ctx->n[1];
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const bool mixed = ctx->precision == LSH_MIXED;
  ctx->off.x64 = take(sizeof(double) * L * F);
  ctx->off.r64 = mixed ? 0 : take(sizeof(double) * L * F);
  ctx->off.p64 = mixed ? 0 : take(sizeof(double) * L * F);
  ctx->off.p64b = mixed ? 0 : take(sizeof(double) * L * F);   // second direction buffer of the fused CG step
  ctx->off.d32 = mixed ? take(sizeof(float) * L * F) : 0;
  ctx->off.r32 = mixed ? take(sizeof(float) * L * F) : 0;
  ctx->off.p32 = mixed ? take(sizeof(float) * L * F) : 0;
  ctx->off.p32b = mixed ? take(sizeof(float) * L * F) : 0;
  ctx->off.s64m = take(sizeof(double) * L * F);
  ctx->off.s64n = take(2 * sizeof(double) * L * nyq);
  ctx->off.s32m = mixed ? take(sizeof(float) * L * F) : 0;
  ctx->off.s32n = mixed ? take(2 * sizeof(float) * L * nyq) : 0;
  ctx->off.phase = take(V + 16);
  ctx->off.i0 = take(256);
  const int tabw = 2 * ctx->c * ctx->c + 5;
  ctx->off.ptab64 = take(sizeof(double) * kMaxPhases * tabw);
  ctx->off.ptab32 = take(sizeof(float) * kMaxPhases * tabw);
  ctx->off.vc64 = take(sizeof(double) * 2 * V);
  ctx->off.vc32 = mixed ? take(sizeof(float) * 2 * V) : 0;
  const int ntw = ctx->n[0] + ctx->n[1] + ctx->n[2];
  ctx->twoff[0] = 0;
  ctx->twoff[1] = ctx->n[0];
  ctx->twoff[2] = ctx->n[0] + ctx->n[1];
  ctx->off.tw64 = take(2 * sizeof(double) * ntw);
  ctx->off.tw32 = take(2 * sizeof(float) * ntw);
  ctx->wstride = std::max(ctx->n[0], std::max(ctx->n[1], ctx->n[2]));
  ctx->off.wt64 = take(2 * sizeof(double) * 3 * ctx->wstride);
  ctx->off.wt32 = take(2 * sizeof(float) * 3 * ctx->wstride);
  ctx->off.loads = take(sizeof(double) * L * c);
  ctx->off.wgrad = take(sizeof(double) * L * L);
  ctx->off.st_out = take(sizeof(LoadState) * L);
  ctx->off.st_in = take(sizeof(LoadState) * L);
  ctx->off.mstate = take(sizeof(MinresState) * L);
  ctx->off.guess = take(L);
  ctx->h_guess.assign(L, 0);
  // partial sums: the largest grid of any reducing kernel, per group
  // (the fused CG step writes the x pass's and the z pass's partials side by side)
  long long pmax = xinv_blocks(ctx->geo, 2) + zg_blocks_max<float>(ctx->geo);
  pmax = std::max(pmax, (F + 1023) / 1024 + 1);
  ctx->pstride = pmax;
  ctx->off.partials = take(sizeof(double) * L * c * pmax);
  ctx->nsums = L * c;
  ctx->off.sums = take(sizeof(double) * L * c);
  // stored z-pass operator: NG quads of the field type per half-spectrum wave-vector
  ctx->off.gst = 0;
  if (gst_shape(ctx)) {
    const long long nk = (long long)ctx->n[2] * ctx->n[1] * (ctx->n[0] / 2 + 1);
    const int ng = c == 6 ? store_groups<6>() : store_groups<3>();
    ctx->off.gst = take((mixed ? sizeof(float) : sizeof(double)) * 4 * ng * nk);
  }
  // residual history: a ring of kHistCap (value, level) pairs and a count per load
  ctx->off.hist = take(sizeof(double) * 2 * kHistCap * L);
  ctx->off.hcnt = take(sizeof(unsigned long long) * L);
  ctx->off.end = o;
  ctx->ws_need = o;
}

// twiddles W_N^m = exp(-2 pi i m / N) and filter weights per axis
void build_consts(lsh_ctx* ctx) {
  const int ntw = ctx->n[0] + ctx->n[1] + ctx->n[2];
  ctx->h_tw64.assign(2 * ntw, 0.0);
  ctx->h_tw32.assign(2 * ntw, 0.f);
  for (int a = 0; a < 3; ++a) {
    const int N = ctx->n[a];
    for (int m = 0; m < N; ++m) {
      const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)N;
      double cr = (double)cosl(ang), ci = (double)(-sinl(ang));
      if (4 * m == N) { cr = 0.0; ci = -1.0; }
      if (2 * m == N) { cr = -1.0; ci = 0.0; }
      if (4 * m == 3 * N) { cr = 0.0; ci = 1.0; }
      const int i = ctx->twoff[a] + m;
      ctx->h_tw64[2 * i] = cr;
      ctx->h_tw64[2 * i + 1] = ci;
      ctx->h_tw32[2 * i] = (float)cr;
      ctx->h_tw32[2 * i + 1] = (float)ci;
    }
  }
  const int W = ctx->wstride;
  ctx->h_wt64.assign(2 * 3 * W, 0.0);
  ctx->h_wt32.assign(2 * 3 * W, 0.f);
  for (int a = 0; a < 3; ++a) {
    const int N = ctx->n[a];
    for (int k = 0; k < N; ++k) {
      const long double t = 3.14159265358979323846264338327950288L * (long double)k / (2.0L * N);
      const long double cc = cosl(t), ss = sinl(t);
      const int i = a * W + k;
      ctx->h_wt64[2 * i] = (double)(cc * cc);
      ctx->h_wt64[2 * i + 1] = (double)(ss * ss);
      ctx->h_wt32[2 * i] = (float)(cc * cc);
      ctx->h_wt32[2 * i + 1] = (float)(ss * ss);
    }
  }
}

lsh_status upload_consts(lsh_ctx* ctx) {
  build_consts(ctx);
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.tw64, ctx->h_tw64.data(), ctx->h_tw64.size() * sizeof(double),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.tw32, ctx->h_tw32.data(), ctx->h_tw32.size() * sizeof(float),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.wt64, ctx->h_wt64.data(), ctx->h_wt64.size() * sizeof(double),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.wt32, ctx->h_wt32.data(), ctx->h_wt32.size() * sizeof(float),
                        hipMemcpyHostToDevice, ctx->stream));
  STCHK(wait_stream(ctx));
  ctx->consts_ready = true;
  return LSH_OK;
}

// Phase tables against the current A0: (A-A0)^{-1}, (A-A0), I0 flag; checks hypothesis (2).
lsh_status build_tables(lsh_ctx* ctx) {
  TraceRange tr("lsh setup: material tables");
  const int c = ctx->c;
  const int tabw = 2 * c * c + 5;
  ctx->h_ptab64.assign((size_t)kMaxPhases * tabw, 0.0);
  bool all_iso = true;
  ctx->h_ptab32.assign((size_t)kMaxPhases * tabw, 0.f);
  ctx->h_i0.assign(256, 0);
  double lmax = 0.0;   // max over phases of ||(A - A0)^{-1}||_2
  for (int p = 0; p < ctx->nphase; ++p) {
    double D[36], Dinv[36];
    bool zero = true;
    double scale = 0.0;
    for (int i = 0; i < c * c; ++i) {
      D[i] = ctx->moduli[(size_t)p * c * c + i] - ctx->A0[i];
      zero &= (D[i] == 0.0);
      scale = std::max(scale, std::fabs(ctx->moduli[(size_t)p * c * c + i]) + std::fabs(ctx->A0[i]));
    }
    double* row = &ctx->h_ptab64[(size_t)p * tabw];
    if (zero) continue;  // outside I0: all zero, flag 0
    double ev[6];
    sym_eigvals(c, D, ev);
    double lo = ev[0], hi = ev[0];
    for (int i = 1; i < c; ++i) {
      lo = std::min(lo, ev[i]);
      hi = std::max(hi, ev[i]);
    }
    const double eps = 1e-12 * scale;
    if (!((lo > eps) || (hi < -eps)))
      return fail(ctx, LSH_EHYP2,
                  "phase " + std::to_string(p) + ": A - A0 is neither zero nor definite (hypothesis (2))");
    if (!invert(c, D, Dinv)) return fail(ctx, LSH_EHYP2, "phase " + std::to_string(p) + ": A - A0 is singular");
    for (int i = 0; i < c; ++i) lmax = std::max(lmax, 1.0 / std::fabs(ev[i]));
    // second matrix: A - A0 (basic scheme) or (A - A0)(A + A0)^{-1} (Eyre--Milton)
    double S2[36];
    if (ctx->tab_em) {
      double Sum[36], SumInv[36];
      for (int i = 0; i < c * c; ++i) Sum[i] = D[i] + 2.0 * ctx->A0[i];
      if (!invert(c, Sum, SumInv)) return fail(ctx, LSH_EHYP2, "phase " + std::to_string(p) + ": A + A0 is singular");
      for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j) {
          double a = 0.0;
          for (int k = 0; k < c; ++k) a += D[i * c + k] * SumInv[k * c + j];
          S2[i * c + j] = a;
        }
    } else {
      for (int i = 0; i < c * c; ++i) S2[i] = D[i];
    }
    for (int i = 0; i < c * c; ++i) {
      row[i] = Dinv[i];
      row[c * c + i] = S2[i];
    }
    row[2 * c * c] = 1.0;
    // short form a Id + b m m^T (m: normal Mandel components; b = 0 for scalar)
    for (int which = 0; which < 2; ++which) {
      const double* M = which == 0 ? Dinv : S2;
      const bool el = ctx->physics == LSH_ELASTIC;
      const double b = el ? M[1] : 0.0;
      const double a = M[0] - b;
      double mscale = 0.0;
      for (int i = 0; i < c * c; ++i) mscale = std::max(mscale, std::fabs(M[i]));
      for (int i = 0; i < c; ++i)
        for (int j = 0; j < c; ++j) {
          const double expect = (i == j ? a : 0.0) + ((el && i < 3 && j < 3) ? b : 0.0);
          if (std::fabs(M[i * c + j] - expect) > 1e-13 * mscale) all_iso = false;
        }
      row[2 * c * c + 1 + 2 * which] = a;
      row[2 * c * c + 2 + 2 * which] = b;
    }
    ctx->h_i0[p] = 1;
  }
  ctx->iso = (all_iso || ctx->mat_voxel) ? 1 : 0;
  {
    // per-voxel media: ||A0^{-1}|| alone (a smaller bound, a stricter test)
    double ev0[6];
    sym_eigvals(c, ctx->A0.data(), ev0);
    double e0 = ev0[0];
    for (int i = 1; i < c; ++i) e0 = std::min(e0, ev0[i]);
    const double lbound = lmax + 1.0 / e0;
    ctx->bd_guard[0] = 1e-6 * lbound;
    ctx->bd_guard[1] = 1e-12 * lbound;
  }
  for (size_t i = 0; i < ctx->h_ptab64.size(); ++i) ctx->h_ptab32[i] = (float)ctx->h_ptab64[i];

  // Green parameters
  GreenParams& gp = ctx->gp;
  std::memset(&gp, 0, sizeof(gp));
  gp.variant = ctx->green == LSH_GREEN_TRUNCATED    ? kGreenTruncated
               : ctx->green == LSH_GREEN_CONSISTENT ? kGreenConsistent
               : ctx->green == LSH_GREEN_FD         ? kGreenFD
                                                    : kGreenFiltered;
  for (int a = 0; a < 3; ++a) gp.n[a] = ctx->n[a];
  if (ctx->physics == LSH_SCALAR) {
    double inv[9];
    invert(c, ctx->A0.data(), inv);
    for (int i = 0; i < c; ++i)
      for (int j = 0; j < c; ++j) {
        gp.a0[3 * i + j] = ctx->A0[i * c + j];
        gp.a0inv[3 * i + j] = inv[i * c + j];
      }
  } else {
    const double lam0 = ctx->A0[1], mu0 = 0.5 * ctx->A0[3 * 6 + 3];
    const double K0 = lam0 + 2.0 * mu0 / 3.0;
    gp.mu0 = mu0;
    gp.kappa = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0));
    gp.s0_diag = 1.0 / (2.0 * mu0);
    gp.s0_vol = 1.0 / (9.0 * K0) - 1.0 / (6.0 * mu0);
  }
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.ptab64, ctx->h_ptab64.data(), ctx->h_ptab64.size() * sizeof(double),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.ptab32, ctx->h_ptab32.data(), ctx->h_ptab32.size() * sizeof(float),
                        hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.i0, ctx->h_i0.data(), 256, hipMemcpyHostToDevice, ctx->stream));
  if (ctx->green == LSH_GREEN_CONSISTENT) {
    const long long nk = main_cpx(ctx->geo) / ctx->c + nyq_cpx(ctx->geo) / ctx->c;
    const int nb = (int)((nk + 255) / 256);
    const int ne = ctx->c * (ctx->c + 1) / 2;
    double* t64 = reinterpret_cast<double*>(ctx->gtab);
    float* t32 = reinterpret_cast<float*>(ctx->gtab + align_up(sizeof(double) * nk * ne));
    switch (ctx->c) {
      case 2: hipLaunchKernelGGL((k_consistent_table<2>), dim3(nb), dim3(256), 0, ctx->stream, ctx->geo, gp,
                                 ctx->series, t64, t32); break;
      case 3: hipLaunchKernelGGL((k_consistent_table<3>), dim3(nb), dim3(256), 0, ctx->stream, ctx->geo, gp,
                                 ctx->series, t64, t32); break;
      default: hipLaunchKernelGGL((k_consistent_table<6>), dim3(nb), dim3(256), 0, ctx->stream, ctx->geo, gp,
                                  ctx->series, t64, t32); break;
    }
    STCHK(check_launch(ctx, 0, "consistent table"));
  }
  if (gst_shape(ctx) && ctx->gstore && ctx->green == LSH_GREEN_FILTERED && ctx->gst_dirty) {
    const long long nk = main_cpx(ctx->geo) / ctx->c + nyq_cpx(ctx->geo) / ctx->c;
    const int nb = (int)((nk + 255) / 256);
    GreenTabs<double> tb64{ctx->ptr<cpx<double>>(ctx->off.wt64), ctx->wstride, {nullptr, nullptr, nullptr}, nullptr,
                           nullptr};
    const bool mixed = ctx->precision == LSH_MIXED;
#define LSH_GSTORE_BUILD(TO, CC)                                                                             \
  hipLaunchKernelGGL((k_green_store<TO, CC>), dim3(nb), dim3(256), 0, ctx->stream, ctx->geo, gp, tb64,       \
                     ctx->ptr<Quad<TO>>(ctx->off.gst))
    if (ctx->c == 6) {
      if (mixed) LSH_GSTORE_BUILD(float, 6);
      else LSH_GSTORE_BUILD(double, 6);
    } else {
      if (mixed) LSH_GSTORE_BUILD(float, 3);
      else LSH_GSTORE_BUILD(double, 3);
    }
#undef LSH_GSTORE_BUILD
    STCHK(check_launch(ctx, 0, "stored Green operator"));
    ctx->gst_dirty = false;
  }
  STCHK(wait_stream(ctx));
  ctx->tables_dirty = false;
  ctx->graph_epoch++;
  return LSH_OK;
}

// Hypothesis (2) on the host, before anything touches the GPU.
lsh_status validate_phases(lsh_ctx* ctx) {
  const int c = ctx->c;
  for (int p = 0; p < ctx->nphase; ++p) {
    double D[36], Dinv[36];
    bool zero = true;
    double scale = 0.0;
    for (int i = 0; i < c * c; ++i) {
      D[i] = ctx->moduli[(size_t)p * c * c + i] - ctx->A0[i];
      zero &= (D[i] == 0.0);
      scale = std::max(scale, std::fabs(ctx->moduli[(size_t)p * c * c + i]) + std::fabs(ctx->A0[i]));
    }
    if (zero) continue;
    double ev[6];
    sym_eigvals(c, D, ev);
    double lo = ev[0], hi = ev[0];
    for (int i = 1; i < c; ++i) {
      lo = std::min(lo, ev[i]);
      hi = std::max(hi, ev[i]);
    }
    const double eps = 1e-12 * scale;
    if (!((lo > eps) || (hi < -eps)) || !invert(c, D, Dinv))
      return fail(ctx, LSH_EHYP2,
                  "phase " + std::to_string(p) + ": A - A0 is neither zero nor definite (hypothesis (2))");
  }
  return LSH_OK;
}

lsh_status prepare(lsh_ctx* ctx) {
  if (!ctx->have_ref) return fail(ctx, LSH_ESTATE, "reference medium not set");
  if (!ctx->have_phase) return fail(ctx, LSH_ESTATE, "material (phases or per-voxel moduli) not set");
  if (ctx->tables_dirty && !ctx->mat_voxel) STCHK(validate_phases(ctx));
  if (!ctx->ws) return fail(ctx, LSH_ESTATE, "no workspace bound");
  if (ctx->green == LSH_GREEN_CONSISTENT && !ctx->gtab)
    return fail(ctx, LSH_ESTATE, "the consistent operator needs a bound table (lsh_bind_green_table)");
  if (!ctx->consts_ready) {
    lsh_status s = upload_consts(ctx);
    if (s != LSH_OK) return s;
  }
  if (ctx->phase_dirty && !ctx->mat_voxel) {
    const size_t V = (size_t)ctx->geo.nvox;
    if (ctx->phase_dev_src) {
      HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.phase, ctx->phase_dev_src, V, hipMemcpyDeviceToDevice, ctx->stream));
    } else {
      HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.phase, ctx->phase_host.data(), V, hipMemcpyHostToDevice,
                            ctx->stream));
    }
    STCHK(wait_stream(ctx));
    ctx->phase_dev_src = nullptr;
    ctx->phase_dirty = false;
  }
  if (ctx->tables_dirty) {
    lsh_status s = build_tables(ctx);
    if (s != LSH_OK) return s;
  }
  return LSH_OK;
}

// ------------------------- operator pieces -------------------------------
template <typename T> struct Sel;
template <> struct Sel<double> {
  static cpx<double>* sm(lsh_ctx* c) {
    return c->ovr_sm ? static_cast<cpx<double>*>(c->ovr_sm) : c->ptr<cpx<double>>(c->off.s64m);
  }
  static cpx<double>* sn(lsh_ctx* c) {
    return c->ovr_sn ? static_cast<cpx<double>*>(c->ovr_sn) : c->ptr<cpx<double>>(c->off.s64n);
  }
  static const cpx<double>* tw(lsh_ctx* c, int a) { return c->ptr<cpx<double>>(c->off.tw64) + c->twoff[a]; }
  static const cpx<double>* wt(lsh_ctx* c) { return c->ptr<cpx<double>>(c->off.wt64); }
  static const double* ptab(lsh_ctx* c) { return c->ptr<double>(c->off.ptab64); }
  static const double* vc(lsh_ctx* c) { return c->mat_voxel ? c->ptr<double>(c->off.vc64) : nullptr; }
  static const double* gtab(lsh_ctx* c) { return reinterpret_cast<const double*>(c->gtab); }
  static const double* gst(lsh_ctx* c) {
    return (gst_shape(c) && c->gstore && c->green == LSH_GREEN_FILTERED && c->precision == LSH_FP64)
               ? c->ptr<double>(c->off.gst)
               : nullptr;
  }
};
template <> struct Sel<float> {
  static cpx<float>* sm(lsh_ctx* c) {
    return c->ovr_sm ? static_cast<cpx<float>*>(c->ovr_sm) : c->ptr<cpx<float>>(c->off.s32m);
  }
  static cpx<float>* sn(lsh_ctx* c) {
    return c->ovr_sn ? static_cast<cpx<float>*>(c->ovr_sn) : c->ptr<cpx<float>>(c->off.s32n);
  }
  static const cpx<float>* tw(lsh_ctx* c, int a) { return c->ptr<cpx<float>>(c->off.tw32) + c->twoff[a]; }
  static const cpx<float>* wt(lsh_ctx* c) { return c->ptr<cpx<float>>(c->off.wt32); }
  static const float* ptab(lsh_ctx* c) { return c->ptr<float>(c->off.ptab32); }
  static const float* vc(lsh_ctx* c) { return c->mat_voxel ? c->ptr<float>(c->off.vc32) : nullptr; }
  static const float* gtab(lsh_ctx* c) {
    if (!c->gtab) return nullptr;
    const long long nk = main_cpx(c->geo) / c->c + nyq_cpx(c->geo) / c->c;
    return reinterpret_cast<const float*>(c->gtab + align_up(sizeof(double) * nk * (c->c * (c->c + 1) / 2)));
  }
  static const float* gst(lsh_ctx* c) {
    return (gst_shape(c) && c->gstore && c->green == LSH_GREEN_FILTERED && c->precision == LSH_MIXED)
               ? c->ptr<float>(c->off.gst)
               : nullptr;
  }
};



template <typename T> int tv(const lsh_ctx* ctx, int pass) { return ctx->tune[sizeof(T) == 8 ? 1 : 0][pass]; }

// Variants from LSH_TUNE, e.g. "zg32=3,y32=1,xinv64=2" (pass name + 32/64 = variant).
void tune_from_env(lsh_ctx* ctx) {
  const char* f = std::getenv("LSH_CG_FUSED");
  if (f && f[0] == '0') ctx->cg_fused = false;
  const char* pe = std::getenv("LSH_PERSISTENT");
  if (pe && pe[0] == '0') ctx->persistent = false;
  const char* gs = std::getenv("LSH_GSTORE");
  if (gs && gs[0] == '0') ctx->gstore = false;
  const char* e = std::getenv("LSH_TUNE");
  if (!e) return;
  const char* names[NPASS] = {"xfwd", "y", "zg", "xinv"};
  std::string s(e);
  size_t pos = 0;
  while (pos < s.size()) {
    size_t end = s.find(',', pos);
    if (end == std::string::npos) end = s.size();
    const std::string item = s.substr(pos, end - pos);
    const size_t eq = item.find('=');
    if (eq != std::string::npos) {
      const std::string key = item.substr(0, eq);
      const int val = std::atoi(item.c_str() + eq + 1);
      for (int p = 0; p < NPASS; ++p)
        for (int prec = 0; prec < 2; ++prec)
          if (key == std::string(names[p]) + (prec ? "64" : "32") && val >= 0 && val < pass_variants(p))
            ctx->tune[prec][p] = val;
    }
    pos = end + 1;
  }
}

// The component-paired spectrum layout of the Green pass's 8-pencil shape
// (z variant kZPaired): FP32 six-component fields of a mixed context with the
// stored operator and 128- or 256-point y and z axes.
template <typename T>
bool paired_shape(lsh_ctx* ctx) {
  if constexpr (sizeof(T) == 4) {
    const Geo& g = ctx->geo;
    auto ax = [](int n) { return n == 128 || n == 256; };
    return ctx->precision == LSH_MIXED && !ctx->ovr_sm && ctx->tune[0][PASS_ZG] == kZPaired && g.c == 6 &&
           ax(g.ny) && ax(g.nz) && Sel<float>::gst(ctx) != nullptr;
  }
  return false;
}

// Where the x passes use the plain layout (the operator passes of
// forward_part), the y forward pass writes the paired spectrum out of place
// and the y inverse pass reads it back: it lives in the FP64 spectrum buffer
// (4F of its 8F bytes per load), which holds nothing between FP64
// applications.  Null where the shape does not apply: the passes then run in
// place on the plain layout.  (The fused CG step writes and reads the paired
// layout in its x passes and runs every pass in place.)
template <typename T>
cpx<T>* paired_spectrum(lsh_ctx* ctx, int l0) {
  if (!paired_shape<T>(ctx)) return nullptr;
  return reinterpret_cast<cpx<T>*>(ctx->ptr<char>(ctx->off.s64m)) + (long long)l0 * main_cpx(ctx->geo);
}

// Forward passes on load slots [l0, l0+nload): x (mode), y, z (+Gamma and inverse z), y inverse.
template <typename T>
lsh_status forward_part(lsh_ctx* ctx, int l0, int nload, int xmode, const T* src, T* pdir, T* xacc,
                        const float* dsrc, const LoadState* st, bool gamma, const IrxFold& fold = IrxFold{}) {
  const Geo& g = ctx->geo;
  cpx<T>* sm = Sel<T>::sm(ctx) + (long long)l0 * main_cpx(g);
  cpx<T>* sn = Sel<T>::sn(ctx) + (long long)l0 * nyq_cpx(g);
  XfwdArgs<T> xa{g, xmode, src, pdir, xacc, dsrc, sm, sn, Sel<T>::tw(ctx, 0), st, fold};
  // algorithmic bytes per launch (loads still iterating x per-load traffic)
  const double nl = std::min(ctx->nact, nload);
  const double cvs = (double)ctx->F * sizeof(T);
  const double spec = cvs + 2.0 * sizeof(T) * (double)nyq_cpx(g);
  // CG: read r, p, write p, and (after the first step) read and write x
  const double xin = xmode == XF_CG ? (ctx->xf_first ? 3.0 : 5.0) * cvs
                                    : (xmode == XF_IRX ? 2.0 * cvs + 4.0 * ctx->F : cvs);
  {
    Scope sc(ctx, kcls<T>(K_XFWD), nl * (xin + spec));
    STCHK(check_launch(ctx, launch_xfwd<T>(ctx->stream, xa, nload, tv<T>(ctx, PASS_XFWD)), "x forward"));
  }
  cpx<T>* sp = gamma ? paired_spectrum<T>(ctx, l0) : nullptr;
  {
    Scope sc(ctx, kcls<T>(K_Y), nl * 2.0 * spec);
    const int nb = sp ? launch_y_paired<T>(ctx->stream, g, -1, sm, sp, sn, Sel<T>::tw(ctx, 1), st, nload,
                                           tv<T>(ctx, PASS_Y))
                      : launch_y<T>(ctx->stream, g, -1, sm, sn, Sel<T>::tw(ctx, 1), st, nload, tv<T>(ctx, PASS_Y));
    STCHK(check_launch(ctx, nb, "y forward"));
  }
  {
    Scope sc(ctx, kcls<T>(K_ZG), nl * 2.0 * spec);
    GreenTabs<T> tb{Sel<T>::wt(ctx), ctx->wstride, {Sel<T>::tw(ctx, 0), Sel<T>::tw(ctx, 1), Sel<T>::tw(ctx, 2)},
                    Sel<T>::gtab(ctx), Sel<T>::gst(ctx)};
    const int nb = sp ? launch_zg_paired<T>(ctx->stream, g, ctx->gp, tb, sp, sn, Sel<T>::tw(ctx, 2), st, nload,
                                            nullptr, 0)
                      : launch_zg<T>(ctx->stream, g, ctx->gp, tb, gamma ? Z_GAMMA : Z_FWD, sm, sn, Sel<T>::tw(ctx, 2),
                                     st, nload, tv<T>(ctx, PASS_ZG));
    STCHK(check_launch(ctx, nb, "z/Green"));
  }
  if (gamma) {
    Scope sc(ctx, kcls<T>(K_Y), nl * 2.0 * spec);
    const int nb = sp ? launch_y_paired<T>(ctx->stream, g, 1, sm, sp, sn, Sel<T>::tw(ctx, 1), st, nload,
                                           tv<T>(ctx, PASS_Y))
                      : launch_y<T>(ctx->stream, g, 1, sm, sn, Sel<T>::tw(ctx, 1), st, nload, tv<T>(ctx, PASS_Y));
    STCHK(check_launch(ctx, nb, "y inverse"));
  }
  return LSH_OK;
}

template <typename T>
lsh_status inverse_x(lsh_ctx* ctx, int l0, int nload, int mode, const T* tau, T* out, float* rout,
                     const LoadState* st, double* partials, int* nparts, const T* rin = nullptr,
                     bool paired = false) {
  const Geo& g = ctx->geo;
  XinvArgs<T> a{};
  a.g = g;
  a.mode = mode;
  a.nphase = ctx->nphase;
  a.iso = ctx->iso;
  a.smain = Sel<T>::sm(ctx) + (long long)l0 * main_cpx(g);
  a.snyq = Sel<T>::sn(ctx) + (long long)l0 * nyq_cpx(g);
  a.twx = Sel<T>::tw(ctx, 0);
  a.tau = tau;
  a.out = out;
  a.rin = rin;
  a.rout = rout;
  a.ptab = Sel<T>::ptab(ctx);
  a.phase = ctx->ptr<uint8_t>(ctx->off.phase);
  a.vcoef = Sel<T>::vc(ctx);
  a.loads = ctx->ptr<double>(ctx->off.loads) + (long long)l0 * ctx->c;
  a.st = st;
  a.partials = partials;
  a.pstride = (int)ctx->pstride;
  a.paired = paired ? 1 : 0;
  a.scale = static_cast<T>(1.0 / (double)g.nvox);
  for (int i = 0; i < 9; ++i) a.em2[i] = T(0);
  if (ctx->physics == LSH_ELASTIC) {
    a.em2[0] = static_cast<T>(2.0 * ctx->A0[3 * 6 + 3]);   // 4 mu0
    a.em2[1] = static_cast<T>(2.0 * ctx->A0[1]);           // 2 lambda0
  } else {
    for (int i = 0; i < ctx->c * ctx->c; ++i) a.em2[i] = static_cast<T>(2.0 * ctx->A0[i]);
  }
  const double nl = std::min(ctx->nact, nload);
  const double cvs = (double)ctx->F * sizeof(T);
  // spectrum + material (phase ids, or two coefficients per voxel)
  double bytes = cvs + 2.0 * sizeof(T) * (double)nyq_cpx(g) + (ctx->mat_voxel ? 2.0 * sizeof(T) : 1.0) * g.nvox;
  if (mode != XI_STRAIN) bytes += cvs;                                          // the field transformed
  if (mode == XI_CGR) bytes += cvs;                                             // residual read
  if (mode == XI_IRRES) bytes += 4.0 * ctx->F;                                  // FP32 residual out
  else if (mode != XI_RESNORM) bytes += cvs;                                    // real output
  Scope sc(ctx, kcls<T>(K_XINV), nl * bytes);
  const int nb = launch_xinv<T>(ctx->stream, a, nload, tv<T>(ctx, PASS_XINV));
  STCHK(check_launch(ctx, nb, "x inverse"));
  if (nparts) *nparts = nb;
  return LSH_OK;
}

lsh_status scal(lsh_ctx* ctx, int mode, int ngroups, int nparts, LoadState* st, double tol, int l0 = 0,
                int aux = -1);

// One CG step with p.Lp known before the inverse passes: the x pass forms p
// and sums p.(A - A0)^{-1} p, the z pass sums p.Gamma p over the spectrum
// (Parseval), alpha follows, and the x-inverse pass updates r in place with
// ||r||^2; q = Lp is never stored.  The direction goes to buffer `par` (pout),
// the previous one is read from the other (pin); the x pass applies the
// pending solution updates in pairs (k_xfwdc).
// x, r, pin, pout and st are the bases of load 0; the step covers loads [l0, l0 + nload).
template <typename T>
lsh_status cg_fused_step(lsh_ctx* ctx, int l0, int nload, T* x, T* r, const T* pin, T* pout, int par,
                         LoadState* st, bool scalars = true) {
  const Geo& g = ctx->geo;
  x += (long long)l0 * ctx->F;
  r += (long long)l0 * ctx->F;
  pin += (long long)l0 * ctx->F;
  pout += (long long)l0 * ctx->F;
  st += l0;
  cpx<T>* sm = Sel<T>::sm(ctx) + (long long)l0 * main_cpx(g);
  cpx<T>* sn = Sel<T>::sn(ctx) + (long long)l0 * nyq_cpx(g);
  double* parts = ctx->ptr<double>(ctx->off.partials) + (long long)l0 * ctx->pstride;
  const double nl = std::min(ctx->nact, nload);
  const double cvs = (double)ctx->F * sizeof(T);
  const double spec = cvs + 2.0 * sizeof(T) * (double)nyq_cpx(g);
  const double mat = (ctx->mat_voxel ? 2.0 * sizeof(T) : 1.0) * g.nvox;
  // the paired z shape: every pass of the step in place on the paired layout
  const bool pr = paired_shape<T>(ctx);
  XfwdcArgs<T> xa{g, r, pin, pout, x, sm, sn, Sel<T>::tw(ctx, 0), st, ctx->nphase, ctx->iso, Sel<T>::ptab(ctx),
                  ctx->ptr<uint8_t>(ctx->off.phase), Sel<T>::vc(ctx), parts, (int)ctx->pstride, pr ? 1 : 0};
  int nbx = 0, nbz = 0, nbi = 0;
  {
    // fields: first step r in, p out; then r and p_{k-1} in, p_k out, and every
    // second step (two pending updates) p_{k-2} and x in, x out as well
    const double fields = ctx->xf_first ? 2.0 : (par == 0 ? 6.0 : 3.0);
    Scope sc(ctx, kcls<T>(K_XFWD), nl * (fields * cvs + spec + mat));
    nbx = launch_xfwdc<T>(ctx->stream, xa, nload);
    STCHK(check_launch(ctx, nbx, "x forward (CG)"));
  }
  {
    Scope sc(ctx, kcls<T>(K_Y), nl * 2.0 * spec);
    const int nb = pr ? launch_y_paired_inplace<T>(ctx->stream, g, -1, sm, sn, Sel<T>::tw(ctx, 1), st, nload,
                                                   tv<T>(ctx, PASS_Y))
                      : launch_y<T>(ctx->stream, g, -1, sm, sn, Sel<T>::tw(ctx, 1), st, nload, tv<T>(ctx, PASS_Y));
    STCHK(check_launch(ctx, nb, "y forward"));
  }
  {
    Scope sc(ctx, kcls<T>(K_ZG), nl * 2.0 * spec);
    GreenTabs<T> tb{Sel<T>::wt(ctx), ctx->wstride, {Sel<T>::tw(ctx, 0), Sel<T>::tw(ctx, 1), Sel<T>::tw(ctx, 2)},
                    Sel<T>::gtab(ctx), Sel<T>::gst(ctx)};
    nbz = pr ? launch_zg_paired<T>(ctx->stream, g, ctx->gp, tb, sm, sn, Sel<T>::tw(ctx, 2), st, nload, parts + nbx,
                                   (int)ctx->pstride)
             : launch_zg<T>(ctx->stream, g, ctx->gp, tb, Z_GAMMA, sm, sn, Sel<T>::tw(ctx, 2), st, nload,
                            tv<T>(ctx, PASS_ZG), parts + nbx, (int)ctx->pstride);
    STCHK(check_launch(ctx, nbz, "z/Green"));
  }
  if (scalars) STCHK(scal(ctx, SC_ALPHA, nload, nbx + nbz, st, ctx->bd_guard[sizeof(T) == 8 ? 1 : 0], l0, par));
  {
    Scope sc(ctx, kcls<T>(K_Y), nl * 2.0 * spec);
    const int nb = pr ? launch_y_paired_inplace<T>(ctx->stream, g, 1, sm, sn, Sel<T>::tw(ctx, 1), st, nload,
                                                   tv<T>(ctx, PASS_Y))
                      : launch_y<T>(ctx->stream, g, 1, sm, sn, Sel<T>::tw(ctx, 1), st, nload, tv<T>(ctx, PASS_Y));
    STCHK(check_launch(ctx, nb, "y inverse"));
  }
  STCHK(inverse_x<T>(ctx, l0, nload, XI_CGR, pout, r, nullptr, st, parts, &nbi, r, pr));
  return scalars ? scal(ctx, SC_BETA, nload, nbi, st, 0.0, l0) : LSH_OK;
}

// groups [l0, l0 + ngroups): the partials of group l at (l0 + l) pstride; st is already offset
// Residual history of loads [l0, ...) at `level` (see hist_push).
HistRef hist_ref(lsh_ctx* ctx, int l0, int level) {
  return HistRef{ctx->ptr<double>(ctx->off.hist) + (long long)l0 * 2 * kHistCap,
                 ctx->ptr<unsigned long long>(ctx->off.hcnt) + l0, level};
}

lsh_status scal(lsh_ctx* ctx, int mode, int ngroups, int nparts, LoadState* st, double tol, int l0, int aux) {
  Scope sc(ctx, K_SCAL);
  // the inner FP32 states of a mixed solve record at level 1, every other state at 0
  const LoadState* sin = ctx->ptr<LoadState>(ctx->off.st_in);
  const int level = (st >= sin && st < sin + ctx->max_loads) ? 1 : 0;
  hipLaunchKernelGGL(k_scal, dim3(ngroups), dim3(256), 0, ctx->stream, mode,
                     ctx->ptr<double>(ctx->off.partials) + (long long)l0 * ctx->pstride, (int)ctx->pstride, nparts,
                     st, ctx->ptr<double>(ctx->off.sums) + l0, tol, aux, hist_ref(ctx, l0, level));
  return check_launch(ctx, 0, "scalars");
}

template <typename T>
lsh_status cg_init(lsh_ctx* ctx, int nload, T* x, T* r, LoadState* st, double tol) {
  const Geo& g = ctx->geo;
  const int nb = ew_blocks(g.nvox);
  {
    Scope sc(ctx, K_INIT);
    hipLaunchKernelGGL((k_cginit<T>), dim3(nb, nload), dim3(256), 0, ctx->stream, g, x, r,
                       ctx->ptr<uint8_t>(ctx->off.phase), ctx->ptr<uint8_t>(ctx->off.i0), Sel<double>::vc(ctx),
                       ctx->ptr<double>(ctx->off.loads), ctx->ptr<double>(ctx->off.partials), (int)ctx->pstride);
    STCHK(check_launch(ctx, 0, "init"));
  }
  return scal(ctx, SC_INIT, nload, nb, st, tol);
}

// flags of the solve in progress (lsh_solve stages them in h_guess_up)
bool any_guess(const lsh_ctx* ctx, int nload) {
  for (int l = 0; l < nload && l < (int)ctx->h_guess_up.size(); ++l)
    if (ctx->h_guess_up[l]) return true;
  return false;
}

// Start of an FP64 solve on x (the solution slots).  Without initial guesses:
// cg_init (x = 0, r = b).  With them (flags uploaded to off.guess): the
// guesses are masked to I0 and the other loads zeroed; with r given, one
// operator application q = L x gives r = b - q, and the solver scalars start
// from ||r||^2 with the tolerance relative to ||b|| (SC_INITG); without r,
// only ||b||^2 is formed and x keeps the guesses.
lsh_status guess_init(lsh_ctx* ctx, int nload, double* x, double* r, LoadState* st, double tol,
                      bool zero_x = true) {
  if (!any_guess(ctx, nload)) return cg_init<double>(ctx, nload, zero_x ? x : nullptr, r, st, tol);
  const Geo& g = ctx->geo;
  const int nb = ew_blocks(g.nvox);
  const uint8_t* gflag = ctx->ptr<uint8_t>(ctx->off.guess);
  {
    Scope sc(ctx, K_INIT);
    hipLaunchKernelGGL((k_guessmask<double>), dim3(nb, nload), dim3(256), 0, ctx->stream, g, x,
                       ctx->ptr<uint8_t>(ctx->off.phase), ctx->ptr<uint8_t>(ctx->off.i0), Sel<double>::vc(ctx), gflag,
                       ctx->ptr<double>(ctx->off.loads));
    STCHK(check_launch(ctx, 0, "guess mask"));
  }
  if (r == nullptr) return cg_init<double>(ctx, nload, nullptr, nullptr, st, tol);
  STCHK(forward_part<double>(ctx, 0, nload, XF_PLAIN, x, nullptr, nullptr, nullptr, nullptr, true));
  double* q = reinterpret_cast<double*>(Sel<double>::sm(ctx));
  STCHK(inverse_x<double>(ctx, 0, nload, XI_APPLY, x, q, nullptr, nullptr, nullptr, nullptr));
  {
    Scope sc(ctx, K_INIT);
    hipLaunchKernelGGL((k_guessinit<double>), dim3(nb, nload), dim3(256), 0, ctx->stream, g, q, r,
                       ctx->ptr<uint8_t>(ctx->off.phase), ctx->ptr<uint8_t>(ctx->off.i0), Sel<double>::vc(ctx),
                       ctx->ptr<double>(ctx->off.loads), gflag, ctx->ptr<double>(ctx->off.partials),
                       (int)ctx->pstride, nload);
    STCHK(check_launch(ctx, 0, "guess init"));
  }
  return scal(ctx, SC_INITG, nload, nb, st, tol);
}

template <typename T>
lsh_status cg_update(lsh_ctx* ctx, int nload, T* r, const T* q, LoadState* st) {
  const long long nvec = ctx->F / Vec16<T>::n;
  const int nb = (int)((nvec + 256 * kEwUnroll - 1) / (256 * kEwUnroll));
  {
    Scope sc(ctx, kcls<T>(K_CGUPD), std::min(ctx->nact, nload) * 3.0 * (double)ctx->F * sizeof(T));
    hipLaunchKernelGGL((k_cgupd<T>), dim3(nb, nload), dim3(256), 0, ctx->stream, nvec, r, q, st,
                       ctx->ptr<double>(ctx->off.partials), (int)ctx->pstride);
    STCHK(check_launch(ctx, 0, "cg update"));
  }
  return scal(ctx, SC_BETA, nload, nb, st, 0.0);
}

// x += alpha p for the loads whose last step is pending (end of a CG solve);
// with two direction buffers (fused step, pb != nullptr) the pending steps of
// each load, one or two, from the buffers its states name
template <typename T>
lsh_status cg_flush(lsh_ctx* ctx, int nload, T* x, const T* p, const T* pb, LoadState* st) {
  const long long nvec = ctx->F / Vec16<T>::n;
  const int nb = (int)((nvec + 256 * kEwUnroll - 1) / (256 * kEwUnroll));
  Scope sc(ctx, kcls<T>(K_CGUPD), nload * (pb ? 4.0 : 3.0) * (double)ctx->F * sizeof(T));
  if (pb) hipLaunchKernelGGL((k_xflush2<T>), dim3(nb, nload), dim3(256), 0, ctx->stream, nvec, x, p, pb, st);
  else hipLaunchKernelGGL((k_xflush<T>), dim3(nb, nload), dim3(256), 0, ctx->stream, nvec, x, p, st);
  return check_launch(ctx, 0, "cg flush");
}

lsh_status read_states(lsh_ctx* ctx, size_t off, int nload, std::vector<LoadState>& h) {
  h.resize(nload);
  return read_back(ctx, h.data(), ctx->ws + off, sizeof(LoadState) * nload, 0);
}

int check_period(lsh_ctx* ctx, int nload) {
  const long long work = ctx->geo.nvox * (long long)nload * ctx->c;
  return work >= (1LL << 22) ? 1 : 8;
}

// Queue one solver iteration.  With graphs enabled (and kernel timing off)
// the iteration is captured once on a private stream, instantiated, and the
// graph is launched on the context's stream thereafter; `key` identifies the
// argument set the capture baked in.
template <typename F>
lsh_status run_iteration(lsh_ctx* ctx, int slot, long long key, F&& enqueue) {
  if (!ctx->use_graphs || ctx->timing) return enqueue();
  auto& G = ctx->graphs[slot];
  key = key * 1000003LL + ctx->graph_epoch;
  if (G.exec == nullptr || G.key != key) {
    if (G.exec) {
      (void)hipGraphExecDestroy(G.exec);
      G.exec = nullptr;
    }
    if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
    hipStream_t user = ctx->stream;
    ctx->stream = ctx->cap_stream;
    const lsh_status s = enqueue();
    ctx->stream = user;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (s != LSH_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return fail(ctx, LSH_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      G.exec = nullptr;
      return fail(ctx, LSH_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
    }
    G.key = key;
  }
  HIPCHK(hipGraphLaunch(G.exec, ctx->stream));
  return LSH_OK;
}

// CG iterations on (x, r, p) with q held in the spectrum buffer; returns after
// convergence of every load, or maxit iterations.  The fused step alternates
// its directions between p (even iterations) and pb (odd ones), one captured
// graph per parity; the unfused step and the persistent loop use p alone.
template <typename T>
lsh_status cg_loop(lsh_ctx* ctx, int nload, T* x, T* r, T* p, T* pb, LoadState* st, size_t st_off, int maxit,
                   std::vector<LoadState>& hst, bool flush = true) {
  const int period = check_period(ctx, nload);
  T* q = reinterpret_cast<T*>(Sel<T>::sm(ctx));
  STCHK(read_states(ctx, st_off, nload, hst));
  bool any = false;
  ctx->nact = 0;
  for (auto& s : hst) any |= s.active != 0, ctx->nact += s.active != 0;
  if (!any) return LSH_OK;
  if (ctx->persistent && ctx->cg_fused && tiny_grid(ctx->geo)) {
    // the whole loop in one launch: one workgroup per load
    TinyArgs<T> ta{};
    ta.g = ctx->geo;
    ta.gp = ctx->gp;
    ta.tb = GreenTabs<T>{Sel<T>::wt(ctx), ctx->wstride, {Sel<T>::tw(ctx, 0), Sel<T>::tw(ctx, 1), Sel<T>::tw(ctx, 2)},
                         Sel<T>::gtab(ctx), nullptr};
    ta.hist = hist_ref(ctx, 0, (sizeof(T) == 4 && ctx->precision == LSH_MIXED) ? 1 : 0);
    ta.x = x;
    ta.r = r;
    ta.p = p;
    ta.sm = Sel<T>::sm(ctx);
    ta.sn = Sel<T>::sn(ctx);
    for (int a = 0; a < 3; ++a) ta.tw[a] = Sel<T>::tw(ctx, a);
    ta.nphase = ctx->nphase;
    ta.iso = ctx->iso;
    ta.ptab = Sel<T>::ptab(ctx);
    ta.phase = ctx->ptr<uint8_t>(ctx->off.phase);
    ta.vcoef = Sel<T>::vc(ctx);
    ta.st = st;
    ta.maxit = maxit;
    ta.guard = ctx->bd_guard[sizeof(T) == 8 ? 1 : 0];
    {
      Scope sc(ctx, K_TINY);
      STCHK(check_launch(ctx, launch_tiny_cg<T>(ctx->stream, ta, nload), "persistent CG"));
    }
    return LSH_OK;
  }
  int par = 0;
  auto iteration = [&]() -> lsh_status {
    if (ctx->cg_fused) return cg_fused_step<T>(ctx, 0, nload, x, r, par ? p : pb, par ? pb : p, par, st);
    STCHK(forward_part<T>(ctx, 0, nload, XF_CG, r, p, x, nullptr, st, true));
    int np = 0;
    STCHK(inverse_x<T>(ctx, 0, nload, XI_CG, p, q, nullptr, st, ctx->ptr<double>(ctx->off.partials), &np));
    STCHK(scal(ctx, SC_ALPHA, nload, np, st, ctx->bd_guard[sizeof(T) == 8 ? 1 : 0]));
    return cg_update<T>(ctx, nload, r, q, st);
  };
  const long long key = (long long)nload * 4 + (st_off == ctx->off.st_in ? 1 : 0) + (ctx->cg_fused ? 2 : 0);
  for (int it = 0; it < maxit; ++it) {
    ctx->xf_first = it == 0;
    par = ctx->cg_fused ? (it & 1) : 0;
    STCHK(run_iteration(ctx, (sizeof(T) == 8 ? 0 : 1) + 3 * par, key, iteration));
    if ((it + 1) % period == 0 || it + 1 == maxit) {
      STCHK(read_states(ctx, st_off, nload, hst));
      any = false;
      ctx->nact = 0;
      for (auto& s : hst) any |= s.active != 0, ctx->nact += s.active != 0;
      if (!any) break;
    }
  }
  ctx->xf_first = false;
  // without flush the caller applies the pending steps (the mixed path's refinement pass)
  return flush ? cg_flush<T>(ctx, nload, x, p, ctx->cg_fused ? pb : nullptr, st) : LSH_OK;
}

// Fixed-point schemes on tau in place: basic (XI_BASIC) or Eyre--Milton (XI_EM).
lsh_status basic_loop(lsh_ctx* ctx, int nload, double* x, LoadState* st, size_t st_off, int maxit,
                      std::vector<LoadState>& hst, int ximode = XI_BASIC) {
  const int period = check_period(ctx, nload);
  STCHK(read_states(ctx, st_off, nload, hst));
  bool any = false;
  ctx->nact = 0;
  for (auto& s : hst) any |= s.active != 0, ctx->nact += s.active != 0;
  if (!any) return LSH_OK;
  auto iteration = [&]() -> lsh_status {
    STCHK(forward_part<double>(ctx, 0, nload, XF_PLAIN, x, nullptr, nullptr, nullptr, st, true));
    int np = 0;
    STCHK(inverse_x<double>(ctx, 0, nload, ximode, x, x, nullptr, st, ctx->ptr<double>(ctx->off.partials), &np));
    return scal(ctx, SC_BASIC, nload, np, st, 0.0);
  };
  for (int it = 0; it < maxit; ++it) {
    STCHK(run_iteration(ctx, 2, (long long)nload * 8 + ximode, iteration));
    if ((it + 1) % period == 0 || it + 1 == maxit) {
      STCHK(read_states(ctx, st_off, nload, hst));
      any = false;
      ctx->nact = 0;
      for (auto& s : hst) any |= s.active != 0, ctx->nact += s.active != 0;
      if (!any) break;
    }
  }
  return LSH_OK;
}

// MINRES on x64 with the Lanczos and direction fields in the bound solver
// buffer (v_{k-1}, v_k, w_{k-1}, w_{k-2}); q = L v_k lands in the FP64
// spectrum buffer.  The four fields rotate roles between steps, so the steps
// are queued eagerly (no graph capture).
lsh_status mr_loop(lsh_ctx* ctx, int nload, double tol, int maxit, std::vector<LoadState>& hst) {
  const long long F = ctx->F;
  const long long LF = (long long)ctx->max_loads * F;
  double* f[4];
  for (int i = 0; i < 4; ++i) f[i] = reinterpret_cast<double*>(ctx->sbuf) + i * LF;
  double* vp = f[0];
  double* v = f[1];
  double* w1 = f[2];
  double* w2 = f[3];
  double* x = ctx->ptr<double>(ctx->off.x64);
  LoadState* st = ctx->ptr<LoadState>(ctx->off.st_out);
  MinresState* ms = ctx->ptr<MinresState>(ctx->off.mstate);
  double* parts = ctx->ptr<double>(ctx->off.partials);
  // x = 0 (or the guess), v = b - L x and its norm; then v = r_0/||r_0|| and the rotation state
  STCHK(guess_init(ctx, nload, x, v, st, tol));
  {
    Scope sc(ctx, K_INIT);
    hipLaunchKernelGGL(k_mr_start, dim3((unsigned)((F + 255) / 256), nload), dim3(256), 0, ctx->stream, F, v, vp, w1,
                       w2, st);
    STCHK(check_launch(ctx, 0, "minres start"));
  }
  {
    Scope sc(ctx, K_SCAL);
    hipLaunchKernelGGL(k_mr_scal, dim3(nload), dim3(256), 0, ctx->stream, (int)MR_INIT, parts, (int)ctx->pstride, 0,
                       st, ms, hist_ref(ctx, 0, 0));
    STCHK(check_launch(ctx, 0, "minres init"));
  }
  const int period = check_period(ctx, nload);
  STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
  ctx->nact = 0;
  bool any = false;
  for (auto& sv : hst) any |= sv.active != 0, ctx->nact += sv.active != 0;
  if (!any) return LSH_OK;
  double* q = reinterpret_cast<double*>(Sel<double>::sm(ctx));
  const int nbe = (int)((F + 256 * kEwUnroll - 1) / (256 * kEwUnroll));
  for (int it = 0; it < maxit; ++it) {
    STCHK(forward_part<double>(ctx, 0, nload, XF_PLAIN, v, nullptr, nullptr, nullptr, st, true));
    int np = 0;
    STCHK(inverse_x<double>(ctx, 0, nload, XI_CG, v, q, nullptr, st, parts, &np));
    {
      Scope sc(ctx, K_SCAL);
      hipLaunchKernelGGL(k_mr_scal, dim3(nload), dim3(256), 0, ctx->stream, (int)MR_ALPHA, parts, (int)ctx->pstride,
                         np, st, ms, hist_ref(ctx, 0, 0));
      STCHK(check_launch(ctx, 0, "minres alpha"));
    }
    {
      Scope sc(ctx, kcls<double>(K_CGUPD), std::min(ctx->nact, nload) * 4.0 * (double)F * 8.0);
      hipLaunchKernelGGL(k_mr_lanczos, dim3(nbe, nload), dim3(256), 0, ctx->stream, F, q, v, vp, st, ms, parts,
                         (int)ctx->pstride);
      STCHK(check_launch(ctx, 0, "minres lanczos"));
    }
    {
      Scope sc(ctx, K_SCAL);
      hipLaunchKernelGGL(k_mr_scal, dim3(nload), dim3(256), 0, ctx->stream, (int)MR_ROT, parts, (int)ctx->pstride,
                         nbe, st, ms, hist_ref(ctx, 0, 0));
      STCHK(check_launch(ctx, 0, "minres rotation"));
    }
    {
      Scope sc(ctx, kcls<double>(K_CGUPD), std::min(ctx->nact, nload) * 8.0 * (double)F * 8.0);
      hipLaunchKernelGGL(k_mr_update, dim3(nbe, nload), dim3(256), 0, ctx->stream, F, v, vp, w1, w2, x, ms);
      STCHK(check_launch(ctx, 0, "minres update"));
    }
    std::swap(v, vp);    // v_{k+1} now in the old v_{k-1} slot
    std::swap(w1, w2);   // w_k now in the old w_{k-2} slot
    if ((it + 1) % period == 0 || it + 1 == maxit) {
      STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
      any = false;
      ctx->nact = 0;
      for (auto& sv : hst) any |= sv.active != 0, ctx->nact += sv.active != 0;
      if (!any) break;
    }
  }
  return LSH_OK;
}

// SYMMLQ on x64: MINRES's Lanczos step, then the LQ step or the transfer to
// the CG point (k_sy_scal, k_sy_update); fields v_{k-1}/v_{k+1}, v_k, wbar_k
// in the bound solver buffer.
lsh_status sy_loop(lsh_ctx* ctx, int nload, double tol, int maxit, std::vector<LoadState>& hst) {
  const long long F = ctx->F;
  const long long LF = (long long)ctx->max_loads * F;
  double* vp = reinterpret_cast<double*>(ctx->sbuf);
  double* v = vp + LF;
  double* wbar = vp + 2 * LF;
  double* x = ctx->ptr<double>(ctx->off.x64);
  LoadState* st = ctx->ptr<LoadState>(ctx->off.st_out);
  MinresState* ms = ctx->ptr<MinresState>(ctx->off.mstate);
  double* parts = ctx->ptr<double>(ctx->off.partials);
  STCHK(guess_init(ctx, nload, x, v, st, tol));   // x = 0 (or the guess), v = b - L x, norms
  {
    Scope sc(ctx, K_INIT);
    hipLaunchKernelGGL(k_sy_start, dim3((unsigned)((F + 255) / 256), nload), dim3(256), 0, ctx->stream, F, v, vp,
                       wbar, st);
    STCHK(check_launch(ctx, 0, "symmlq start"));
  }
  {
    Scope sc(ctx, K_SCAL);
    hipLaunchKernelGGL(k_sy_scal, dim3(nload), dim3(256), 0, ctx->stream, (int)SY_INIT, parts, (int)ctx->pstride, 0,
                       0, st, ms, hist_ref(ctx, 0, 0));
    STCHK(check_launch(ctx, 0, "symmlq init"));
  }
  const int period = check_period(ctx, nload);
  STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
  ctx->nact = 0;
  bool any = false;
  for (auto& sv : hst) any |= sv.active != 0, ctx->nact += sv.active != 0;
  if (!any) return LSH_OK;
  double* q = reinterpret_cast<double*>(Sel<double>::sm(ctx));
  const int nbe = (int)((F + 256 * kEwUnroll - 1) / (256 * kEwUnroll));
  for (int it = 0; it < maxit; ++it) {
    STCHK(forward_part<double>(ctx, 0, nload, XF_PLAIN, v, nullptr, nullptr, nullptr, st, true));
    int np = 0;
    STCHK(inverse_x<double>(ctx, 0, nload, XI_CG, v, q, nullptr, st, parts, &np));
    {
      Scope sc(ctx, K_SCAL);
      hipLaunchKernelGGL(k_mr_scal, dim3(nload), dim3(256), 0, ctx->stream, (int)MR_ALPHA, parts, (int)ctx->pstride,
                         np, st, ms, hist_ref(ctx, 0, 0));
      STCHK(check_launch(ctx, 0, "symmlq alpha"));
    }
    {
      Scope sc(ctx, kcls<double>(K_CGUPD), std::min(ctx->nact, nload) * 4.0 * (double)F * 8.0);
      hipLaunchKernelGGL(k_mr_lanczos, dim3(nbe, nload), dim3(256), 0, ctx->stream, F, q, v, vp, st, ms, parts,
                         (int)ctx->pstride);
      STCHK(check_launch(ctx, 0, "symmlq lanczos"));
    }
    {
      Scope sc(ctx, K_SCAL);
      hipLaunchKernelGGL(k_sy_scal, dim3(nload), dim3(256), 0, ctx->stream, (int)SY_ROT, parts, (int)ctx->pstride,
                         nbe, it + 1 == maxit ? 1 : 0, st, ms, hist_ref(ctx, 0, 0));
      STCHK(check_launch(ctx, 0, "symmlq rotation"));
    }
    {
      Scope sc(ctx, kcls<double>(K_CGUPD), std::min(ctx->nact, nload) * 6.0 * (double)F * 8.0);
      hipLaunchKernelGGL(k_sy_update, dim3(nbe, nload), dim3(256), 0, ctx->stream, F, vp, wbar, x, ms);
      STCHK(check_launch(ctx, 0, "symmlq update"));
    }
    std::swap(v, vp);    // v_{k+1} now in the old v_{k-1} slot
    if ((it + 1) % period == 0 || it + 1 == maxit) {
      STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
      any = false;
      ctx->nact = 0;
      for (auto& sv : hst) any |= sv.active != 0, ctx->nact += sv.active != 0;
      if (!any) break;
    }
  }
  return LSH_OK;
}

// ||b - L x||^2 per load into sums[0..nload) (FP64 application on x64)
lsh_status true_residual(lsh_ctx* ctx, int nload) {
  double* x = ctx->ptr<double>(ctx->off.x64);
  STCHK(forward_part<double>(ctx, 0, nload, XF_PLAIN, x, nullptr, nullptr, nullptr, nullptr, true));
  int np = 0;
  STCHK(inverse_x<double>(ctx, 0, nload, XI_RESNORM, x, nullptr, nullptr, nullptr,
                          ctx->ptr<double>(ctx->off.partials), &np));
  return scal(ctx, SC_SUM, nload, np, nullptr, 0.0);
}

lsh_status effective(lsh_ctx* ctx, int nload) {
  const Geo& g = ctx->geo;
  const int nb = ew_blocks(g.nvox);
  {
    Scope sc(ctx, K_MEAN);
    hipLaunchKernelGGL((k_mean<double>), dim3(nb, nload * ctx->c), dim3(256), 0, ctx->stream, g,
                       ctx->ptr<double>(ctx->off.x64), ctx->ptr<double>(ctx->off.partials), (int)ctx->pstride);
    STCHK(check_launch(ctx, 0, "mean"));
  }
  STCHK(scal(ctx, SC_SUM, nload * ctx->c, nb, nullptr, 0.0));
  std::vector<double> sums((size_t)nload * ctx->c);
  STCHK(read_back(ctx, sums.data(), ctx->ws + ctx->off.sums, sums.size() * sizeof(double),
                  sizeof(LoadState) * ctx->max_loads));
  const int c = ctx->c;
  ctx->sigma.assign((size_t)nload * c, 0.0);
  for (int l = 0; l < nload; ++l)
    for (int i = 0; i < c; ++i) {
      double a = 0.0;
      for (int j = 0; j < c; ++j) a += ctx->A0[i * c + j] * ctx->last_loads[(size_t)l * c + j];
      ctx->sigma[(size_t)l * c + i] = a + sums[(size_t)l * c + i] / (double)g.nvox;
    }
  return LSH_OK;
}

// ------------------------- kernel-shape tuning ---------------------------
// Passes compiled in several shapes: the 128/256-point axes.
bool pass_has_variants(const lsh_ctx* ctx, int pass) {
  switch (pass) {
    case PASS_XFWD:
    case PASS_XINV: return ctx->geo.mx == 64 || ctx->geo.mx == 128;
    case PASS_Y: return ctx->n[1] == 128 || ctx->n[1] == 256;
    case PASS_ZG: return ctx->c != 2 && (ctx->n[2] == 128 || ctx->n[2] == 256);
    default: return false;
  }
}

int pass_class(int pass, bool fp64) {
  const int base = pass == PASS_XFWD ? K_XFWD : pass == PASS_Y ? K_Y : pass == PASS_ZG ? K_ZG : K_XINV;
  return base + (fp64 ? 1 : 0);
}

// One operator application in the modes the solvers run, on the workspace's
// own fields (timing input): the CG modes (x += alpha p and p = r + beta p
// fused into the x pass, q and p.q out of the last) for FP32 fields of a mixed
// context and FP64 fields of an FP64 context, the refinement modes (x64 += d,
// FP64 residual to FP32) for the FP64 passes of a mixed context.
lsh_status timing_iteration(lsh_ctx* ctx, int nload, bool fp64) {
  double* parts = ctx->ptr<double>(ctx->off.partials);
  if (!fp64 && ctx->cg_fused)
    return cg_fused_step<float>(ctx, 0, nload, ctx->ptr<float>(ctx->off.d32), ctx->ptr<float>(ctx->off.r32),
                                ctx->ptr<float>(ctx->off.p32b), ctx->ptr<float>(ctx->off.p32), 0,
                                ctx->ptr<LoadState>(ctx->off.st_in), false);
  if (fp64 && ctx->cg_fused && ctx->precision != LSH_MIXED)
    return cg_fused_step<double>(ctx, 0, nload, ctx->ptr<double>(ctx->off.x64), ctx->ptr<double>(ctx->off.r64),
                                 ctx->ptr<double>(ctx->off.p64b), ctx->ptr<double>(ctx->off.p64), 0,
                                 ctx->ptr<LoadState>(ctx->off.st_out), false);
  if (!fp64) {
    LoadState* st = ctx->ptr<LoadState>(ctx->off.st_in);
    float* q = reinterpret_cast<float*>(Sel<float>::sm(ctx));
    STCHK(forward_part<float>(ctx, 0, nload, XF_CG, ctx->ptr<float>(ctx->off.r32), ctx->ptr<float>(ctx->off.p32),
                              ctx->ptr<float>(ctx->off.d32), nullptr, st, true));
    return inverse_x<float>(ctx, 0, nload, XI_CG, ctx->ptr<float>(ctx->off.p32), q, nullptr, st, parts, nullptr);
  }
  LoadState* st = ctx->ptr<LoadState>(ctx->off.st_out);
  double* x = ctx->ptr<double>(ctx->off.x64);
  if (ctx->precision == LSH_MIXED) {
    STCHK(forward_part<double>(ctx, 0, nload, XF_IRX, nullptr, x, nullptr, ctx->ptr<float>(ctx->off.d32), st, true));
    return inverse_x<double>(ctx, 0, nload, XI_IRRES, x, nullptr, ctx->ptr<float>(ctx->off.r32), st, parts, nullptr);
  }
  double* q = reinterpret_cast<double*>(Sel<double>::sm(ctx));
  STCHK(forward_part<double>(ctx, 0, nload, XF_CG, ctx->ptr<double>(ctx->off.r64), ctx->ptr<double>(ctx->off.p64), x,
                             nullptr, st, true));
  return inverse_x<double>(ctx, 0, nload, XI_CG, ctx->ptr<double>(ctx->off.p64), q, nullptr, st, parts, nullptr);
}

std::string tune_key(const lsh_ctx* ctx, int nload) {
  std::ostringstream k;
  k << "gfx950 " << ctx->n[0] << "x" << ctx->n[1] << "x" << ctx->n[2] << " c" << ctx->c
    << (ctx->precision == LSH_MIXED ? " mixed" : " fp64") << " L" << nload << " green" << ctx->green
    << (ctx->mat_voxel ? " voxel" : (ctx->iso ? " iso" : " full"))
    << ((Sel<float>::gst(const_cast<lsh_ctx*>(ctx)) || Sel<double>::gst(const_cast<lsh_ctx*>(ctx))) ? " stored" : "");
  return k.str();
}

// Cache file: one line per key, "<key> = v00 v01 v02 v03 v10 v11 v12 v13"
// (FP32 passes xfwd y zg xinv, then FP64).
std::map<std::string, std::vector<int>> read_tune_cache(const char* path) {
  std::map<std::string, std::vector<int>> m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t eq = line.find(" = ");
    if (eq == std::string::npos) continue;
    std::istringstream vs(line.substr(eq + 3));
    std::vector<int> v;
    int x;
    while (vs >> x) v.push_back(x);
    if (v.size() != 2 * NPASS) continue;
    bool ok = true;
    for (size_t i = 0; i < v.size(); ++i) ok &= (v[i] >= 0 && v[i] < pass_variants((int)(i % NPASS)));
    if (ok) m[line.substr(0, eq)] = v;
  }
  return m;
}

bool write_tune_cache(const char* path, const std::map<std::string, std::vector<int>>& m) {
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)std::hash<std::thread::id>()(std::this_thread::get_id()) % 100000);
  {
    std::ofstream f(tmp);
    if (!f) return false;
    for (const auto& kv : m) {
      f << kv.first << " =";
      for (int v : kv.second) f << " " << v;
      f << "\n";
    }
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

// Isotropic reference of per-voxel mode: a0 (scalar, A0 = a0 Id) or (K0, mu0).
bool isotropic_reference(const lsh_ctx* ctx, double* a0, double* K0, double* mu0) {
  const int c = ctx->c;
  if (ctx->physics == LSH_ELASTIC) {
    const double lam0 = ctx->A0[1];
    *mu0 = 0.5 * ctx->A0[3 * 6 + 3];
    *K0 = lam0 + 2.0 * *mu0 / 3.0;
    *a0 = 0.0;
    return true;
  }
  *a0 = ctx->A0[0];
  *K0 = *mu0 = 0.0;
  for (int i = 0; i < c; ++i)
    for (int j = 0; j < c; ++j)
      if (std::fabs(ctx->A0[i * c + j] - (i == j ? *a0 : 0.0)) > 1e-14 * std::fabs(*a0)) return false;
  return true;
}

// Hypothesis (2) for one voxel of per-voxel mode (the rule of k_voxset).
bool voxel_admissible(bool elastic, double x, double y, double a0, double K0, double mu0) {
  if (!elastic) {
    const double d = x - a0;
    if (!std::isfinite(x)) return false;
    return d == 0.0 || std::fabs(d) > 1e-12 * (std::fabs(x) + std::fabs(a0));
  }
  if (!std::isfinite(x) || !std::isfinite(y)) return false;
  const double dK = x - K0, dm = y - mu0;
  if (dK == 0.0 && dm == 0.0) return true;
  const bool tiny = std::fabs(dK) <= 1e-12 * (std::fabs(x) + std::fabs(K0)) ||
                    std::fabs(dm) <= 1e-12 * (std::fabs(y) + std::fabs(mu0));
  return !tiny && ((dK > 0.0) == (dm > 0.0));
}

template <typename TI>
lsh_status voxel_setup(lsh_ctx* ctx, const TI* m, bool count_only, long long* nbad) {
  double a0, K0, mu0;
  isotropic_reference(ctx, &a0, &K0, &mu0);
  const long long V = ctx->geo.nvox;
  const int nb = (int)((V + 255) / 256);
  const int el = ctx->physics == LSH_ELASTIC ? 1 : 0;
  if (count_only) {
    // one partial per workgroup; the partials buffer holds at least L c pstride doubles
    const long long cap = (long long)ctx->max_loads * ctx->c * ctx->pstride;
    double* parts = ctx->ptr<double>(ctx->off.partials);
    std::vector<double> h;
    long long bad = 0;
    for (long long b0 = 0; b0 < nb; b0 += cap) {
      const long long nbk = std::min<long long>(cap, nb - b0);
      const long long v0 = b0 * 256;
      hipLaunchKernelGGL((k_voxset<TI>), dim3((unsigned)nbk), dim3(256), 0, ctx->stream, v0,
                         std::min(V, v0 + nbk * 256), V, el, m, a0, K0, mu0, nullptr, nullptr, parts);
      STCHK(check_launch(ctx, 0, "voxel check"));
      h.resize((size_t)nbk);
      HIPCHK(hipMemcpyAsync(h.data(), parts, sizeof(double) * nbk, hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));
      for (double x : h) bad += (long long)x;
    }
    *nbad = bad;
    return LSH_OK;
  }
  float* o32 = ctx->precision == LSH_MIXED ? ctx->ptr<float>(ctx->off.vc32) : nullptr;
  hipLaunchKernelGGL((k_voxset<TI>), dim3(nb), dim3(256), 0, ctx->stream, 0LL, V, V, el, m, a0, K0, mu0,
                     ctx->ptr<double>(ctx->off.vc64), o32, ctx->ptr<double>(ctx->off.partials));
  STCHK(check_launch(ctx, 0, "voxel moduli"));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LSH_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free operator (lsh_apply_noalloc): the Nyquist
// plane of the spectrum (the main spectrum occupies exactly the caller's
// output buffer).  A file-scope device array: every GPU the library runs on
// holds one copy of kScratchBytes until the process ends.  Host code never
// uses the array's name as an address (it is a host-side stand-in): the
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and is kept per device.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {nullptr};

lsh_status scratch_address(lsh_ctx* ctx, void** out) {
  int dev = ctx->ws_device;
  if (dev < 0) HIPCHK(hipGetDevice(&dev));
  if (dev >= kMaxDevices) return fail(ctx, LSH_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != dev) HIPCHK(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || p == nullptr)
      return fail(ctx, LSH_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return LSH_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* lsh_version(void) { return "lsh 0.1.0 (gfx950)"; }

const char* lsh_last_error(const lsh_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

lsh_status lsh_create(lsh_ctx** out, int dim, const int64_t* n, int physics, int precision, int max_loads,
                      void* stream) {
  if (!out || !n) return LSH_EINVAL;
  *out = nullptr;
  if (dim != 2 && dim != 3) return LSH_EINVAL;
  if (physics != LSH_SCALAR && physics != LSH_ELASTIC) return LSH_EINVAL;
  if (physics == LSH_ELASTIC && dim != 3) return LSH_EINVAL;
  if (precision != LSH_FP64 && precision != LSH_MIXED) return LSH_EINVAL;
  if (max_loads < 1 || max_loads > 65535) return LSH_EINVAL;
  for (int a = 0; a < dim; ++a) {
    if (!supported_axis(n[a])) return LSH_EINVAL;
    if (a == 0 && n[a] < 4) return LSH_EINVAL;
    if (a > 0 && n[a] < 2) return LSH_EINVAL;
  }
  lsh_ctx* ctx = new lsh_ctx();
  ctx->dim = dim;
  ctx->physics = physics;
  ctx->precision = precision;
  ctx->max_loads = max_loads;
  ctx->c = physics == LSH_ELASTIC ? 6 : dim;
  for (int a = 0; a < dim; ++a) ctx->n[a] = (int)n[a];
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  ctx->geo.nx = ctx->n[0];
  ctx->geo.ny = ctx->n[1];
  ctx->geo.nz = ctx->n[2];
  ctx->geo.mx = ctx->n[0] / 2;
  ctx->geo.c = ctx->c;
  ctx->geo.nvox = (long long)ctx->n[0] * ctx->n[1] * ctx->n[2];
  ctx->F = (long long)ctx->c * ctx->geo.nvox;
  ctx->A0.assign((size_t)ctx->c * ctx->c, 0.0);
  compute_layout(ctx);
  tune_from_env(ctx);
  *out = ctx;
  return LSH_OK;
}

lsh_status lsh_destroy(lsh_ctx* ctx) {
  if (!ctx) return LSH_EINVAL;
  drain_timers(ctx);
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  for (auto& G : ctx->graphs)
    if (G.exec) (void)hipGraphExecDestroy(G.exec);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->wait_ev) (void)hipEventDestroy(ctx->wait_ev);
  if (ctx->hpin) (void)hipHostFree(ctx->hpin);
  delete ctx;
  return LSH_OK;
}

lsh_status lsh_workspace_bytes(const lsh_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return LSH_EINVAL;
  *bytes = ctx->ws_need;
  return LSH_OK;
}

lsh_status lsh_bind_workspace(lsh_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return LSH_EINVAL;
  if (!dev_ptr) return fail(ctx, LSH_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign != 0) return fail(ctx, LSH_EINVAL, "workspace not 256-byte aligned");
  if (bytes < ctx->ws_need)
    return fail(ctx, LSH_ENOMEM, "workspace too small: need " + std::to_string(ctx->ws_need) + " bytes");
  if (ctx->have_phase && ctx->phase_host.empty())
    return fail(ctx, LSH_ESTATE,
                "a device phase map or per-voxel moduli must be set again after rebinding the workspace");
  ctx->ws = static_cast<char*>(dev_ptr);
  ctx->ws_size = bytes;
  {
    hipPointerAttribute_t attr;
    ctx->ws_device = hipPointerGetAttributes(&attr, dev_ptr) == hipSuccess ? attr.device : -1;
    (void)hipGetLastError();
  }
  ctx->graph_epoch++;
  ctx->consts_ready = false;
  ctx->tables_dirty = true;
  ctx->gst_dirty = true;
  ctx->phase_dirty = ctx->have_phase;
  ctx->have_solution = false;
  return LSH_OK;
}

lsh_status lsh_set_reference(lsh_ctx* ctx, const double* A0) {
  if (!ctx) return LSH_EINVAL;
  if (!A0) return fail(ctx, LSH_EINVAL, "null A0");
  const int c = ctx->c;
  for (int i = 0; i < c * c; ++i)
    if (!std::isfinite(A0[i])) return fail(ctx, LSH_EINVAL, "A0 has a non-finite entry");
  if (!symmetric(c, A0)) return fail(ctx, LSH_EINVAL, "A0 is not symmetric");
  double ev[6];
  sym_eigvals(c, A0, ev);
  for (int i = 0; i < c; ++i)
    if (!(ev[i] > 0.0)) return fail(ctx, LSH_EINVAL, "A0 is not positive definite");
  if (ctx->physics == LSH_ELASTIC) {
    const double lam = A0[1], mu2 = A0[3 * 6 + 3];
    double scale = 0.0;
    for (int i = 0; i < 36; ++i) scale = std::max(scale, std::fabs(A0[i]));
    const double tol = 1e-12 * scale;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double expect = 0.0;
        if (i < 3 && j < 3) expect = lam + (i == j ? mu2 : 0.0);
        else if (i == j) expect = mu2;
        if (std::fabs(A0[i * 6 + j] - expect) > tol)
          return fail(ctx, LSH_EINVAL, "elastic A0 must be isotropic (lambda0, mu0) in Mandel form");
      }
  }
  ctx->A0.assign(A0, A0 + c * c);
  ctx->have_ref = true;
  ctx->gst_dirty = true;
  if (ctx->mat_voxel) ctx->have_phase = false;  // per-voxel coefficients were formed against the old A0
  ctx->tables_dirty = true;
  ctx->have_solution = false;
  return LSH_OK;
}

lsh_status lsh_set_phases(lsh_ctx* ctx, const uint8_t* phase, int mem, int nphase, const double* moduli) {
  if (!ctx) return LSH_EINVAL;
  if (!phase || !moduli) return fail(ctx, LSH_EINVAL, "null phase map or moduli");
  if (nphase < 1 || nphase > kMaxPhases) return fail(ctx, LSH_EINVAL, "nphase must be in 1..32");
  if (mem != LSH_HOST && mem != LSH_DEVICE) return fail(ctx, LSH_EINVAL, "bad memory space");
  const int c = ctx->c;
  for (int p = 0; p < nphase; ++p) {
    for (int i = 0; i < c * c; ++i)
      if (!std::isfinite(moduli[(size_t)p * c * c + i]))
        return fail(ctx, LSH_EINVAL, "non-finite modulus in phase " + std::to_string(p));
    if (!symmetric(c, moduli + (size_t)p * c * c))
      return fail(ctx, LSH_EINVAL, "phase " + std::to_string(p) + " modulus is not symmetric");
  }
  const size_t V = (size_t)ctx->geo.nvox;
  if (mem == LSH_HOST) {
    for (size_t i = 0; i < V; ++i)
      if (phase[i] >= nphase) return fail(ctx, LSH_EINVAL, "phase id out of range at voxel " + std::to_string(i));
    ctx->phase_host.assign(phase, phase + V);
    ctx->phase_dev_src = nullptr;
  } else {
    if (!ctx->ws) return fail(ctx, LSH_ESTATE, "bind the workspace before passing a device phase map");
    // ids are checked on the device before the map is accepted (the flag
    // lives in the reduction-results slot of the workspace)
    int* flag = ctx->ptr<int>(ctx->off.sums);
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), ctx->stream));
    const long long nb = std::min<long long>(((long long)V + 255) / 256, 8192);
    hipLaunchKernelGGL(k_phase_check, dim3((unsigned)nb), dim3(256), 0, ctx->stream, phase, (long long)V, nphase, flag);
    STCHK(check_launch(ctx, 0, "phase check"));
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (hflag != 0) return fail(ctx, LSH_EINVAL, "device phase map holds an id >= nphase");
    ctx->phase_host.clear();
    ctx->phase_dev_src = phase;
  }
  ctx->nphase = nphase;
  ctx->moduli.assign(moduli, moduli + (size_t)nphase * c * c);
  ctx->mat_voxel = false;
  ctx->have_phase = true;
  ctx->phase_dirty = true;
  ctx->tables_dirty = true;
  ctx->have_solution = false;
  return LSH_OK;
}

lsh_status lsh_set_voxel_moduli(lsh_ctx* ctx, const void* m, int dtype, int mem, int ncoef) {
  if (!ctx) return LSH_EINVAL;
  if (!m) return fail(ctx, LSH_EINVAL, "null moduli");
  if (dtype != LSH_F64 && dtype != LSH_F32) return fail(ctx, LSH_EINVAL, "bad dtype");
  if (mem != LSH_HOST && mem != LSH_DEVICE) return fail(ctx, LSH_EINVAL, "bad memory space");
  const bool el = ctx->physics == LSH_ELASTIC;
  if (ncoef != (el ? 2 : 1))
    return fail(ctx, LSH_EINVAL, el ? "elasticity takes two coefficients per voxel (K, mu)"
                                    : "scalar problems take one coefficient per voxel");
  if (!ctx->have_ref) return fail(ctx, LSH_ESTATE, "set the reference medium before per-voxel moduli");
  double a0, K0, mu0;
  if (!isotropic_reference(ctx, &a0, &K0, &mu0))
    return fail(ctx, LSH_EINVAL, "per-voxel moduli need an isotropic reference A0 = a0 Id");
  if (!ctx->ws) return fail(ctx, LSH_ESTATE, "bind the workspace before setting per-voxel moduli");
  const long long V = ctx->geo.nvox;
  const size_t es = dtype == LSH_F64 ? sizeof(double) : sizeof(float);
  const void* src = m;
  if (mem == LSH_HOST) {
    for (long long v = 0; v < V; ++v) {
      double x, y = 0.0;
      if (dtype == LSH_F64) {
        x = static_cast<const double*>(m)[v];
        if (el) y = static_cast<const double*>(m)[V + v];
      } else {
        x = static_cast<const float*>(m)[v];
        if (el) y = static_cast<const float*>(m)[V + v];
      }
      if (!voxel_admissible(el, x, y, a0, K0, mu0))
        return fail(ctx, LSH_EHYP2, "voxel " + std::to_string(v) +
                                        ": A - A0 is neither zero nor definite, or not finite (hypothesis (2))");
    }
    // staged through the FP64 spectrum buffer (at least c nvox doubles)
    HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.s64m, m, es * ncoef * V, hipMemcpyHostToDevice, ctx->stream));
    src = ctx->ws + ctx->off.s64m;
  } else {
    long long nbad = 0;
    if (dtype == LSH_F64) STCHK(voxel_setup<double>(ctx, static_cast<const double*>(m), true, &nbad));
    else STCHK(voxel_setup<float>(ctx, static_cast<const float*>(m), true, &nbad));
    if (nbad > 0)
      return fail(ctx, LSH_EHYP2, std::to_string(nbad) +
                                      " voxels have A - A0 neither zero nor definite, or not finite (hypothesis (2))");
  }
  if (dtype == LSH_F64) STCHK(voxel_setup<double>(ctx, static_cast<const double*>(src), false, nullptr));
  else STCHK(voxel_setup<float>(ctx, static_cast<const float*>(src), false, nullptr));
  ctx->mat_voxel = true;
  ctx->nphase = 0;
  ctx->phase_host.clear();
  ctx->phase_dev_src = nullptr;
  ctx->have_phase = true;
  ctx->phase_dirty = false;
  ctx->tables_dirty = true;
  ctx->have_solution = false;
  return LSH_OK;
}

lsh_status lsh_gradient(lsh_ctx* ctx, const double* W, void* grad, int dtype) {
  if (!ctx) return LSH_EINVAL;
  TraceRange tr("lsh_gradient");
  if (!W || !grad) return fail(ctx, LSH_EINVAL, "null weights or gradient buffer");
  if (dtype != LSH_F64 && dtype != LSH_F32) return fail(ctx, LSH_EINVAL, "bad dtype");
  if (!ctx->have_solution) return fail(ctx, LSH_ESTATE, "no solution");
  const int L = ctx->last_nload;
  std::vector<double> w((size_t)L * L);
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j) {
      if (!std::isfinite(W[i * L + j])) return fail(ctx, LSH_EINVAL, "non-finite weight");
      w[(size_t)i * L + j] = 0.5 * (W[i * L + j] + W[j * L + i]);
    }
  ctx->nact = 1 << 30;
  // strain estimates p_l - Gamma tau_l of every solved load, in the FP64 spectrum buffer
  double* x = ctx->ptr<double>(ctx->off.x64);
  double* eps = reinterpret_cast<double*>(Sel<double>::sm(ctx));
  STCHK(forward_part<double>(ctx, 0, L, XF_PLAIN, x, nullptr, nullptr, nullptr, nullptr, true));
  STCHK(inverse_x<double>(ctx, 0, L, XI_STRAIN, x, eps, nullptr, nullptr, nullptr, nullptr));
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.wgrad, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice,
                        ctx->stream));
  const Geo& g = ctx->geo;
  const int nb = (int)((g.nvox + 255) / 256);
  const double* wd = ctx->ptr<double>(ctx->off.wgrad);
  {
    Scope sc(ctx, K_GRAD, (double)L * ctx->F * 8.0 + (ctx->c == 6 ? 2.0 : 1.0) * g.nvox * (dtype == LSH_F64 ? 8 : 4));
#define LSH_GRAD(CC, TO) \
  hipLaunchKernelGGL((k_grad<CC, TO>), dim3(nb), dim3(256), 0, ctx->stream, g, L, eps, wd, static_cast<TO*>(grad))
    if (dtype == LSH_F64) {
      if (ctx->c == 2) LSH_GRAD(2, double);
      else if (ctx->c == 3) LSH_GRAD(3, double);
      else LSH_GRAD(6, double);
    } else {
      if (ctx->c == 2) LSH_GRAD(2, float);
      else if (ctx->c == 3) LSH_GRAD(3, float);
      else LSH_GRAD(6, float);
    }
#undef LSH_GRAD
    STCHK(check_launch(ctx, 0, "gradient"));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LSH_OK;
}

lsh_status lsh_set_green(lsh_ctx* ctx, int variant) {
  if (!ctx) return LSH_EINVAL;
  if (variant < LSH_GREEN_TRUNCATED || variant > LSH_GREEN_FD) return fail(ctx, LSH_EINVAL, "unknown Green operator");
  if (variant == LSH_GREEN_FD && ctx->physics != LSH_SCALAR)
    return fail(ctx, LSH_EINVAL, "the finite-difference operator is defined for scalar problems only");
  ctx->green = variant;
  ctx->tables_dirty = true;
  ctx->gst_dirty = true;
  ctx->have_solution = false;
  return LSH_OK;
}

lsh_status lsh_green_table_bytes(const lsh_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return LSH_EINVAL;
  const long long nk = main_cpx(ctx->geo) / ctx->c + nyq_cpx(ctx->geo) / ctx->c;
  const int ne = ctx->c * (ctx->c + 1) / 2;
  *bytes = align_up(sizeof(double) * nk * ne) + align_up(sizeof(float) * nk * ne);
  return LSH_OK;
}

lsh_status lsh_bind_green_table(lsh_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return LSH_EINVAL;
  size_t need = 0;
  lsh_green_table_bytes(ctx, &need);
  if (!dev_ptr) return fail(ctx, LSH_EINVAL, "null table buffer");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign != 0) return fail(ctx, LSH_EINVAL, "table not 256-byte aligned");
  if (bytes < need) return fail(ctx, LSH_ENOMEM, "table buffer too small: need " + std::to_string(need) + " bytes");
  ctx->gtab = static_cast<char*>(dev_ptr);
  ctx->gtab_size = bytes;
  ctx->tables_dirty = true;
  ctx->have_solution = false;
  return LSH_OK;
}

lsh_status lsh_set_green_series(lsh_ctx* ctx, int nmax) {
  if (!ctx) return LSH_EINVAL;
  if (nmax < 0 || nmax > 64) return fail(ctx, LSH_EINVAL, "nmax must be in 0..64");
  ctx->series = nmax;
  ctx->tables_dirty = true;
  ctx->have_solution = false;
  return LSH_OK;
}

lsh_status lsh_solver_buffer_bytes(const lsh_ctx* ctx, int solver, size_t* bytes) {
  if (!ctx || !bytes) return LSH_EINVAL;
  if (solver < LSH_SOLVER_BASIC || solver > LSH_SOLVER_SYMMLQ) return LSH_EINVAL;
  const bool krylov = solver == LSH_SOLVER_MINRES || solver == LSH_SOLVER_SYMMLQ;
  *bytes = krylov ? align_up(4 * sizeof(double) * (size_t)ctx->max_loads * ctx->F) : 0;
  return LSH_OK;
}

lsh_status lsh_bind_solver_buffer(lsh_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return LSH_EINVAL;
  size_t need = 0;
  lsh_solver_buffer_bytes(ctx, LSH_SOLVER_MINRES, &need);
  if (!dev_ptr) return fail(ctx, LSH_EINVAL, "null solver buffer");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign != 0)
    return fail(ctx, LSH_EINVAL, "solver buffer not 256-byte aligned");
  if (bytes < need) return fail(ctx, LSH_ENOMEM, "solver buffer too small: need " + std::to_string(need) + " bytes");
  ctx->sbuf = static_cast<char*>(dev_ptr);
  ctx->sbuf_size = bytes;
  return LSH_OK;
}

lsh_status lsh_solve(lsh_ctx* ctx, int solver, int nload, const double* loads, double tol, int maxit,
                     lsh_load_report* reports, lsh_solve_report* summary) {
  if (!ctx) return LSH_EINVAL;
  if (solver != LSH_SOLVER_BASIC && solver != LSH_SOLVER_CG && solver != LSH_SOLVER_MINRES &&
      solver != LSH_SOLVER_EYRE_MILTON && solver != LSH_SOLVER_SYMMLQ)
    return fail(ctx, LSH_EINVAL, "unknown solver");
  if (nload < 1 || nload > ctx->max_loads) return fail(ctx, LSH_EINVAL, "nload out of range");
  if (!loads) return fail(ctx, LSH_EINVAL, "null loads");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(ctx, LSH_EINVAL, "tol must be positive");
  if (maxit < 1) return fail(ctx, LSH_EINVAL, "maxit must be >= 1");
  const int c = ctx->c;
  for (int i = 0; i < nload * c; ++i)
    if (!std::isfinite(loads[i])) return fail(ctx, LSH_EINVAL, "non-finite load");
  if ((solver == LSH_SOLVER_MINRES || solver == LSH_SOLVER_SYMMLQ) && !ctx->sbuf)
    return fail(ctx, LSH_ESTATE, "MINRES and SYMMLQ need a bound solver buffer (lsh_solver_buffer_bytes)");
  if (solver == LSH_SOLVER_BASIC || solver == LSH_SOLVER_EYRE_MILTON) {
    const bool em = solver == LSH_SOLVER_EYRE_MILTON;
    if (ctx->tab_em != em) {
      ctx->tab_em = em;
      ctx->tables_dirty = true;
    }
  }
  TraceRange tr("lsh_solve");
  STCHK(prepare(ctx));
  ctx->nact = 1 << 30;
  const auto t0 = std::chrono::steady_clock::now();
  ctx->have_solution = false;
  // residual histories start empty (outside any captured graph)
  HIPCHK(hipMemsetAsync(ctx->ws + ctx->off.hcnt, 0, sizeof(unsigned long long) * nload, ctx->stream));
  ctx->hist_loads = nload;
  ctx->last_nload = nload;
  ctx->last_loads.assign(loads, loads + (size_t)nload * c);
  ctx->h_loads = ctx->last_loads;
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.loads, ctx->h_loads.data(), ctx->h_loads.size() * sizeof(double),
                        hipMemcpyHostToDevice, ctx->stream));
  // initial guesses apply to this solve only
  ctx->h_guess_up.assign(ctx->h_guess.begin(), ctx->h_guess.begin() + nload);
  std::fill(ctx->h_guess.begin(), ctx->h_guess.end(), 0);
  HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.guess, ctx->h_guess_up.data(), (size_t)nload, hipMemcpyHostToDevice,
                        ctx->stream));

  LoadState* sto = ctx->ptr<LoadState>(ctx->off.st_out);
  LoadState* sti = ctx->ptr<LoadState>(ctx->off.st_in);
  double* x64 = ctx->ptr<double>(ctx->off.x64);
  std::vector<LoadState> hst, hin;
  std::vector<long long> iters(nload, 0);
  long long apps64 = 0, apps32 = 0;
  int outer = 0;
  bool residual_known = false;
  std::vector<double> res2(nload, 0.0), bb(nload, 0.0);

  if (solver == LSH_SOLVER_BASIC || solver == LSH_SOLVER_EYRE_MILTON) {
    STCHK(guess_init(ctx, nload, x64, nullptr, sto, tol));   // tau_0 = 0 or the guess
    STCHK(basic_loop(ctx, nload, x64, sto, ctx->off.st_out, maxit, hst,
                     solver == LSH_SOLVER_BASIC ? XI_BASIC : XI_EM));
    STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
    for (int l = 0; l < nload; ++l) iters[l] = hst[l].iters, apps64 += hst[l].iters;
  } else if (solver == LSH_SOLVER_MINRES || solver == LSH_SOLVER_SYMMLQ) {
    STCHK(solver == LSH_SOLVER_MINRES ? mr_loop(ctx, nload, tol, maxit, hst) : sy_loop(ctx, nload, tol, maxit, hst));
    STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
    for (int l = 0; l < nload; ++l) iters[l] = hst[l].iters, apps64 += hst[l].iters;
  } else if (ctx->precision == LSH_FP64) {
    double* r = ctx->ptr<double>(ctx->off.r64);
    double* p = ctx->ptr<double>(ctx->off.p64);
    STCHK(guess_init(ctx, nload, x64, r, sto, tol));
    STCHK(cg_loop<double>(ctx, nload, x64, r, p, ctx->ptr<double>(ctx->off.p64b), sto, ctx->off.st_out, maxit, hst));
    STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
    for (int l = 0; l < nload; ++l) iters[l] = hst[l].iters, apps64 += hst[l].iters;
  } else {
    // mixed precision: FP32 CG on the correction, FP64 residual refinement
    float* d = ctx->ptr<float>(ctx->off.d32);
    float* r = ctx->ptr<float>(ctx->off.r32);
    float* p = ctx->ptr<float>(ctx->off.p32);
    // x64 = 0 or the guess, outer ||b||^2.  Without guesses the first
    // refinement pass writes x64 = d (zero for the loads it does not refine),
    // so x64 is not zeroed here.
    bool xzero = !any_guess(ctx, nload);
    STCHK(guess_init(ctx, nload, x64, nullptr, sto, tol, !xzero));
    STCHK(cg_init<float>(ctx, nload, d, r, sti, 1e-4));      // d = 0, r = b
    STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
    double eta = 1e-4;
    int budget = maxit;
    // from initial guesses the first pass is the refinement alone (d = 0):
    // r = b - L x64 in FP64, then the inner solve restarts from it
    bool refine_first = any_guess(ctx, nload);
    // breakdown or non-finite values met by a load's inner solve end that load
    // (with that status) once its progress so far is refined into x64
    std::vector<int> inner_bad(nload, 0);
    bool stalled = false;
    while (true) {
      if (!refine_first) {
        // inner FP32 solve, then refresh the residual in FP64 (x64 += d inside)
        {
          TraceRange tr_in("lsh_solve: inner FP32 CG");
          // pending x updates stay for the refinement pass to apply
          STCHK(cg_loop<float>(ctx, nload, d, r, p, ctx->ptr<float>(ctx->off.p32b), sti, ctx->off.st_in, budget, hin,
                               false));
        }
        STCHK(read_states(ctx, ctx->off.st_in, nload, hin));
        int used = 0;
        for (int l = 0; l < nload; ++l) {
          iters[l] += hin[l].iters;
          apps32 += hin[l].iters;
          used = std::max(used, hin[l].iters);
          if (hst[l].active && hin[l].status != kStatusOk) inner_bad[l] = hin[l].status;
        }
        // every pass costs budget, and a pass in which no inner solve moved
        // (all stopped at once: breakdown, NaN/Inf, or an FP32 residual that
        // vanished while the FP64 one did not) is the last
        budget -= std::max(used, 1);
        stalled = used == 0;
      }
      refine_first = false;
      ctx->nact = 0;
      for (auto& sv : hst) ctx->nact += sv.active != 0;
      {
        TraceRange tr_ref("lsh_solve: FP64 refinement residual");
        // x64 += d plus the inner solve's pending steps (x64 = that, on the first pass from zero)
        const IrxFold fold{p, ctx->cg_fused ? ctx->ptr<float>(ctx->off.p32b) : nullptr, sti, xzero ? 1 : 0};
        STCHK(forward_part<double>(ctx, 0, nload, XF_IRX, nullptr, x64, nullptr, d, sto, true, fold));
        xzero = false;
        int np = 0;
        STCHK(inverse_x<double>(ctx, 0, nload, XI_IRRES, x64, nullptr, r, sto, ctx->ptr<double>(ctx->off.partials),
                                &np));
        STCHK(scal(ctx, SC_OUTER, nload, np, sto, 0.0));
      }
      ++outer;
      STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
      bool ended = false;
      for (int l = 0; l < nload; ++l)
        if (hst[l].active && inner_bad[l] != kStatusOk) {
          hst[l].active = 0;
          hst[l].status = inner_bad[l];
          ended = true;
        }
      if (ended) {
        HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.st_out, hst.data(), sizeof(LoadState) * nload,
                              hipMemcpyHostToDevice, ctx->stream));
        STCHK(wait_stream(ctx));
      }
      bool any = false;
      double worst = 0.0;
      for (int l = 0; l < nload; ++l) {
        if (hst[l].active) {
          any = true;
          worst = std::max(worst, std::sqrt(hst[l].res2 / hst[l].bb));
        }
      }
      if (!any || budget <= 0 || stalled) break;
      eta = std::max(1e-4, 0.5 * tol / std::max(worst, 1e-300));
      eta = std::min(eta, 0.5);
      // restart the inner solve on the loads still refining
      const int nb = ew_blocks(ctx->F);
      {
        Scope sc(ctx, K_INIT);
        hipLaunchKernelGGL((k_innerinit<float>), dim3(nb, nload), dim3(256), 0, ctx->stream, (long long)ctx->F, d, r,
                           sto, ctx->ptr<double>(ctx->off.partials), (int)ctx->pstride);
        STCHK(check_launch(ctx, 0, "inner init"));
      }
      STCHK(scal(ctx, SC_INIT, nload, nb, sti, eta));
      // loads already refined stay frozen in the inner solve
      STCHK(read_states(ctx, ctx->off.st_in, nload, hin));
      bool patched = false;
      for (int l = 0; l < nload; ++l)
        if (!hst[l].active && hin[l].active) {
          hin[l].active = 0;
          patched = true;
        }
      if (patched) {
        HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.st_in, hin.data(), sizeof(LoadState) * nload,
                              hipMemcpyHostToDevice, ctx->stream));
        STCHK(wait_stream(ctx));
      }
    }
    for (int l = 0; l < nload; ++l) {
      iters[l] += hst[l].iters;
      apps64 += hst[l].iters;
      res2[l] = hst[l].res2;
      bb[l] = hst[l].bb;
    }
    residual_known = true;
  }

  // FP64 true residual of the result (CG and basic), A*
  ctx->nact = 1 << 30;
  if (!residual_known) {
    STCHK(true_residual(ctx, nload));
    std::vector<double> s(nload);
    STCHK(read_back(ctx, s.data(), ctx->ws + ctx->off.sums, sizeof(double) * nload,
                    sizeof(LoadState) * ctx->max_loads));
    STCHK(read_states(ctx, ctx->off.st_out, nload, hst));
    for (int l = 0; l < nload; ++l) {
      res2[l] = s[l];
      bb[l] = hst[l].bb;
    }
    for (int l = 0; l < nload; ++l) apps64 += 1;
  }
  STCHK(effective(ctx, nload));
  const auto t1 = std::chrono::steady_clock::now();

  lsh_status overall = LSH_OK;
  for (int l = 0; l < nload; ++l) {
    lsh_status ls = LSH_OK;
    if (hst[l].status == kStatusBreakdown) ls = LSH_EBREAKDOWN;
    else if (hst[l].status == kStatusNumeric) ls = LSH_ENUMERIC;
    else if (hst[l].active) ls = LSH_MAXIT;
    if (reports) {
      reports[l].iterations = (int32_t)iters[l];
      reports[l].status = ls;
      reports[l].rel_residual = bb[l] > 0 ? std::sqrt(res2[l] / bb[l]) : 0.0;
    }
    if (ls < 0 && overall >= 0) overall = ls;
    if (ls == LSH_MAXIT && overall == LSH_OK) overall = LSH_MAXIT;
  }
  if (summary) {
    summary->applications_fp64 = apps64;
    summary->applications_fp32 = apps32;
    summary->outer_iterations = outer;
    summary->pad = 0;
    summary->seconds = std::chrono::duration<double>(t1 - t0).count();
  }
  ctx->have_solution = true;
  if (overall == LSH_EBREAKDOWN) ctx->err = "CG breakdown: the system is not positive definite for this A0";
  if (overall == LSH_ENUMERIC) ctx->err = "NaN or Inf during the solve";
  return overall;
}

lsh_status lsh_get_effective(lsh_ctx* ctx, double* sigma_mean) {
  if (!ctx || !sigma_mean) return LSH_EINVAL;
  if (!ctx->have_solution) return fail(ctx, LSH_ESTATE, "no solution");
  std::memcpy(sigma_mean, ctx->sigma.data(), ctx->sigma.size() * sizeof(double));
  return LSH_OK;
}

static lsh_status copy_field_out(lsh_ctx* ctx, const double* src, long long n, void* dst, int dtype, int mem) {
  if (mem == LSH_DEVICE) {
    if (dtype == LSH_F64) {
      HIPCHK(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    } else {
      Scope sc(ctx, K_COPY);
      hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, n,
                         src, static_cast<float*>(dst));
      STCHK(check_launch(ctx, 0, "convert"));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return LSH_OK;
  }
  std::vector<double> h((size_t)n);
  HIPCHK(hipMemcpyAsync(h.data(), src, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (dtype == LSH_F64) {
    std::memcpy(dst, h.data(), n * sizeof(double));
  } else {
    float* f = static_cast<float*>(dst);
    for (long long i = 0; i < n; ++i) f[i] = (float)h[(size_t)i];
  }
  return LSH_OK;
}

lsh_status lsh_set_initial_guess(lsh_ctx* ctx, int load, const void* tau, int dtype, int mem) {
  if (!ctx) return LSH_EINVAL;
  if (load < 0 || load >= ctx->max_loads) return fail(ctx, LSH_EINVAL, "load out of range");
  if (!tau) {
    ctx->h_guess[load] = 0;
    return LSH_OK;
  }
  if (dtype != LSH_F64 && dtype != LSH_F32) return fail(ctx, LSH_EINVAL, "bad dtype");
  if (mem != LSH_HOST && mem != LSH_DEVICE) return fail(ctx, LSH_EINVAL, "bad memory space");
  if (!ctx->ws) return fail(ctx, LSH_ESTATE, "workspace not bound");
  const long long F = ctx->F;
  double* x = ctx->ptr<double>(ctx->off.x64) + (long long)load * F;
  if (mem == LSH_DEVICE) {
    if (dtype == LSH_F64) {
      HIPCHK(hipMemcpyAsync(x, tau, F * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    } else {
      Scope sc(ctx, K_COPY);
      hipLaunchKernelGGL((k_convert<float, double>), dim3((unsigned)((F + 255) / 256)), dim3(256), 0, ctx->stream, F,
                         static_cast<const float*>(tau), x);
      STCHK(check_launch(ctx, 0, "convert"));
    }
  } else if (dtype == LSH_F64) {
    HIPCHK(hipMemcpyAsync(x, tau, F * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  } else {
    std::vector<double> h((size_t)F);
    const float* f = static_cast<const float*>(tau);
    for (long long i = 0; i < F; ++i) h[(size_t)i] = (double)f[i];
    HIPCHK(hipMemcpyAsync(x, h.data(), F * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->h_guess[load] = 1;
  ctx->have_solution = false;   // the solution slot of this load now holds the guess
  return LSH_OK;
}

lsh_status lsh_get_field(lsh_ctx* ctx, int load, int which, void* dst, int dtype, int mem) {
  if (!ctx) return LSH_EINVAL;
  if (!dst) return fail(ctx, LSH_EINVAL, "null destination");
  if (!ctx->have_solution) return fail(ctx, LSH_ESTATE, "no solution");
  if (load < 0 || load >= ctx->last_nload) return fail(ctx, LSH_EINVAL, "load out of range");
  if (dtype != LSH_F64 && dtype != LSH_F32) return fail(ctx, LSH_EINVAL, "bad dtype");
  if (mem != LSH_HOST && mem != LSH_DEVICE) return fail(ctx, LSH_EINVAL, "bad memory space");
  if (which != LSH_FIELD_TAU && which != LSH_FIELD_STRAIN) return fail(ctx, LSH_EINVAL, "bad field");
  const long long F = ctx->F;
  double* x = ctx->ptr<double>(ctx->off.x64) + (long long)load * F;
  if (which == LSH_FIELD_TAU) return copy_field_out(ctx, x, F, dst, dtype, mem);
  // strain p - Gamma tau, computed into the FP64 spectrum slot of this load
  STCHK(forward_part<double>(ctx, load, 1, XF_PLAIN, x, nullptr, nullptr, nullptr, nullptr, true));
  double* out = reinterpret_cast<double*>(Sel<double>::sm(ctx) + (long long)load * main_cpx(ctx->geo));
  STCHK(inverse_x<double>(ctx, load, 1, XI_STRAIN, x, out, nullptr, nullptr, nullptr, nullptr));
  return copy_field_out(ctx, out, F, dst, dtype, mem);
}

lsh_status lsh_apply(lsh_ctx* ctx, int nload, const void* tau, void* out, int dtype) {
  if (!ctx) return LSH_EINVAL;
  TraceRange tr("lsh_apply");
  if (nload < 1 || nload > ctx->max_loads) return fail(ctx, LSH_EINVAL, "nload out of range");
  if (!tau || !out || tau == out) return fail(ctx, LSH_EINVAL, "bad buffers");
  if (dtype != LSH_F64 && dtype != LSH_F32) return fail(ctx, LSH_EINVAL, "bad dtype");
  if (dtype == LSH_F32 && ctx->precision != LSH_MIXED)
    return fail(ctx, LSH_EINVAL, "FP32 application needs a mixed-precision context");
  STCHK(prepare(ctx));
  if (dtype == LSH_F64) {
    STCHK(forward_part<double>(ctx, 0, nload, XF_PLAIN, static_cast<const double*>(tau), nullptr, nullptr, nullptr,
                               nullptr, true));
    STCHK(inverse_x<double>(ctx, 0, nload, XI_APPLY, static_cast<const double*>(tau), static_cast<double*>(out),
                            nullptr, nullptr, nullptr, nullptr));
  } else {
    STCHK(forward_part<float>(ctx, 0, nload, XF_PLAIN, static_cast<const float*>(tau), nullptr, nullptr, nullptr,
                              nullptr, true));
    STCHK(inverse_x<float>(ctx, 0, nload, XI_APPLY, static_cast<const float*>(tau), static_cast<float*>(out), nullptr,
                           nullptr, nullptr, nullptr));
  }
  ctx->have_solution = false;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LSH_OK;
}

lsh_status lsh_apply_noalloc(lsh_ctx* ctx, int nload, const void* tau, void* out, int dtype) {
  if (!ctx) return LSH_EINVAL;
  if (nload < 1 || nload > ctx->max_loads) return fail(ctx, LSH_EINVAL, "nload out of range");
  if (!tau || !out || tau == out) return fail(ctx, LSH_EINVAL, "bad buffers");
  if (reinterpret_cast<uintptr_t>(out) % kAlign != 0) return fail(ctx, LSH_EINVAL, "out not 256-byte aligned");
  if (dtype != LSH_F64 && dtype != LSH_F32) return fail(ctx, LSH_EINVAL, "bad dtype");
  if (dtype == LSH_F32 && ctx->precision != LSH_MIXED)
    return fail(ctx, LSH_EINVAL, "FP32 application needs a mixed-precision context");
  const size_t nyq = (size_t)nload * nyq_cpx(ctx->geo) * (dtype == LSH_F64 ? 16 : 8);
  if (nyq > kScratchBytes)
    return fail(ctx, LSH_ENOMEM, "the Nyquist plane of " + std::to_string(nload) + " loads needs " +
                                     std::to_string(nyq) + " bytes, beyond the " + std::to_string(kScratchBytes) +
                                     "-byte scratch of lsh_apply_noalloc");
  STCHK(prepare(ctx));
  void* sp = nullptr;
  STCHK(scratch_address(ctx, &sp));
  ctx->ovr_sm = out;
  ctx->ovr_sn = sp;
  lsh_status s;
  if (dtype == LSH_F64) {
    s = forward_part<double>(ctx, 0, nload, XF_PLAIN, static_cast<const double*>(tau), nullptr, nullptr, nullptr,
                             nullptr, true);
    if (s == LSH_OK)
      s = inverse_x<double>(ctx, 0, nload, XI_APPLY, static_cast<const double*>(tau), static_cast<double*>(out),
                            nullptr, nullptr, nullptr, nullptr);
  } else {
    s = forward_part<float>(ctx, 0, nload, XF_PLAIN, static_cast<const float*>(tau), nullptr, nullptr, nullptr,
                            nullptr, true);
    if (s == LSH_OK)
      s = inverse_x<float>(ctx, 0, nload, XI_APPLY, static_cast<const float*>(tau), static_cast<float*>(out), nullptr,
                           nullptr, nullptr, nullptr);
  }
  ctx->ovr_sm = nullptr;
  ctx->ovr_sn = nullptr;
  STCHK(s);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LSH_OK;
}

lsh_status lsh_spectrum_bytes(const lsh_ctx* ctx, int dtype, size_t* bytes) {
  if (!ctx || !bytes) return LSH_EINVAL;
  if (dtype != LSH_F64 && dtype != LSH_F32) return LSH_EINVAL;
  const size_t s = dtype == LSH_F64 ? 16 : 8;
  *bytes = s * (size_t)(main_cpx(ctx->geo) + nyq_cpx(ctx->geo));
  return LSH_OK;
}

lsh_status lsh_forward_dft(lsh_ctx* ctx, int nload, const void* field, void* spec, int dtype) {
  if (!ctx) return LSH_EINVAL;
  if (nload < 1 || nload > ctx->max_loads) return fail(ctx, LSH_EINVAL, "nload out of range");
  if (!field || !spec) return fail(ctx, LSH_EINVAL, "bad buffers");
  if (dtype != LSH_F64 && dtype != LSH_F32) return fail(ctx, LSH_EINVAL, "bad dtype");
  if (dtype == LSH_F32 && ctx->precision != LSH_MIXED)
    return fail(ctx, LSH_EINVAL, "FP32 transforms need a mixed-precision context");
  STCHK(prepare(ctx));
  const long long nm = main_cpx(ctx->geo) * nload, nn = nyq_cpx(ctx->geo) * nload;
  if (dtype == LSH_F64) {
    STCHK(forward_part<double>(ctx, 0, nload, XF_PLAIN, static_cast<const double*>(field), nullptr, nullptr, nullptr,
                               nullptr, false));
    HIPCHK(hipMemcpyAsync(spec, Sel<double>::sm(ctx), nm * 16, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(static_cast<char*>(spec) + nm * 16, Sel<double>::sn(ctx), nn * 16, hipMemcpyDeviceToDevice,
                          ctx->stream));
  } else {
    STCHK(forward_part<float>(ctx, 0, nload, XF_PLAIN, static_cast<const float*>(field), nullptr, nullptr, nullptr,
                              nullptr, false));
    HIPCHK(hipMemcpyAsync(spec, Sel<float>::sm(ctx), nm * 8, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(static_cast<char*>(spec) + nm * 8, Sel<float>::sn(ctx), nn * 8, hipMemcpyDeviceToDevice,
                          ctx->stream));
  }
  ctx->have_solution = false;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LSH_OK;
}

lsh_status lsh_set_variant(lsh_ctx* ctx, int pass, int fp64, int variant) {
  if (!ctx) return LSH_EINVAL;
  if (pass < 0 || pass >= NPASS || variant < 0 || variant >= pass_variants(pass))
    return fail(ctx, LSH_EINVAL, "bad pass or variant");
  ctx->tune[fp64 ? 1 : 0][pass] = variant;
  ctx->graph_epoch++;
  return LSH_OK;
}

lsh_status lsh_get_residual_history(lsh_ctx* ctx, int load, int cap, double* rel, int32_t* level, int64_t* total) {
  if (!ctx) return LSH_EINVAL;
  if (load < 0 || load >= ctx->hist_loads) return fail(ctx, LSH_EINVAL, "no residual history for that load");
  if (cap < 0 || (cap > 0 && (!rel || !level))) return fail(ctx, LSH_EINVAL, "bad history buffers");
  unsigned long long cnt = 0;
  std::vector<double> ring((size_t)2 * kHistCap);
  HIPCHK(hipMemcpyAsync(&cnt, ctx->ws + ctx->off.hcnt + sizeof(unsigned long long) * load, sizeof(cnt),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipMemcpyAsync(ring.data(), ctx->ws + ctx->off.hist + sizeof(double) * 2 * kHistCap * load,
                        sizeof(double) * ring.size(), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (total) *total = (int64_t)cnt;
  // the last n entries in order (the ring keeps the last kHistCap)
  const unsigned long long n = std::min<unsigned long long>({cnt, (unsigned long long)kHistCap, (unsigned long long)cap});
  for (unsigned long long i = 0; i < n; ++i) {
    const unsigned long long k = (cnt - n + i) % kHistCap;
    rel[i] = std::sqrt(ring[2 * k]);
    level[i] = (int32_t)ring[2 * k + 1];
  }
  return LSH_OK;
}

lsh_status lsh_get_variants(const lsh_ctx* ctx, int32_t* variants) {
  if (!ctx || !variants) return LSH_EINVAL;
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < NPASS; ++q) variants[p * NPASS + q] = ctx->tune[p][q];
  return LSH_OK;
}

lsh_status lsh_autotune(lsh_ctx* ctx, int nload, const char* cache_path, int32_t* variants, int* from_cache) {
  if (!ctx) return LSH_EINVAL;
  TraceRange tr("lsh_autotune");
  if (nload < 1 || nload > ctx->max_loads) return fail(ctx, LSH_EINVAL, "nload out of range");
  STCHK(prepare(ctx));
  const std::string key = tune_key(ctx, nload);
  std::map<std::string, std::vector<int>> cache;
  if (from_cache) *from_cache = 0;
  if (cache_path) {
    cache = read_tune_cache(cache_path);
    auto it = cache.find(key);
    if (it != cache.end()) {
      for (int p = 0; p < 2; ++p)
        for (int q = 0; q < NPASS; ++q) ctx->tune[p][q] = it->second[p * NPASS + q];
      ctx->graph_epoch++;
      if (from_cache) *from_cache = 1;
      if (variants) lsh_get_variants(ctx, variants);
      return LSH_OK;
    }
  }
  // search: each pass of each precision in turn, the others at their current choice
  const bool saved_timing = ctx->timing;
  drain_timers(ctx);
  ctx->timing = true;
  ctx->nact = 1 << 30;
  const int reps = 3;
  // inputs: smooth finite fields, and load states that take the full CG path
  // (active, not the first step, x updates pending: two, so that the fused x
  // pass takes its heavier paired form; zero steps keep the fields bounded)
  {
    const long long n = (long long)nload * ctx->F;
    const unsigned nb = (unsigned)((n + 255) / 256);
    std::vector<double*> f64 = {ctx->ptr<double>(ctx->off.x64)};
    std::vector<float*> f32;
    if (ctx->precision == LSH_MIXED) {
      f32 = {ctx->ptr<float>(ctx->off.d32), ctx->ptr<float>(ctx->off.r32), ctx->ptr<float>(ctx->off.p32),
             ctx->ptr<float>(ctx->off.p32b)};
    } else {
      f64.push_back(ctx->ptr<double>(ctx->off.r64));
      f64.push_back(ctx->ptr<double>(ctx->off.p64));
      f64.push_back(ctx->ptr<double>(ctx->off.p64b));
    }
    for (double* f : f64) hipLaunchKernelGGL((k_fill<double>), dim3(nb), dim3(256), 0, ctx->stream, n, f);
    for (float* f : f32) hipLaunchKernelGGL((k_fill<float>), dim3(nb), dim3(256), 0, ctx->stream, n, f);
    STCHK(check_launch(ctx, 0, "fill"));
    LoadState s0{};
    s0.rr = s0.pq = s0.bb = s0.res2 = 1.0;
    s0.active = 1;
    s0.pending = 2;
    std::vector<LoadState> hs((size_t)nload, s0);
    HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.st_in, hs.data(), sizeof(LoadState) * nload, hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->ws + ctx->off.st_out, hs.data(), sizeof(LoadState) * nload, hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  for (int prec = ctx->precision == LSH_MIXED ? 0 : 1; prec < 2; ++prec) {
    const bool fp64 = prec == 1;
    // the z pass before the y passes: its shape 5 sets the spectrum layout the
    // y passes convert, so they are timed in the layout they will run in
    const int order[NPASS] = {PASS_XFWD, PASS_ZG, PASS_Y, PASS_XINV};
    for (int pi = 0; pi < NPASS; ++pi) {
      const int pass = order[pi];
      if (!pass_has_variants(ctx, pass)) continue;
      // the fused CG x pass has one shape (CG fields: FP32 of a mixed context, FP64 of an FP64 one)
      if (pass == PASS_XFWD && ctx->cg_fused && (!fp64 || ctx->precision != LSH_MIXED)) continue;
      const int cls = pass_class(pass, fp64);
      double best_t = 1e300;
      int best_v = ctx->tune[prec][pass];
      for (int v = 0; v < pass_variants(pass); ++v) {
        ctx->tune[prec][pass] = v;
        // one warm-up application, then the timed ones
        STCHK(timing_iteration(ctx, nload, fp64));
        drain_timers(ctx);
        const double t0 = ctx->tsum[cls];
        const long long c0 = ctx->tcount[cls];
        for (int r = 0; r < reps; ++r) STCHK(timing_iteration(ctx, nload, fp64));
        drain_timers(ctx);
        const long long dc = ctx->tcount[cls] - c0;
        const double t = dc > 0 ? (ctx->tsum[cls] - t0) / (double)dc : 1e300;
        if (t < best_t) {
          best_t = t;
          best_v = v;
        }
      }
      ctx->tune[prec][pass] = best_v;
    }
  }
  // timing sums of the search are not the caller's
  for (int k = 0; k < K_NCLASS; ++k) {
    ctx->tsum[k] = 0.0;
    ctx->tbytes[k] = 0.0;
    ctx->tcount[k] = 0;
  }
  ctx->timing = saved_timing;
  ctx->graph_epoch++;
  ctx->have_solution = false;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (cache_path) {
    std::vector<int> v(2 * NPASS);
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < NPASS; ++q) v[p * NPASS + q] = ctx->tune[p][q];
    cache = read_tune_cache(cache_path);   // entries other processes may have added meanwhile
    cache[key] = v;
    if (!write_tune_cache(cache_path, cache)) return fail(ctx, LSH_EINVAL, std::string("cannot write ") + cache_path);
  }
  if (variants) lsh_get_variants(ctx, variants);
  return LSH_OK;
}

lsh_status lsh_solve_many(int n, lsh_ctx* const* ctxs, int solver, const int32_t* nloads, const double* const* loads,
                          double tol, int maxit, lsh_load_report* const* reports, lsh_solve_report* summaries,
                          int32_t* statuses, int nthreads) {
  if (n < 1 || !ctxs || !nloads || !loads) return LSH_EINVAL;
  TraceRange tr("lsh_solve_many");
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !loads[i]) return LSH_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(ctxs[i], LSH_EINVAL, "a context appears twice in one ensemble solve");
  }
  if (t_fibers.cur != nullptr) return fail(ctxs[0], LSH_ESTATE, "lsh_solve_many called from inside an ensemble solve");
  const int slots = std::min(std::max(nthreads, 1), n);
  std::vector<lsh_status> st(n, LSH_OK);
  // one member at a time per slot; a slot is a fiber with its own stack
  // (reserved address space with a guard page, pages committed on use)
  constexpr size_t kStack = 16u << 20, kGuard = 64u << 10;
  std::vector<Fiber> fib(slots);
  int next = 0;
  bool setup_ok = true;
  for (auto& f : fib) {
    void* mem = mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (mem == MAP_FAILED) {
      setup_ok = false;
      break;
    }
    (void)mprotect(mem, kGuard, PROT_NONE);
    f.stack = mem;
    f.stack_bytes = kStack;
    f.body = [&]() {
      while (true) {
        const int i = next++;
        if (i >= n) break;
        lsh_ctx* c = ctxs[i];
        if (c->ws_device >= 0) {
          int cur = -1;
          if (hipGetDevice(&cur) == hipSuccess && cur != c->ws_device) (void)hipSetDevice(c->ws_device);
        }
        st[i] = lsh_solve(c, solver, nloads[i], loads[i], tol, maxit, reports ? reports[i] : nullptr,
                          summaries ? &summaries[i] : nullptr);
      }
    };
    getcontext(&f.uc);
    f.uc.uc_stack.ss_sp = static_cast<char*>(mem) + kGuard;
    f.uc.uc_stack.ss_size = kStack - kGuard;
    f.uc.uc_link = nullptr;
    makecontext(&f.uc, fiber_entry, 0);
  }
  if (setup_ok) {
    // round robin over the slots until every member is solved; each turn runs
    // a fiber up to its next wait for the GPU
    bool any = true;
    while (any) {
      any = false;
      for (auto& f : fib) {
        if (f.done) continue;
        any = true;
        t_fibers.cur = &f;
        swapcontext(&t_fibers.main, &f.uc);
        t_fibers.cur = nullptr;
      }
    }
  }
  for (auto& f : fib)
    if (f.stack) munmap(f.stack, f.stack_bytes);
  if (!setup_ok) return fail(ctxs[0], LSH_ENOMEM, "cannot reserve fiber stacks");
  lsh_status overall = LSH_OK;
  for (int i = 0; i < n; ++i) {
    if (statuses) statuses[i] = st[i];
    if (st[i] < 0 && overall >= 0) overall = st[i];
    if (st[i] == LSH_MAXIT && overall == LSH_OK) overall = LSH_MAXIT;
  }
  return overall;
}

lsh_status lsh_set_persistent(lsh_ctx* ctx, int enable) {
  if (!ctx) return LSH_EINVAL;
  ctx->persistent = enable != 0;
  return LSH_OK;
}

lsh_status lsh_set_graphs(lsh_ctx* ctx, int enable) {
  if (!ctx) return LSH_EINVAL;
  ctx->use_graphs = enable != 0;
  return LSH_OK;
}

lsh_status lsh_set_timing(lsh_ctx* ctx, int enable) {
  if (!ctx) return LSH_EINVAL;
  drain_timers(ctx);
  ctx->timing = enable != 0;
  for (int k = 0; k < K_NCLASS; ++k) {
    ctx->tsum[k] = 0.0;
    ctx->tbytes[k] = 0.0;
    ctx->tcount[k] = 0;
  }
  return LSH_OK;
}

lsh_status lsh_kernel_times(lsh_ctx* ctx, const char** names, double* total_ms, int64_t* launches,
                            double* alg_bytes, int cap, int* count) {
  if (!ctx || !count) return LSH_EINVAL;
  drain_timers(ctx);
  for (int i = 0; i < K_NCLASS && i < cap; ++i) {
    if (names) names[i] = kClassNames[i];
    if (total_ms) total_ms[i] = ctx->tsum[i];
    if (launches) launches[i] = ctx->tcount[i];
    if (alg_bytes) alg_bytes[i] = ctx->tbytes[i];
  }
  *count = K_NCLASS;
  return LSH_OK;
}

}  // extern "C"
