// C ABI (include/fl.h): validation, operator handles, device buffers and
// the host-side control of the solvers.  No exception crosses the boundary.
#include "../../include/fl.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fl_internal.h"

#include <unordered_map>

namespace fl {
namespace {

struct Allocator {
  fl_alloc_fn alloc = nullptr;
  fl_release_fn release = nullptr;
  void* ctx = nullptr;
};

std::mutex g_alloc_mu;
Allocator g_alloc;                               // current (null: hipMalloc)
std::unordered_map<void*, Allocator> g_owner;    // blocks from a registered allocator

}  // namespace

void* dev_alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  Allocator a;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
  }
  void* p = nullptr;
  if (!a.alloc) {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(FL_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
  }
  p = a.alloc(bytes, a.ctx);
  if (!p) throw Error(FL_E_NOMEM, "the registered allocator failed for " + std::to_string(bytes) +
                                      " bytes");
  if (reinterpret_cast<uintptr_t>(p) % 256) {
    a.release(p, a.ctx);
    throw Error(FL_E_NOMEM, "the registered allocator returned memory not aligned to 256 bytes");
  }
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_owner[p] = a;
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  Allocator a;
  bool registered = false;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_owner.find(p);
    if (it != g_owner.end()) {
      a = it->second;
      g_owner.erase(it);
      registered = true;
    }
  }
  if (!registered) {
    (void)hipFree(p);
    return;
  }
  // hipFree waits for the device; a caller's allocator may reuse the block at
  // once, so wait here for every queued use of it to finish
  (void)hipDeviceSynchronize();
  a.release(p, a.ctx);
}

struct SetupScratch::Area {
  std::mutex mu;
  char* p = nullptr;
  size_t bytes = 0;
};

namespace {
std::mutex g_area_mu;
std::unordered_map<int, SetupScratch::Area*> g_areas;   // per device, never freed
}  // namespace

SetupScratch::SetupScratch(size_t bytes, hipStream_t st) : size_(scratch_round(bytes)), st_(st) {
  if (size_ == 0) size_ = 256;
  if (size_ > kSetupScratchCap) {
    base_ = (char*)dev_alloc(size_);
    return;
  }
  int dev = 0;
  FL_HIP(hipGetDevice(&dev));
  Area* a = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_area_mu);
    auto it = g_areas.find(dev);
    if (it == g_areas.end()) it = g_areas.emplace(dev, new Area).first;
    a = it->second;
  }
  a->mu.lock();
  if (a->bytes < size_) {
    size_t grow = size_t(1) << 20;
    while (grow < size_) grow <<= 1;
    if (a->p) (void)hipFree(a->p);
    a->p = nullptr;
    a->bytes = 0;
    if (hipMalloc(&a->p, grow) != hipSuccess) {
      (void)hipGetLastError();
      a->p = nullptr;
      a->mu.unlock();
      throw Error(FL_E_NOMEM, "hipMalloc of " + std::to_string(grow) +
                                  " bytes of setup scratch failed");
    }
    a->bytes = grow;
  }
  area_ = a;
  base_ = a->p;
}

SetupScratch::~SetupScratch() {
  (void)hipStreamSynchronize(st_);
  if (area_)
    area_->mu.unlock();
  else
    dev_free(base_);
}

void* SetupScratch::take(size_t bytes) {
  const size_t b = scratch_round(bytes == 0 ? 1 : bytes);
  if (used_ + b > size_) throw Error(FL_E_DEVICE, "setup scratch lease exceeded");
  void* p = base_ + used_;
  used_ += b;
  return p;
}

}  // namespace fl

using fl::Error;

namespace {

thread_local std::string g_last_error;

fl_status fail(int code, const std::string& msg) {
  g_last_error = msg;
  return (fl_status)code;
}

template <typename F>
fl_status guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(FL_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(FL_E_DEVICE, e.what());
  }
}

void* dmalloc(size_t bytes) { return fl::dev_alloc(bytes); }

// Grow-only device buffer.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void* get(size_t need) {
    if (need > bytes) {
      if (p) fl::dev_free(p);
      p = nullptr;
      bytes = 0;
      p = dmalloc(need);
      bytes = need;
    }
    return p;
  }
  void release() {
    if (p) fl::dev_free(p);
    p = nullptr;
    bytes = 0;
  }
};

constexpr int kMaxBlocks = 8192;

// Device-resident CG bookkeeping for up to `cap` right-hand sides.
struct CgState {
  DBuf mem;
  int cap = 0;
  fl::CgScalars s{};
  void ensure(int nrhs, hipStream_t st) {
    if (nrhs <= cap) return;
    const size_t nd8 = (size_t)nrhs * sizeof(double);
    const size_t ni4 = (size_t)nrhs * sizeof(int);
    const size_t part = (size_t)nrhs * kMaxBlocks * sizeof(double);
    const size_t total = 5 * nd8 + 3 * ni4 + sizeof(int) + 3 * part + 12 * 256;
    char* b = (char*)mem.get(total);
    auto take = [&](size_t n) {
      char* r = b;
      b += (n + 255) / 256 * 256;
      return r;
    };
    char* base = b;
    s.rr_cur = (double*)take(nd8);
    s.rr_prev = (double*)take(nd8);
    s.thresh2 = (double*)take(nd8);
    s.alpha = (double*)take(nd8);
    s.res2 = (double*)take(nd8);
    s.active = (int*)take(ni4);
    s.iters = (int*)take(ni4);
    s.status = (int*)take(ni4);
    s.n_active = (int*)take(sizeof(int));
    s.part_a = (double*)take(part);
    s.part_b = (double*)take(part);
    s.part_c = (double*)take(part);
    s.max_blocks = kMaxBlocks;
    fl::fill_zero_bytes(base, (size_t)(b - base), st);
    cap = nrhs;
  }
};

// A chunk of CG iterations captured once into a HIP graph and replayed.
// The key lists every value baked into the captured launches (buffers,
// schedule, sizes, tolerances); any change recaptures.
struct ChunkGraph {
  hipGraphExec_t exec = nullptr;
  std::vector<double> key;
  std::vector<double> seen;   // key of the last eager launch (captured on its next use)
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    key.clear();
    seen.clear();
  }
};

}  // namespace

struct fl_op_s {
  fl::Geometry g{};
  int degree = 0, device = 0;
  double alpha = 0, h = 0, c = 0;
  double* G = nullptr;
  double* lam64 = nullptr;
  float* lam32 = nullptr;
  double* linv64 = nullptr;   // preconditioner multiplier 1/lambda-hat (floored)
  float* linv32 = nullptr;
  // the tau preconditioner's multiplier for the mixed-radix sine passes (some
  // 2 N_s not a power of two; null otherwise)
  double* tinv64 = nullptr;
  float* tinv32 = nullptr;
  int precond = 2;            // 0 plain CG, 1 circulant, 2 tau preconditioner
  fl::Twiddles tw64{}, tw32{};   // per axis
  fl::Schedule sc64{}, sc32{};  // transform passes of the product A u
  fl::Schedule sp64{}, sp32{};  // transform passes of the preconditioner
  double delta = 1e-5;      // reliable-update trigger (mixed = 1)
  double inner_tol = 1e-4;  // inner solve tolerance (mixed = 2)
  int max_outer = 40;
  DBuf ws;                // FFT intermediates
  DBuf tau_ws;            // the tau preconditioner's intermediate between its split halves
  DBuf vecs;              // solver vectors
  CgState cg, cg_out;     // CG state; partial sums of residual norms
  DBuf outer_flags;       // per-RHS flags and norms of the refinement loop
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool used = false;
  // solver stream (default priority) and its input event
  hipStream_t solve_stream = nullptr;
  hipEvent_t ev_in = nullptr;
  ChunkGraph grel;        // captured reliable-update step of mixed = 1
  ChunkGraph glen[5];     // FP64 CG chunks of 1, 2, 4, 8, 16 iterations
  ChunkGraph glen32[5];   // FP32 CG chunks of 1, 2, 4, 8, 16 iterations (mixed = 1)
  DBuf ext_khat;          // transformed wrapped generator of the exterior term
  DBuf ext_work;          // exterior-term transform workspace
  bool ext_ready = false;
  DBuf ext_rhs;           // f - b for solves with exterior data
  // held by every call that uses the workspaces, CG state or settings
  // (fl_apply, fl_apply_precond, fl_exterior, fl_profile_*, fl_set_*,
  // fl_get_*schedule, fl_solve and the solves of fl_solve_async): one such
  // call at a time per handle
  std::mutex mu;
  DBuf poll_dev;          // packed CG state for the host (device side)
  double* poll_host = nullptr;   // pinned copy
  size_t poll_cap = 0;
  int iter_hint = 0;      // iterations of the last FP64 solve (first chunk length)
  double mixed_rate = 0;  // slowest r.r contraction per FP32 iteration of the last mixed solve
  int graph_mode = 1;     // 0 direct launches, 1 capture at first use, 2 at the second

  // Order this call after the previous one if it ran on another stream
  // (the workspace is shared).
  void begin(hipStream_t st) {
    if (used && st != last_stream) FL_HIP(hipStreamWaitEvent(st, done, 0));
  }
  void end(hipStream_t st) {
    FL_HIP(hipEventRecord(done, st));
    last_stream = st;
    used = true;
  }
};

namespace fl {

static size_t line_bytes(int M, int E, bool fp32) {
  return (size_t)2 * (M + M / E) * (fp32 ? 4 : 8);
}

// E_first / W_first drive the axis-0 passes (length Ma[0]), E_c2c / W_c2c
// the 3D axis-1 passes (Ma[1]), E_mid / LPB_mid the last axis (Ma[d-1]).
bool schedule_ok(const Geometry& g, const Schedule& s, bool fp32) {
  auto ok = [&](int M, int E, int W, bool tiled) {
    if (!(E == 8 || E == 16 || E == 32) || E > M) return false;
    if (W < 1 || (tiled && !pow2(W))) return false;
    if ((long)W * (M / E) > 512) return false;
    const size_t b = tiled ? tile_lds(M, E, W, fp32 ? 4 : 8).bytes : line_bytes(M, E, fp32) * W;
    if (b > kMaxLds - 1024) return false;  // room for static LDS
    return true;
  };
  return ok(g.Ma[0], s.E_first, s.W_first, true) && ok(g.Ma[g.d - 1], s.E_mid, s.LPB_mid, false) &&
         ok(g.d == 3 ? g.Ma[1] : g.Ma[0], s.E_c2c, s.W_c2c, true);
}

// Starting schedule before tuning: radix-16 register stages (radix 32 in the
// strided FP32 passes for lines of 512 and more), blocks of up to 256 threads, up to 96 KiB of
// LDS, and as many lines per block as that allows (wider column tiles in the
// strided passes).
Schedule default_schedule(const Geometry& g, bool fp32) {
  auto pickE = [&](int M, int cap) {
    const int e = fp32 && M >= 512 ? 32 : (M >= 256 ? 16 : 8);
    return std::min(std::min(e, cap), M);
  };
  auto fitW = [&](int M, int E, int want) {
    const int tpl = M / E;
    int w = std::max(1, std::min(want, 256 / std::max(1, tpl)));
    w = 1 << ilog2i(w + 1) >> 1;   // largest power of two <= w
    while (w > 1 && tile_lds(M, E, w, fp32 ? 4 : 8).bytes > 96 * 1024) w /= 2;
    return w;
  };
  const int M0 = g.Ma[0], Ml = g.Ma[g.d - 1], M1 = g.d == 3 ? g.Ma[1] : g.Ma[0];
  Schedule s{};
  s.E_first = pickE(M0, 32);
  s.E_mid = pickE(Ml, 16);
  s.E_c2c = pickE(M1, 32);
  s.W_first = fitW(M0, s.E_first, 16);
  s.W_c2c = fitW(M1, s.E_c2c, 16);
  s.LPB_mid = fitW(Ml, s.E_mid, 64);
  return s;
}

}  // namespace fl

namespace {

void set_device(fl_op A) { FL_HIP(hipSetDevice(A->device)); }

// multiplier of the preconditioners (kind 1 zero-padded, kind 2 odd-extended
// passes share it)
template <typename T>
const T* pc_symbol(fl_op A);
template <>
const double* pc_symbol<double>(fl_op A) {
  return A->precond == 2 && A->tinv64 ? A->tinv64 : A->linv64;
}
template <>
const float* pc_symbol<float>(fl_op A) {
  return A->precond == 2 && A->tinv32 ? A->tinv32 : A->linv32;
}

// schedule of the preconditioner's passes
template <typename T>
const fl::Schedule& pc_sched(fl_op A) {
  return sizeof(T) == 4 ? A->sp32 : A->sp64;
}

void check_schedule(const fl::Geometry& g, const fl::Schedule& s, bool fp32) {
  if (!fl::schedule_ok(g, s, fp32)) throw Error(FL_E_INVAL, "schedule out of range");
}

}  // namespace

extern "C" {

const char* fl_last_error(void) { return g_last_error.c_str(); }

fl_status fl_weights(int d, double alpha, int degree, double h, int kernel, double lambda,
                     void* stream, fl_op* out) {
  return fl_weights_gamma(d, alpha, degree, h, kernel, lambda, 2.0, stream, out);
}

// Operator setup shared by the cube (fl_weights_gamma) and the box
// (fl_weights_box): generator on {0..N}^d with h = 2/N, grid of Nax[s]
// intervals along axis s.
static_assert(FL_MAX_KERNEL_TERMS == fl::kMaxKernelTerms, "kernel term limit");

struct KernelTerms {
  int n;
  double coef[fl::kMaxKernelTerms], rate[fl::kMaxKernelTerms];
};

static KernelTerms single_term(int kernel, double lambda) {
  KernelTerms kt{};
  kt.n = 1;
  kt.coef[0] = 1.0;
  kt.rate[0] = kernel == FL_KERNEL_TEMPERED ? lambda : 0.0;
  return kt;
}

static fl_status create_op(int d, double alpha, int degree, int N, const int* Nax,
                           const KernelTerms& kt, double gamma, void* stream, fl_op* out) {
  if (!(gamma > alpha && gamma <= 2.0)) return fail(FL_E_INVAL, "gamma must lie in (alpha, 2]");
  if (N < 4) return fail(FL_E_INVAL, "N = 2/h must be >= 4");
  if (degree == 2 && N % 2) return fail(FL_E_INVAL, "degree 2 needs N even");
  if (N > 1024) return fail(FL_E_UNSUPPORTED, "N must be at most 1024 (embedding M <= 2048)");
  // embedding length per axis: any M >= 2 Na - 3 makes the restricted
  // circulant product exact; the transforms take powers of two (8..2048).
  // The tau preconditioner's sine transforms have length 2 Na: the
  // power-of-two passes when that is M, else mixed-radix passes
  int Ma[3] = {1, 1, 1};
  for (int s = 0; s < d; ++s) {
    if (Nax[s] < 2 || Nax[s] > N) return fail(FL_E_INVAL, "box intervals must lie in [2, N]");
    Ma[s] = 8;
    while (Ma[s] < 2 * Nax[s]) Ma[s] *= 2;
  }
  hipStream_t st = (hipStream_t)stream;
  fl_op A = new fl_op_s();
  try {
    FL_HIP(hipGetDevice(&A->device));
    A->g.d = d;
    A->g.N = N;
    A->g.nd = 1;
    for (int s = 0; s < 3; ++s) {
      const bool on = s < d;
      A->g.Na[s] = on ? Nax[s] : 2;
      A->g.na[s] = on ? Nax[s] - 1 : 1;
      A->g.Ma[s] = on ? Ma[s] : 1;
      A->g.Ha[s] = on ? Ma[s] / 2 + 1 : 1;
      A->g.La[s] = on ? 2 * Nax[s] : 1;
      A->g.nd *= A->g.na[s];
    }
    A->precond = A->g.tau_ok() ? 2 : 1;
    A->degree = degree;
    A->alpha = alpha;
    A->h = 2.0 / N;
    // c_{d,alpha} = 2^{alpha-1} alpha Gamma((d+alpha)/2) / (pi^{d/2} Gamma(1-alpha/2))
    A->c = std::pow(2.0, alpha - 1.0) * alpha * std::tgamma((d + alpha) / 2.0) /
           (std::pow(M_PI, d / 2.0) * std::tgamma(1.0 - alpha / 2.0));
    long nf = 1;
    for (int s = 0; s < d; ++s) nf *= (N + 1);
    const long nh = A->g.nh();
    A->G = (double*)dmalloc((size_t)nf * sizeof(double));
    A->lam64 = (double*)dmalloc((size_t)nh * sizeof(double));
    A->lam32 = (float*)dmalloc((size_t)nh * sizeof(float));
    A->linv64 = (double*)dmalloc((size_t)nh * sizeof(double));
    A->linv32 = (float*)dmalloc((size_t)nh * sizeof(float));
    fl::GenParams gp{};
    gp.d = d;
    gp.p = degree;
    gp.N = N;
    gp.alpha = alpha;
    gp.h = A->h;
    gp.c = A->c;
    gp.gamma = gamma;
    gp.nterm = kt.n;
    for (int i = 0; i < kt.n; ++i) {
      gp.coef[i] = kt.coef[i];
      gp.rate[i] = kt.rate[i];
    }
    fl::build_generator(gp, A->G, st);
    fl::build_symbol(A->g, A->G, A->lam64, A->lam32, st);
    {
      fl::SetupScratch scr(256, st);
      fl::build_inverse_symbol(A->g, A->lam64, nh, A->linv64, A->linv32,
                               (double*)scr.take(256), st);
      FL_HIP(hipStreamSynchronize(st));
    }
    for (int s = 0; s < 3; ++s) {
      const int M = A->g.Ma[s >= d ? 0 : s];
      A->tw64.ax[s] = fl::twiddles(M, false, st);
      A->tw32.ax[s] = fl::twiddles(M, true, st);
      A->tw64.sx[s] = A->tw64.ax[s];
      A->tw32.sx[s] = A->tw32.ax[s];
    }
    if (!A->g.sine_ok() && A->g.sine_any_ok()) {
      // the tau preconditioner on mixed-radix sine passes of length 2 N_s
      const long nt = fl::tau_any_entries(A->g);
      A->tinv64 = (double*)dmalloc((size_t)nt * sizeof(double));
      A->tinv32 = (float*)dmalloc((size_t)nt * sizeof(float));
      fl::build_tau_multiplier(A->g, A->G, A->tinv64, A->tinv32, st);
      for (int s = 0; s < d; ++s) {
        A->tw64.sx[s] = fl::twiddles(A->g.La[s], false, st);
        A->tw32.sx[s] = fl::twiddles(A->g.La[s], true, st);
      }
    }
    A->sc64 = fl::default_schedule(A->g, false);
    A->sc32 = fl::default_schedule(A->g, true);
    A->sp64 = A->sc64;
    A->sp32 = A->sc32;
    FL_HIP(hipEventCreateWithFlags(&A->done, hipEventDisableTiming));
    FL_HIP(hipStreamSynchronize(st));
  } catch (...) {
    fl_destroy(A);
    throw;
  }
  *out = A;
  return FL_OK;
}

static fl_status check_common(int d, double alpha, int degree, int kernel, double lambda,
                              fl_op* out) {
  if (!out) return fail(FL_E_INVAL, "out is NULL");
  if (d < 1 || d > 3) return fail(FL_E_INVAL, "d must be 1, 2 or 3");
  if (!(alpha > 0.0 && alpha < 2.0)) return fail(FL_E_INVAL, "alpha must lie in (0, 2)");
  if (degree < 0 || degree > 2) return fail(FL_E_INVAL, "degree must be 0, 1 or 2");
  if (kernel != FL_KERNEL_FRACTIONAL && kernel != FL_KERNEL_TEMPERED)
    return fail(FL_E_INVAL, "unknown kernel");
  if (kernel == FL_KERNEL_TEMPERED && (!(lambda >= 0.0) || !std::isfinite(lambda)))
    return fail(FL_E_INVAL, "lambda must be finite and >= 0");
  return FL_OK;
}

fl_status fl_weights_gamma(int d, double alpha, int degree, double h, int kernel, double lambda,
                           double gamma, void* stream, fl_op* out) {
  return guarded([&]() -> fl_status {
    const fl_status e = check_common(d, alpha, degree, kernel, lambda, out);
    if (e != FL_OK) return e;
    if (!(h > 0.0) || !std::isfinite(h)) return fail(FL_E_INVAL, "h must be positive");
    const double Nf = 2.0 / h;
    const double Nr = std::round(Nf);
    if (!(Nr >= 1.0) || std::fabs(Nf - Nr) > 1e-12 * Nr)
      return fail(FL_E_INVAL, "2/h must be an integer");
    if (Nr > 1e6) return fail(FL_E_UNSUPPORTED, "N too large");
    const int N = (int)Nr;
    const int Nax[3] = {N, N, N};
    return create_op(d, alpha, degree, N, Nax, single_term(kernel, lambda), gamma, stream, out);
  });
}

fl_status fl_weights_box(int d, double alpha, int degree, const int* intervals, int kernel,
                         double lambda, double gamma, void* stream, fl_op* out) {
  return guarded([&]() -> fl_status {
    const fl_status e = check_common(d, alpha, degree, kernel, lambda, out);
    if (e != FL_OK) return e;
    if (!intervals) return fail(FL_E_INVAL, "intervals is NULL");
    int N = 0;
    for (int s = 0; s < d; ++s) N = std::max(N, intervals[s]);
    return create_op(d, alpha, degree, N, intervals, single_term(kernel, lambda), gamma, stream,
                     out);
  });
}

fl_status fl_weights_expsum(int d, double alpha, int degree, const int* intervals, int nterm,
                            const double* coef, const double* rate, double gamma, void* stream,
                            fl_op* out) {
  return guarded([&]() -> fl_status {
    const fl_status e = check_common(d, alpha, degree, FL_KERNEL_FRACTIONAL, 0.0, out);
    if (e != FL_OK) return e;
    if (!intervals || !coef || !rate) return fail(FL_E_INVAL, "intervals, coef or rate is NULL");
    if (nterm < 1 || nterm > FL_MAX_KERNEL_TERMS)
      return fail(FL_E_INVAL, "nterm must lie in [1, FL_MAX_KERNEL_TERMS]");
    KernelTerms kt{};
    kt.n = nterm;
    double total = 0.0;
    for (int i = 0; i < nterm; ++i) {
      if (!(coef[i] >= 0.0) || !std::isfinite(coef[i]))
        return fail(FL_E_INVAL, "kernel coefficients must be finite and >= 0");
      if (!(rate[i] >= 0.0) || !std::isfinite(rate[i]))
        return fail(FL_E_INVAL, "kernel rates must be finite and >= 0");
      kt.coef[i] = coef[i];
      kt.rate[i] = rate[i];
      total += coef[i];
    }
    if (!(total > 0.0)) return fail(FL_E_INVAL, "kernel coefficients are all zero");
    int N = 0;
    for (int s = 0; s < d; ++s) N = std::max(N, intervals[s]);
    return create_op(d, alpha, degree, N, intervals, kt, gamma, stream, out);
  });
}

fl_status fl_set_allocator(fl_alloc_fn alloc, fl_release_fn release, void* ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(FL_E_INVAL, "give both alloc and release, or neither");
  std::lock_guard<std::mutex> lk(fl::g_alloc_mu);
  fl::g_alloc.alloc = alloc;
  fl::g_alloc.release = release;
  fl::g_alloc.ctx = ctx;
  return FL_OK;
}

void fl_destroy(fl_op A) {
  if (!A) return;
  (void)hipSetDevice(A->device);
  // wait for this handle's own work only (other streams keep running)
  if (A->solve_stream) (void)hipStreamSynchronize(A->solve_stream);
  if (A->used && A->done) (void)hipEventSynchronize(A->done);
  fl::dev_free(A->G);
  fl::dev_free(A->lam64);
  fl::dev_free(A->lam32);
  fl::dev_free(A->linv64);
  fl::dev_free(A->linv32);
  fl::dev_free(A->tinv64);
  fl::dev_free(A->tinv32);
  A->ws.release();
  A->tau_ws.release();
  A->vecs.release();
  A->cg.mem.release();
  A->cg_out.mem.release();
  A->outer_flags.release();
  if (A->done) (void)hipEventDestroy(A->done);
  A->grel.reset();
  for (auto& gph : A->glen) gph.reset();
  for (auto& gph : A->glen32) gph.reset();
  A->poll_dev.release();
  A->ext_khat.release();
  A->ext_work.release();
  A->ext_rhs.release();
  if (A->poll_host) (void)hipHostFree(A->poll_host);
  if (A->ev_in) (void)hipEventDestroy(A->ev_in);
  if (A->solve_stream) (void)hipStreamDestroy(A->solve_stream);
  delete A;
}

fl_status fl_query(fl_op A, int* d, int* N, int* n, int* M) {
  if (!A) return fail(FL_E_INVAL, "null handle");
  if (d) *d = A->g.d;
  if (N) *N = A->g.N;
  if (n) *n = A->g.na[0];
  if (M) *M = A->g.Ma[0];
  return FL_OK;
}

fl_status fl_query_axes(fl_op A, int* intervals, int* n, int* M) {
  if (!A) return fail(FL_E_INVAL, "null handle");
  for (int s = 0; s < A->g.d; ++s) {
    if (intervals) intervals[s] = A->g.Na[s];
    if (n) n[s] = A->g.na[s];
    if (M) M[s] = A->g.Ma[s];
  }
  return FL_OK;
}

static fl_status copy_out(fl_op A, const void* src, void* host, size_t count, size_t need,
                          size_t esz) {
  if (!A || !host) return fail(FL_E_INVAL, "null argument");
  if (count < need) return fail(FL_E_INVAL, "output buffer too small");
  set_device(A);
  FL_HIP(hipDeviceSynchronize());
  FL_HIP(hipMemcpy(host, src, need * esz, hipMemcpyDeviceToHost));
  return FL_OK;
}

fl_status fl_generator(fl_op A, double* host_out, size_t count) {
  return guarded([&]() -> fl_status {
    if (!A) return fail(FL_E_INVAL, "null handle");
    size_t nf = 1;
    for (int s = 0; s < A->g.d; ++s) nf *= (size_t)(A->g.N + 1);
    return copy_out(A, A->G, host_out, count, nf, sizeof(double));
  });
}

fl_status fl_symbol(fl_op A, double* host_out, size_t count) {
  return guarded([&]() -> fl_status {
    if (!A) return fail(FL_E_INVAL, "null handle");
    const size_t nf = (size_t)A->g.nh();
    return copy_out(A, A->lam64, host_out, count, nf, sizeof(double));
  });
}

fl_status fl_embedding(fl_op A, double* host_out, size_t count) {
  return guarded([&]() -> fl_status {
    if (!A || !host_out) return fail(FL_E_INVAL, "null argument");
    const size_t nm = (size_t)A->g.nm();
    if (count < nm) return fail(FL_E_INVAL, "output buffer too small");
    set_device(A);
    double* tmp = (double*)dmalloc(nm * sizeof(double));
    fl::embed_generator(A->g, A->G, tmp, nullptr);
    hipError_t e = hipMemcpy(host_out, tmp, nm * sizeof(double), hipMemcpyDeviceToHost);
    fl::dev_free(tmp);
    if (e != hipSuccess) return fail(FL_E_DEVICE, hipGetErrorString(e));
    return FL_OK;
  });
}

static fl_status set_sched(fl_op A, bool pc, int fp32, int e_first, int e_mid, int e_c2c,
                           int w_first, int w_c2c, int lpb_mid) {
  return guarded([&]() -> fl_status {
    if (!A) return fail(FL_E_INVAL, "null handle");
    std::lock_guard<std::mutex> lock(A->mu);
    fl::Schedule& dst = pc ? (fp32 ? A->sp32 : A->sp64) : (fp32 ? A->sc32 : A->sc64);
    fl::Schedule s = dst;
    if (e_first > 0) s.E_first = e_first;
    if (e_mid > 0) s.E_mid = e_mid;
    if (e_c2c > 0) s.E_c2c = e_c2c;
    if (w_first > 0) s.W_first = w_first;
    if (w_c2c > 0) s.W_c2c = w_c2c;
    if (lpb_mid > 0) s.LPB_mid = lpb_mid;
    check_schedule(A->g, s, fp32 != 0);
    dst = s;
    return FL_OK;
  });
}

fl_status fl_set_schedule(fl_op A, int fp32, int e_first, int e_mid, int e_c2c, int w_first,
                          int w_c2c, int lpb_mid) {
  return set_sched(A, false, fp32, e_first, e_mid, e_c2c, w_first, w_c2c, lpb_mid);
}

fl_status fl_set_precond_schedule(fl_op A, int fp32, int e_first, int e_mid, int e_c2c,
                                  int w_first, int w_c2c, int lpb_mid) {
  return set_sched(A, true, fp32, e_first, e_mid, e_c2c, w_first, w_c2c, lpb_mid);
}

fl_status fl_set_preconditioner(fl_op A, int kind) {
  if (!A) return fail(FL_E_INVAL, "null handle");
  if (kind < 0 || kind > 2) return fail(FL_E_INVAL, "kind must be 0, 1 or 2");
  if (kind == 2 && !A->g.tau_ok())
    return fail(FL_E_UNSUPPORTED,
                "the tau preconditioner needs every 2 N_s to be a power of two or to have no "
                "prime factor above 7");
  std::lock_guard<std::mutex> lock(A->mu);
  A->precond = kind;
  return FL_OK;
}

fl_status fl_get_preconditioner(fl_op A, int* kind) {
  if (!A || !kind) return fail(FL_E_INVAL, "null argument");
  std::lock_guard<std::mutex> lock(A->mu);
  *kind = A->precond;
  return FL_OK;
}

fl_status fl_apply_precond(fl_op A, const void* u, void* y, int nrhs, int fp32, void* stream) {
  return guarded([&]() -> fl_status {
    if (!A) return fail(FL_E_INVAL, "null handle");
    if (!u || !y) return fail(FL_E_INVAL, "null vector");
    if (u == y) return fail(FL_E_INVAL, "u and y must be distinct");
    if (nrhs < 1) return fail(FL_E_INVAL, "nrhs must be >= 1");
    std::lock_guard<std::mutex> lock(A->mu);
    if (A->precond == 0) return fail(FL_E_INVAL, "no preconditioner selected");
    set_device(A);
    hipStream_t st = (hipStream_t)stream;
    A->begin(st);
    void* ws = A->ws.get(fl::apply_workspace_bytes(A->g, nrhs, fp32 != 0));
    const bool odd = A->precond == 2;
    if (fp32)
      fl::apply_passes<float>(A->g, A->sp32, pc_symbol<float>(A), A->tw32, (const float*)u,
                              (float*)y, nrhs, ws, st, fl::PM_PLAIN, nullptr, nullptr, nullptr,
                              nullptr, nullptr, nullptr, -1, odd);
    else
      fl::apply_passes<double>(A->g, A->sp64, pc_symbol<double>(A), A->tw64, (const double*)u,
                               (double*)y, nrhs, ws, st, fl::PM_PLAIN, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, -1, odd);
    A->end(st);
    return FL_OK;
  });
}

fl_status fl_set_graphs(fl_op A, int enable) {
  if (!A) return fail(FL_E_INVAL, "null handle");
  std::lock_guard<std::mutex> lock(A->mu);
  if (enable < 0 || enable > 2) return fail(FL_E_INVAL, "enable must be 0, 1 or 2");
  A->graph_mode = enable;
  return FL_OK;
}

static fl_status get_sched(fl_op A, bool pc, int fp32, int* s6) {
  if (!A || !s6) return fail(FL_E_INVAL, "null argument");
  std::lock_guard<std::mutex> lock(A->mu);
  const fl::Schedule& s = pc ? (fp32 ? A->sp32 : A->sp64) : (fp32 ? A->sc32 : A->sc64);
  s6[0] = s.E_first;
  s6[1] = s.E_mid;
  s6[2] = s.E_c2c;
  s6[3] = s.W_first;
  s6[4] = s.W_c2c;
  s6[5] = s.LPB_mid;
  return FL_OK;
}

fl_status fl_get_schedule(fl_op A, int fp32, int* s6) { return get_sched(A, false, fp32, s6); }

fl_status fl_get_precond_schedule(fl_op A, int fp32, int* s6) {
  return get_sched(A, true, fp32, s6);
}

fl_status fl_set_refinement(fl_op A, double delta, double inner_tol, int max_outer) {
  if (!A) return fail(FL_E_INVAL, "null handle");
  if (!(delta > 0.0 && delta < 1.0) || !(inner_tol > 0.0 && inner_tol < 1.0) || max_outer < 1)
    return fail(FL_E_INVAL, "delta and inner_tol in (0,1) and max_outer >= 1 required");
  std::lock_guard<std::mutex> lock(A->mu);
  A->delta = delta;
  A->inner_tol = inner_tol;
  A->max_outer = max_outer;
  return FL_OK;
}

fl_status fl_apply(fl_op A, const void* u, void* y, int nrhs, int fp32, void* stream) {
  return guarded([&]() -> fl_status {
    if (!A) return fail(FL_E_INVAL, "null handle");
    if (!u || !y) return fail(FL_E_INVAL, "null vector");
    if (u == y) return fail(FL_E_INVAL, "u and y must be distinct");
    if (nrhs < 1) return fail(FL_E_INVAL, "nrhs must be >= 1");
    std::lock_guard<std::mutex> lock(A->mu);
    set_device(A);
    hipStream_t st = (hipStream_t)stream;
    A->begin(st);
    void* ws = A->ws.get(fl::apply_workspace_bytes(A->g, nrhs, fp32 != 0));
    if (fp32)
      fl::apply_passes<float>(A->g, A->sc32, A->lam32, A->tw32, (const float*)u, (float*)y, nrhs,
                              ws, st, fl::PM_PLAIN, nullptr, nullptr, nullptr, nullptr, nullptr);
    else
      fl::apply_passes<double>(A->g, A->sc64, A->lam64, A->tw64, (const double*)u, (double*)y,
                               nrhs, ws, st, fl::PM_PLAIN, nullptr, nullptr, nullptr, nullptr,
                               nullptr);
    A->end(st);
    return FL_OK;
  });
}

}  // extern "C"

int fl::apply_in_area(fl_op A, const void* u, void* y, int nrhs, int fp32, void* stream,
                      void* (*area_of_device)(int dev), size_t area_bytes) {
  return guarded([&]() -> fl_status {
    if (!A) return fail(FL_E_INVAL, "null handle");
    if (!u || !y) return fail(FL_E_INVAL, "null vector");
    if (u == y) return fail(FL_E_INVAL, "u and y must be distinct");
    if (nrhs < 1) return fail(FL_E_INVAL, "nrhs must be >= 1");
    // the same checks, schedule and passes as fl_apply; the handle's
    // buffers are not touched (only its generator-derived data is read), so
    // no ordering against the handle's earlier calls is needed
    std::lock_guard<std::mutex> lock(A->mu);
    const size_t need = fl::apply_workspace_bytes(A->g, nrhs, fp32 != 0);
    if (need > area_bytes)
      return fail(FL_E_UNSUPPORTED,
                  "fl_apply_noalloc: the product needs " + std::to_string(need) +
                      " bytes of intermediates, the fixed scratch area holds " +
                      std::to_string(area_bytes) + "; use fl_apply or fewer right-hand sides");
    set_device(A);
    void* ws = need ? area_of_device(A->device) : nullptr;
    hipStream_t st = (hipStream_t)stream;
    if (fp32)
      fl::apply_passes<float>(A->g, A->sc32, A->lam32, A->tw32, (const float*)u, (float*)y, nrhs,
                              ws, st, fl::PM_PLAIN, nullptr, nullptr, nullptr, nullptr, nullptr);
    else
      fl::apply_passes<double>(A->g, A->sc64, A->lam64, A->tw64, (const double*)u, (double*)y,
                               nrhs, ws, st, fl::PM_PLAIN, nullptr, nullptr, nullptr, nullptr,
                               nullptr);
    return FL_OK;
  });
}

extern "C" {

// Shared body of fl_profile_apply (pc false: y = A u) and fl_profile_precond
// (pc true: y = P u).
static fl_status profile_passes(fl_op A, const void* u, void* y, int nrhs, int fp32, int reps,
                                void* stream, double* ms_per_pass, int max_passes,
                                int* n_passes, bool pc) {
  return guarded([&]() -> fl_status {
    if (!A) return fail(FL_E_INVAL, "null handle");
    if (!u || !y || !ms_per_pass || !n_passes) return fail(FL_E_INVAL, "null argument");
    if (u == y) return fail(FL_E_INVAL, "u and y must be distinct");
    if (nrhs < 1 || reps < 1) return fail(FL_E_INVAL, "nrhs and reps must be >= 1");
    std::lock_guard<std::mutex> lock(A->mu);
    if (pc && A->precond == 0) return fail(FL_E_INVAL, "no preconditioner selected");
    const int np = fl::apply_npasses(A->g.d);
    if (max_passes < np) return fail(FL_E_INVAL, "max_passes too small");
    set_device(A);
    hipStream_t st = (hipStream_t)stream;
    A->begin(st);
    void* ws = A->ws.get(fl::apply_workspace_bytes(A->g, nrhs, fp32 != 0));
    const bool odd = pc && A->precond == 2;
    auto run = [&](int only) {
      if (fp32)
        fl::apply_passes<float>(A->g, pc ? A->sp32 : A->sc32, pc ? pc_symbol<float>(A) : A->lam32, A->tw32,
                                (const float*)u, (float*)y, nrhs, ws, st, fl::PM_PLAIN, nullptr,
                                nullptr, nullptr, nullptr, nullptr, nullptr, only, odd);
      else
        fl::apply_passes<double>(A->g, pc ? A->sp64 : A->sc64, pc ? pc_symbol<double>(A) : A->lam64, A->tw64,
                                 (const double*)u, (double*)y, nrhs, ws, st, fl::PM_PLAIN,
                                 nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, only, odd);
    };
    // one whole application puts every pass's input in place; then each pass
    // runs reps times back to back between two events; a last whole
    // application leaves the result in y
    hipEvent_t ev[2];
    FL_HIP(hipEventCreate(&ev[0]));
    FL_HIP(hipEventCreate(&ev[1]));
    run(-1);
    for (int k = 0; k < np; ++k) {
      FL_HIP(hipEventRecord(ev[0], st));
      for (int r = 0; r < reps; ++r) run(k);
      FL_HIP(hipEventRecord(ev[1], st));
      FL_HIP(hipEventSynchronize(ev[1]));
      float ms = 0.f;
      FL_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
      ms_per_pass[k] = (double)ms / reps;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (max_passes >= 2 * np) {
      // each launch between an event pair of its own (the duration of one
      // dispatch, as a kernel trace reports it), averaged over reps
      std::vector<hipEvent_t> evs(2 * (size_t)reps, nullptr);
      try {
        for (auto& e : evs) FL_HIP(hipEventCreate(&e));
        for (int k = 0; k < np; ++k) {
          for (int r = 0; r < reps; ++r) {
            FL_HIP(hipEventRecord(evs[2 * r], st));
            run(k);
            FL_HIP(hipEventRecord(evs[2 * r + 1], st));
          }
          FL_HIP(hipEventSynchronize(evs[2 * reps - 1]));
          double tot = 0.0;
          for (int r = 0; r < reps; ++r) {
            float ms = 0.f;
            FL_HIP(hipEventElapsedTime(&ms, evs[2 * r], evs[2 * r + 1]));
            tot += ms;
          }
          ms_per_pass[np + k] = tot / reps;
        }
      } catch (...) {
        for (auto& e : evs)
          if (e) (void)hipEventDestroy(e);
        throw;
      }
      for (auto& e : evs) (void)hipEventDestroy(e);
    }
    run(-1);
    FL_HIP(hipStreamSynchronize(st));
    *n_passes = np;
    A->end(st);
    return FL_OK;
  });
}

fl_status fl_profile_apply(fl_op A, const void* u, void* y, int nrhs, int fp32, int reps,
                           void* stream, double* ms_per_pass, int max_passes, int* n_passes) {
  return profile_passes(A, u, y, nrhs, fp32, reps, stream, ms_per_pass, max_passes, n_passes,
                        false);
}

fl_status fl_profile_precond(fl_op A, const void* u, void* y, int nrhs, int fp32, int reps,
                             void* stream, double* ms_per_pass, int max_passes, int* n_passes) {
  return profile_passes(A, u, y, nrhs, fp32, reps, stream, ms_per_pass, max_passes, n_passes,
                        true);
}

}  // extern "C"

namespace {

// Per-call view of the CG state: block counts, iteration cap, tolerance.
fl::CgScalars cg_view(const fl::CgScalars& base, const fl::Geometry& g, const fl::Schedule& sc,
                      const fl::Schedule& scp, int nrhs, int maxiter, double tol, int precond) {
  fl::CgScalars c = base;
  c.nb_a = fl::last_pass_blocks(g, sc);
  c.nb_c = fl::vec_blocks(g.nd, nrhs);
  // r.z from the preconditioner (its own schedule): the tau middle pass or
  // the last pass
  c.nb_b = precond == 2   ? fl::tau_dot_blocks(g, scp, c.max_blocks)
           : precond == 1 ? fl::last_pass_blocks(g, scp)
                          : c.nb_c;
  if (c.nb_a > c.max_blocks || c.nb_b > c.max_blocks || c.nb_c > c.max_blocks)
    throw Error(FL_E_UNSUPPORTED, "too many blocks for the reduction buffers");
  c.maxiter = maxiter;
  c.precond = precond;
  c.rel_last = nullptr;
  c.rel_f2 = nullptr;
  c.rel_trig = nullptr;
  c.rel_delta2 = c.rel_tol2 = 0.0;
  c.tol2 = tol * tol;
  return c;
}

void ensure_solver_stream(fl_op A) {
  if (A->solve_stream) return;
  FL_HIP(hipStreamCreateWithFlags(&A->solve_stream, hipStreamNonBlocking));
  FL_HIP(hipEventCreateWithFlags(&A->ev_in, hipEventDisableTiming));
}

// Replay the captured chunk if `key` matches; otherwise run `enqueue` once
// directly and capture it into a new graph for the next calls (mode 1), or
// (mode 2) capture it only when the same sequence comes a second time, so
// that an operator solved once, as most are in a serving stream, never pays
// for capture and instantiation.  Mode 0: direct launches only.
template <typename F>
void launch_chunk(ChunkGraph& g, const std::vector<double>& key, hipStream_t st, int mode,
                  F&& enqueue) {
  if (mode == 0) {
    enqueue();
    return;
  }
  if (g.exec && g.key == key) {
    FL_HIP(hipGraphLaunch(g.exec, st));
    return;
  }
  if (mode == 2 && g.seen != key) {
    g.seen = key;
    enqueue();
    return;
  }
  g.reset();
  enqueue();
  hipGraph_t graph = nullptr;
  FL_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    enqueue();
  } catch (...) {
    (void)hipStreamEndCapture(st, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  FL_HIP(hipStreamEndCapture(st, &graph));
  const hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g.exec = nullptr;
    throw Error(FL_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  g.key = key;
}

// Device and pinned host buffers of the poll record (fl::pack_poll).
double* poll_buffers(fl_op A, int nrhs, double** dev, size_t* bytes) {
  const size_t pb = (1 + fl::POLL_STRIDE * (size_t)nrhs) * sizeof(double);
  *dev = (double*)A->poll_dev.get(pb);
  if (A->poll_cap < pb) {
    if (A->poll_host) FL_HIP(hipHostFree(A->poll_host));
    A->poll_host = nullptr;
    A->poll_cap = 0;
    FL_HIP(hipHostMalloc((void**)&A->poll_host, pb, hipHostMallocDefault));
    A->poll_cap = pb;
  }
  *bytes = pb;
  return A->poll_host;
}

// n CG iterations as captured graphs of 16, 8, 4, 2 and 1 iterations.
template <typename F>
void launch_iterations(fl_op A, ChunkGraph* gl, const std::vector<double>& key, int n,
                       hipStream_t st, F&& enqueue_one) {
  static const int lens[5] = {1, 2, 4, 8, 16};
  for (int b = 4; b >= 0; --b) {
    while (n >= lens[b]) {
      std::vector<double> kb = key;
      kb.push_back(lens[b]);
      launch_chunk(gl[b], kb, st, A->graph_mode, [&]() {
        for (int i = 0; i < lens[b]; ++i) enqueue_one();
      });
      n -= lens[b];
    }
  }
}

// Iterations for r.r to fall from rr to target at `rate` per iteration
// (8 if the rate is unknown or too slow to extrapolate).
inline int iterations_to(double rr, double target, double rate) {
  if (!(rr > target)) return 0;
  if (!(rate > 0.0 && rate < 0.95) || !(target > 0.0)) return 8;
  return (int)std::ceil(std::log(target / rr) / std::log(rate));
}

// Run CG iterations in chunks whose length is predicted from each active
// right-hand side's observed contraction of r.r (iterations to reach its
// threshold at the rate seen so far, from r_0 on, at most 16); the host
// reads the state after every chunk, so no work is queued past convergence
// beyond a misprediction.  The first chunk is the previous solve's
// iteration count plus the one that detects convergence (8 on the first
// solve).  Chunks are composed of captured graphs of 16, 8, 4, 2 and 1
// iterations; iterations of stopped right-hand sides are masked no-ops.
// detect: iterations after the last useful one needed to detect
// convergence (1 when the stopping test runs at the iteration start, 0 with
// the split tau preconditioner, which tests at the end of the iteration).
template <typename F>
void predictive_loop(fl_op A, const std::vector<double>& key, int cap, const fl::CgScalars& cg,
                     int nrhs, hipStream_t st, int detect, F&& enqueue_one) {
  double* dpoll = nullptr;
  size_t pb = 0;
  const double* h = poll_buffers(A, nrhs, &dpoll, &pb);
  std::vector<double> rr_prev(nrhs, 0.0);
  std::vector<int> it_prev(nrhs, 0);
  int done = 0, next = A->iter_hint > 0 ? std::min(A->iter_hint + detect, 16) : 8;
  int max_it = 0;
  while (done < cap) {
    const int k = std::min(next, cap - done);
    launch_iterations(A, A->glen, key, k, st, enqueue_one);
    done += k;
    fl::pack_poll(cg, nrhs, nullptr, nullptr, nullptr, dpoll, st);
    FL_HIP(hipMemcpyAsync(A->poll_host, dpoll, pb, hipMemcpyDeviceToHost, st));
    FL_HIP(hipStreamSynchronize(st));
    for (int o = 0; o < nrhs; ++o) max_it = std::max(max_it, (int)h[1 + fl::POLL_STRIDE * o + 3]);
    if (h[0] == 0.0) break;
    int need = 1;
    for (int o = 0; o < nrhs; ++o) {
      const double* q = h + 1 + fl::POLL_STRIDE * o;
      if (q[2] == 0.0) continue;
      // r.r after the last update (what the next iteration start tests)
      const double rr = q[4], th = q[1];
      const int it = (int)q[3];
      // before the first poll the reference is r_0: ||r_0||^2 = thresh2 / tol^2
      if (rr_prev[o] == 0.0 && cg.tol2 > 0.0) rr_prev[o] = th / cg.tol2;
      double rate = 0.0;
      if (rr_prev[o] > 0.0 && it > it_prev[o] && rr > 0.0)
        rate = std::pow(rr / rr_prev[o], 1.0 / (it - it_prev[o]));
      // plus the iteration whose start detects convergence (detect = 1)
      need = std::max(need, iterations_to(rr, th, rate) + detect);
      rr_prev[o] = rr;
      it_prev[o] = it;
    }
    next = std::min(std::max(need, 1), 16);
  }
  FL_HIP(hipStreamSynchronize(st));
  A->iter_hint = max_it;
}

// Mixed precision (FP32 CG with FP64 reliable updates) in predicted chunks:
// FP32 iterations as captured graphs, then the reliable step (fold the FP32
// correction and replace the residual by the FP64 one for the right-hand
// sides whose recursion stopped at its trigger, stop those that meet the
// tolerance, resume the others), then a poll.  The trigger is tested at
// every iteration start on the device, so chunk lengths change only when
// the reliable step runs, never the arithmetic.  The next chunk lasts until
// the slowest active right-hand side reaches its next trigger,
// max(delta^2 rr_last, tol^2 ||f||^2), at the contraction of its FP32 r.r
// observed between replacements.  The first chunk uses the previous mixed
// solve's rate.
template <typename F, typename G>
void predictive_mixed_loop(fl_op A, const std::vector<double>& key, int maxiter,
                           const fl::CgScalars& cg, int nrhs, const double* rr_last,
                           const double* f2, const int* nupd, double delta2, double tol2,
                           hipStream_t st, int detect, F&& enqueue_one, G&& enqueue_reliable) {
  double* dpoll = nullptr;
  size_t pb = 0;
  const double* h = poll_buffers(A, nrhs, &dpoll, &pb);
  std::vector<double> rr_ref(nrhs, 0.0), rate(nrhs, 0.0);
  std::vector<int> it_ref(nrhs, 0), nu_ref(nrhs, 0);
  int next = 8;
  if (A->mixed_rate > 0.0 && A->mixed_rate < 0.95)
    next = std::min(std::max(iterations_to(1.0, std::max(delta2, tol2), A->mixed_rate) + detect, 1),
                    16);
  std::vector<double> krel = key;
  krel.push_back(-1.0);
  double slowest = 0.0;
  // maxiter is enforced per RHS on the device; a right-hand side waiting for
  // its reliable update skips the rest of the chunk, so launched iterations
  // overcount.  Every chunk advances each active RHS by an iteration or a
  // replacement, which bounds the number of chunks.
  const int max_chunks = 2 * (maxiter + 2) + 8;
  for (int c = 0; c < max_chunks; ++c) {
    launch_iterations(A, A->glen32, key, next, st, enqueue_one);
    launch_chunk(A->grel, krel, st, A->graph_mode, enqueue_reliable);
    fl::pack_poll(cg, nrhs, rr_last, f2, nupd, dpoll, st);
    FL_HIP(hipMemcpyAsync(A->poll_host, dpoll, pb, hipMemcpyDeviceToHost, st));
    FL_HIP(hipStreamSynchronize(st));
    if (h[0] == 0.0) break;
    int need = 1;
    for (int o = 0; o < nrhs; ++o) {
      const double* q = h + 1 + fl::POLL_STRIDE * o;
      if (q[2] == 0.0) continue;
      const double res2 = q[0], rr = q[4], rl = q[5], ff = q[6];
      const int it = (int)q[3], nu = (int)q[7];
      if (rr_ref[o] == 0.0) rr_ref[o] = ff;   // x_0 = 0: r_0 = f
      // contraction of the FP32 recursion since the reference: from r.r now
      // if no replacement happened, else from r.r at the start of the last
      // iteration (before the replacement)
      double cur = rr;
      int itc = it;
      if (nu != nu_ref[o]) {
        cur = res2;
        itc = it - 1;
      }
      if (itc > it_ref[o] && cur > 0.0 && rr_ref[o] > 0.0) {
        const double r = std::pow(cur / rr_ref[o], 1.0 / (itc - it_ref[o]));
        if (r < 1.0) rate[o] = r;
      }
      slowest = std::max(slowest, rate[o]);
      const double target = std::max(delta2 * rl, tol2 * ff);
      // plus the iteration whose start detects the trigger (detect = 1)
      need = std::max(need, iterations_to(rr, target, rate[o]) + detect);
      rr_ref[o] = rr;
      it_ref[o] = it;
      nu_ref[o] = nu;
    }
    next = std::min(std::max(need, 1), 16);
  }
  FL_HIP(hipStreamSynchronize(st));
  if (slowest > 0.0) A->mixed_rate = slowest;
}

template <typename... P>
std::vector<double> make_key(P... v) {
  return {static_cast<double>(v)...};
}

inline double pkey(const void* p) { return (double)(uintptr_t)p; }

inline std::vector<double> sched_key(const fl::Schedule& s) {
  return {(double)s.E_first, (double)s.E_mid, (double)s.E_c2c, (double)s.W_first,
          (double)s.W_c2c, (double)s.LPB_mid};
}

// z = P r and partials of r.z: P the restricted inverse of the embedding
// circulant (kind 1, zero-padded passes) or the inverse of the tau
// approximation (kind 2, odd-extended passes); `linv` is its multiplier.
template <typename T>
void precond_apply(fl_op A, const T* linv, const fl::Twiddles& tw, const T* r, T* z, int nrhs, void* ws,
                   const fl::CgScalars& cg, const int* active, hipStream_t st) {
  fl::apply_passes<T>(A->g, pc_sched<T>(A), linv, tw, r, z, nrhs, ws, st, fl::PM_DOT, nullptr,
                      nullptr, nullptr, &cg, active, nullptr, -1, A->precond == 2);
}

// Whether preconditioned CG runs the tau preconditioner split around the
// iteration start (fl::tau_front / fl::tau_back_direction: z = P r is never
// stored and the direction kernel is not launched): the tau preconditioner
// on the power-of-two sine passes with d >= 2 and the middle pass's r.z
// partials within the buffers.
bool tau_split(fl_op A, const fl::Schedule& scp) {
  return A->precond == 2 && A->g.d >= 2 && A->g.sine_ok() &&
         fl::sine_mid_blocks(A->g, scp) <= kMaxBlocks;
}

// CG start: x = 0, r = rhs, p = 0; preconditioned: z = P r (with the split
// tau preconditioner, S1 != null: its first half, into S1).
template <typename T>
void cg_start(fl_op A, const fl::Schedule& sc, const T* linv, const fl::Twiddles& tw, const T* rhs,
              T* x, T* r, T* p, T* z, int nrhs, const fl::CgScalars& cg,
              const int* outer_active, void* ws, hipStream_t st, T* S1) {
  fl::fill_int(cg.n_active, 0, 1, st);
  fl::cg_init<T>(A->g, rhs, x, r, p, nrhs, cg, outer_active, st);
  if (S1)
    fl::tau_front<T>(A->g, pc_sched<T>(A), linv, tw, r, S1, nrhs, st, cg, cg.active, true);
  else if (cg.precond)
    precond_apply<T>(A, linv, tw, r, z, nrhs, ws, cg, cg.active, st);
}

// One CG (or preconditioned CG) iteration for all active right-hand sides.
// With the split tau preconditioner (S1 != null) the iteration is: second
// half of z = P r fused with the iteration start (p = z + beta p) and the
// product's first pass, the product's other passes, the update, first half
// of the next z = P r.
template <typename T>
void cg_iteration(fl_op A, const fl::Schedule& sc, const T* lam, const T* linv, const fl::Twiddles& tw,
                  T* x, T* r, T* p, T* q, T* z, int nrhs, const fl::CgScalars& cg, void* ws,
                  hipStream_t st, T* S1) {
  if (S1) {
    // z's last pass, p = z + beta p and the product's first pass in one kernel
    fl::tau_back_direction<T>(A->g, sc, pc_sched<T>(A), tw, S1, p, ws, nrhs, st, cg);
    fl::apply_passes<T>(A->g, sc, lam, tw, p, q, nrhs, ws, st, fl::PM_PQ, nullptr, nullptr,
                        nullptr, &cg, cg.active, nullptr, -1, false, true);
    fl::cg_update<T>(A->g, x, r, p, q, nrhs, cg, st);
    fl::tau_front<T>(A->g, pc_sched<T>(A), linv, tw, r, S1, nrhs, st, cg, cg.active, true);
    return;
  }
  if (A->g.d >= 2) {
    // iteration start and p = z + beta p streamed; the strided first pass
    // then reads p alone
    fl::cg_direction<T>(A->g, p, cg.precond ? z : r, nrhs, cg, st);
    fl::apply_passes<T>(A->g, sc, lam, tw, p, q, nrhs, ws, st, fl::PM_PQ, nullptr, nullptr,
                        nullptr, &cg, cg.active);
  } else {
    fl::apply_passes<T>(A->g, sc, lam, tw, nullptr, q, nrhs, ws, st, fl::PM_CG,
                        cg.precond ? z : r, p, nullptr, &cg, cg.active);
  }
  fl::cg_update<T>(A->g, x, r, p, q, nrhs, cg, st);
  if (cg.precond) precond_apply<T>(A, linv, tw, r, z, nrhs, ws, cg, cg.active, st);
}

// CG from x0 = 0 on A x = rhs until no right-hand side is active.  The
// number of active right-hand sides is read back every `chunk` iterations
// (one 4-byte copy); masked launches past convergence cost only launch time.
template <typename T>
void cg_run(fl_op A, const fl::Schedule& sc, const T* lam, const T* linv, const fl::Twiddles& tw,
            const T* rhs, T* x, T* r, T* p, T* q, T* z, int nrhs, const fl::CgScalars& cg,
            const int* outer_active, void* ws, hipStream_t st, T* S1) {
  cg_start<T>(A, sc, linv, tw, rhs, x, r, p, z, nrhs, cg, outer_active, ws, st, S1);
  int done = 0;
  int chunk = 8;
  const int cap = cg.maxiter + 2;
  while (done < cap) {
    const int k = std::min(chunk, cap - done);
    for (int i = 0; i < k; ++i)
      cg_iteration<T>(A, sc, lam, linv, tw, x, r, p, q, z, nrhs, cg, ws, st, S1);
    done += k;
    int nact = 0;
    FL_HIP(hipMemcpyAsync(&nact, cg.n_active, sizeof(int), hipMemcpyDeviceToHost, st));
    FL_HIP(hipStreamSynchronize(st));
    if (nact == 0) break;
    chunk = std::min(chunk * 2, 32);
  }
}

// ||f - A u||^2 per RHS (FP64 product) into out; r receives the residual.
void fp64_residual(fl_op A, const double* f, const double* u, double* r, int nrhs,
                   const fl::CgScalars& co, const int* active, double* out, void* ws,
                   hipStream_t st) {
  fl::apply_passes<double>(A->g, A->sc64, A->lam64, A->tw64, u, r, nrhs, ws, st, fl::PM_RESID,
                           nullptr, nullptr, f, &co, active);
  fl::reduce_parts(co.part_a, fl::last_pass_blocks(A->g, A->sc64), co.max_blocks, nrhs, out,
                   active, st);
}

// Per-RHS results of a finished solve: packed on the device and copied to
// the pinned poll record in one transfer, then unpacked (synchronizes st).
void read_results(fl_op A, int nrhs, const int* iters, const int* status, const int* nupd,
                  const double* res2, const double* rro, const double* f2, hipStream_t st,
                  std::vector<int>& h_iters, std::vector<int>& h_status, std::vector<int>& h_nupd,
                  std::vector<double>& h_res2, std::vector<double>& h_rro,
                  std::vector<double>& h_f2) {
  double* dev = nullptr;
  size_t pb = 0;
  const double* h = poll_buffers(A, nrhs, &dev, &pb);
  static_assert(fl::RESULT_STRIDE <= fl::POLL_STRIDE, "the result record fits the poll record");
  fl::pack_results(nrhs, iters, status, nupd, res2, rro, f2, dev, st);
  FL_HIP(hipMemcpyAsync(A->poll_host, dev, (size_t)fl::RESULT_STRIDE * nrhs * sizeof(double),
                        hipMemcpyDeviceToHost, st));
  FL_HIP(hipStreamSynchronize(st));
  for (int o = 0; o < nrhs; ++o) {
    const double* q = h + fl::RESULT_STRIDE * (size_t)o;
    h_iters[o] = (int)q[0];
    h_status[o] = (int)q[1];
    h_nupd[o] = (int)q[2];
    h_res2[o] = q[3];
    h_rro[o] = q[4];
    h_f2[o] = q[5];
  }
}

void sum_squares(fl_op A, const double* v, int nrhs, const fl::CgScalars& co, double* out,
                 hipStream_t st) {
  fl::sum_squares_parts(v, A->g.nd, nrhs, co.part_b, co.max_blocks, st);
  fl::reduce_parts(co.part_b, fl::vec_blocks(A->g.nd, nrhs), co.max_blocks, nrhs, out, nullptr,
                   st);
}

}  // namespace

extern "C" fl_status fl_exterior(fl_op A, const double* g_lat, const double* tail, double* b,
                                 int nrhs, void* stream) {
  return guarded([&]() -> fl_status {
    if (!A) return fail(FL_E_INVAL, "null handle");
    if (!g_lat || !b) return fail(FL_E_INVAL, "null argument");
    if (nrhs < 1) return fail(FL_E_INVAL, "nrhs must be >= 1");
    if (!fl::exterior_supported(A->g))
      return fail(FL_E_UNSUPPORTED,
                  "exterior data: d = 3 needs at most 1024^3 transform points (N <= 256)");
    std::lock_guard<std::mutex> lock(A->mu);
    set_device(A);
    hipStream_t st = (hipStream_t)stream;
    A->begin(st);
    const size_t kb = fl::exterior_khat_bytes(A->g);
    void* kh = kb ? A->ext_khat.get(kb) : nullptr;
    const size_t wb = fl::exterior_work_bytes(A->g);
    void* wk = wb ? A->ext_work.get(wb) : nullptr;
    fl::exterior_term(A->g, A->G, A->c, g_lat, tail, b, nrhs, kh, A->ext_ready, wk, st);
    A->ext_ready = kb != 0;
    A->end(st);
    return FL_OK;
  });
}

// Argument checks of fl_solve and fl_solve_async (no device work).
static fl_status check_solve(fl_op A, const double* f, const double* b, double tol, int maxiter,
                             int mixed, const double* u, int nrhs) {
  if (!A) return fail(FL_E_INVAL, "null handle");
  if (!f || !u) return fail(FL_E_INVAL, "null vector");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(FL_E_INVAL, "tol must be positive");
  if (maxiter < 1) return fail(FL_E_INVAL, "maxiter must be >= 1");
  if (nrhs < 1) return fail(FL_E_INVAL, "nrhs must be >= 1");
  if (mixed < 0 || mixed > 2) return fail(FL_E_INVAL, "mixed must be 0, 1 or 2");
  if ((const void*)f == (const void*)u) return fail(FL_E_INVAL, "f and u must be distinct");
  if (b && (const void*)b == (const void*)u) return fail(FL_E_INVAL, "b and u must be distinct");
  return FL_OK;
}

// The solve, on the operator's own stream, one at a time per operator.  It
// starts after `user`'s work so far, or, given `after`, after that event
// (the asynchronous form, which also leaves `user` free of the result).
static fl_status solve_body(fl_op A, const double* f, const double* b, double tol, int maxiter,
                            int mixed, double* u, int nrhs, fl_info* info, hipStream_t user,
                            hipEvent_t after) {
  std::lock_guard<std::mutex> lock(A->mu);
  set_device(A);
  ensure_solver_stream(A);
  hipStream_t st = A->solve_stream;
  if (after) {
    FL_HIP(hipStreamWaitEvent(st, after, 0));
  } else {
    FL_HIP(hipEventRecord(A->ev_in, user));
    FL_HIP(hipStreamWaitEvent(st, A->ev_in, 0));
  }
  A->begin(st);
  const long nd = A->g.nd;
  const size_t v8 = (size_t)nrhs * nd * sizeof(double);
  if (b) {
    // exterior-data term b: solve A u = f - b (norms relative to ||f - b||)
    double* fb = (double*)A->ext_rhs.get(v8);
    fl::difference(f, b, fb, (long)nrhs * nd, st);
    f = fb;
  }
  const size_t v4 = (size_t)nrhs * nd * sizeof(float);
  const size_t a8 = ((v8 + 255) / 256) * 256, a4 = ((v4 + 255) / 256) * 256;
  std::vector<int> iters(nrhs, 0), outer(nrhs, 0), status(nrhs, 0);
  std::vector<double> rec(nrhs, 0.0), tru(nrhs, 0.0);
  A->cg.ensure(nrhs, st);
  A->cg_out.ensure(nrhs, st);
  const fl::CgScalars& co = A->cg_out.s;
  // per-RHS host-visible norms and flags: f2, rr (outer), scale, flags
  char* fb = (char*)A->outer_flags.get(4 * (size_t)nrhs * sizeof(double) +
                                       3 * (size_t)nrhs * sizeof(int) + 1024);
  double* f2 = (double*)fb;
  double* rro = f2 + nrhs;
  double* scale = rro + nrhs;
  double* rr_last = scale + nrhs;
  int* oact = (int*)(rr_last + nrhs);
  int* trig = oact + nrhs;
  int* nupd = trig + nrhs;
  void* ws = A->ws.get(fl::apply_workspace_bytes(A->g, nrhs, false));
  std::vector<double> hf2(nrhs), hrr(nrhs);
  sum_squares(A, f, nrhs, co, f2, st);
  const int pc = A->precond;
  if (!mixed) {
    const fl::CgScalars cg = cg_view(A->cg.s, A->g, A->sc64, A->sp64, nrhs, maxiter, tol, pc);
    char* vb = (char*)A->vecs.get(5 * a8);
    double* r = (double*)vb;
    double* p = (double*)(vb + a8);
    double* q = (double*)(vb + 2 * a8);
    double* x = (double*)(vb + 3 * a8);
    double* z = (double*)(vb + 4 * a8);
    if (A->g.d == 1 && !(pc == 2 && !A->g.sine_ok())) {
      // the line fits a workgroup: the whole solve in one launch (radix 8:
      // the most threads per line and no register spills); the tau
      // preconditioner of a 2N that is not a power of two runs the
      // multi-kernel iteration with the mixed-radix sine pass
      fl::cg1d_solve(A->g, 8, f, x, A->lam64, pc ? pc_symbol<double>(A) : nullptr, pc == 2, cg,
                     nrhs, maxiter, tol, A->tw64.ax[0], st);
    } else {
      double* S1 = tau_split(A, A->sp64)
                       ? (double*)A->tau_ws.get((size_t)nrhs * nd * sizeof(double))
                       : nullptr;
      cg_start<double>(A, A->sc64, pc_symbol<double>(A), A->tw64, f, x, r, p, z, nrhs, cg,
                       nullptr, ws, st, S1);
      const int chunk = 8;
      std::vector<double> key = make_key(0, nrhs, chunk, maxiter, tol, pc);
      for (double v : {pkey(ws), pkey(vb), pkey(A->cg.mem.p), pkey(A->lam64), pkey(S1)})
        key.push_back(v);
      for (double v : sched_key(A->sc64)) key.push_back(v);
      for (double v : sched_key(A->sp64)) key.push_back(v);
      predictive_loop(A, key, maxiter + 2, cg, nrhs, st, S1 ? 0 : 1, [&]() {
        cg_iteration<double>(A, A->sc64, A->lam64, pc_symbol<double>(A), A->tw64, x, r, p, q, z,
                             nrhs, cg, ws, st, S1);
      });
    }
    FL_HIP(hipMemcpyAsync(u, x, v8, hipMemcpyDeviceToDevice, st));
    // true residual with an FP64 product (into q); the results travel in
    // one pinned record (copies into pageable memory would each wait)
    fp64_residual(A, f, u, q, nrhs, co, nullptr, rro, ws, st);
    std::vector<double> rr(nrhs);
    read_results(A, nrhs, cg.iters, cg.status, nullptr, cg.res2, rro, f2, st, iters, status,
                 outer, rr, hrr, hf2);
    for (int o = 0; o < nrhs; ++o) {
      const double fn = std::sqrt(hf2[o]);
      rec[o] = fn > 0 ? std::sqrt(rr[o]) / fn : 0.0;
      tru[o] = fn > 0 ? std::sqrt(hrr[o]) / fn : 0.0;
      if (status[o] == 0 && !(rec[o] <= tol) && fn > 0) status[o] = FL_E_NOCONV;
    }
  } else if (mixed == 1) {
    // FP32 CG with FP64 reliable updates: the FP32 recursion runs on a
    // correction xlo; after every predicted chunk of iterations each RHS
    // whose FP32 r.r fell below delta^2 of its value at the last update
    // (or below the tolerance) folds xlo into the FP64 iterate, recomputes
    // r = f - A u in FP64, stops if ||r|| <= tol ||f||, and otherwise
    // continues from r (rounded to FP32); preconditioned, the search
    // direction restarts there.
    fl::CgScalars cg = cg_view(A->cg.s, A->g, A->sc32, A->sp32, nrhs, maxiter, tol, pc);
    cg.tol2 = 0.0;  // the FP32 recursion never stops on its own residual
    const double delta2 = A->delta * A->delta;
    // ... but waits for a reliable update at the iteration start where its
    // r.r reaches the trigger (cg_begin)
    cg.rel_last = rr_last;
    cg.rel_f2 = f2;
    cg.rel_trig = trig;
    cg.rel_delta2 = delta2;
    cg.rel_tol2 = tol * tol;
    const int nb64 = fl::last_pass_blocks(A->g, A->sc64);
    char* vb = (char*)A->vecs.get(3 * a8 + 6 * a4);
    double* r64 = (double*)vb;
    double* xhi = (double*)(vb + a8);
    double* fc = (double*)(vb + 2 * a8);
    float* rhs32 = (float*)(vb + 3 * a8);
    float* xlo = (float*)(vb + 3 * a8 + a4);
    float* r32 = (float*)(vb + 3 * a8 + 2 * a4);
    float* p32 = (float*)(vb + 3 * a8 + 3 * a4);
    float* q32 = (float*)(vb + 3 * a8 + 4 * a4);
    float* z32 = (float*)(vb + 3 * a8 + 5 * a4);
    fl::fill_zero_bytes(xhi, v8, st);
    FL_HIP(hipMemcpyAsync(fc, f, v8, hipMemcpyDeviceToDevice, st));
    fl::to_float(f, rhs32, (long)nrhs * nd, st);
    FL_HIP(hipMemcpyAsync(rr_last, f2, nrhs * sizeof(double), hipMemcpyDeviceToDevice, st));
    fl::fill_int(nupd, 0, nrhs, st);
    fl::fill_int(trig, 0, nrhs, st);
    float* S1 = tau_split(A, A->sp32)
                    ? (float*)A->tau_ws.get((size_t)nrhs * nd * sizeof(float))
                    : nullptr;
    cg_start<float>(A, A->sc32, pc_symbol<float>(A), A->tw32, rhs32, xlo, r32, p32, z32, nrhs, cg,
                    nullptr, ws, st, S1);
    const int chunk = 8;
    std::vector<double> key = make_key(1, nrhs, chunk, maxiter, tol, A->delta, pc);
    for (double v : {pkey(ws), pkey(vb), pkey(A->cg.mem.p), pkey(A->cg_out.mem.p),
                     pkey(A->outer_flags.p), pkey(A->lam32), pkey(S1)})
      key.push_back(v);
    for (double v : sched_key(A->sc32)) key.push_back(v);
    for (double v : sched_key(A->sp32)) key.push_back(v);
    for (double v : sched_key(A->sc64)) key.push_back(v);
    predictive_mixed_loop(
        A, key, maxiter, cg, nrhs, rr_last, f2, nupd, delta2, tol * tol, st, S1 ? 0 : 1,
        [&]() {
          cg_iteration<float>(A, A->sc32, A->lam32, pc_symbol<float>(A), A->tw32, xlo, r32, p32,
                              q32, z32, nrhs, cg, ws, st, S1);
        },
        [&]() {
          fl::reliable_accum(A->g, xhi, xlo, nrhs, cg, trig, false, st);
          fl::apply_passes<double>(A->g, A->sc64, A->lam64, A->tw64, xhi, r64, nrhs, ws, st,
                                   fl::PM_RESID, nullptr, nullptr, fc, &co, trig);
          fl::reliable_replace(A->g, r64, r32, nrhs, cg, co.part_a, nb64, co.max_blocks,
                               rr_last, f2, tol * tol, trig, nupd, st);
          // the restarted right-hand sides' z = P r (or its first half,
          // into S1, which the FP64 residual's passes above do not touch)
          if (S1)
            fl::tau_front<float>(A->g, A->sp32, pc_symbol<float>(A), A->tw32, r32, S1, nrhs, st,
                                 cg, trig, false);
          else if (pc)
            precond_apply<float>(A, pc_symbol<float>(A), A->tw32, r32, z32, nrhs, ws, cg, trig,
                                 st);
        });
    // fold what is left (RHS stopped by maxiter) and report true residuals:
    // a converged RHS has its final iterate's FP64 residual from its last
    // replacement; the others get a fresh FP64 product
    fl::reliable_accum(A->g, xhi, xlo, nrhs, cg, trig, true, st);
    FL_HIP(hipMemcpyAsync(u, xhi, v8, hipMemcpyDeviceToDevice, st));
    fl::reliable_final(cg.status, rr_last, trig, rro, nrhs, st);
    fp64_residual(A, f, u, r64, nrhs, co, trig, rro, ws, st);
    std::vector<double> rr(nrhs);
    read_results(A, nrhs, cg.iters, cg.status, nupd, nullptr, rro, f2, st, iters, status, outer,
                 rr, hrr, hf2);
    for (int o = 0; o < nrhs; ++o) {
      const double rel = hf2[o] > 0 ? std::sqrt(hrr[o] / hf2[o]) : 0.0;
      rec[o] = rel;
      tru[o] = rel;
      if (status[o] == 0 && !(rel <= tol) && hf2[o] > 0) status[o] = FL_E_NOCONV;
    }
  } else {
    // FP64 residual and iterate; FP32 CG on A delta = r / ||r|| (inner_tol)
    const fl::CgScalars cg = cg_view(A->cg.s, A->g, A->sc32, A->sp32, nrhs, maxiter, A->inner_tol, pc);
    char* vb = (char*)A->vecs.get(a8 + 6 * a4);
    double* r64 = (double*)vb;
    float* rhs32 = (float*)(vb + a8);
    float* d32 = (float*)(vb + a8 + a4);
    float* r32 = (float*)(vb + a8 + 2 * a4);
    float* p32 = (float*)(vb + a8 + 3 * a4);
    float* q32 = (float*)(vb + a8 + 4 * a4);
    float* z32 = (float*)(vb + a8 + 5 * a4);
    float* S1 = tau_split(A, A->sp32)
                    ? (float*)A->tau_ws.get((size_t)nrhs * nd * sizeof(float))
                    : nullptr;
    fl::fill_zero_bytes(u, v8, st);
    FL_HIP(hipMemcpyAsync(r64, f, v8, hipMemcpyDeviceToDevice, st));
    FL_HIP(hipMemcpyAsync(rro, f2, nrhs * sizeof(double), hipMemcpyDeviceToDevice, st));
    std::vector<int> hact(nrhs), hit(nrhs), hst(nrhs);
    FL_HIP(hipMemcpyAsync(hf2.data(), f2, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    FL_HIP(hipStreamSynchronize(st));
    hrr = hf2;
    for (int step = 0;; ++step) {
      int nact = 0;
      for (int o = 0; o < nrhs; ++o) {
        const double rel = hf2[o] > 0 ? std::sqrt(hrr[o] / hf2[o]) : 0.0;
        const bool bad = !std::isfinite(rel);
        hact[o] = (!bad && rel > tol && status[o] == 0) ? 1 : 0;
        if (bad) status[o] = FL_E_BREAKDOWN;
        nact += hact[o];
      }
      if (nact == 0) break;
      if (step >= A->max_outer) {
        for (int o = 0; o < nrhs; ++o)
          if (hact[o]) status[o] = FL_E_NOCONV;
        break;
      }
      FL_HIP(hipMemcpyAsync(oact, hact.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
      fl::refine_scale(r64, rhs32, rro, scale, nd, nrhs, oact, st);
      cg_run<float>(A, A->sc32, A->lam32, pc_symbol<float>(A), A->tw32, rhs32, d32, r32, p32, q32, z32,
                    nrhs, cg, oact, ws, st, S1);
      fl::refine_axpy(u, d32, scale, nd, nrhs, oact, st);
      fp64_residual(A, f, u, r64, nrhs, co, oact, rro, ws, st);
      FL_HIP(hipMemcpyAsync(hit.data(), cg.iters, nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
      FL_HIP(hipMemcpyAsync(hst.data(), cg.status, nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
      FL_HIP(hipMemcpyAsync(hrr.data(), rro, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
      FL_HIP(hipStreamSynchronize(st));
      for (int o = 0; o < nrhs; ++o)
        if (hact[o]) {
          iters[o] += hit[o];
          outer[o] += 1;
          if (hst[o] == FL_E_BREAKDOWN && hit[o] == 0) status[o] = FL_E_BREAKDOWN;
        }
    }
    for (int o = 0; o < nrhs; ++o) {
      const double rel = hf2[o] > 0 ? std::sqrt(hrr[o] / hf2[o]) : 0.0;
      rec[o] = rel;
      tru[o] = rel;
    }
  }
  A->end(st);
  if (!after) FL_HIP(hipStreamWaitEvent(user, A->done, 0));
  fl_status worst = FL_OK;
  for (int o = 0; o < nrhs; ++o) {
    if (info) {
      info[o].iters = iters[o];
      info[o].outer_iters = outer[o];
      info[o].status = status[o];
      info[o].converged = status[o] == 0;
      info[o].relres_rec = rec[o];
      info[o].relres_true = tru[o];
    }
    if (status[o] != 0 && worst == FL_OK) worst = (fl_status)status[o];
  }
  if (worst != FL_OK) g_last_error = "some right-hand sides did not converge";
  return worst;
}

extern "C" fl_status fl_solve(fl_op A, const double* f, const double* b, double tol, int maxiter,
                              int mixed, double* u, int nrhs, fl_info* info, void* stream) {
  return guarded([&]() -> fl_status {
    const fl_status e = check_solve(A, f, b, tol, maxiter, mixed, u, nrhs);
    if (e != FL_OK) return e;
    return solve_body(A, f, b, tol, maxiter, mixed, u, nrhs, info, (hipStream_t)stream, nullptr);
  });
}

// A solve running on its own host thread (fl_solve_async).
struct fl_request_s {
  std::thread worker;
  std::atomic<int> done{0};
  fl_status status = FL_OK;
  std::string error;
  std::vector<fl_info> info;
};

extern "C" fl_status fl_solve_async(fl_op A, const double* f, const double* b, double tol,
                                    int maxiter, int mixed, double* u, int nrhs, void* stream,
                                    fl_request* out) {
  return guarded([&]() -> fl_status {
    if (!out) return fail(FL_E_INVAL, "out is NULL");
    const fl_status e = check_solve(A, f, b, tol, maxiter, mixed, u, nrhs);
    if (e != FL_OK) return e;
    // order the solve after the caller's work on `stream` submitted so far
    set_device(A);
    hipEvent_t after = nullptr;
    FL_HIP(hipEventCreateWithFlags(&after, hipEventDisableTiming));
    hipError_t he = hipEventRecord(after, (hipStream_t)stream);
    if (he != hipSuccess) {
      (void)hipEventDestroy(after);
      return fail(FL_E_DEVICE, hipGetErrorString(he));
    }
    fl_request R = new fl_request_s();
    R->info.resize(nrhs);
    try {
      R->worker = std::thread([=]() {
        R->status = guarded([&]() -> fl_status {
          return solve_body(A, f, b, tol, maxiter, mixed, u, nrhs, R->info.data(), nullptr, after);
        });
        if (R->status != FL_OK) R->error = fl_last_error();
        (void)hipEventDestroy(after);
        R->done.store(1, std::memory_order_release);
      });
    } catch (...) {
      delete R;
      (void)hipEventDestroy(after);
      throw;
    }
    *out = R;
    return FL_OK;
  });
}

extern "C" fl_status fl_poll(fl_request R, int* done) {
  if (!R || !done) return fail(FL_E_INVAL, "null argument");
  *done = R->done.load(std::memory_order_acquire);
  return FL_OK;
}

extern "C" fl_status fl_wait(fl_request R, fl_info* info) {
  if (!R) return fail(FL_E_INVAL, "null request");
  if (R->worker.joinable()) R->worker.join();
  if (info) std::copy(R->info.begin(), R->info.end(), info);
  const fl_status st = R->status;
  if (st != FL_OK) g_last_error = R->error;
  else g_last_error.clear();
  delete R;
  return st;
}
