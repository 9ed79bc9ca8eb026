// Host-side interfaces between the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <stdexcept>
#include <string>

namespace fl {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define FL_HIP(call)                                                             \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      throw ::fl::Error(4, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

// ---------------------------------------------------------------------------
// per-RHS CG bookkeeping (device pointers, all arrays of length nrhs unless
// noted).  Shared by the pass epilogues and the update kernels.
// ---------------------------------------------------------------------------
struct CgScalars {
  double* rr;        // current ||r||^2
  double* alpha;     // rr / (p.Ap)
  double* beta;      // rr_new / rr_old (0 on the first iteration)
  double* thresh2;   // stop when rr <= thresh2
  double* rr0;       // ||rhs||^2 at start
  int* active;       // 1 while iterating
  int* iters;        // iterations done
  int* status;       // 0 running/converged, 5 no convergence, 6 breakdown
  int* n_active;     // single int: number of active RHS
  double* part_a;    // partial sums, nrhs * max_blocks
  double* part_b;
  unsigned* cnt_a;   // last-block counters, nrhs
  unsigned* cnt_b;
  int max_blocks;
};

// Epilogue/prologue selection of the first and last FFT passes.
enum PassMode {
  PM_PLAIN = 0,     // y = A u
  PM_CG = 1,        // first pass: p = r + beta p ; last pass: q = A p, alpha = rr / p.q
  PM_RESID = 2,     // last pass: y = f - A u and ||y||^2 per RHS (FP64 only)
};

struct ApplyPlan;  // defined in the passes unit

// Geometry of one operator application.
struct Geometry {
  int d;       // 1, 2, 3
  int N;       // intervals per axis
  int n;       // interior points per axis = N - 1
  int M;       // embedding length per axis = 2N
  long nd;     // n^d
};

// Launch schedule (tunable).
struct Schedule {
  int E_first;   // elements per thread, strided passes along axis 0
  int E_mid;     // elements per thread, contiguous middle pass
  int E_c2c;     // elements per thread, 3D axis-1 passes
  int W_first;   // lines per block in strided passes
  int W_c2c;
  int LPB_mid;   // lines per block in the middle pass
};

Schedule default_schedule(const Geometry& g, bool fp32);

// Workspace bytes for nrhs right-hand sides (FFT intermediates).
size_t apply_workspace_bytes(const Geometry& g, int nrhs, bool fp32);

// y = A u (mode PM_PLAIN), CG fused step (PM_CG: uses r, p in place of u,
// writes q into y), or FP64 residual (PM_RESID: y = f - A u).
template <typename T>
void apply_passes(const Geometry& g, const Schedule& sc, const T* lam, const void* tw,
                  const T* u, T* y, int nrhs, void* ws, hipStream_t st, int mode,
                  const T* rvec, T* pvec, const double* fvec, const CgScalars* cg,
                  const int* active, hipEvent_t* ev = nullptr);

// Number of kernel launches (passes) of one application: 1, 3 or 5 for d = 1, 2, 3.
inline int apply_npasses(int d) { return d == 1 ? 1 : (d == 2 ? 3 : 5); }

// Twiddle table exp(-2 pi i j / M), j < M (cx<T> array), cached per device.
const void* twiddles(int M, bool fp32, hipStream_t st);

// Generator, symbol: see weights unit.
struct GenParams {
  int d, p, N, kernel;
  double alpha, h, lambda, c;
};
void build_generator(const GenParams& gp, double* G, hipStream_t st);
void build_symbol(const Geometry& g, const double* G, double* lam64, float* lam32,
                  hipStream_t st);
void embed_generator(const Geometry& g, const double* G, double* out, hipStream_t st);

// CG kernels (cg unit).
template <typename T>
void cg_init(const Geometry& g, const T* rhs, T* x, T* r, T* p, int nrhs, double tol,
             const CgScalars& cg, const int* outer_active, hipStream_t st);
template <typename T>
void cg_update(const Geometry& g, T* x, T* r, const T* p, const T* q, int nrhs, int maxiter,
               const CgScalars& cg, hipStream_t st);
void fill_int(int* p, int v, int n, hipStream_t st);
void fill_zero_bytes(void* p, size_t bytes, hipStream_t st);
// refinement helpers
void refine_scale(const double* r64, float* r32, const double* rr, double* scale, long nd,
                  int nrhs, const int* active, hipStream_t st);
void refine_axpy(double* u, const float* d32, const double* scale, long nd, int nrhs,
                 const int* active, hipStream_t st);
void sum_squares(const double* v, long nd, int nrhs, double* out, double* part, unsigned* cnt,
                 int max_blocks, hipStream_t st);

}  // namespace fl
