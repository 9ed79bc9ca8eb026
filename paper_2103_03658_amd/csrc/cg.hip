// Conjugate-gradient vector kernels for many right-hand sides at once.
// A is symmetric positive definite (Sec. 2.2), so plain CG applies; the
// paper names no solver.  Vectors are [nrhs][n^d] in T (double, or float for
// the inner solves of the mixed-precision path); every scalar and every
// reduction is FP64 and in a fixed order, so a right-hand side gives the
// same bits whatever else is in the batch.  A right-hand side that has
// converged, broken down or hit maxiter is masked out of later launches.
//
// One iteration is: first pass (beta, stopping test, p = r + beta p, forward
// transform), middle pass, last pass (q = A p and partials of p.q), update
// (alpha = rr / p.q, x += alpha p, r -= alpha q, partials of r.r).
#include <algorithm>

#include "passes_impl.h"

namespace fl {

namespace {

constexpr int VT = 256;  // threads per vector block

template <typename T>
__global__ void __launch_bounds__(VT) k_cg_init(const T* rhs, T* x, T* r, T* p, long nd,
                                                CgScalars cg, const int* outer_active) {
  __shared__ double red[8];
  const int o = blockIdx.y;
  if (outer_active && !outer_active[o]) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg.active[o] = 0;
      cg.iters[o] = 0;
      cg.status[o] = 0;
    }
    return;
  }
  const long base = (long)o * nd;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT) {
    const T v = rhs[base + i];
    r[base + i] = v;
    x[base + i] = 0;
    p[base + i] = 0;
    acc += (double)v * (double)v;
  }
  const double blk = block_sum(acc, red);
  if (threadIdx.x == 0) {
    (cg.precond ? cg.part_c : cg.part_b)[(long)o * cg.max_blocks + blockIdx.x] = blk;
    if (blockIdx.x == 0) {
      cg.iters[o] = 0;
      cg.status[o] = 0;
      cg.active[o] = 1;
      cg.rr_prev[o] = 0.0;
      cg.alpha[o] = 0.0;
      atomicAdd(cg.n_active, 1);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(VT) k_cg_update(T* x, T* r, const T* p, const T* q, long nd,
                                                  CgScalars cg) {
  __shared__ double red[64];
  const int o = blockIdx.y;
  if (!cg.active[o]) return;
  const double pq = sum_partials(cg.part_a + (long)o * cg.max_blocks, cg.nb_a, red);
  const double rr = cg.rr_cur[o];
  const double al = rr / pq;
  if (!(pq > 0.0) || !isfinite(al)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg.active[o] = 0;
      cg.status[o] = 6;
      atomicSub(cg.n_active, 1);
    }
    return;
  }
  const long base = (long)o * nd;
  const T a = (T)al;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT) {
    x[base + i] += a * p[base + i];
    const T rv = r[base + i] - a * q[base + i];
    r[base + i] = rv;
    acc += (double)rv * (double)rv;
  }
  const double blk = block_sum(acc, red);
  if (threadIdx.x == 0) {
    (cg.precond ? cg.part_c : cg.part_b)[(long)o * cg.max_blocks + blockIdx.x] = blk;
    if (blockIdx.x == 0) {
      cg.rr_prev[o] = rr;
      cg.iters[o] = cg.iters[o] + 1;
      cg.alpha[o] = al;
    }
  }
}

// Start of a CG iteration for d >= 2 as a streaming pass: the stopping test
// and beta (cg_begin), then p = zr + beta p (zr = z preconditioned, else r).
// A right-hand side that stops returns in every block: the lead block's
// deactivation can only turn later blocks of it away, which is what they do.
template <typename T>
__global__ void __launch_bounds__(VT) k_cg_direction(T* p, const T* zr, long nd, CgScalars cg) {
  __shared__ double red[64];
  const int o = blockIdx.y;
  if (!cg.active[o]) return;
  double beta;
  if (cg_begin(cg, o, blockIdx.x == 0, red, &beta)) return;
  const T b = (T)beta;
  const long base = (long)o * nd;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT)
    p[base + i] = zr[base + i] + b * p[base + i];
}

__global__ void k_fill_int(int* p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Per-RHS CG state gathered for the host: [n_active, then per RHS
// POLL_STRIDE values: r.r at the last iteration start, stopping threshold,
// active, iterations, r.r now (sum of the partials of the last update or
// replacement), r.r at the last reliable update, ||f||^2, reliable updates].
// The last three are 0 when their arrays are not given.  One wave per RHS.
__global__ void __launch_bounds__(64) k_pack_poll(CgScalars cg, int nrhs, const double* rr_last,
                                                  const double* f2, const int* nupd,
                                                  double* out) {
  const int o = blockIdx.x;
  if (o == 0 && threadIdx.x == 0) out[0] = (double)cg.n_active[0];
  const double* part = (cg.precond ? cg.part_c : cg.part_b) + (long)o * cg.max_blocks;
  double now = 0.0;
  for (int i = threadIdx.x; i < cg.nb_c; i += 64) now += part[i];
  now = wave_sum(now);
  if (threadIdx.x == 0) {
    double* q = out + 1 + POLL_STRIDE * (long)o;
    q[0] = cg.res2[o];
    q[1] = cg.thresh2[o];
    q[2] = (double)cg.active[o];
    q[3] = (double)cg.iters[o];
    q[4] = now;
    q[5] = rr_last ? rr_last[o] : 0.0;
    q[6] = f2 ? f2[o] : 0.0;
    q[7] = nupd ? (double)nupd[o] : 0.0;
  }
}

// Per-RHS results of a finished solve in one record of RESULT_STRIDE doubles:
// iterations, status, reliable updates (0 if nupd is null), r.r of the
// recursion (0 if res2 is null), r.r of the FP64 residual, ||f||^2.
__global__ void k_pack_results(int nrhs, const int* iters, const int* status, const int* nupd,
                               const double* res2, const double* rro, const double* f2,
                               double* out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nrhs) return;
  double* q = out + RESULT_STRIDE * (long)o;
  q[0] = (double)iters[o];
  q[1] = (double)status[o];
  q[2] = nupd ? (double)nupd[o] : 0.0;
  q[3] = res2 ? res2[o] : 0.0;
  q[4] = rro[o];
  q[5] = f2[o];
}

__global__ void k_fill_zero(unsigned* p, size_t nwords) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) p[i] = 0u;
}

__global__ void k_reduce_parts(const double* part, int nb, int max_blocks, double* out,
                               const int* active) {
  __shared__ double red[64];
  const int o = blockIdx.x;
  if (active && !active[o]) return;
  const double t = sum_partials(part + (long)o * max_blocks, nb, red);
  if (threadIdx.x == 0) out[o] = t;
}

__global__ void __launch_bounds__(VT) k_refine_scale(const double* r64, float* r32,
                                                     const double* rr, double* scale, long nd,
                                                     const int* active) {
  const int o = blockIdx.y;
  if (active && !active[o]) return;
  const double s = sqrt(rr[o]);
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) scale[o] = s;
  const long base = (long)o * nd;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT)
    r32[base + i] = (float)(r64[base + i] * inv);
}

__global__ void __launch_bounds__(VT) k_refine_axpy(double* u, const float* d32,
                                                    const double* scale, long nd,
                                                    const int* active) {
  const int o = blockIdx.y;
  if (active && !active[o]) return;
  const double s = scale[o];
  const long base = (long)o * nd;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT)
    u[base + i] += s * (double)d32[base + i];
}

__global__ void __launch_bounds__(VT) k_sumsq_parts(const double* v, long nd, double* part,
                                                    int max_blocks) {
  __shared__ double red[8];
  const int o = blockIdx.y;
  const long base = (long)o * nd;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT)
    acc += v[base + i] * v[base + i];
  const double blk = block_sum(acc, red);
  if (threadIdx.x == 0) part[(long)o * max_blocks + blockIdx.x] = blk;
}

__global__ void __launch_bounds__(VT) k_to_float(const double* src, float* dst, long n) {
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < n; i += (long)gridDim.x * VT)
    dst[i] = (float)src[i];
}

// Reliable update, step 1: for each RHS whose FP32 recursion stopped at an
// iteration start because its r.r fell below delta^2 times its value at the
// last replacement, or below the final tolerance (trig[o] = 1, decided per
// iteration, so the result does not depend on when this step runs), fold
// the FP32 correction into the FP64 iterate: xhi += xlo, xlo = 0.
// force: fold for every RHS (end of the solve).
__global__ void __launch_bounds__(VT) k_reliable_accum(double* xhi, float* xlo, long nd,
                                                       const int* trig, int force) {
  const int o = blockIdx.y;
  if (!force && !trig[o]) return;
  const long base = (long)o * nd;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT) {
    xhi[base + i] += (double)xlo[base + i];
    xlo[base + i] = 0.0f;
  }
}

// End of a reliable-update solve.  A right-hand side that converged did so
// at a replacement (the recursion's tolerance test only flags one), after
// which its FP32 correction was folded and nothing was added: the FP64
// residual of that replacement, rr_last = ||f - A x||^2, belongs to the
// final iterate.  The others (iteration cap or breakdown inside the FP32
// recursion, with a correction folded only now) get mask = 1 for a fresh
// FP64 residual.
__global__ void k_reliable_final(const int* status, const double* rr_last, int* mask,
                                 double* rr_true, int nrhs) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nrhs) return;
  const bool done = status[o] == 0;
  mask[o] = done ? 0 : 1;
  if (done) rr_true[o] = rr_last[o];
}

// Reliable update, step 2 (after r64 = f - A xhi in FP64 for the flagged
// RHS): stop if ||r64|| meets the tolerance (and clear the flag, so the
// preconditioner skips it), else resume the FP32 recursion from r32 = r64
// with fresh partials of r32.r32.
__global__ void __launch_bounds__(VT) k_reliable_replace(const double* r64, float* r32, long nd,
                                                         CgScalars cg, const double* part64,
                                                         int nb64, int mb64, double* rr_last,
                                                         const double* f2, double tol2,
                                                         int* trig, int* nupd) {
  __shared__ double red[64];
  const int o = blockIdx.y;
  if (!trig[o]) return;
  const double rr64 = sum_partials(part64 + (long)o * mb64, nb64, red);
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  if (lead) {
    rr_last[o] = rr64;
    nupd[o] = nupd[o] + 1;
  }
  // the RHS is inactive since its recursion stopped; blocks other than the
  // lead do nothing more on this branch, so clearing the flag cannot race
  if (rr64 <= tol2 * f2[o] || !isfinite(rr64)) {
    if (lead) {
      cg.status[o] = isfinite(rr64) ? 0 : 6;
      trig[o] = 0;
    }
    return;
  }
  // the iteration cap, which the recursion's own test would apply at its
  // next check: the FP64 iterate and residual are final
  if (cg.iters[o] >= cg.maxiter) {
    if (lead) {
      cg.status[o] = 5;
      trig[o] = 0;
    }
    return;
  }
  if (lead) {
    cg.active[o] = 1;
    atomicAdd(cg.n_active, 1);
  }
  // Preconditioned: within one check interval the FP32 recursion reaches
  // FP32 accuracy, so the old search direction no longer matches the
  // replaced residual; restart it (the next beta is rho / inf = 0).
  if (lead && cg.precond) cg.rr_prev[o] = INFINITY;
  const long base = (long)o * nd;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT) {
    const float v = (float)r64[base + i];
    r32[base + i] = v;
    acc += (double)v * (double)v;
  }
  const double blk = block_sum(acc, red);
  if (threadIdx.x == 0)
    (cg.precond ? cg.part_c : cg.part_b)[(long)o * cg.max_blocks + blockIdx.x] = blk;
}

}  // namespace

void to_float(const double* src, float* dst, long n, hipStream_t st) {
  long b = (n + VT * 4 - 1) / (VT * 4);
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_to_float, dim3((unsigned)b), dim3(VT), 0, st, src, dst, n);
  check_launch("to float");
}

void reliable_accum(const Geometry& g, double* xhi, float* xlo, int nrhs, const CgScalars& cg,
                    const int* trig, bool force, hipStream_t st) {
  dim3 grid(cg.nb_c, nrhs);
  hipLaunchKernelGGL(k_reliable_accum, grid, dim3(VT), 0, st, xhi, xlo, g.nd, trig,
                     force ? 1 : 0);
  check_launch("reliable accumulate");
}

void reliable_final(const int* status, const double* rr_last, int* mask, double* rr_true,
                    int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_reliable_final, dim3((nrhs + 63) / 64), dim3(64), 0, st, status, rr_last,
                     mask, rr_true, nrhs);
  check_launch("reliable final");
}

void reliable_replace(const Geometry& g, const double* r64, float* r32, int nrhs,
                      const CgScalars& cg, const double* part64, int nb64, int mb64,
                      double* rr_last, const double* f2, double tol2, int* trig,
                      int* nupd, hipStream_t st) {
  dim3 grid(cg.nb_c, nrhs);
  hipLaunchKernelGGL(k_reliable_replace, grid, dim3(VT), 0, st, r64, r32, g.nd, cg, part64, nb64,
                     mb64, rr_last, f2, tol2, trig, nupd);
  check_launch("reliable replace");
}

int vec_blocks(long nd, int nrhs) {
  // about 2048 blocks in total (8 per CU), at least 1024 elements per block
  long b = (nd + 1023) / 1024;
  const long cap = std::max<long>(8, (2048 + nrhs - 1) / nrhs);
  if (b > cap) b = cap;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
void cg_init(const Geometry& g, const T* rhs, T* x, T* r, T* p, int nrhs, const CgScalars& cg,
             const int* outer_active, hipStream_t st) {
  dim3 grid(cg.nb_c, nrhs);
  hipLaunchKernelGGL((k_cg_init<T>), grid, dim3(VT), 0, st, rhs, x, r, p, g.nd, cg,
                     outer_active);
  check_launch("cg init");
}

template <typename T>
void cg_update(const Geometry& g, T* x, T* r, const T* p, const T* q, int nrhs,
               const CgScalars& cg, hipStream_t st) {
  dim3 grid(cg.nb_c, nrhs);
  hipLaunchKernelGGL((k_cg_update<T>), grid, dim3(VT), 0, st, x, r, p, q, g.nd, cg);
  check_launch("cg update");
}

template <typename T>
void cg_direction(const Geometry& g, T* p, const T* zr, int nrhs, const CgScalars& cg,
                  hipStream_t st) {
  dim3 grid(cg.nb_c, nrhs);
  hipLaunchKernelGGL((k_cg_direction<T>), grid, dim3(VT), 0, st, p, zr, g.nd, cg);
  check_launch("cg direction");
}

template void cg_direction<double>(const Geometry&, double*, const double*, int,
                                   const CgScalars&, hipStream_t);
template void cg_direction<float>(const Geometry&, float*, const float*, int, const CgScalars&,
                                  hipStream_t);
template void cg_init<double>(const Geometry&, const double*, double*, double*, double*, int,
                              const CgScalars&, const int*, hipStream_t);
template void cg_init<float>(const Geometry&, const float*, float*, float*, float*, int,
                             const CgScalars&, const int*, hipStream_t);
template void cg_update<double>(const Geometry&, double*, double*, const double*, const double*,
                                int, const CgScalars&, hipStream_t);
template void cg_update<float>(const Geometry&, float*, float*, const float*, const float*, int,
                               const CgScalars&, hipStream_t);

void fill_int(int* p, int v, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  check_launch("fill");
}

void pack_poll(const CgScalars& cg, int nrhs, const double* rr_last, const double* f2,
               const int* nupd, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_poll, dim3(nrhs), dim3(64), 0, st, cg, nrhs, rr_last, f2, nupd,
                     out);
  check_launch("poll pack");
}

void pack_results(int nrhs, const int* iters, const int* status, const int* nupd,
                  const double* res2, const double* rro, const double* f2, double* out,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_pack_results, dim3((nrhs + 63) / 64), dim3(64), 0, st, nrhs, iters, status,
                     nupd, res2, rro, f2, out);
  check_launch("result pack");
}

void fill_zero_bytes(void* p, size_t bytes, hipStream_t st) {
  const size_t w = bytes / 4;
  if (!w) return;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((w + 255) / 256)), dim3(256), 0, st,
                     (unsigned*)p, w);
  check_launch("fill");
}

void reduce_parts(const double* part, int nb, int max_blocks, int nrhs, double* out,
                  const int* active, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_parts, dim3(nrhs), dim3(64), 0, st, part, nb, max_blocks, out,
                     active);
  check_launch("reduce");
}

void refine_scale(const double* r64, float* r32, const double* rr, double* scale, long nd,
                  int nrhs, const int* active, hipStream_t st) {
  dim3 grid(vec_blocks(nd, nrhs), nrhs);
  hipLaunchKernelGGL(k_refine_scale, grid, dim3(VT), 0, st, r64, r32, rr, scale, nd, active);
  check_launch("refine scale");
}

void refine_axpy(double* u, const float* d32, const double* scale, long nd, int nrhs,
                 const int* active, hipStream_t st) {
  dim3 grid(vec_blocks(nd, nrhs), nrhs);
  hipLaunchKernelGGL(k_refine_axpy, grid, dim3(VT), 0, st, u, d32, scale, nd, active);
  check_launch("refine axpy");
}

void sum_squares_parts(const double* v, long nd, int nrhs, double* part, int max_blocks,
                       hipStream_t st) {
  dim3 grid(vec_blocks(nd, nrhs), nrhs);
  hipLaunchKernelGGL(k_sumsq_parts, grid, dim3(VT), 0, st, v, nd, part, max_blocks);
  check_launch("sum of squares");
}

}  // namespace fl
