// Conjugate-gradient vector kernels for many right-hand sides at once.
// A is symmetric positive definite (Sec. 2.2), so plain CG applies; the
// paper names no solver.  Vectors are [nrhs][n^d] in T (double, or float for
// the inner solves of the mixed-precision path); every scalar and every
// reduction is FP64, in a fixed order (deterministic, independent of what
// else is in the batch).  Per-RHS state lives on the device; a RHS that has
// converged, broken down or hit maxiter is masked out of later launches.
#include "passes_impl.h"

namespace fl {

namespace {

constexpr int VT = 256;  // threads per vector block

inline int vec_blocks(long nd) {
  long b = (nd + VT * 4 - 1) / (VT * 4);
  if (b < 1) b = 1;
  if (b > 512) b = 512;
  return (int)b;
}

template <typename T>
__global__ void __launch_bounds__(VT) k_cg_init(const T* rhs, T* x, T* r, T* p, long nd,
                                                double tol2, CgScalars cg,
                                                const int* outer_active) {
  __shared__ double red[8];
  const int o = blockIdx.y;
  if (outer_active && !outer_active[o]) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg.active[o] = 0;
      cg.iters[o] = 0;
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
  double tot = 0.0;
  if (last_block_total(blk, cg.part_b + (long)o * cg.max_blocks, cg.cnt_b + o, gridDim.x,
                       blockIdx.x, red, &tot)) {
    if (threadIdx.x == 0) {
      cg.rr[o] = tot;
      cg.rr0[o] = tot;
      cg.thresh2[o] = tol2 * tot;
      cg.beta[o] = 0.0;
      cg.alpha[o] = 0.0;
      cg.iters[o] = 0;
      cg.status[o] = 0;
      const int act = tot > 0.0 && isfinite(tot);
      if (!isfinite(tot)) cg.status[o] = 6;
      cg.active[o] = act;
      if (act) atomicAdd(cg.n_active, 1);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(VT) k_cg_update(T* x, T* r, const T* p, const T* q, long nd,
                                                  int maxiter, CgScalars cg) {
  __shared__ double red[8];
  const int o = blockIdx.y;
  if (!cg.active[o]) return;
  const long base = (long)o * nd;
  const T a = (T)cg.alpha[o];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT) {
    x[base + i] += a * p[base + i];
    const T rv = r[base + i] - a * q[base + i];
    r[base + i] = rv;
    acc += (double)rv * (double)rv;
  }
  const double blk = block_sum(acc, red);
  double tot = 0.0;
  if (last_block_total(blk, cg.part_b + (long)o * cg.max_blocks, cg.cnt_b + o, gridDim.x,
                       blockIdx.x, red, &tot)) {
    if (threadIdx.x == 0) {
      const double old = cg.rr[o];
      cg.beta[o] = tot / old;
      cg.rr[o] = tot;
      const int it = cg.iters[o] + 1;
      cg.iters[o] = it;
      if (!isfinite(tot)) {
        cg.active[o] = 0;
        cg.status[o] = 6;
        atomicSub(cg.n_active, 1);
      } else if (tot <= cg.thresh2[o]) {
        cg.active[o] = 0;
        cg.status[o] = 0;
        atomicSub(cg.n_active, 1);
      } else if (it >= maxiter) {
        cg.active[o] = 0;
        cg.status[o] = 5;
        atomicSub(cg.n_active, 1);
      }
    }
  }
}

__global__ void k_fill_int(int* p, int v, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_zero(unsigned* p, size_t nwords) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) p[i] = 0u;
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

__global__ void __launch_bounds__(VT) k_sumsq(const double* v, long nd, double* out, double* part,
                                              unsigned* cnt, int max_blocks) {
  __shared__ double red[8];
  const int o = blockIdx.y;
  const long base = (long)o * nd;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * VT + threadIdx.x; i < nd; i += (long)gridDim.x * VT)
    acc += v[base + i] * v[base + i];
  const double blk = block_sum(acc, red);
  double tot = 0.0;
  if (last_block_total(blk, part + (long)o * max_blocks, cnt + o, gridDim.x, blockIdx.x, red,
                       &tot)) {
    if (threadIdx.x == 0) out[o] = tot;
  }
}

}  // namespace

template <typename T>
void cg_init(const Geometry& g, const T* rhs, T* x, T* r, T* p, int nrhs, double tol,
             const CgScalars& cg, const int* outer_active, hipStream_t st) {
  dim3 grid(vec_blocks(g.nd), nrhs);
  hipLaunchKernelGGL((k_cg_init<T>), grid, dim3(VT), 0, st, rhs, x, r, p, g.nd, tol * tol, cg,
                     outer_active);
  check_launch("cg init");
}

template <typename T>
void cg_update(const Geometry& g, T* x, T* r, const T* p, const T* q, int nrhs, int maxiter,
               const CgScalars& cg, hipStream_t st) {
  dim3 grid(vec_blocks(g.nd), nrhs);
  hipLaunchKernelGGL((k_cg_update<T>), grid, dim3(VT), 0, st, x, r, p, q, g.nd, maxiter, cg);
  check_launch("cg update");
}

template void cg_init<double>(const Geometry&, const double*, double*, double*, double*, int,
                              double, const CgScalars&, const int*, hipStream_t);
template void cg_init<float>(const Geometry&, const float*, float*, float*, float*, int, double,
                             const CgScalars&, const int*, hipStream_t);
template void cg_update<double>(const Geometry&, double*, double*, const double*, const double*,
                                int, int, const CgScalars&, hipStream_t);
template void cg_update<float>(const Geometry&, float*, float*, const float*, const float*, int,
                               int, const CgScalars&, hipStream_t);

void fill_int(int* p, int v, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
  check_launch("fill");
}

void fill_zero_bytes(void* p, size_t bytes, hipStream_t st) {
  const size_t w = bytes / 4;
  if (!w) return;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((w + 255) / 256)), dim3(256), 0, st,
                     (unsigned*)p, w);
  check_launch("fill");
}

void refine_scale(const double* r64, float* r32, const double* rr, double* scale, long nd,
                  int nrhs, const int* active, hipStream_t st) {
  dim3 grid(vec_blocks(nd), nrhs);
  hipLaunchKernelGGL(k_refine_scale, grid, dim3(VT), 0, st, r64, r32, rr, scale, nd, active);
  check_launch("refine scale");
}

void refine_axpy(double* u, const float* d32, const double* scale, long nd, int nrhs,
                 const int* active, hipStream_t st) {
  dim3 grid(vec_blocks(nd), nrhs);
  hipLaunchKernelGGL(k_refine_axpy, grid, dim3(VT), 0, st, u, d32, scale, nd, active);
  check_launch("refine axpy");
}

void sum_squares(const double* v, long nd, int nrhs, double* out, double* part, unsigned* cnt,
                 int max_blocks, hipStream_t st) {
  dim3 grid(vec_blocks(nd), nrhs);
  hipLaunchKernelGGL(k_sumsq, grid, dim3(VT), 0, st, v, nd, out, part, cnt, max_blocks);
  check_launch("sum of squares");
}

}  // namespace fl
