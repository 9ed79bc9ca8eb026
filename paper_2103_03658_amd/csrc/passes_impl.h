// FFT pass kernels of the circulant-embedded multilevel Toeplitz product
//   y = Re IDFT_M( lambda-hat * DFT_M( zero-pad(u) ) ) restricted to [0,n)^d
// (the fast product that the Toeplitz structure of A^(1), A^(2) allows,
// Sec. 2.1 and 2.2).  Included by one translation unit per precision.
//
// Data layout (row-major, last index fastest, RHS-major):
//   u, y          [nrhs][n]^d                 real
//   T1 (2D, 3D)   [nrhs][M/2+1][n^(d-1)]      complex, after the axis-0 pass
//   T2 (3D)       [nrhs][M/2+1][M][n]         complex, after the axis-1 pass
// The axis-0 pass packs two real columns into one complex line and splits
// the result by Hermitian symmetry, so only rows 0..M/2 of the axis-0
// frequency exist (the product of a real input with the real, even symbol
// keeps that symmetry, which the last pass uses to rebuild the other half).
//
// The strided (axis-0 and axis-1) passes run on a one-dimensional grid whose
// block order is permuted so that each of the eight XCDs of the chip works
// on a contiguous range of column tiles: neighbouring tiles share cache
// lines, and this keeps them in one XCD's L2.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <unordered_set>

#include "fl_device.h"
#include "fl_internal.h"

namespace fl {

// ---------------------------------------------------------------------------
// reductions (fixed order: results do not depend on timing)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block sum; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  v = wave_sum(v);
  __syncthreads();
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  double s = 0.0;
  if (tid < 64) {
    s = tid < nw ? sh[tid] : 0.0;
    s = wave_sum(s);
  }
  return s;
}

// Sum of nb per-block partials written by an earlier kernel, in a fixed
// order, returned to every thread of the block: 64 strided sums, then the
// pairwise tree of wave_sum.  Blocks narrower than a wave (strided passes of
// short lines) form the same 64 sums and the same tree in LDS, so the result
// has the same bits for every block size.  sh holds 64 doubles.
__device__ __forceinline__ double sum_partials(const double* part, int nb, double* sh) {
  if (blockDim.x >= 64) {
    if (threadIdx.x < 64) {
      double v = 0.0;
      for (int i = threadIdx.x; i < nb; i += 64) v += part[i];
      v = wave_sum(v);
      if (threadIdx.x == 0) sh[0] = v;
    }
  } else {
    for (int l = threadIdx.x; l < 64; l += blockDim.x) {
      double v = 0.0;
      for (int i = l; i < nb; i += 64) v += part[i];
      sh[l] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0)
      for (int off = 32; off > 0; off >>= 1)
        for (int l = 0; l < off; ++l) sh[l] += sh[l + off];
  }
  __syncthreads();
  const double t = sh[0];
  __syncthreads();
  return t;
}

// Start of a CG iteration for RHS o (every block of the first pass runs it
// and reaches the same decision).  Returns true if the RHS stops here;
// `lead` is true for exactly one block of the RHS, which records the state.
__device__ __forceinline__ bool cg_begin(const CgScalars& cg, int o, bool lead, double* sh,
                                         double* beta) {
  const double rho = sum_partials(cg.part_b + (long)o * cg.max_blocks, cg.nb_b, sh);
  const double rr =
      cg.precond ? sum_partials(cg.part_c + (long)o * cg.max_blocks, cg.nb_c, sh) : rho;
  const int it = cg.iters[o];
  bool stop = false, pending = false;
  int status = 0;
  double b = 0.0;
  if (!isfinite(rr) || !isfinite(rho)) {
    stop = true;
    status = 6;
  } else if (it == 0) {
    stop = rr == 0.0;
  } else if (cg.rel_trig &&
             (!(rr >= cg.rel_delta2 * cg.rel_last[o]) || rr <= cg.rel_tol2 * cg.rel_f2[o])) {
    stop = pending = true;   // wait for the reliable update
  } else if (rr <= cg.thresh2[o]) {
    stop = true;
  } else if (it >= cg.maxiter) {
    stop = true;
    status = 5;
  } else if (!(rho > 0.0)) {
    stop = true;   // r.z <= 0: the preconditioned iteration broke down
    status = 6;
  } else {
    b = rho / cg.rr_prev[o];
  }
  if (lead && threadIdx.x == 0) {
    cg.rr_cur[o] = rho;
    cg.res2[o] = rr;
    if (cg.rel_trig) cg.rel_trig[o] = pending ? 1 : 0;
    if (it == 0) cg.thresh2[o] = cg.tol2 * rr;
    if (stop) {
      cg.active[o] = 0;
      cg.status[o] = status;
      atomicSub(cg.n_active, 1);
    }
  }
  *beta = b;
  return stop;
}

// The iteration start split in two for the tau-preconditioned CG (the
// decisions and state of cg_begin, in its order).  cg_stop_rr runs at the
// end of an iteration, in the pass that starts z = P r: the tests on r.r
// (non-finite, r_0 = 0, the reliable-update trigger, the tolerance,
// maxiter), so that a right-hand side that stops is not preconditioned
// again.  cg_beta_rho runs in the pass that finishes z: the tests on r.z
// (non-finite, r.z <= 0 after the first iteration) and beta.
__device__ __forceinline__ bool cg_stop_rr(const CgScalars& cg, int o, bool lead, double* sh) {
  const double rr = sum_partials(cg.part_c + (long)o * cg.max_blocks, cg.nb_c, sh);
  const int it = cg.iters[o];
  bool stop = false, pending = false;
  int status = 0;
  if (!isfinite(rr)) {
    stop = true;
    status = 6;
  } else if (it == 0) {
    stop = rr == 0.0;
  } else if (cg.rel_trig &&
             (!(rr >= cg.rel_delta2 * cg.rel_last[o]) || rr <= cg.rel_tol2 * cg.rel_f2[o])) {
    stop = pending = true;   // wait for the reliable update
  } else if (rr <= cg.thresh2[o]) {
    stop = true;
  } else if (it >= cg.maxiter) {
    stop = true;
    status = 5;
  }
  if (lead && threadIdx.x == 0) {
    cg.res2[o] = rr;
    if (cg.rel_trig) cg.rel_trig[o] = pending ? 1 : 0;
    if (it == 0) cg.thresh2[o] = cg.tol2 * rr;
    if (stop) {
      cg.active[o] = 0;
      cg.status[o] = status;
      atomicSub(cg.n_active, 1);
    }
  }
  return stop;
}

__device__ __forceinline__ bool cg_beta_rho(const CgScalars& cg, int o, bool lead, double* sh,
                                            double* beta) {
  const double rho = sum_partials(cg.part_b + (long)o * cg.max_blocks, cg.nb_b, sh);
  const int it = cg.iters[o];
  bool stop = false;
  double b = 0.0;
  if (!isfinite(rho)) {
    stop = true;
  } else if (it > 0) {
    if (!(rho > 0.0)) stop = true;   // r.z <= 0: the preconditioned iteration broke down
    else b = rho / cg.rr_prev[o];
  }
  if (lead && threadIdx.x == 0) {
    cg.rr_cur[o] = rho;
    if (stop) {
      cg.active[o] = 0;
      cg.status[o] = 6;
      atomicSub(cg.n_active, 1);
    }
  }
  *beta = b;
  return stop;
}

// Logical (tile, outer) of this block: hardware places block b on XCD b % 8;
// XCD x is given the contiguous logical range starting at x*q + min(x, r).
__device__ __forceinline__ void xcd_tile(long ntiles, long& tile, long& outer) {
  const long nb = gridDim.x, b = blockIdx.x;
  const long x = b & 7, k = b >> 3, q = nb >> 3, r = nb & 7;
  const long l = x * q + (x < r ? x : r) + k;
  tile = l % ntiles;
  outer = l / ntiles;
}

// ---------------------------------------------------------------------------
// Strided passes (axis 0; 3D axis 1).  A block owns a tile of W lines (W
// column pairs in the real passes, W complex columns in the complex pass).
// Global memory is read and written cooperatively in row segments of the
// tile (consecutive threads on consecutive columns), staged through the
// lines' LDS planes; the transforms themselves run line-major (TPL
// consecutive threads per line), so that a wave's LDS traffic stays inside
// one line.  Inputs are zero at index >= M/2 and only outputs below M/2 are
// kept (the embedded data occupies n <= M/2 - 1 rows): those register slots
// are compile-time zeros / never computed.
// ---------------------------------------------------------------------------
template <typename T>
struct FirstArgs {
  const T* u;            // input
  const int* active;     // per RHS, may be null
  cx<T>* out;
  long C;                // real columns per RHS (n^(d-1))
  long in_os;            // elements between RHS in u
  long out_os;           // complex elements between RHS in out
  long ntiles;           // column-pair tiles per RHS
  int n_in;              // rows of input (n <= M/2)
  int W, lw;             // lines per block, log2(W)
  int PO, LS;            // LDS plane offset and line stride (elements)
  const cx<T>* tw;
};

// Transform of one line held in LDS planes (natural order) and write-back in
// natural order of the outputs (only those below M/2 if PRUNE_OUT).  IN: 0
// every input is read; 1 inputs at index >= M/2 are zero; 2 the line is the
// odd extension of its lower half (input at e >= M/2 is -input[M - e], zero
// at M/2), of which only the lower half is in LDS.
template <typename T, int M, int E, int DIR, int IN, bool PRUNE_OUT>
__device__ __forceinline__ void line_in_lds(T* lre, T* lim, int t, const cx<T>* tw) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  cx<T> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = t + j * TPL;
    if (IN == 0 || j < E / 2) {
      const int i = P::pad(e);
      v[j] = {lre[i], lim[i]};
    } else if (IN == 1) {
      v[j] = {0, 0};
    } else {
      const int i = P::pad(M - e);
      v[j] = e == M / 2 ? cx<T>{0, 0} : cx<T>{-lre[i], -lim[i]};
    }
  }
  fft_line<T, M, E, DIR>(v, lre, lim, t, tw);
  __syncthreads();
#pragma unroll
  for (int sl = 0; sl < E; ++sl) {
    if (!PRUNE_OUT || P::jslot(sl) < E / 2) {
      const int i = P::pad(t + TPL * P::jslot(sl));
      lre[i] = v[sl].x;
      lim[i] = v[sl].y;
    }
  }
}

// The same with one exchange plane, lre[0, M + M/E): the line's lower halves
// at lre (real) and lim (imaginary) lie inside it (tile_lds_half), and the
// transform overwrites them after every lane has read its inputs (the
// exchange begins with a barrier).  Only the lower half of the outputs.
template <typename T, int M, int E, int DIR, int IN>
__device__ __forceinline__ void line_in_lds_half(T* lre, T* lim, int t, const cx<T>* tw) {
  static_assert(IN == 1 || IN == 2, "the inputs' upper half is zero or mirrored");
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  cx<T> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = t + j * TPL;
    if (j < E / 2) {
      const int i = P::pad(e);
      v[j] = {lre[i], lim[i]};
    } else if (IN == 1) {
      v[j] = {0, 0};
    } else {
      const int i = P::pad(M - e);
      v[j] = e == M / 2 ? cx<T>{0, 0} : cx<T>{-lre[i], -lim[i]};
    }
  }
  fft_line_1p<T, M, E, DIR>(v, lre, t, tw);
  __syncthreads();
#pragma unroll
  for (int sl = 0; sl < E; ++sl) {
    if (P::jslot(sl) < E / 2) {
      const int i = P::pad(t + TPL * P::jslot(sl));
      lre[i] = v[sl].x;
      lim[i] = v[sl].y;
    }
  }
}

// Hermitian split of the tile's W packed line pairs (transformed in the LDS
// planes) into rows k = 0..M/2 of the axis-0 frequency, row segments of 2W
// complex values: X_a = (Z_k + conj Z_{M-k})/2, X_b = (Z_k - conj Z_{M-k})/(2i).
// out points at (rhs, row 0, first column of the tile); rows are C apart.
template <typename T, int M, int E>
__device__ __forceinline__ void hermitian_split_out(const T* lds, cx<T>* out, long C, int W,
                                                    int lw, int PO, int LS, int ncol) {
  using P = Plan<M, E>;
  const int nthr = W * P::TPL;
  const T half = (T)0.5;
  const int tot3 = (M / 2 + 1) * W;   // E/2 full rounds and a partial one
#pragma unroll
  for (int j = 0; j <= E / 2; ++j) {
    const int e = threadIdx.x + j * nthr;
    const int k = e >> lw, l = e & (W - 1);
    if (e >= tot3 || 2 * l >= ncol) continue;
    const T* re = lds + l * LS;
    const T* im = re + PO;
    const int km = (M - k) & (M - 1);
    const cx<T> z = {re[P::pad(k)], im[P::pad(k)]};
    const cx<T> zm = {re[P::pad(km)], im[P::pad(km)]};
    const long oi = (long)k * C + 2 * l;
    out[oi] = {(z.x + zm.x) * half, (z.y - zm.y) * half};
    if (2 * l + 1 < ncol) out[oi + 1] = {(z.y + zm.y) * half, (zm.x - z.x) * half};
  }
}

template <typename T, int M, int E>
__global__ void __launch_bounds__(512) k_first(FirstArgs<T> a) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  long tile, ol;
  xcd_tile(a.ntiles, tile, ol);
  const int o = (int)ol;
  if (a.active && !a.active[o]) return;
  const int lw1 = a.lw + 1, W2 = 2 * a.W;
  const int nthr = a.W * TPL;
  const long col0 = tile * W2;
  const long cl = a.C - col0;
  const int ncol = cl < W2 ? (int)cl : W2;
  // rows [0, M/2) of the tile into the planes (rows >= n_in are zero):
  // (M/2) * 2W elements, exactly E per thread, all loads issued first
  {
    const long ib = (long)o * a.in_os + col0;
    T x[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = threadIdx.x + j * nthr;
      const int row = e >> lw1, cc = e & (W2 - 1);
      x[j] = (row < a.n_in && cc < ncol) ? a.u[ib + (long)row * a.C + cc] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = threadIdx.x + j * nthr;
      const int row = e >> lw1, cc = e & (W2 - 1);
      lds[(cc >> 1) * a.LS + (cc & 1) * a.PO + P::pad(row)] = x[j];
    }
  }
  __syncthreads();
  {
    const int l = threadIdx.x / TPL, t = threadIdx.x % TPL;
    T* lre = lds + l * a.LS;
    line_in_lds<T, M, E, -1, 1, false>(lre, lre + a.PO, t, a.tw);
  }
  __syncthreads();
  hermitian_split_out<T, M, E>(lds, a.out + (long)o * a.out_os + col0, a.C, a.W, a.lw, a.PO,
                               a.LS, ncol);
}

// ---------------------------------------------------------------------------
// last pass (axis 0, strided): rows 0..M/2 (Hermitian half) -> real pairs
// ---------------------------------------------------------------------------
template <typename T>
struct LastArgs {
  const cx<T>* in;
  T* y;
  const T* p;            // PM_CG / PM_DOT: dot partner
  const double* f;       // PM_RESID: right-hand side (FP64)
  const int* active;
  double* part;          // PM_CG / PM_DOT / PM_RESID: per-block partials [nrhs][max_blocks]
  int max_blocks;
  long C;                // real columns per RHS
  long in_os;            // complex elements between RHS of in
  long y_os;             // elements between RHS of y / p / f
  long ntiles;
  int n_out;             // rows of output (n <= M/2)
  int W, lw;
  int PO, LS;
  int mode;
  const cx<T>* tw;
};

template <typename T, int M, int E>
__global__ void __launch_bounds__(512) k_last(LastArgs<T> a) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[64];
  T* lds = reinterpret_cast<T*>(smem_raw);
  long tile, ol;
  xcd_tile(a.ntiles, tile, ol);
  const int o = (int)ol;
  if (a.active && !a.active[o]) return;
  const int lw1 = a.lw + 1, W2 = 2 * a.W;
  const int nthr = a.W * TPL;
  const long col0 = tile * W2;
  const long cl = a.C - col0;
  const int ncol = cl < W2 ? (int)cl : W2;
  // rows k = 0..M/2 of both halves of each pair: line input Y_a + i Y_b at
  // k, and its Hermitian image conj(Y_a) + i conj(Y_b) at M - k
  {
    const long ib = (long)o * a.in_os + col0;
    const int tot1 = (M / 2 + 1) * a.W;   // E/2 full rounds and a partial one
    cx<T> ya_[E / 2 + 1], yb_[E / 2 + 1];
#pragma unroll
    for (int j = 0; j <= E / 2; ++j) {
      const int e = threadIdx.x + j * nthr;
      const int k = e >> a.lw, l = e & (a.W - 1);
      ya_[j] = {0, 0};
      yb_[j] = {0, 0};
      const long ii = ib + (long)k * a.C + 2 * l;
      if (e < tot1 && 2 * l < ncol) ya_[j] = a.in[ii];
      if (e < tot1 && 2 * l + 1 < ncol) yb_[j] = a.in[ii + 1];
    }
#pragma unroll
    for (int j = 0; j <= E / 2; ++j) {
      const int e = threadIdx.x + j * nthr;
      if (e >= tot1) continue;
      const int k = e >> a.lw, l = e & (a.W - 1);
      const cx<T> ya = ya_[j], yb = yb_[j];
      T* re = lds + l * a.LS;
      T* im = re + a.PO;
      re[P::pad(k)] = ya.x - yb.y;
      im[P::pad(k)] = ya.y + yb.x;
      if (k > 0 && k < M / 2) {
        re[P::pad(M - k)] = ya.x + yb.y;
        im[P::pad(M - k)] = yb.x - ya.y;
      }
    }
  }
  __syncthreads();
  {
    const int l = threadIdx.x / TPL, t = threadIdx.x % TPL;
    T* lre = lds + l * a.LS;
    line_in_lds<T, M, E, +1, 0, true>(lre, lre + a.PO, t, a.tw);
  }
  __syncthreads();
  double acc = 0.0;
  const long yb0 = (long)o * a.y_os + col0;
  const int tot3 = a.n_out * W2;   // at most (M/2) * 2W: E rounds
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = threadIdx.x + j * nthr;
    const int row = e >> lw1, cc = e & (W2 - 1);
    if (e >= tot3 || cc >= ncol) continue;
    const T v = lds[(cc >> 1) * a.LS + (cc & 1) * a.PO + P::pad(row)];
    const long i = yb0 + (long)row * a.C + cc;
    if (a.mode == PM_RESID) {
      const double r = a.f[i] - (double)v;
      a.y[i] = (T)r;
      acc += r * r;
    } else {
      a.y[i] = v;
      if (a.mode == PM_CG || a.mode == PM_DOT) acc += (double)a.p[i] * (double)v;
    }
  }
  if (a.mode == PM_PLAIN) return;
  const double blk = block_sum(acc, red);
  if (threadIdx.x == 0) a.part[(long)o * a.max_blocks + tile] = blk;
}

// ---------------------------------------------------------------------------
// strided complex-to-complex pass (3D axis 1; symbol construction)
// ---------------------------------------------------------------------------
template <typename T>
struct C2CArgs {
  const cx<T>* in;
  cx<T>* out;
  const int* active;     // per RHS (outer index / outer_per_rhs), may be null
  long C;                // complex columns
  long in_os, in_rs;     // per outer slice / per row (complex elements)
  long out_os, out_rs;
  long ntiles;
  int outer_per_rhs;
  int n_in, n_out;
  int W, lw;
  int PO, LS;
  const cx<T>* tw;
};

// PR: 0 full transform, 1 inputs >= M/2 zero (n_in <= M/2), 2 outputs below
// M/2 only (n_out <= M/2).
template <typename T, int M, int E, int DIR, int PR>
__global__ void __launch_bounds__(512) k_c2c(C2CArgs<T> a) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  constexpr int ROWS_IN = PR == 1 ? M / 2 : M;
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  long tile, o;
  xcd_tile(a.ntiles, tile, o);
  if (a.active && !a.active[o / a.outer_per_rhs]) return;
  const int nthr = a.W * TPL;
  const long col0 = tile * a.W;
  const long cl = a.C - col0;
  const int ncol = cl < a.W ? (int)cl : a.W;
  {
    // ROWS_IN * W elements: exactly ROWS_IN / TPL per thread
    constexpr int J = ROWS_IN / TPL;
    const long ib = o * a.in_os + col0;
    cx<T> x[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int e = threadIdx.x + j * nthr;
      const int row = e >> a.lw, l = e & (a.W - 1);
      x[j] = {0, 0};
      if (row < a.n_in && l < ncol) x[j] = a.in[ib + (long)row * a.in_rs + l];
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int e = threadIdx.x + j * nthr;
      const int row = e >> a.lw, l = e & (a.W - 1);
      T* re = lds + l * a.LS;
      re[P::pad(row)] = x[j].x;
      re[a.PO + P::pad(row)] = x[j].y;
    }
  }
  __syncthreads();
  {
    const int l = threadIdx.x / TPL, t = threadIdx.x % TPL;
    T* lre = lds + l * a.LS;
    line_in_lds<T, M, E, DIR, PR == 1 ? 1 : 0, PR == 2>(lre, lre + a.PO, t, a.tw);
  }
  __syncthreads();
  const long obase = o * a.out_os + col0;
  const int tot3 = a.n_out * a.W;   // at most ROWS_OUT * W
  constexpr int ROWS_OUT = PR == 2 ? M / 2 : M;
#pragma unroll
  for (int j = 0; j < ROWS_OUT / TPL; ++j) {
    const int e = threadIdx.x + j * nthr;
    const int row = e >> a.lw, l = e & (a.W - 1);
    if (e >= tot3 || l >= ncol) continue;
    const T* re = lds + l * a.LS;
    a.out[obase + (long)row * a.out_rs + l] = {re[P::pad(row)], re[a.PO + P::pad(row)]};
  }
}

// ---------------------------------------------------------------------------
// middle pass (last axis, contiguous): forward, symbol multiply, inverse
// ---------------------------------------------------------------------------
template <typename T>
struct MidArgs {
  cx<T>* data;
  const T* lam;          // folded symbol, Ha[0] x .. x Ha[d-1]
  const int* active;
  long rows;             // lines per RHS
  long o_stride;         // complex elements between RHS
  long row_stride;       // complex elements between lines
  int n_in, n_out;
  int Hl;                // folded symbol length of the last axis (M/2 + 1)
  int H1, M1;            // 3D: folded symbol length and embedding length of axis 1
  int d;
  int LPB;
  int nrhs;
  const cx<T>* tw;
};

// FP64 radix-16 lines fit 168 registers, which allows three waves per SIMD
// (the compiler's own choice keeps two at some lengths).  At 1024 points
// they fit 128 (four waves), but measured slower: 39.1 -> 40.9 us on the
// 511^2 batch.
template <typename T, int M, int E>
__global__ void __launch_bounds__(512, (E == 16 && sizeof(T) == 8) ? 3 : 1)
    k_mid(MidArgs<T> a) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  // right-hand side fastest within each XCD's contiguous range of blocks:
  // all RHS of a row block run close together and share its symbol rows in
  // that XCD's L2
  long ol, rb;
  xcd_tile(a.nrhs, ol, rb);
  const int o = (int)ol;
  if (a.active && !a.active[o]) return;
  const int l = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long line = rb * a.LPB + l;
  const bool h = line < a.rows;
  T* l1 = lds + (long)l * P::LDSN;
  cx<T>* base = a.data + (long)o * a.o_stride + (h ? line : 0) * a.row_stride;
  cx<T> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int i = t + j * TPL;   // n_in <= M/2: slots j >= E/2 are zero
    v[j] = (j < E / 2 && h && i < a.n_in) ? base[i] : cx<T>{0, 0};
  }
  fft_line_1p<T, M, E, -1>(v, l1, t, a.tw);
  // symbol row of this line
  long lrow = 0;
  if (h) {
    if (a.d == 3) {
      const long k0 = line / a.M1, k1 = line % a.M1;
      lrow = (k0 * a.H1 + (k1 <= a.M1 / 2 ? k1 : a.M1 - k1)) * a.Hl;
    } else if (a.d == 2) {
      lrow = line * a.Hl;
    }
  }
  const T* lr = a.lam + lrow;
#pragma unroll
  for (int sl = 0; sl < E; ++sl) {
    const int k = t + TPL * P::jslot(sl);
    const T s = lr[k <= M / 2 ? k : M - k];
    v[sl] = cscale(v[sl], s);
  }
  to_natural<T, M, E>(v);
  // The second transform takes the lane index through an empty asm: with
  // the same index the compiler shares the two transforms' LDS and twiddle
  // index arithmetic and keeps it in registers across the symbol multiply
  // (FP64 E = 16: 166 -> 134 registers, FP32: 120 -> 92, five waves).
  int t2 = t;
  asm volatile("" : "+v"(t2));
  fft_line_1p<T, M, E, +1>(v, l1, t2, a.tw);
#pragma unroll
  for (int sl = 0; sl < E; ++sl) {
    const int i = t + TPL * P::jslot(sl);   // n_out <= M/2
    if (P::jslot(sl) < E / 2 && h && i < a.n_out) base[i] = v[sl];
  }
}

// contiguous transform of full lines in place (symbol construction, exterior
// term); DIR -1 forward, +1 inverse (unnormalised)
template <typename T, int M, int E, int DIR>
__global__ void __launch_bounds__(512) k_rows(cx<T>* data, long rows, int LPB,
                                              const cx<T>* tw) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const int l = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long line = (long)blockIdx.x * LPB + l;
  const bool h = line < rows;
  T* lre = lds + (long)l * 2 * P::LDSN;
  T* lim = lre + P::LDSN;
  cx<T>* base = data + (h ? line : 0) * (long)M;
  cx<T> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = h ? base[t + j * TPL] : cx<T>{0, 0};
  fft_line<T, M, E, DIR>(v, lre, lim, t, tw);
#pragma unroll
  for (int sl = 0; sl < E; ++sl)
    if (h) base[t + TPL * P::jslot(sl)] = v[sl];
}

// ---------------------------------------------------------------------------
// 1D: one right-hand side per line (imaginary part zero, so its bits do not
// depend on which other right-hand sides share the launch); the whole
// product, and in CG mode the whole iteration start, in one block.
// ---------------------------------------------------------------------------
template <typename T>
struct Line1Args {
  const T* u;
  T* y;
  T* p;
  const T* r;
  const double* f;
  const int* active;
  CgScalars cg;
  double* part;          // PM_CG / PM_DOT / PM_RESID partials, one per RHS
  int max_blocks;
  const T* lam;
  int n;
  int nrhs;
  int mode;
  const cx<T>* tw;
};

// ODD: the line is the odd extension of the n values (no PM_CG then).
template <typename T, int M, int E, bool ODD>
__global__ void __launch_bounds__(512) k_line1d(Line1Args<T> a) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[64];
  T* lds = reinterpret_cast<T*>(smem_raw);
  T* lre = lds;
  T* lim = lds + P::LDSN;
  const int t = threadIdx.x;
  const int o = blockIdx.x;
  if (a.active && !a.active[o]) return;
  T bt = 0;
  if (a.mode == PM_CG) {
    double beta;
    if (cg_begin(a.cg, o, true, red, &beta)) return;
    bt = (T)beta;
  }
  const long n = a.n;
  const long base = (long)o * n;
  cx<T> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int i = t + j * TPL;   // n <= M/2: slots j >= E/2 are zero
    T re = 0;
    if constexpr (ODD) {
      if (j < E / 2) {
        if (i >= 1 && i - 1 < n) re = a.u[base + i - 1];
      } else if (i != M / 2 && M - i - 1 < n) {
        re = -a.u[base + M - i - 1];
      }
    } else if (j < E / 2 && i < n) {
      if (a.mode == PM_CG) {
        re = a.r[base + i] + bt * a.p[base + i];
        a.p[base + i] = re;
      } else {
        re = a.u[base + i];
      }
    }
    v[j] = {re, (T)0};
  }
  fft_line<T, M, E, -1>(v, lre, lim, t, a.tw);
#pragma unroll
  for (int sl = 0; sl < E; ++sl) {
    const int k = t + TPL * P::jslot(sl);
    v[sl] = cscale(v[sl], a.lam[k <= M / 2 ? k : M - k]);
  }
  to_natural<T, M, E>(v);
  fft_line<T, M, E, +1>(v, lre, lim, t, a.tw);
  double acc = 0.0;
#pragma unroll
  for (int sl = 0; sl < E; ++sl) {
    const int i = t + TPL * P::jslot(sl) - (ODD ? 1 : 0);
    if (P::jslot(sl) < E / 2 && i >= 0 && i < n) {
      if (a.mode == PM_RESID) {
        const double q = a.f[base + i] - (double)v[sl].x;
        a.y[base + i] = (T)q;
        acc += q * q;
      } else {
        a.y[base + i] = v[sl].x;
        if (a.mode == PM_CG) acc += (double)a.p[base + i] * (double)v[sl].x;
        if (a.mode == PM_DOT) acc += (double)a.u[base + i] * (double)v[sl].x;
      }
    }
  }
  if (a.mode == PM_PLAIN) return;
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) a.part[(long)o * a.max_blocks] = tot;
}

// ---------------------------------------------------------------------------
// 1D FP64 PCG in one workgroup per right-hand side: the line fits the block,
// so the whole solve runs in one launch, with x, r, p, z in LDS.  The
// iteration and its decisions are those of the multi-kernel solve (cg_begin
// at every iteration start, breakdown when p.q <= 0, the same update).
// ---------------------------------------------------------------------------
struct Cg1Args {
  const double* f;       // [nrhs][n]
  double* x;             // [nrhs][n], the final iterate
  const double* lam;     // folded symbol of A, M/2 + 1 values
  const double* pcs;     // folded preconditioner multiplier, or null (plain CG)
  int pc_odd;            // the tau preconditioner (odd extension), else zero padding
  CgScalars cg;          // iters, status, res2, active per RHS
  int n;
  int maxiter;
  double tol2;
  const cx<double>* tw;
};

// Block sum returned to every thread (slot 15 of red carries the broadcast).
__device__ __forceinline__ double block_sum_all(double v, double* red) {
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) red[15] = s;
  __syncthreads();
  const double r = red[15];
  __syncthreads();
  return r;
}

// The transform y = F^-1 diag(sym) F of the n values `in` (LDS), zero-padded
// or odd-extended to M, into the slots of v: y_i sits in slot sl with
// i = t + TPL jslot(sl) - ODD, jslot(sl) < E/2, 0 <= i < n.
template <int M, int E, bool ODD>
__device__ __forceinline__ void line1_apply(const double* in, int n, const double* sym,
                                            cx<double> (&v)[E], double* lre, double* lim, int t,
                                            const cx<double>* tw) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int i = t + j * TPL;
    double re = 0.0;
    if constexpr (ODD) {
      if (j < E / 2) {
        if (i >= 1 && i - 1 < n) re = in[i - 1];
      } else if (i != M / 2 && M - i - 1 < n) {
        re = -in[M - i - 1];
      }
    } else if (j < E / 2 && i < n) {
      re = in[i];
    }
    v[j] = {re, 0.0};
  }
  fft_line<double, M, E, -1>(v, lre, lim, t, tw);
#pragma unroll
  for (int sl = 0; sl < E; ++sl) {
    const int k = t + TPL * P::jslot(sl);
    v[sl] = cscale(v[sl], sym[k <= M / 2 ? k : M - k]);
  }
  to_natural<double, M, E>(v);
  fft_line<double, M, E, +1>(v, lre, lim, t, tw);
}

// z = P r into Z (LDS); returns r.z (every thread).
template <int M, int E>
__device__ __forceinline__ double line1_precond(const Cg1Args& a, const double* R, double* Z,
                                                cx<double> (&v)[E], double* lre, double* lim,
                                                int t, double* red) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  const int n = a.n;
  double acc = 0.0;
  if (!a.pcs) {
    for (int i = t; i < n; i += TPL) {
      Z[i] = R[i];
      acc += R[i] * R[i];
    }
    return block_sum_all(acc, red);
  }
  if (a.pc_odd) {
    line1_apply<M, E, true>(R, n, a.pcs, v, lre, lim, t, a.tw);
  } else {
    line1_apply<M, E, false>(R, n, a.pcs, v, lre, lim, t, a.tw);
  }
  const int sh = a.pc_odd ? 1 : 0;
#pragma unroll
  for (int sl = 0; sl < E; ++sl) {
    const int i = t + TPL * P::jslot(sl) - sh;
    if (P::jslot(sl) < E / 2 && i >= 0 && i < n) {
      Z[i] = v[sl].x;
      acc += R[i] * v[sl].x;
    }
  }
  return block_sum_all(acc, red);
}

template <int M, int E>
__global__ void __launch_bounds__(512) k_cg1d(Cg1Args a) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[64];
  double* lre = reinterpret_cast<double*>(smem_raw);
  double* lim = lre + P::LDSN;
  double* X = lim + P::LDSN;
  double* R = X + M / 2;
  double* Pv = R + M / 2;
  double* Z = Pv + M / 2;
  const int t = threadIdx.x, o = blockIdx.x, n = a.n;
  const double* f = a.f + (long)o * n;
  cx<double> v[E];
  double acc = 0.0;
  for (int i = t; i < n; i += TPL) {
    const double fi = f[i];
    R[i] = fi;
    X[i] = 0.0;
    Pv[i] = 0.0;
    acc += fi * fi;
  }
  __syncthreads();
  double rr = block_sum_all(acc, red);
  double rz = line1_precond<M, E>(a, R, Z, v, lre, lim, t, red);
  const double thresh2 = a.tol2 * rr;
  double rz_prev = 0.0;
  int it = 0, status = 0;
  for (;;) {
    // iteration start (the order of cg_begin's tests)
    if (!isfinite(rr) || !isfinite(rz)) {
      status = 6;
      break;
    }
    if (it == 0) {
      if (rr == 0.0) break;
    } else if (rr <= thresh2) {
      break;
    } else if (it >= a.maxiter) {
      status = 5;
      break;
    } else if (!(rz > 0.0)) {
      status = 6;
      break;
    }
    const double beta = it == 0 ? 0.0 : rz / rz_prev;
    for (int i = t; i < n; i += TPL) Pv[i] = Z[i] + beta * Pv[i];
    __syncthreads();
    // q = A p in the slots; p.q
    line1_apply<M, E, false>(Pv, n, a.lam, v, lre, lim, t, a.tw);
    acc = 0.0;
#pragma unroll
    for (int sl = 0; sl < E; ++sl) {
      const int i = t + TPL * P::jslot(sl);
      if (P::jslot(sl) < E / 2 && i < n) acc += Pv[i] * v[sl].x;
    }
    const double pq = block_sum_all(acc, red);
    const double alpha = rz / pq;
    if (!(pq > 0.0) || !isfinite(alpha)) {
      status = 6;
      break;
    }
    acc = 0.0;
#pragma unroll
    for (int sl = 0; sl < E; ++sl) {
      const int i = t + TPL * P::jslot(sl);
      if (P::jslot(sl) < E / 2 && i < n) {
        X[i] += alpha * Pv[i];
        const double ri = R[i] - alpha * v[sl].x;
        R[i] = ri;
        acc += ri * ri;
      }
    }
    rr = block_sum_all(acc, red);   // its barriers also publish X and R
    ++it;
    rz_prev = rz;
    rz = line1_precond<M, E>(a, R, Z, v, lre, lim, t, red);
  }
  for (int i = t; i < n; i += TPL) a.x[(long)o * n + i] = X[i];
  if (t == 0) {
    a.cg.iters[o] = it;
    a.cg.status[o] = status;
    a.cg.res2[o] = rr;
    a.cg.active[o] = 0;
  }
}


// ---------------------------------------------------------------------------
// Real sine passes (the tau preconditioner of the CG solves: the natural
// tau approximation of A is diagonalised by the sine transform of every
// axis).  For a real line x_1..x_n (n = N - 1, M = 2N)
// the length-M DFT of its odd extension (0, x_1..x_n, 0, -x_n..-x_1) is
// -2i S x with (S x)_k = sum_j x_j sin(pi j k / N).  Two real lines a, b
// packed as a + i b therefore give Z = 2 S b - 2i S a: sigma(a) := -2 S a =
// Im Z and sigma(b) = -Re Z come out without a Hermitian split, and every
// intermediate stays real, n values per line (half the bytes of a complex
// half spectrum, whose real part would be zero).  The preconditioner is
// sigma_0 .. sigma_{d-1} diag(m) sigma_{d-1} .. sigma_0 = 2^{2d} S diag(m) S.
// ---------------------------------------------------------------------------
template <typename T>
struct SineArgs {
  const T* in;
  T* out;                // may equal in: a block owns whole columns
  const T* partner;      // dot != 0: partials of partner . out
  const int* active;     // per RHS (outer index / outer_per_rhs), may be null
  double* part;          // dot != 0: [nrhs][max_blocks]
  int max_blocks;
  long C;                // real columns per outer slice (= row stride)
  long os;               // elements between outer slices
  long ntiles;           // column-pair tiles per outer slice
  int outer_per_rhs;
  int n;                 // rows (= M/2 - 1)
  int W, lw;             // column pairs per block, log2(W)
  int PO, LS;
  int dot;
  const cx<T>* tw;
  // DIRF kernels (the last pass of the preconditioner fused with the next CG
  // iteration start): the search direction, updated in place, and the CG
  // state whose stopping test and beta every block evaluates first
  T* pdir;
  CgScalars cg;
  // FIRST kernels (DIRF too): the product's axis-0 forward pass of the new p
  // on the same tile, into T1 [nrhs][M/2+1][C] complex (t1_os per RHS)
  cx<T>* t1;
  long t1_os;
};

// Strided sine pass along the row axis of [outer][n][C]: each block owns 2W
// columns (W packed pairs), loads all n rows into the LDS planes (row e
// holds input row e - 1), transforms the odd-extended lines and writes
// sigma of each column.  DIRF: the pass that completes z = P r also starts
// the next CG iteration (cg_begin: stopping test and beta, the same decision
// in every block of the right-hand side) and writes p = z + beta p instead
// of z, so z is never stored (the old p is loaded with the input tile).
// FIRST: the tile's new p then goes on through the product's first pass
// (zero-padded forward transform along axis 0 and Hermitian split into T1),
// so that pass does not read p back.  STOP (the pass that starts z = P r):
// the end-of-iteration tests on r.r first (cg_stop_rr); DIRF then takes only
// the tests on r.z and beta (cg_beta_rho).
template <typename T, int M, int E, bool DIRF, bool FIRST, bool STOP>
__global__ void __launch_bounds__(512) k_sine_cols(SineArgs<T> a) {
  static_assert(DIRF || !FIRST, "the fused first pass follows the direction update");
  static_assert(!(DIRF && STOP), "one test per pass");
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[64];
  T* lds = reinterpret_cast<T*>(smem_raw);
  long tile, o;
  xcd_tile(a.ntiles, tile, o);
  if (a.active && !a.active[o / a.outer_per_rhs]) return;
  const int lw1 = a.lw + 1, W2 = 2 * a.W;
  const int nthr = a.W * TPL;
  const long col0 = tile * W2;
  const long cl = a.C - col0;
  const int ncol = cl < W2 ? (int)cl : W2;
  const long base = o * a.os + col0;
  const int tot = a.n * W2;
  // DIRF: the tile's loads are issued before the iteration tests, whose
  // partial sums then wait on them together; the old p is loaded after the
  // transform, so that it is not held in registers across it
  T pold[DIRF ? E : 1];
  if constexpr (STOP) {
    // only the right-hand side's lead block takes the decision; the others
    // transform their tiles anyway (nothing reads them if it stops).  The
    // test comes before the tile's loads: held across it, they cost every
    // block some 25 registers (a wave per SIMD)
    if (tile == 0 && cg_stop_rr(a.cg, (int)o, true, red)) return;
  }
  // rows [0, M/2) of the tile: (M/2) * 2W elements, exactly E per thread
  T x[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = threadIdx.x + j * nthr;
    const int row = e >> lw1, cc = e & (W2 - 1);
    const int src = row - 1;
    x[j] = (src >= 0 && src < a.n && cc < ncol) ? a.in[base + (long)src * a.C + cc] : (T)0;
  }
  T bt = 0;
  if constexpr (DIRF) {
    double beta;
    if (cg_beta_rho(a.cg, (int)o, tile == 0, red, &beta)) return;
    bt = (T)beta;
  }
  {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = threadIdx.x + j * nthr;
      const int row = e >> lw1, cc = e & (W2 - 1);
      lds[(cc >> 1) * a.LS + (cc & 1) * a.PO + P::pad(row)] = x[j];
    }
  }
  __syncthreads();
  {
    const int l = threadIdx.x / TPL, t = threadIdx.x % TPL;
    T* lre = lds + l * a.LS;
    if constexpr (DIRF)
      line_in_lds<T, M, E, -1, 2, true>(lre, lre + a.PO, t, a.tw);
    else
      line_in_lds_half<T, M, E, -1, 2>(lre, lre + a.PO, t, a.tw);
  }
  // the thread index of the tile's stores, opaque to the compiler: it then
  // forms their addresses here instead of keeping those of the loads in
  // registers across the transform
  int tx = threadIdx.x;
  asm volatile("" : "+v"(tx));
  if constexpr (DIRF) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = tx + j * nthr;
      const int row = e >> lw1, cc = e & (W2 - 1);
      pold[j] = (e < tot && cc < ncol) ? a.pdir[base + (long)row * a.C + cc] : (T)0;
    }
  }
  __syncthreads();
  // positions 1..n: first column of a pair from the imaginary plane, second
  // from the negated real plane
  double acc = 0.0;
  T pnew[FIRST ? E : 1];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = tx + j * nthr;
    const int row = e >> lw1, cc = e & (W2 - 1);
    if constexpr (FIRST) pnew[j] = 0;
    if (e >= tot || cc >= ncol) continue;
    const T* ln = lds + (cc >> 1) * a.LS + P::pad(row + 1);
    const T v = (cc & 1) ? -ln[0] : ln[a.PO];
    const long i = base + (long)row * a.C + cc;
    if constexpr (DIRF) {
      const T pv = v + bt * pold[j];
      a.pdir[i] = pv;
      if constexpr (FIRST) pnew[j] = pv;
    } else {
      a.out[i] = v;
      if (a.dot) acc += (double)a.partner[i] * (double)v;
    }
  }
  if constexpr (FIRST) {
    // the new p as the first pass's input tile: rows [0, M/2), zero from n on
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int e = tx + j * nthr;
      const int row = e >> lw1, cc = e & (W2 - 1);
      lds[(cc >> 1) * a.LS + (cc & 1) * a.PO + P::pad(row)] = pnew[j];
    }
    __syncthreads();
    {
      // opaque lane index: the index arithmetic of the sine transform above
      // is not kept for this one (FP64: 137 -> 116 registers, four waves)
      int tx3 = threadIdx.x;
      asm volatile("" : "+v"(tx3));
      const int l = tx3 / TPL, t = tx3 % TPL;
      T* lre = lds + l * a.LS;
      line_in_lds<T, M, E, -1, 1, false>(lre, lre + a.PO, t, a.tw);
    }
    __syncthreads();
    hermitian_split_out<T, M, E>(lds, a.t1 + o * a.t1_os + col0, a.C, a.W, a.lw, a.PO, a.LS,
                                 ncol);
    return;
  }
  if (DIRF || !a.dot) return;
  const double blk = block_sum(acc, red);
  if (threadIdx.x == 0) a.part[(o / a.outer_per_rhs) * a.max_blocks + tile] = blk;
}

template <typename T>
struct SineMidArgs {
  T* data;               // [nrhs][rows][n], transformed in place
  const T* m;            // folded multiplier, Ha[0] x .. x Ha[d-1]
  const int* active;
  long rows;             // lines per RHS (product of the other axes' n)
  long o_stride;         // elements between RHS
  int n;                 // line length (last axis)
  int n1;                // 3D: interior points of axis 1 (lines per axis-0 index)
  int Hl, H1;            // folded multiplier lengths of the last axis and of axis 1
  int d;
  int LPB;               // line pairs per block
  int nrhs;
  const cx<T>* tw;
  // dot != 0: partials of r.z = sum_k m_k sigma(r)_k^2 (z = sigma diag(m)
  // sigma r, sigma symmetric), one per block, into part[rhs][block]
  int dot;
  double* part;
  int max_blocks;
};

// Multiplier row of line L of the last axis: the frequencies of the other
// axes are k = (index along that axis) + 1.
// (L < n0 n1 <= 2047^2: 32-bit arithmetic; a 64-bit division here costs
// registers that the transforms need)
__device__ __forceinline__ long sine_mrow(long L, int n1, int H1, int Hl, int d) {
  const int l = (int)L;
  if (d == 3) return (long)((l / n1 + 1) * H1 + (l % n1 + 1)) * Hl;
  return (long)(l + 1) * Hl;
}

// Contiguous last-axis pass on pairs of lines: sigma, multiply each line by
// its own multiplier row, sigma again.  After the first transform slot k
// holds (-sigma(b)_k, sigma(a)_k); the second transform's packed input is
// (m_a sigma(a), m_b sigma(b)) = (m_a Z.y, -m_b Z.x), odd in k because Z is
// odd and the multiplier is even.
template <typename T, int M, int E>
__global__ void __launch_bounds__(512) k_sine_mid(SineMidArgs<T> a) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  long ol, rb;
  xcd_tile(a.nrhs, ol, rb);
  const int o = (int)ol;
  if (a.active && !a.active[o]) return;
  const int l = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const long la = 2 * (rb * a.LPB + l);
  const bool ha = la < a.rows, hb = la + 1 < a.rows;
  T* l1 = lds + (long)l * P::LDSN;
  T* pa = a.data + (long)o * a.o_stride + (ha ? la : 0) * a.n;
  T* pb = pa + a.n;   // dereferenced only if hb
  const int n = a.n;
  cx<T> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int i = t + j * TPL;
    const int src = j < E / 2 ? i - 1 : M - i - 1;   // i = 0 and i = M/2 give -1 and n
    const bool ok = src >= 0 && src < n;
    T xa = (ha && ok) ? pa[src] : (T)0;
    T xb = (hb && ok) ? pb[src] : (T)0;
    if (j >= E / 2) {
      xa = -xa;
      xb = -xb;
    }
    v[j] = {xa, xb};
  }
  fft_line_1p<T, M, E, -1>(v, l1, t, a.tw);
  const T* ma = a.m + (ha ? sine_mrow(la, a.n1, a.H1, a.Hl, a.d) : 0);
  const T* mb = a.m + (hb ? sine_mrow(la + 1, a.n1, a.H1, a.Hl, a.d) : 0);
  // The r.z sum is pinned after each quarter of the slots (an empty asm with
  // the sum as an in/out register): left to the compiler it is sunk to its
  // use after the second transform, which then holds the transformed values
  // across that transform, and the multiplier loads of all slots are issued
  // at once (FP64 E = 16: 256 registers with spills -> 150 with the opaque
  // lane index below, three waves).  The sum keeps its order.
  double acc = 0.0;
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
#pragma unroll
    for (int sl = qq * (E / 4); sl < (qq + 1) * (E / 4); ++sl) {
      const int k = t + TPL * P::jslot(sl);
      const int kk = k <= M / 2 ? k : M - k;
      const T sa = ha ? ma[kk] : (T)0;
      const T sb = hb ? mb[kk] : (T)0;
      // slots 1..n hold the sine coefficients (the others mirror them)
      if (k >= 1 && k <= n)
        acc += (double)sa * (double)v[sl].y * (double)v[sl].y +
               (double)sb * (double)v[sl].x * (double)v[sl].x;
      v[sl] = {sa * v[sl].y, -(sb * v[sl].x)};
    }
    asm volatile("" : "+v"(acc));
  }
  to_natural<T, M, E>(v);
  // opaque lane index for the second transform, as in k_mid (FP64 E = 8:
  // 148 -> 94 registers with the quarters above, five waves per SIMD)
  int t2 = t;
  asm volatile("" : "+v"(t2));
  fft_line_1p<T, M, E, -1>(v, l1, t2, a.tw);
#pragma unroll
  for (int sl = 0; sl < E; ++sl) {
    const int pos = t + TPL * P::jslot(sl);
    if (P::jslot(sl) < E / 2 && pos >= 1 && pos <= n) {
      if (ha) pa[pos - 1] = v[sl].y;
      if (hb) pb[pos - 1] = -v[sl].x;
    }
  }
  if (!a.dot) return;
  __shared__ double red[64];
  const double blk = block_sum(acc, red);
  if (threadIdx.x == 0) a.part[(long)o * a.max_blocks + rb] = blk;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
#define FL_CASE_ME(M_, E_, ...) \
  case (M_ * 64 + E_): {        \
    constexpr int M = M_;       \
    constexpr int E = E_;       \
    __VA_ARGS__;                \
  } break;

#define FL_CASES_M(M_, ...)            \
  FL_CASE_ME(M_, 8, __VA_ARGS__)       \
  FL_CASE_ME(M_, 16, __VA_ARGS__)      \
  FL_CASE_ME(M_, 32, __VA_ARGS__)

#define FL_DISPATCH(Mv, Ev, ...)                                                         \
  switch ((Mv) * 64 + (Ev)) {                                                            \
    FL_CASE_ME(8, 8, __VA_ARGS__)                                                        \
    FL_CASE_ME(16, 8, __VA_ARGS__)                                                       \
    FL_CASE_ME(16, 16, __VA_ARGS__)                                                      \
    FL_CASES_M(32, __VA_ARGS__)                                                          \
    FL_CASES_M(64, __VA_ARGS__)                                                          \
    FL_CASES_M(128, __VA_ARGS__)                                                         \
    FL_CASES_M(256, __VA_ARGS__)                                                         \
    FL_CASES_M(512, __VA_ARGS__)                                                         \
    FL_CASES_M(1024, __VA_ARGS__)                                                        \
    FL_CASES_M(2048, __VA_ARGS__)                                                        \
    default:                                                                             \
      throw Error(2, "unsupported transform length / radix (M=" + std::to_string(Mv) +   \
                         ", E=" + std::to_string(Ev) + ")");                             \
  }

template <typename T>
inline size_t line_lds_bytes(int M, int E) {
  return (size_t)2 * (M + M / E) * sizeof(T);
}

// one exchange plane per line (the contiguous passes)
template <typename T>
inline size_t plane_lds_bytes(int M, int E) {
  return (size_t)(M + M / E) * sizeof(T);
}

inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(4, std::string(what) + ": " + hipGetErrorString(e));
}

// Allow up to the full 160 KiB of dynamic LDS of a gfx950 workgroup; set
// once per kernel (so never inside a stream capture after the first run).
template <typename K>
inline void lds_attr(K kernel, size_t bytes) {
  if (bytes <= 65536) return;
  static std::mutex mu;
  static std::unordered_set<const void*> done;
  const void* key = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(key)) return;
  hipFuncAttributes fa{};
  FL_HIP(hipFuncGetAttributes(&fa, key));
  const int avail = (int)kMaxLds - (int)fa.sharedSizeBytes;  // minus static LDS
  if ((int)bytes > avail) throw Error(2, "LDS request exceeds the workgroup limit");
  FL_HIP(hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, avail));
  done.insert(key);
}

#define FL_LAUNCH(KERNEL, GRID, BLOCK, SH, ST, ...) \
  do {                                              \
    auto kfn_ = KERNEL;                             \
    lds_attr(kfn_, SH);                             \
    hipLaunchKernelGGL(kfn_, GRID, BLOCK, SH, ST, __VA_ARGS__); \
  } while (0)

inline long pair_tiles(long C, int W) { return ((C + 1) / 2 + W - 1) / W; }

template <typename T>
void launch_first(int M, int E, FirstArgs<T> a, int nrhs, hipStream_t st) {
  if (!pow2(a.W) || a.n_in > M / 2) throw Error(2, "first pass: bad tile width or rows");
  a.ntiles = pair_tiles(a.C, a.W);
  a.lw = ilog2i(a.W);
  const TileLds tl = tile_lds(M, E, a.W, sizeof(T));
  a.PO = tl.PO;
  a.LS = tl.LS;
  dim3 grid((unsigned)(a.ntiles * nrhs));
  const int threads = a.W * (M / E);
  FL_DISPATCH(M, E, FL_LAUNCH((k_first<T, M, E>), grid, dim3(threads), tl.bytes, st, a));
  check_launch("first pass");
}

template <typename T>
void launch_last(int M, int E, LastArgs<T> a, int nrhs, hipStream_t st) {
  if (!pow2(a.W) || a.n_out > M / 2) throw Error(2, "last pass: bad tile width or rows");
  a.ntiles = pair_tiles(a.C, a.W);
  if (a.mode != PM_PLAIN && a.ntiles > a.max_blocks)
    throw Error(2, "too many blocks for the reduction buffers");
  a.lw = ilog2i(a.W);
  const TileLds tl = tile_lds(M, E, a.W, sizeof(T));
  a.PO = tl.PO;
  a.LS = tl.LS;
  dim3 grid((unsigned)(a.ntiles * nrhs));
  const int threads = a.W * (M / E);
  FL_DISPATCH(M, E, FL_LAUNCH((k_last<T, M, E>), grid, dim3(threads), tl.bytes, st, a));
  check_launch("last pass");
}

template <typename T>
void launch_c2c(int M, int E, int dir, C2CArgs<T> a, long outer, hipStream_t st) {
  if (!pow2(a.W)) throw Error(2, "c2c pass: bad tile width");
  a.ntiles = (a.C + a.W - 1) / a.W;
  a.lw = ilog2i(a.W);
  const TileLds tl = tile_lds(M, E, a.W, sizeof(T));
  a.PO = tl.PO;
  a.LS = tl.LS;
  dim3 grid((unsigned)(a.ntiles * outer));
  const int threads = a.W * (M / E);
  const size_t sh = tl.bytes;
  if (dir < 0 && a.n_in <= M / 2 && a.n_out == M) {
    FL_DISPATCH(M, E, FL_LAUNCH((k_c2c<T, M, E, -1, 1>), grid, dim3(threads), sh, st, a));
  } else if (dir > 0 && a.n_in == M && a.n_out <= M / 2) {
    FL_DISPATCH(M, E, FL_LAUNCH((k_c2c<T, M, E, 1, 2>), grid, dim3(threads), sh, st, a));
  } else if (dir < 0 && a.n_in == M && a.n_out == M) {
    FL_DISPATCH(M, E, FL_LAUNCH((k_c2c<T, M, E, -1, 0>), grid, dim3(threads), sh, st, a));
  } else if (dir > 0 && a.n_in == M && a.n_out == M) {
    FL_DISPATCH(M, E, FL_LAUNCH((k_c2c<T, M, E, 1, 0>), grid, dim3(threads), sh, st, a));
  } else {
    throw Error(2, "c2c pass: unsupported row ranges");
  }
  check_launch("c2c pass");
}

template <typename T>
void launch_mid(int M, int E, const MidArgs<T>& a, int nrhs, hipStream_t st) {
  if (a.n_in > M / 2 || a.n_out > M / 2) throw Error(2, "middle pass: rows beyond M/2");
  MidArgs<T> b = a;
  b.nrhs = nrhs;
  dim3 grid((unsigned)(((a.rows + a.LPB - 1) / a.LPB) * nrhs));
  const int threads = a.LPB * (M / E);
  const size_t sh = plane_lds_bytes<T>(M, E) * a.LPB;
  FL_DISPATCH(M, E, FL_LAUNCH((k_mid<T, M, E>), grid, dim3(threads), sh, st, b));
  check_launch("middle pass");
}

template <typename T>
void launch_rows(int M, int E, int dir, cx<T>* data, long rows, int LPB, const cx<T>* tw,
                 hipStream_t st) {
  dim3 grid((unsigned)((rows + LPB - 1) / LPB));
  const int threads = LPB * (M / E);
  const size_t sh = line_lds_bytes<T>(M, E) * LPB;
  if (dir < 0) {
    FL_DISPATCH(M, E, FL_LAUNCH((k_rows<T, M, E, -1>), grid, dim3(threads), sh, st, data, rows,
                                LPB, tw));
  } else {
    FL_DISPATCH(M, E, FL_LAUNCH((k_rows<T, M, E, 1>), grid, dim3(threads), sh, st, data, rows,
                                LPB, tw));
  }
  check_launch("row transform");
}

template <typename T>
void launch_sine_cols(int M, int E, SineArgs<T> a, long outer, hipStream_t st,
                      bool stop_test = false) {
  if (!pow2(a.W) || a.n != M / 2 - 1) throw Error(2, "sine pass: bad tile width or rows");
  a.ntiles = pair_tiles(a.C, a.W);
  if (a.dot && (a.ntiles > a.max_blocks || a.outer_per_rhs != 1))
    throw Error(2, "sine pass: bad reduction layout");
  if (a.pdir && (a.dot || a.outer_per_rhs != 1))
    throw Error(2, "sine pass: the fused iteration start needs one slice per RHS, no dot");
  a.lw = ilog2i(a.W);
  // the fused passes keep both planes (the product's first pass needs whole
  // lines); the others one (line_in_lds_half)
  const TileLds tl = a.pdir ? tile_lds(M, E, a.W, sizeof(T)) : tile_lds_half(M, E, a.W, sizeof(T));
  a.PO = tl.PO;
  a.LS = tl.LS;
  dim3 grid((unsigned)(a.ntiles * outer));
  const int threads = a.W * (M / E);
  if (a.pdir && a.t1) {
    FL_DISPATCH(M, E, FL_LAUNCH((k_sine_cols<T, M, E, true, true, false>), grid, dim3(threads),
                                tl.bytes, st, a));
  } else if (a.pdir) {
    FL_DISPATCH(M, E, FL_LAUNCH((k_sine_cols<T, M, E, true, false, false>), grid, dim3(threads),
                                tl.bytes, st, a));
  } else if (stop_test) {
    if (a.dot || a.outer_per_rhs != 1) throw Error(2, "sine pass: the stop test needs one slice per RHS");
    FL_DISPATCH(M, E, FL_LAUNCH((k_sine_cols<T, M, E, false, false, true>), grid, dim3(threads),
                                tl.bytes, st, a));
  } else {
    FL_DISPATCH(M, E, FL_LAUNCH((k_sine_cols<T, M, E, false, false, false>), grid, dim3(threads),
                                tl.bytes, st, a));
  }
  check_launch("sine pass");
}

template <typename T>
void launch_sine_mid(int M, int E, const SineMidArgs<T>& a, hipStream_t st) {
  if (a.n != M / 2 - 1 || a.LPB < 1) throw Error(2, "sine middle pass: bad rows");
  const long pairs = (a.rows + 1) / 2;
  dim3 grid((unsigned)(((pairs + a.LPB - 1) / a.LPB) * a.nrhs));
  const int threads = a.LPB * (M / E);
  const size_t sh = plane_lds_bytes<T>(M, E) * a.LPB;
  FL_DISPATCH(M, E, FL_LAUNCH((k_sine_mid<T, M, E>), grid, dim3(threads), sh, st, a));
  check_launch("sine middle pass");
}

template <typename T>
void launch_line1d(int M, int E, const Line1Args<T>& a, hipStream_t st, bool odd = false) {
  if (a.n > M / 2) throw Error(2, "1D line: rows beyond M/2");
  dim3 grid((unsigned)a.nrhs);
  const int threads = M / E;
  const size_t sh = line_lds_bytes<T>(M, E);
  if (odd) {
    if (a.mode == PM_CG) throw Error(2, "1D line: odd extension with a CG prologue");
    FL_DISPATCH(M, E, FL_LAUNCH((k_line1d<T, M, E, true>), grid, dim3(threads), sh, st, a));
  } else {
    FL_DISPATCH(M, E, FL_LAUNCH((k_line1d<T, M, E, false>), grid, dim3(threads), sh, st, a));
  }
  check_launch("1D line");
}

// LDS of k_cg1d: the two exchange planes and four vectors of M/2 values.
inline size_t cg1d_lds_bytes(int M, int E) {
  return line_lds_bytes<double>(M, E) + (size_t)4 * (M / 2) * sizeof(double);
}

inline void launch_cg1d(int M, int E, const Cg1Args& a, int nrhs, hipStream_t st) {
  if (a.n > M / 2) throw Error(2, "1D solve: rows beyond M/2");
  dim3 grid((unsigned)nrhs);
  const int threads = M / E;
  const size_t sh = cg1d_lds_bytes(M, E);
  FL_DISPATCH(M, E, FL_LAUNCH((k_cg1d<M, E>), grid, dim3(threads), sh, st, a));
  check_launch("1D solve");
}

}  // namespace fl
