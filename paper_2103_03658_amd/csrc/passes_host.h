// Host side of the operator application: pass sequence per dimension.
// Included by one translation unit per precision.
#pragma once

#include "passes_impl.h"

namespace fl {

template <typename T>
size_t ws_bytes_t(const Geometry& g, int nrhs) {
  const size_t h = (size_t)(g.M / 2 + 1);
  const size_t n = (size_t)g.n;
  size_t cells = 0;
  if (g.d == 2) cells = h * n;
  if (g.d == 3) cells = h * n * n + h * (size_t)g.M * n;
  return cells * (size_t)nrhs * 2 * sizeof(T);
}

template <typename T>
void apply_passes_t(const Geometry& g, const Schedule& sc, const T* lam, const void* twv,
                    const T* u, T* y, int nrhs, void* ws, hipStream_t st, int mode,
                    const T* rvec, T* pvec, const double* fvec, const CgScalars* cg,
                    const int* active, hipEvent_t* ev, int only, bool odd) {
  // optional timing: ev[k] recorded before pass k, ev[npasses] after the last;
  // only >= 0 launches that pass alone (its input must already be in place)
  int pass = 0;
  auto go = [&]() {
    if (ev) FL_HIP(hipEventRecord(ev[pass], st));
    return only < 0 || only == pass++;
  };
  auto done = [&]() {
    if (ev) FL_HIP(hipEventRecord(ev[pass], st));
  };
  const cx<T>* tw = reinterpret_cast<const cx<T>*>(twv);
  const int M = g.M, n = g.n, N1 = g.H;   // folded symbol row length
  const long h = M / 2 + 1;
  CgScalars nocg{};
  const CgScalars& c = cg ? *cg : nocg;
  if (mode != PM_PLAIN && !cg) throw Error(1, "missing reduction buffers");
  double* part = mode == PM_DOT ? c.part_b : c.part_a;
  if (g.d == 1) {
    Line1Args<T> a{u, y, pvec, rvec, fvec, active, c, part, c.max_blocks, lam, n, nrhs,
                   mode, tw};
    if (go()) launch_line1d<T>(M, sc.E_mid, a, st, odd);
    done();
    return;
  }
  const long C0 = g.d == 2 ? (long)n : (long)n * n;   // columns of the axis-0 passes
  const long nd = g.nd;
  if (odd) {
    // real sine passes: axis 0 (r -> S1), 3D axis 1 (in place), last axis
    // with the multiplier (in place), 3D axis 1, axis 0 (S1 -> y, partials
    // of u.y in PM_DOT)
    if (mode != PM_PLAIN && mode != PM_DOT) throw Error(2, "odd passes: plain or dot mode only");
    T* S1 = reinterpret_cast<T*>(ws);
    SineArgs<T> a0{u, S1, nullptr, active, nullptr, 0, C0, nd, 0, 1, n,
                   sc.W_first, 0, 0, 0, 0, tw};
    SineArgs<T> a1{S1, S1, nullptr, active, nullptr, 0, n, (long)n * n, 0, n, n,
                   sc.W_c2c, 0, 0, 0, 0, tw};
    if (go()) launch_sine_cols<T>(M, sc.E_first, a0, nrhs, st);
    if (g.d == 3 && go()) launch_sine_cols<T>(M, sc.E_c2c, a1, (long)nrhs * n, st);
    SineMidArgs<T> m{S1, lam, active, nd / n, nd, n, N1, g.d, sc.LPB_mid, nrhs, tw};
    if (go()) launch_sine_mid<T>(M, sc.E_mid, m, st);
    if (g.d == 3 && go()) launch_sine_cols<T>(M, sc.E_c2c, a1, (long)nrhs * n, st);
    SineArgs<T> a2{S1, y, mode == PM_DOT ? u : nullptr, active, part, c.max_blocks, C0, nd, 0,
                   1, n, sc.W_first, 0, 0, 0, mode == PM_DOT ? 1 : 0, tw};
    if (go()) launch_sine_cols<T>(M, sc.E_first, a2, nrhs, st);
    done();
    return;
  }
  cx<T>* T1 = reinterpret_cast<cx<T>*>(ws);
  // axis 0, forward (real pairs -> Hermitian half); CG: iteration start
  {
    FirstArgs<T> a{u, pvec, rvec, active, c, T1, C0, nd, h * C0, 0, n,
                   sc.W_first, 0, 0, 0, mode == PM_CG ? PM_CG : PM_PLAIN, tw};
    if (go()) launch_first<T>(M, sc.E_first, a, nrhs, st);
  }
  if (g.d == 2) {
    MidArgs<T> m{T1, lam, active, h, h * n, n, n, n, N1, 2, sc.LPB_mid, nrhs, tw};
    if (go()) launch_mid<T>(M, sc.E_mid, m, nrhs, st);
  } else {
    cx<T>* T2 = T1 + (long)nrhs * h * n * n;
    // axis 1 forward: slices (rhs, k0), rows i1 < n -> k1 < M, columns i2
    C2CArgs<T> f1{T1, T2, active, n, (long)n * n, n, (long)M * n, n, 0, (int)h, n, M,
                  sc.W_c2c, 0, 0, 0, tw};
    if (go()) launch_c2c<T>(M, sc.E_c2c, -1, f1, (long)nrhs * h, st);
    MidArgs<T> m{T2, lam, active, h * M, h * M * n, n, n, n, N1, 3, sc.LPB_mid, nrhs, tw};
    if (go()) launch_mid<T>(M, sc.E_mid, m, nrhs, st);
    C2CArgs<T> i1{T2, T1, active, n, (long)M * n, n, (long)n * n, n, 0, (int)h, M, n,
                  sc.W_c2c, 0, 0, 0, tw};
    if (go()) launch_c2c<T>(M, sc.E_c2c, +1, i1, (long)nrhs * h, st);
  }
  {
    LastArgs<T> a{T1, y, mode == PM_DOT ? u : pvec, fvec, active, part, c.max_blocks, C0,
                  h * C0, nd, 0, n, sc.W_first, 0, 0, 0, mode, tw};
    if (go()) launch_last<T>(M, sc.E_first, a, nrhs, st);
    done();
  }
}

template <typename T>
__global__ void k_twiddle(cx<T>* tw, int M) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < M) {
    double s, c;
    sincospi(2.0 * (double)j / (double)M, &s, &c);
    tw[j] = {(T)c, (T)(-s)};
  }
}

}  // namespace fl
