// Host side of the operator application: pass sequence per dimension.
// Included by one translation unit per precision.
#pragma once

#include "passes_impl.h"
#include "sine_any.h"

namespace fl {

template <typename T>
size_t ws_bytes_t(const Geometry& g, int nrhs) {
  const size_t h0 = (size_t)g.Ha[0];
  const size_t n1 = (size_t)g.na[1], n2 = (size_t)g.na[2];
  size_t cells = 0;
  if (g.d == 2) cells = h0 * n1;
  if (g.d == 3) cells = h0 * n1 * n2 + h0 * (size_t)g.Ma[1] * n2;
  return cells * (size_t)nrhs * 2 * sizeof(T);
}

template <typename T>
void apply_passes_t(const Geometry& g, const Schedule& sc, const T* lam, const Twiddles& twv,
                    const T* u, T* y, int nrhs, void* ws, hipStream_t st, int mode,
                    const T* rvec, T* pvec, const double* fvec, const CgScalars* cg,
                    const int* active, hipEvent_t* ev, int only, bool odd, bool first_done) {
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
  // per axis: interior points, embedding length, folded symbol length, twiddles
  const int n0 = g.na[0], n1 = g.na[1], n2 = g.na[2];
  const int M0 = g.Ma[0], M1 = g.Ma[1], M2 = g.Ma[2];
  const cx<T>* tw0 = reinterpret_cast<const cx<T>*>(twv.ax[0]);
  const cx<T>* tw1 = reinterpret_cast<const cx<T>*>(twv.ax[1]);
  const cx<T>* tw2 = reinterpret_cast<const cx<T>*>(twv.ax[2]);
  const long h0 = g.Ha[0];
  CgScalars nocg{};
  const CgScalars& c = cg ? *cg : nocg;
  if (mode != PM_PLAIN && !cg) throw Error(1, "missing reduction buffers");
  double* part = mode == PM_DOT ? c.part_b : c.part_a;
  if (mode == PM_PQ && g.d == 1) throw Error(2, "PM_PQ: d >= 2 only");
  if (g.d == 1 && odd && !g.sine_ok()) {
    // mixed-radix sine passes of length 2N (not a power of two): the middle
    // pass on the one line, u -> y (with the u.y = sum_k m_k sigma(u)_k^2
    // partials in PM_DOT, one block per RHS)
    if (mode != PM_PLAIN && mode != PM_DOT) throw Error(2, "odd passes: plain or dot mode only");
    if (!g.sine_any_ok()) throw Error(2, "sine passes: 2N with prime factors 2, 3, 5, 7 only");
    SineAnyMidArgs<T> m{y, lam, active, 1, n0, n0, 1, g.Na[0] + 1, 1, 1, 0, 0,
                        mode == PM_DOT ? 1 : 0, part, c.max_blocks,
                        reinterpret_cast<const cx<T>*>(twv.sx[0]), radix_plan_or_throw(g.La[0]),
                        u};
    if (go()) launch_sine_any_mid<T>(m, nrhs, st);
    done();
    return;
  }
  if (g.d == 1) {
    Line1Args<T> a{u, y, pvec, rvec, fvec, active, c, part, c.max_blocks, lam, n0, nrhs,
                   mode, tw0};
    if (go()) launch_line1d<T>(M0, sc.E_mid, a, st, odd);
    done();
    return;
  }
  const long C0 = (long)n1 * n2;   // columns of the axis-0 passes
  const long nd = g.nd;
  if (odd) {
    // real sine passes: axis 0 (r -> S1), 3D axis 1 (in place), last axis
    // with the multiplier (in place), 3D axis 1, axis 0 (S1 -> y, partials
    // of u.y in PM_DOT)
    if (mode != PM_PLAIN && mode != PM_DOT) throw Error(2, "odd passes: plain or dot mode only");
    T* S1 = reinterpret_cast<T*>(ws);
    if (!g.sine_ok()) {
      // mixed-radix sine passes (2 N_s not a power of two on some axis); the
      // same sequence, r.z in the middle pass when its blocks fit
      if (!g.sine_any_ok())
        throw Error(2, "sine passes: d >= 2 and 2 N_s with prime factors 2, 3, 5, 7 only");
      const cx<T>* sw0 = reinterpret_cast<const cx<T>*>(twv.sx[0]);
      const cx<T>* sw1 = reinterpret_cast<const cx<T>*>(twv.sx[1]);
      const cx<T>* sw2 = reinterpret_cast<const cx<T>*>(twv.sx[2]);
      const RadixPlan p0 = radix_plan_or_throw(g.La[0]);
      const RadixPlan p1 = radix_plan_or_throw(g.La[1]);
      SineAnyArgs<T> b0{u, S1, nullptr, active, nullptr, 0, C0, nd, 0, 1, n0, 0, 0, sw0, p0};
      SineAnyArgs<T> b1{S1, S1, nullptr, active, nullptr, 0, n2, (long)n1 * n2, 0, n0, n1,
                        0, 0, sw1, p1};
      if (go()) launch_sine_any_cols<T>(b0, nrhs, st);
      if (g.d == 3 && go()) launch_sine_any_cols<T>(b1, (long)nrhs * n0, st);
      const int nl = g.d == 2 ? n1 : n2;
      const RadixPlan pl = radix_plan_or_throw(g.La[g.d - 1]);
      const bool dot = mode == PM_DOT;
      const bool mid_dot = dot && sine_any_mid_blocks(g) <= c.max_blocks;
      SineAnyMidArgs<T> m{S1, lam, active, nd / nl, nd, nl, n1, g.Na[g.d - 1] + 1, g.Na[1] + 1,
                          g.d, 0, 0, mid_dot ? 1 : 0, part, c.max_blocks,
                          g.d == 2 ? sw1 : sw2, pl};
      if (go()) launch_sine_any_mid<T>(m, nrhs, st);
      if (g.d == 3 && go()) launch_sine_any_cols<T>(b1, (long)nrhs * n0, st);
      const bool last_dot = dot && !mid_dot;
      SineAnyArgs<T> b2{S1, y, last_dot ? u : nullptr, active, part, c.max_blocks, C0, nd, 0,
                        1, n0, 0, last_dot ? 1 : 0, sw0, p0};
      if (go()) launch_sine_any_cols<T>(b2, nrhs, st);
      done();
      return;
    }
    SineArgs<T> a0{u, S1, nullptr, active, nullptr, 0, C0, nd, 0, 1, n0,
                   sc.W_first, 0, 0, 0, 0, tw0};
    SineArgs<T> a1{S1, S1, nullptr, active, nullptr, 0, n2, (long)n1 * n2, 0, n0, n1,
                   sc.W_c2c, 0, 0, 0, 0, tw1};
    if (go()) launch_sine_cols<T>(M0, sc.E_first, a0, nrhs, st);
    if (g.d == 3 && go()) launch_sine_cols<T>(M1, sc.E_c2c, a1, (long)nrhs * n0, st);
    const int nl = g.d == 2 ? n1 : n2;            // line length of the last axis
    const int ml = g.d == 2 ? M1 : M2;
    // PM_DOT: r.z = sum_k m_k sigma(r)_k^2 in the middle pass, from the
    // transformed values, when its blocks fit the partials; else in the
    // last pass against u
    const bool dot = mode == PM_DOT;
    const bool mid_dot = dot && sine_mid_blocks(g, sc) <= c.max_blocks;
    SineMidArgs<T> m{S1, lam, active, nd / nl, nd, nl, n1, g.Ha[g.d - 1], g.Ha[1], g.d,
                     sc.LPB_mid, nrhs, g.d == 2 ? tw1 : tw2, mid_dot ? 1 : 0, part, c.max_blocks};
    if (go()) launch_sine_mid<T>(ml, sc.E_mid, m, st);
    if (g.d == 3 && go()) launch_sine_cols<T>(M1, sc.E_c2c, a1, (long)nrhs * n0, st);
    const bool last_dot = dot && !mid_dot;
    SineArgs<T> a2{S1, y, last_dot ? u : nullptr, active, part, c.max_blocks, C0, nd, 0,
                   1, n0, sc.W_first, 0, 0, 0, last_dot ? 1 : 0, tw0};
    if (go()) launch_sine_cols<T>(M0, sc.E_first, a2, nrhs, st);
    done();
    return;
  }
  cx<T>* T1 = reinterpret_cast<cx<T>*>(ws);
  // axis 0, forward (real pairs -> Hermitian half); the CG iteration start
  // runs before it (cg_direction), so d >= 2 takes PM_PQ rather than PM_CG
  if (mode == PM_CG) throw Error(2, "PM_CG: d = 1 only (d >= 2 uses PM_PQ)");
  if (!first_done) {
    // (first_done: the axis-0 forward pass has already written T1, fused
    // into the preconditioner's last pass)
    FirstArgs<T> a{u, active, T1, C0, nd, h0 * C0, 0, n0, sc.W_first, 0, 0, 0, tw0};
    if (go()) launch_first<T>(M0, sc.E_first, a, nrhs, st);
  }
  if (g.d == 2) {
    // lines k0 < h0 of n1 values; symbol row k0 * Ha[1]
    MidArgs<T> m{T1, lam, active, h0, h0 * n1, n1, n1, n1, g.Ha[1], 1, 1, 2, sc.LPB_mid, nrhs,
                 tw1};
    if (go()) launch_mid<T>(M1, sc.E_mid, m, nrhs, st);
  } else {
    cx<T>* T2 = T1 + (long)nrhs * h0 * n1 * n2;
    // axis 1 forward: slices (rhs, k0), rows i1 < n1 -> k1 < M1, columns i2
    C2CArgs<T> f1{T1, T2, active, n2, (long)n1 * n2, n2, (long)M1 * n2, n2, 0, (int)h0, n1, M1,
                  sc.W_c2c, 0, 0, 0, tw1};
    if (go()) launch_c2c<T>(M1, sc.E_c2c, -1, f1, (long)nrhs * h0, st);
    // lines (k0, k1) of n2 values; symbol row (k0 Ha[1] + fold(k1)) Ha[2]
    MidArgs<T> m{T2, lam, active, h0 * M1, h0 * M1 * n2, n2, n2, n2, g.Ha[2], g.Ha[1], M1, 3,
                 sc.LPB_mid, nrhs, tw2};
    if (go()) launch_mid<T>(M2, sc.E_mid, m, nrhs, st);
    C2CArgs<T> i1{T2, T1, active, n2, (long)M1 * n2, n2, (long)n1 * n2, n2, 0, (int)h0, M1, n1,
                  sc.W_c2c, 0, 0, 0, tw1};
    if (go()) launch_c2c<T>(M1, sc.E_c2c, +1, i1, (long)nrhs * h0, st);
  }
  {
    // PM_PQ: the CG last pass (q = A p, p.q partials) with p the input u
    LastArgs<T> a{T1, y, (mode == PM_DOT || mode == PM_PQ) ? u : pvec, fvec, active, part,
                  c.max_blocks, C0, h0 * C0, nd, 0, n0, sc.W_first, 0, 0, 0,
                  mode == PM_PQ ? (int)PM_CG : mode, tw0};
    if (go()) launch_last<T>(M0, sc.E_first, a, nrhs, st);
    done();
  }
}

// The tau preconditioner split around the CG iteration start (d >= 2, the
// middle pass's blocks within the partial buffers).  tau_front: the sine
// passes of r up to the middle pass, which writes S1 = sigma diag(m) sigma r
// (all but the axis-0 back transform) and the r.z partials into part_b.
// tau_back_direction: the rest; its axis-0 pass starts the next iteration
// (k_sine_cols DIRF: stopping test, beta, p = z + beta p).  Between the two
// S1 must stay untouched (it is not the product's workspace).
template <typename T>
void tau_front_t(const Geometry& g, const Schedule& sc, const T* m, const Twiddles& twv,
                 const T* r, T* S1, int nrhs, hipStream_t st, const CgScalars& c,
                 const int* active, bool stop_test) {
  if (g.d < 2 || !g.sine_ok() || sine_mid_blocks(g, sc) > c.max_blocks)
    throw Error(2, "split tau preconditioner: d >= 2, 2N a power of two, mid-pass partials");
  const int n0 = g.na[0], n1 = g.na[1], n2 = g.na[2];
  const int M0 = g.Ma[0], M1 = g.Ma[1], M2 = g.Ma[2];
  const cx<T>* tw0 = reinterpret_cast<const cx<T>*>(twv.ax[0]);
  const cx<T>* tw1 = reinterpret_cast<const cx<T>*>(twv.ax[1]);
  const cx<T>* tw2 = reinterpret_cast<const cx<T>*>(twv.ax[2]);
  const long C0 = (long)n1 * n2, nd = g.nd;
  // stop_test: the first pass begins with the end-of-iteration tests on r.r
  // (cg_stop_rr: a right-hand side that stops is not preconditioned again)
  SineArgs<T> a0{r, S1, nullptr, active, nullptr, 0, C0, nd, 0, 1, n0,
                 sc.W_first, 0, 0, 0, 0, tw0, nullptr, c};
  launch_sine_cols<T>(M0, sc.E_first, a0, nrhs, st, stop_test);
  if (g.d == 3) {
    SineArgs<T> a1{S1, S1, nullptr, active, nullptr, 0, n2, (long)n1 * n2, 0, n0, n1,
                   sc.W_c2c, 0, 0, 0, 0, tw1};
    launch_sine_cols<T>(M1, sc.E_c2c, a1, (long)nrhs * n0, st);
  }
  const int nl = g.d == 2 ? n1 : n2;
  SineMidArgs<T> mid{S1, m, active, nd / nl, nd, nl, n1, g.Ha[g.d - 1], g.Ha[1], g.d,
                     sc.LPB_mid, nrhs, g.d == 2 ? tw1 : tw2, 1, c.part_b, c.max_blocks};
  launch_sine_mid<T>(g.d == 2 ? M1 : M2, sc.E_mid, mid, st);
}

// T1 != null: the axis-0 pass also runs the product's first pass on the new
// p (into T1, the product's workspace), on the product's tile schedule sc;
// the 3D axis-1 sine pass keeps the preconditioner's schedule sp.
template <typename T>
void tau_back_direction_t(const Geometry& g, const Schedule& sc, const Schedule& sp,
                          const Twiddles& twv, T* S1, T* p, void* T1, int nrhs, hipStream_t st,
                          const CgScalars& c) {
  const int n0 = g.na[0], n1 = g.na[1], n2 = g.na[2];
  const int M0 = g.Ma[0], M1 = g.Ma[1];
  const cx<T>* tw0 = reinterpret_cast<const cx<T>*>(twv.ax[0]);
  const cx<T>* tw1 = reinterpret_cast<const cx<T>*>(twv.ax[1]);
  const long C0 = (long)n1 * n2, nd = g.nd;
  if (g.d == 3) {
    SineArgs<T> a1{S1, S1, nullptr, c.active, nullptr, 0, n2, (long)n1 * n2, 0, n0, n1,
                   sp.W_c2c, 0, 0, 0, 0, tw1};
    launch_sine_cols<T>(M1, sp.E_c2c, a1, (long)nrhs * n0, st);
  }
  const Schedule& s0 = T1 ? sc : sp;
  SineArgs<T> a2{S1, nullptr, nullptr, c.active, nullptr, 0, C0, nd, 0, 1, n0,
                 s0.W_first, 0, 0, 0, 0, tw0, p, c, reinterpret_cast<cx<T>*>(T1),
                 (long)g.Ha[0] * C0};
  launch_sine_cols<T>(M0, s0.E_first, a2, nrhs, st);
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
