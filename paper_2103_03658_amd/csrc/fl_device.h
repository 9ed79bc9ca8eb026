// Device-side building blocks shared by the library's kernels: complex
// arithmetic, small in-register DFTs (radix 2 to 32) and the register+LDS
// Stockham engine that transforms one line of length M held by M/E threads
// (E elements per thread).  gfx950 (CDNA4, wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }

// Multiply by DIR*i:  DIR = -1 gives -i (forward kernel e^{-2 pi i/4}), +1 gives +i.
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  if constexpr (DIR < 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}

// ---------------------------------------------------------------------------
// In-register DFTs, natural order in and out.  X_k = sum_j v_j w^{jk},
// w = exp(DIR * 2 pi i / R).  DIR = -1 forward, +1 inverse (unnormalised).
// ---------------------------------------------------------------------------
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  cx<T> b0 = cadd(v[1], v[3]), b1 = mul_i<DIR>(csub(v[1], v[3]));
  v[0] = cadd(a0, b0);
  v[2] = csub(a0, b0);
  v[1] = cadd(a1, b1);
  v[3] = csub(a1, b1);
}

// w8^1 = (1 + DIR i)/sqrt2 ; w8^3 = (-1 + DIR i)/sqrt2
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_w8_1(cx<T> a) {
  const T s = (T)0.70710678118654752440084436210485;
  if constexpr (DIR < 0) return {(a.x + a.y) * s, (a.y - a.x) * s};
  else return {(a.x - a.y) * s, (a.y + a.x) * s};
}
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_w8_3(cx<T> a) {
  const T s = (T)0.70710678118654752440084436210485;
  if constexpr (DIR < 0) return {(a.y - a.x) * s, -(a.x + a.y) * s};
  else return {-(a.x + a.y) * s, (a.x - a.y) * s};
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  o[1] = mul_w8_1<DIR>(o[1]);
  o[2] = mul_i<DIR>(o[2]);
  o[3] = mul_w8_3<DIR>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

// cos(2 pi j / 16), sin(2 pi j / 16) for j = 0..4
template <typename T>
__device__ __forceinline__ cx<T> w16(int jk) {
  // returns exp(-2 pi i jk/16) for the forward sign; caller conjugates.
  const T c1 = (T)0.92387953251128675612818318939679;
  const T s1 = (T)0.38268343236508977172845998403040;
  const T c2 = (T)0.70710678118654752440084436210485;
  switch (jk & 15) {
    case 0: return {(T)1, (T)0};
    case 1: return {c1, -s1};
    case 2: return {c2, -c2};
    case 3: return {s1, -c1};
    case 4: return {(T)0, (T)-1};
    case 5: return {-s1, -c1};
    case 6: return {-c2, -c2};
    case 7: return {-c1, -s1};
    case 8: return {(T)-1, (T)0};
    case 9: return {-c1, s1};
    case 10: return {-c2, c2};
    case 11: return {-s1, c1};
    case 12: return {(T)0, (T)1};
    case 13: return {s1, c1};
    case 14: return {c2, c2};
    default: return {c1, s1};
  }
}

template <int DIR, typename T>
__device__ __forceinline__ void dft16(cx<T>* v) {
  // n = 4 n1 + n2, k = k1 + 4 k2
  cx<T> a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
    dft4<DIR>(a[n2]);  // a[n2][k1]
  }
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2) {
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) {
      cx<T> w = w16<T>(n2 * k1);
      if constexpr (DIR > 0) w.y = -w.y;
      a[n2][k1] = cmul(a[n2][k1], w);
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft4<DIR>(b);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
  }
}

// cos(pi k/16), sin(pi k/16), k = 0..15: w32^k = (c, DIR s)
__device__ __forceinline__ constexpr double c32(int k) {
  constexpr double t[16] = {1.0,
                            0.98078528040323044912618223613424,
                            0.92387953251128675612818318939679,
                            0.83146961230254523707878837761791,
                            0.70710678118654752440084436210485,
                            0.55557023301960222474283081394853,
                            0.38268343236508977172845998403040,
                            0.19509032201612826784828486847702,
                            0.0,
                            -0.19509032201612826784828486847702,
                            -0.38268343236508977172845998403040,
                            -0.55557023301960222474283081394853,
                            -0.70710678118654752440084436210485,
                            -0.83146961230254523707878837761791,
                            -0.92387953251128675612818318939679,
                            -0.98078528040323044912618223613424};
  return t[k];
}
__device__ __forceinline__ constexpr double s32(int k) { return k <= 8 ? c32(8 - k) : c32(k - 8); }

template <int DIR, typename T>
__device__ __forceinline__ void dft32(cx<T>* v) {
  cx<T> e[16], o[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    e[k] = v[2 * k];
    o[k] = v[2 * k + 1];
  }
  dft16<DIR>(e);
  dft16<DIR>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    cx<T> t = o[k];
    if (k == 8) {
      t = mul_i<DIR>(t);
    } else if (k != 0) {
      const T c = (T)c32(k);
      const T sn = (T)(DIR < 0 ? -s32(k) : s32(k));
      t = cmul(t, cx<T>{c, sn});
    }
    v[k] = cadd(e[k], t);
    v[k + 16] = csub(e[k], t);
  }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
  else if constexpr (R == 16) dft16<DIR>(v);
  else if constexpr (R == 32) dft32<DIR>(v);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Stockham plan for a line of length M = E^(S-1) * R_last, E elements per
// thread, TPL = M/E threads per line.  Stage s combines sub-transforms of
// length Ls = E^s with radix R_s (E, ..., E, R_last).
// ---------------------------------------------------------------------------
constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int M, int E>
struct Plan {
  static_assert((M & (M - 1)) == 0 && (E & (E - 1)) == 0 && E <= M, "powers of two, E <= M");
  static constexpr int TPL = M / E;
  static constexpr int LOGE = ilog2(E);
  static constexpr int S = (ilog2(M) + LOGE - 1) / LOGE;
  static constexpr int RLAST = M / ipow(E, S - 1);
  static constexpr int radix(int s) { return s < S - 1 ? E : RLAST; }
  static constexpr int ls(int s) { return ipow(E, s); }
  // register slot -> j such that the slot holds element t + TPL * j after
  // the last stage (the first stage reads element t + TPL*j into slot j).
  static constexpr int jslot(int slot) {
    return (slot / RLAST) + (slot % RLAST) * (E / RLAST);
  }
  static constexpr int slot_of_j(int j) {
    // inverse of jslot
    return (j % (E / RLAST)) * RLAST + j / (E / RLAST);
  }
  // LDS words per line (padding one word per E elements breaks the stride-E
  // bank pattern of the first exchange).
  static constexpr int LDSN = M + M / E;
  __device__ static __forceinline__ int pad(int i) { return i + (i >> LOGE); }
};

// Cross-lane exchanges of a wave's registers (gfx950 lane-swap instructions).
// For a register pair (a, b) that differs in one register bit:
//   permlane32_swap: lanes 32..63 of a <-> lanes 0..31 of b, which swaps lane
//     bit 5 with that register bit;
//   permlane16_swap: odd rows (16 lanes) of a <-> even rows of b, which swaps
//     lane bit 4 with that register bit.
// Each 32-bit word of a value goes through its own instruction.
template <typename V>
__device__ __forceinline__ void lane_swap32(V& a, V& b) {
  constexpr int W = sizeof(V) / 4;
  uint32_t wa[W], wb[W];
  __builtin_memcpy(wa, &a, sizeof(V));
  __builtin_memcpy(wb, &b, sizeof(V));
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(wa[i], wb[i], false, false);
    wa[i] = r[0];
    wb[i] = r[1];
  }
  __builtin_memcpy(&a, wa, sizeof(V));
  __builtin_memcpy(&b, wb, sizeof(V));
}
template <typename V>
__device__ __forceinline__ void lane_swap16(V& a, V& b) {
  constexpr int W = sizeof(V) / 4;
  uint32_t wa[W], wb[W];
  __builtin_memcpy(wa, &a, sizeof(V));
  __builtin_memcpy(wb, &b, sizeof(V));
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(wa[i], wb[i], false, false);
    wa[i] = r[0];
    wb[i] = r[1];
  }
  __builtin_memcpy(&a, wa, sizeof(V));
  __builtin_memcpy(&b, wb, sizeof(V));
}

// The exchange before the last stage of a line held by exactly one wave
// (TPL = 64), when the previous stages span Lp >= 16 elements.  With t =
// Lp h + c, the previous stage leaves element h Lp E + r Lp + c in lane t,
// register r; the last stage (radix R = 64/Lp) wants in lane t, slot q R + j
// the element t + 64 q + j M/R, which lane Lp j + c holds in register q R + h.
// So the lane bits above log2 Lp trade places with the low register bits:
// lane bits 4, 5 with register bits 0, 1 (Lp = 16), or lane bit 5 with
// register bit 0 (Lp = 32).  No LDS and no barrier.
template <int M, int E, int s>
struct LaneExchange {
  using P = Plan<M, E>;
  static constexpr bool ok = s == P::S - 1 && P::TPL == 64 && P::radix(s - 1) == E &&
                             (P::ls(s - 1) == 16 || P::ls(s - 1) == 32);
};

template <typename T, int E, int LP>
__device__ __forceinline__ void lane_exchange(cx<T> (&v)[E]) {
  if constexpr (LP == 16) {
#pragma unroll
    for (int r = 0; r < E; ++r)
      if ((r & 2) == 0) lane_swap32(v[r], v[r + 2]);
#pragma unroll
    for (int r = 0; r < E; ++r)
      if ((r & 1) == 0) lane_swap16(v[r], v[r + 1]);
  } else {
#pragma unroll
    for (int r = 0; r < E; ++r)
      if ((r & 1) == 0) lane_swap32(v[r], v[r + 1]);
  }
}

// One Stockham stage s >= 1: exchange the previous stage's outputs through
// LDS (or, before the last stage of a one-wave line, across lanes), then
// twiddle and DFT.  lre/lim: this line's LDS planes; ONE: a single
// plane (lre) carries the real and then the imaginary parts (half the LDS
// of a line, so more lines fit a CU, for two more barriers per stage).
// Twiddles: of the R - 1 factors w^j (w = e^{-2 pi i k / (Ls R)}) only
// w^(2^b), b < log2 R, are read from the table (before the exchange, so that
// the reads overlap it); the others are products of at most log2 R - 1 of
// those, by the binary digits of j.  Reading all R - 1 per stage held more
// registers than the transform itself and left each stage waiting on them.
template <typename T, int M, int E, int DIR, int s, bool ONE>
__device__ __forceinline__ void stockham_stage(cx<T> (&v)[E], T* lre, T* lim, int t,
                                               const cx<T>* __restrict__ tw) {
  using P = Plan<M, E>;
  constexpr int TPL = P::TPL;
  constexpr int Rp = P::radix(s - 1);
  constexpr int Lp = P::ls(s - 1);
  constexpr int R = P::radix(s);
  constexpr int Ls = P::ls(s);
  constexpr int LR = ilog2(R);
  cx<T> pw[E / R][LR];
#pragma unroll
  for (int q = 0; q < E / R; ++q) {
    const int k = (t + q * TPL) & (Ls - 1);
    const int i1 = k * (M / (Ls * R));
#pragma unroll
    for (int bit = 0; bit < LR; ++bit) pw[q][bit] = tw[i1 << bit];
  }
  if constexpr (LaneExchange<M, E, s>::ok) {
    lane_exchange<T, E, Lp>(v);
  } else {
#pragma unroll
    for (int part = 0; part < (ONE ? 2 : 1); ++part) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < E / Rp; ++q) {
        const int b = t + q * TPL;
        const int k = b & (Lp - 1);
#pragma unroll
        for (int r = 0; r < Rp; ++r) {
          const int o = P::pad((b - k) * Rp + k + r * Lp);
          if (!ONE || part == 0) lre[o] = v[q * Rp + r].x;
          if (!ONE) lim[o] = v[q * Rp + r].y;
          if (ONE && part == 1) lre[o] = v[q * Rp + r].y;
        }
      }
      __syncthreads();
      T nx[E], ny[E];
#pragma unroll
      for (int q = 0; q < E / R; ++q) {
        const int b = t + q * TPL;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const int i = P::pad(b + j * (M / R));
          nx[q * R + j] = lre[i];
          if (!ONE) ny[q * R + j] = lim[i];
        }
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (!ONE) {
          v[e] = {nx[e], ny[e]};
        } else if (part == 0) {
          v[e].x = nx[e];
        } else {
          v[e].y = nx[e];
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < E / R; ++q) {
#pragma unroll
    for (int j = 1; j < R; ++j) {
      cx<T> w = {1, 0};
      bool first = true;
#pragma unroll
      for (int bit = 0; bit < LR; ++bit) {
        if (j & (1 << bit)) {
          w = first ? pw[q][bit] : cmul(w, pw[q][bit]);
          first = false;
        }
      }
      if constexpr (DIR > 0) w.y = -w.y;
      v[q * R + j] = cmul(v[q * R + j], w);
    }
    dft<R, DIR>(&v[q * R]);
  }
}

template <typename T, int M, int E, int DIR, int s, bool ONE>
__device__ __forceinline__ void stockham_from(cx<T> (&v)[E], T* lre, T* lim, int t,
                                              const cx<T>* __restrict__ tw) {
  if constexpr (s < Plan<M, E>::S) {
    stockham_stage<T, M, E, DIR, s, ONE>(v, lre, lim, t, tw);
    stockham_from<T, M, E, DIR, s + 1, ONE>(v, lre, lim, t, tw);
  }
}

// Full length-M transform of one line.  On entry slot j holds element
// t + TPL*j; on exit slot `sl` holds output element t + TPL*Plan::jslot(sl).
// Every thread of the block must call this (it contains barriers).
template <typename T, int M, int E, int DIR>
__device__ __forceinline__ void fft_line(cx<T> (&v)[E], T* lre, T* lim, int t,
                                         const cx<T>* __restrict__ tw) {
  dft<Plan<M, E>::radix(0), DIR>(v);
  stockham_from<T, M, E, DIR, 1, false>(v, lre, lim, t, tw);
}

// The same with one LDS plane of Plan::LDSN elements for the exchanges.
template <typename T, int M, int E, int DIR>
__device__ __forceinline__ void fft_line_1p(cx<T> (&v)[E], T* l, int t,
                                            const cx<T>* __restrict__ tw) {
  dft<Plan<M, E>::radix(0), DIR>(v);
  stockham_from<T, M, E, DIR, 1, true>(v, l, nullptr, t, tw);
}

// Reorder slots so that slot j holds element t + TPL*j (compile-time permutation).
template <typename T, int M, int E>
__device__ __forceinline__ void to_natural(cx<T> (&v)[E]) {
  cx<T> w[E];
#pragma unroll
  for (int j = 0; j < E; ++j) w[j] = v[Plan<M, E>::slot_of_j(j)];
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = w[j];
}

}  // namespace fl
