// Sine passes of the tau preconditioner for transform lengths L = 2 N_s that
// are not powers of two: mixed-radix Stockham transforms (radix 8, 4, 2, then
// 3, 5, 7) of the odd-extended line pairs, the whole line held in LDS.  The
// passes compute what the power-of-two sine passes compute (sigma of each
// line: for a packed pair a + ib the spectrum's imaginary part is sigma(a) =
// -2 S a and minus its real part sigma(b)), for grids whose 2 N_s has no
// prime factor above 7.  Included by one translation unit per precision.
//
// Each stage reads the R inputs of a butterfly from one LDS buffer and writes
// its R outputs to the other (Stockham autosort: stage s of sub-transform
// length Ls reads index b + j L/R, applies w^(j k), k = b mod Ls, w =
// exp(-2 pi i / (Ls R)), and writes (b - k) R + k + m Ls), so the result is
// in natural order after the last stage.  The butterflies of all lines of a
// block are spread over its threads.
#pragma once

#include "passes_impl.h"

namespace fl {

constexpr int kMaxRadices = 14;
struct RadixPlan {
  int L;
  int n;
  int r[kMaxRadices];
};

// Radix-8 stages for the power of two, then one radix 4 or 2, then 3, 5, 7.
// False if L has a prime factor above 7.
inline bool radix_plan(int L, RadixPlan& p) {
  p.L = L;
  p.n = 0;
  int m = L, e2 = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++e2;
  }
  auto push = [&](int r) {
    if (p.n >= kMaxRadices) return false;
    p.r[p.n++] = r;
    return true;
  };
  for (; e2 >= 3; e2 -= 3)
    if (!push(8)) return false;
  if (e2 == 2 && !push(4)) return false;
  if (e2 == 1 && !push(2)) return false;
  for (int r : {3, 5, 7}) {
    while (m % r == 0) {
      if (!push(r)) return false;
      m /= r;
    }
  }
  return m == 1 && L >= 2;
}

// Forward DFT of R = 3, 5, 7 values, X_k = sum_j v_j w^(j k), w = exp(-2 pi
// i / R), from the symmetric pairs a_j = v_j + v_{R-j}, b_j = v_j - v_{R-j}:
// X_k = v_0 + sum_j a_j cos(2 pi j k / R) - i sum_j b_j sin(2 pi j k / R) and
// X_{R-k} the same with +i.  cos and sin of 2 pi m / R come from the
// length-L table (entry m L / R).
template <typename T, int R>
__device__ __forceinline__ void dft_odd(cx<T>* v, const cx<T>* __restrict__ tw, int L) {
  constexpr int H = (R - 1) / 2;
  T c[H], s[H];
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    const cx<T> w = tw[m * (L / R)];
    c[m - 1] = w.x;
    s[m - 1] = -w.y;
  }
  cx<T> a[H], b[H];
  cx<T> s0 = v[0];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    a[j - 1] = cadd(v[j], v[R - j]);
    b[j - 1] = csub(v[j], v[R - j]);
    s0 = cadd(s0, a[j - 1]);
  }
  const cx<T> x0 = v[0];
  v[0] = s0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cx<T> re = x0, im = {0, 0};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const int m = (j * k) % R;
      const T cm = m <= H ? c[m - 1] : c[R - m - 1];
      const T sm = m <= H ? s[m - 1] : -s[R - m - 1];
      re = cadd(re, cscale(a[j - 1], cm));
      im = cadd(im, cscale(b[j - 1], sm));
    }
    v[k] = {re.x + im.y, re.y - im.x};       // re - i im
    v[R - k] = {re.x - im.y, re.y + im.x};   // re + i im
  }
}

// One stage of radix R over `nlines` lines (line l at l * L in src and dst).
template <typename T, int R>
__device__ __forceinline__ void any_stage(const cx<T>* src, cx<T>* dst, int L, int Ls,
                                          int nlines, const cx<T>* __restrict__ tw) {
  const int nb = L / R;
  const int step = L / (Ls * R);
  const int tot = nlines * nb;
  for (int f = threadIdx.x; f < tot; f += blockDim.x) {
    const int line = f / nb, b = f - line * nb;
    const cx<T>* in = src + (long)line * L;
    cx<T>* out = dst + (long)line * L;
    const int k = b % Ls;
    cx<T> v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) v[j] = in[b + j * nb];
#pragma unroll
    for (int j = 1; j < R; ++j) v[j] = cmul(v[j], tw[j * k * step]);
    if constexpr (R == 3 || R == 5 || R == 7) dft_odd<T, R>(v, tw, L);
    else dft<R, -1>(v);
    const int o = (b - k) * R + k;
#pragma unroll
    for (int m = 0; m < R; ++m) out[o + m * Ls] = v[m];
  }
}

// Forward transform of nlines lines of length p.L held in b0; b1 is the
// other buffer.  Returns the buffer holding the result.  Every thread of the
// block must call it (barriers).
template <typename T>
__device__ cx<T>* any_fft(cx<T>* b0, cx<T>* b1, const RadixPlan& p, int nlines,
                          const cx<T>* __restrict__ tw) {
  cx<T>* src = b0;
  cx<T>* dst = b1;
  int Ls = 1;
  for (int s = 0; s < p.n; ++s) {
    const int R = p.r[s];
    switch (R) {
      case 8: any_stage<T, 8>(src, dst, p.L, Ls, nlines, tw); break;
      case 4: any_stage<T, 4>(src, dst, p.L, Ls, nlines, tw); break;
      case 2: any_stage<T, 2>(src, dst, p.L, Ls, nlines, tw); break;
      case 3: any_stage<T, 3>(src, dst, p.L, Ls, nlines, tw); break;
      case 5: any_stage<T, 5>(src, dst, p.L, Ls, nlines, tw); break;
      default: any_stage<T, 7>(src, dst, p.L, Ls, nlines, tw); break;
    }
    __syncthreads();
    cx<T>* t = src;
    src = dst;
    dst = t;
    Ls *= R;
  }
  return src;
}

// Lines (column pairs, line pairs) per block: two LDS buffers of L complex
// values per line within 128 KB in FP64 (the same count in FP32, so that the
// number of partial sums a pass writes does not depend on the precision).
constexpr size_t kSineAnyLds = size_t(128) << 10;
constexpr int kSineAnyThreads = 1024;
inline int sine_any_lines(int L) {
  int w = (int)(kSineAnyLds / (2 * (size_t)L * sizeof(cx<double>)));
  if (w > 8) w = 8;
  return w < 1 ? 1 : w;
}
// The contiguous middle pass runs one line pair per block (its loads are
// whole lines, so the lines per block do not matter for coalescing): two LDS
// buffers of at most 32 KB (FP64, L <= 2048), so that several blocks share
// a CU and hide each other's stage barriers and twiddle loads; 256 threads
// up to L = 1600, 512 above (measured: L = 1200 and 1400 faster with 256,
// L = 2000 with 512).
constexpr int kSineAnyMidThreads = 512;
inline int sine_any_mid_threads(int L) { return L <= 1600 ? 256 : 512; }
inline long sine_any_mid_blocks(const Geometry& g) {
  const long rows = g.nd / g.na[g.d - 1];
  return (rows + 1) / 2;
}
inline long sine_any_last_blocks(const Geometry& g) {
  return pair_tiles((long)g.na[1] * g.na[2], sine_any_lines(g.La[0]));
}

// Strided sine pass along the row axis of [outer][n][C] (the arguments of
// the power-of-two pass; E and the schedule are not used): a block owns W
// column pairs, reads their rows (consecutive threads on consecutive
// columns), builds the odd extensions in LDS, transforms, writes sigma of
// each column (and with dot, partials of partner . out).
template <typename T>
struct SineAnyArgs {
  const T* in;
  T* out;
  const T* partner;
  const int* active;
  double* part;
  int max_blocks;
  long C, os, ntiles;
  int outer_per_rhs;
  int n;
  int W;
  int dot;
  const cx<T>* tw;
  RadixPlan plan;
};

template <typename T>
__global__ void __launch_bounds__(kSineAnyThreads) k_sine_any_cols(SineAnyArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[64];
  const int L = a.plan.L, N = L / 2, W2 = 2 * a.W;
  cx<T>* b0 = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* b1 = b0 + (long)a.W * L;
  T* bt = reinterpret_cast<T*>(b0);
  long tile, o;
  xcd_tile(a.ntiles, tile, o);
  if (a.active && !a.active[o / a.outer_per_rhs]) return;
  const long col0 = tile * W2;
  const long cl = a.C - col0;
  const int ncol = cl < W2 ? (int)cl : W2;
  const long base = o * a.os + col0;
  for (int l = threadIdx.x; l < a.W; l += blockDim.x) {
    b0[(long)l * L] = {0, 0};
    b0[(long)l * L + N] = {0, 0};
  }
  const int tot = a.n * W2;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int row = e / W2, cc = e - row * W2;
    const T x = cc < ncol ? a.in[base + (long)row * a.C + cc] : (T)0;
    const long l = cc >> 1;
    const int comp = cc & 1;
    bt[2 * (l * L + row + 1) + comp] = x;
    bt[2 * (l * L + L - row - 1) + comp] = -x;
  }
  __syncthreads();
  const cx<T>* res = any_fft<T>(b0, b1, a.plan, a.W, a.tw);
  double acc = 0.0;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int row = e / W2, cc = e - row * W2;
    if (cc >= ncol) continue;
    const cx<T> z = res[(long)(cc >> 1) * L + row + 1];
    const T v = (cc & 1) ? -z.x : z.y;
    const long i = base + (long)row * a.C + cc;
    a.out[i] = v;
    if (a.dot) acc += (double)a.partner[i] * (double)v;
  }
  if (!a.dot) return;
  const double blk = block_sum(acc, red);
  if (threadIdx.x == 0) a.part[(o / a.outer_per_rhs) * a.max_blocks + tile] = blk;
}

// Contiguous last-axis pass on pairs of lines, in place: sigma, multiply
// each line by its own multiplier row, sigma again (as the power-of-two
// middle pass: after the first transform slot k holds (-sigma(b)_k,
// sigma(a)_k); the second transform's packed input is (m_a Z.y, -m_b Z.x)),
// with the partials of r.z = sum_k m_k sigma(r)_k^2 when dot.
template <typename T>
struct SineAnyMidArgs {
  T* data;             // output (may equal `in`: a block reads all its lines first)
  const T* m;          // folded multiplier, (N_0 + 1) x .. x (N_{d-1} + 1)
  const int* active;
  long rows;           // lines per RHS
  long o_stride;
  int n;               // line length
  int n1;              // 3D: interior points of axis 1
  int Hl, H1;          // multiplier row lengths of the last axis and of axis 1
  int d;
  int LPB;             // line pairs per block
  long nblk;           // blocks per RHS
  int dot;
  double* part;
  int max_blocks;
  const cx<T>* tw;
  RadixPlan plan;
  const T* in;         // input lines (null: data)
};

// Multiplier row of line L of the last axis (the other axes' frequencies are
// their indices + 1); d = 1: the one line.
__device__ __forceinline__ long any_mrow(long L, int n1, int H1, int Hl, int d) {
  if (d == 1) return 0;
  const int l = (int)L;
  if (d == 3) return (long)((l / n1 + 1) * H1 + (l % n1 + 1)) * Hl;
  return (long)(l + 1) * Hl;
}

template <typename T>
__global__ void __launch_bounds__(kSineAnyMidThreads) k_sine_any_mid(SineAnyMidArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[64];
  const int L = a.plan.L, N = L / 2, n = a.n;
  cx<T>* b0 = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* b1 = b0 + (long)a.LPB * L;
  T* bt = reinterpret_cast<T*>(b0);
  long ol, rb;
  xcd_tile(a.nblk, rb, ol);
  const int o = (int)ol;
  if (a.active && !a.active[o]) return;
  T* base = a.data + (long)o * a.o_stride;
  const T* src = (a.in ? a.in : a.data) + (long)o * a.o_stride;
  const long la0 = 2 * rb * a.LPB;
  for (int l = threadIdx.x; l < a.LPB; l += blockDim.x) {
    b0[(long)l * L] = {0, 0};
    b0[(long)l * L + N] = {0, 0};
  }
  const int tot = a.LPB * 2 * n;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int lp = e / n, pos = e - lp * n;   // lp = 2 * pair + comp
    const long line = la0 + lp;
    const T x = line < a.rows ? src[line * n + pos] : (T)0;
    const long pr = lp >> 1;
    const int comp = lp & 1;
    bt[2 * (pr * L + pos + 1) + comp] = x;
    bt[2 * (pr * L + L - pos - 1) + comp] = -x;
  }
  __syncthreads();
  cx<T>* res = any_fft<T>(b0, b1, a.plan, a.LPB, a.tw);
  cx<T>* other = res == b0 ? b1 : b0;
  double acc = 0.0;
  for (int f = threadIdx.x; f < a.LPB * L; f += blockDim.x) {
    const int pr = f / L, k = f - pr * L;
    const int kk = k <= N ? k : L - k;
    const long la = la0 + 2 * pr;
    const bool ha = la < a.rows, hb = la + 1 < a.rows;
    const T sa = ha ? a.m[any_mrow(la, a.n1, a.H1, a.Hl, a.d) + kk] : (T)0;
    const T sb = hb ? a.m[any_mrow(la + 1, a.n1, a.H1, a.Hl, a.d) + kk] : (T)0;
    const cx<T> z = res[f];
    if (a.dot && k >= 1 && k <= n)
      acc += (double)sa * (double)z.y * (double)z.y + (double)sb * (double)z.x * (double)z.x;
    res[f] = {sa * z.y, -(sb * z.x)};
  }
  __syncthreads();
  const cx<T>* y = any_fft<T>(res, other, a.plan, a.LPB, a.tw);
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int lp = e / n, pos = e - lp * n;
    const long line = la0 + lp;
    if (line >= a.rows) continue;
    const cx<T> v = y[(long)(lp >> 1) * L + pos + 1];
    base[line * n + pos] = (lp & 1) ? -v.x : v.y;
  }
  if (!a.dot) return;
  const double blk = block_sum(acc, red);
  if (threadIdx.x == 0) a.part[(long)o * a.max_blocks + rb] = blk;
}

inline RadixPlan radix_plan_or_throw(int L) {
  RadixPlan p{};
  if (!radix_plan(L, p)) throw Error(2, "sine transform length with a prime factor above 7");
  return p;
}

template <typename T>
void launch_sine_any_cols(SineAnyArgs<T> a, long outer, hipStream_t st) {
  a.W = sine_any_lines(a.plan.L);
  a.ntiles = pair_tiles(a.C, a.W);
  const size_t sh = 2 * (size_t)a.W * a.plan.L * sizeof(cx<T>);
  dim3 grid((unsigned)(a.ntiles * outer));
  FL_LAUNCH((k_sine_any_cols<T>), grid, dim3(kSineAnyThreads), sh, st, a);
  check_launch("mixed-radix sine pass");
}

template <typename T>
void launch_sine_any_mid(SineAnyMidArgs<T> a, int nrhs, hipStream_t st) {
  a.LPB = 1;
  a.nblk = (a.rows + 1) / 2;
  const size_t sh = 2 * (size_t)a.LPB * a.plan.L * sizeof(cx<T>);
  dim3 grid((unsigned)(a.nblk * nrhs));
  FL_LAUNCH((k_sine_any_mid<T>), grid, dim3(sine_any_mid_threads(a.plan.L)), sh, st, a);
  check_launch("mixed-radix sine middle pass");
}

}  // namespace fl
