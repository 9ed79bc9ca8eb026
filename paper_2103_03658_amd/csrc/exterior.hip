// Exterior-data term of the scheme with nonhomogeneous data u = g outside
// Omega (Sec. 2.1 eq. (1D-scheme), Sec. 2.2 eq. (2D-scheme) and the terms b
// of their matrix forms):
//   b_i = sum over exterior lattice nodes j, |j - i|_inf <= N, of G_{|j-i|} g(x_j)
//         - c_{d,alpha} tail_i
// The lattice sum is a multilevel Toeplitz product of G with g on the node
// lattice [-N, 2N]^d (zero on the interior nodes).  In 2D and 3D it is done
// by circulant embedding in P = 4N points per axis: with the data at offset
// j + N in [0, 3N] and G wrapped to k mod P for |k| <= N, every offset i - j
// of an interior i and a lattice j falls in [1 - 2N, 2N - 1], and those with
// |i - j| > N land in the zero band (N, 3N) of the wrapped generator, so the
// circular product restricted to the interior is the lattice sum.  When 4N
// points exceed the longest transform (2D, N > 512) each axis of the lattice
// is cut into the blocks [-N, -1], [0, N] and [N+1, 2N]: for an interior i
// and a node j of a block from lo to hi the offset i - j spans fewer than
// 2N <= M values, so with the block's data placed from position 0 and the
// generator at (i - j + lo) mod M, a circular product of length M is exact at
// positions i; the 3^d block products are summed as spectra and transformed
// back once.  In 1D the sum over the 2N + 1 offsets is taken directly.

#include <hip/hip_runtime.h>

#include "passes_impl.h"

namespace fl {
namespace {

// Wrapped generator on P^d: K[q] = G_{|k|}, k = q or q - P, |k_s| <= N.
__global__ void k_wrap_generator(const double* G, int d, int N, int P, long total,
                                 cx<double>* K) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  long rem = e, gi = 0;
  bool inside = true;
  int q[3] = {0, 0, 0};
  for (int s = d - 1; s >= 0; --s) {
    q[s] = (int)(rem % P);
    rem /= P;
  }
  for (int s = 0; s < d; ++s) {
    const int k = q[s] <= N ? q[s] : (q[s] >= P - N ? P - q[s] : -1);
    if (k < 0) inside = false;
    gi = gi * (N + 1) + (k < 0 ? 0 : k);
  }
  K[e] = {inside ? G[gi] : 0.0, 0.0};
}

// Exterior lattice data on P^d: position j + N for j in [-N, 2N]^d, zero on
// interior nodes (1 <= j_s <= N - 1 for every s) and beyond 3N.
__global__ void k_place_exterior(const double* g, int d, int N, int P, long total,
                                 cx<double>* D) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int L = 3 * N + 1;
  long rem = e, gi = 0;
  bool inlat = true, interior = true;
  int q[3] = {0, 0, 0};
  for (int s = d - 1; s >= 0; --s) {
    q[s] = (int)(rem % P);
    rem /= P;
  }
  for (int s = 0; s < d; ++s) {
    if (q[s] >= L) inlat = false;
    const int j = q[s] - N;
    if (j < 1 || j > N - 1) interior = false;
    gi = gi * L + (q[s] < L ? q[s] : 0);
  }
  D[e] = {(inlat && !interior) ? g[gi] : 0.0, 0.0};
}

__global__ void k_mul_spectra(cx<double>* D, const cx<double>* K, long total) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) D[e] = cmul(D[e], K[e]);
}

// Lattice blocks per axis: index a = 0, 1, 2 covers nodes [lo, hi].
struct AxisBlocks {
  int lo[3], hi[3];
};

__host__ __device__ inline AxisBlocks axis_blocks(int N) {
  return {{-N, 0, N + 1}, {-1, N, 2 * N}};
}

// Generator of block (a_0, .., a_{d-1}) on P^d: position q_s holds the offset
// k_s = v_s - lo_s, v_s = q_s (q_s <= N - 1) or q_s - P, for the offsets of
// the block's range with |k_s| <= N; zero elsewhere.
__global__ void k_block_generator(const double* G, int d, int N, int P, int blk, long total,
                                  cx<double>* K) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const AxisBlocks ab = axis_blocks(N);
  long rem = e, gi = 0;
  bool ok = true;
  int q[3] = {0, 0, 0}, a[3] = {0, 0, 0};
  for (int s = d - 1; s >= 0; --s) {
    q[s] = (int)(rem % P);
    rem /= P;
  }
  for (int s = d - 1, b = blk; s >= 0; --s) {
    a[s] = b % 3;
    b /= 3;
  }
  for (int s = 0; s < d; ++s) {
    const int lo = ab.lo[a[s]], hi = ab.hi[a[s]];
    const int v = q[s] <= N - 1 ? q[s] : q[s] - P;
    const int k = v - lo;
    // offsets of interior i in [1, N-1] and j in [lo, hi]
    if (k < 1 - hi || k > N - 1 - lo || k < -N || k > N) ok = false;
    gi = gi * (N + 1) + (ok ? (k < 0 ? -k : k) : 0);
  }
  K[e] = {ok ? G[gi] : 0.0, 0.0};
}

// Exterior data of block blk on P^d: position q_s holds node lo_s + q_s for
// q_s <= hi_s - lo_s; interior nodes are zero.
__global__ void k_place_block(const double* g, int d, int N, int P, int blk, long total,
                              cx<double>* D) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const AxisBlocks ab = axis_blocks(N);
  const int L = 3 * N + 1;
  long rem = e, gi = 0;
  bool in = true, interior = true;
  int q[3] = {0, 0, 0}, a[3] = {0, 0, 0};
  for (int s = d - 1; s >= 0; --s) {
    q[s] = (int)(rem % P);
    rem /= P;
  }
  for (int s = d - 1, b = blk; s >= 0; --s) {
    a[s] = b % 3;
    b /= 3;
  }
  for (int s = 0; s < d; ++s) {
    const int lo = ab.lo[a[s]], hi = ab.hi[a[s]];
    const int j = lo + q[s];
    if (j > hi) in = false;
    if (j < 1 || j > N - 1) interior = false;
    gi = gi * L + (j <= hi ? j + N : 0);
  }
  D[e] = {(in && !interior) ? g[gi] : 0.0, 0.0};
}

// acc (+)= D * K
__global__ void k_mac_spectra(cx<double>* acc, const cx<double>* D, const cx<double>* K,
                              long total, int first) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const cx<double> t = cmul(D[e], K[e]);
  acc[e] = first ? t : cx<double>{acc[e].x + t.x, acc[e].y + t.y};
}

// b_i = Re D[i + shift] / P^d - c tail_i over the interior i in [1, N-1]^d.
__global__ void k_take_interior(const cx<double>* D, int d, int N, int P, int shift, long nd,
                                double scale, const double* tail, double c, double* b) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nd) return;
  const int n = N - 1;
  long rem = e, pi = 0;
  int i[3] = {0, 0, 0};
  for (int s = d - 1; s >= 0; --s) {
    i[s] = (int)(rem % n) + 1;
    rem /= n;
  }
  for (int s = 0; s < d; ++s) pi = pi * P + (i[s] + shift);
  b[e] = D[pi].x * scale - (tail ? c * tail[e] : 0.0);
}

// 1D: b_i = sum_{j in [i-N, 0] u [N, i+N]} G_{|j-i|} g_j - c tail_i.
__global__ void k_exterior_1d(const double* G, const double* g, int N, const double* tail,
                              double c, double* b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (i > N - 1) return;
  double s = 0.0;
  for (int j = i - N; j <= 0; ++j) s += G[i - j] * g[j + N];
  for (int j = N; j <= i + N; ++j) s += G[j - i] * g[j + N];
  b[i - 1] = s - (tail ? c * tail[i - 1] : 0.0);
}

__global__ void k_difference(const double* a, const double* b, double* out, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = a[e] - b[e];
}

inline unsigned blocks(long n, int thr) { return (unsigned)((n + thr - 1) / thr); }

}  // namespace

void difference(const double* a, const double* b, double* out, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_difference, dim3(blocks(n, 256)), dim3(256), 0, st, a, b, out, n);
  check_launch("difference");
}

// 2D beyond 4N = 2048 points: the block form on M points per axis.
static bool blocked(const Geometry& g) { return g.d == 2 && 2 * g.Ma[0] > 2048; }

bool exterior_supported(const Geometry& g) {
  // the cube only (the exterior lattice of a box is not built); the
  // transforms take at most 2048 points per axis, and in 3D P <= 1024 keeps
  // the two P^3 complex buffers at 17 GB each
  if (!g.cube()) return false;
  const int P = 2 * g.Ma[0];
  return g.d == 1 || g.d == 2 || (g.d == 3 && P <= 1024);
}

static long exterior_points(const Geometry& g) {
  const long P = blocked(g) ? g.Ma[0] : 2L * g.Ma[0];
  long total = 1;
  for (int s = 0; s < g.d; ++s) total *= P;
  return total;
}

size_t exterior_khat_bytes(const Geometry& g) {
  if (g.d == 1) return 0;
  const int nblk = blocked(g) ? 9 : 1;
  return (size_t)nblk * exterior_points(g) * sizeof(cx<double>);
}

size_t exterior_work_bytes(const Geometry& g) {
  if (g.d == 1) return 0;
  return (size_t)(blocked(g) ? 2 : 1) * exterior_points(g) * sizeof(cx<double>);
}

void exterior_term(const Geometry& g, const double* G, double c, const double* g_lat,
                   const double* tail, double* b, int nrhs, void* khat, bool khat_ready,
                   void* work, hipStream_t st) {
  const int N = g.N, d = g.d, thr = 256;
  const long nd = g.nd;
  const long L = 3L * N + 1;
  if (d == 1) {
    for (int o = 0; o < nrhs; ++o) {
      hipLaunchKernelGGL(k_exterior_1d, dim3(blocks(N - 1, thr)), dim3(thr), 0, st, G,
                         g_lat + (long)o * L, N, tail ? tail + (long)o * nd : nullptr, c,
                         b + (long)o * nd);
      check_launch("exterior 1D");
    }
    return;
  }
  const bool blk = blocked(g);
  const int P = blk ? g.Ma[0] : 2 * g.Ma[0];
  const int Pd[3] = {P, P, P};
  long total = 1, Ld = 1;
  for (int s = 0; s < d; ++s) {
    total *= P;
    Ld *= L;
  }
  cx<double>* K = reinterpret_cast<cx<double>*>(khat);
  cx<double>* D = reinterpret_cast<cx<double>*>(work);
  const double scale = 1.0 / (double)total;
  if (blk) {
    const int nb = 9;
    if (!khat_ready) {
      for (int b = 0; b < nb; ++b) {
        hipLaunchKernelGGL(k_block_generator, dim3(blocks(total, thr)), dim3(thr), 0, st, G, d,
                           N, P, b, total, K + (long)b * total);
        check_launch("block generator");
        fft_full(Pd, d, K + (long)b * total, -1, st);
      }
    }
    cx<double>* acc = D + total;
    for (int o = 0; o < nrhs; ++o) {
      for (int b = 0; b < nb; ++b) {
        hipLaunchKernelGGL(k_place_block, dim3(blocks(total, thr)), dim3(thr), 0, st,
                           g_lat + (long)o * Ld, d, N, P, b, total, D);
        check_launch("place block");
        fft_full(Pd, d, D, -1, st);
        hipLaunchKernelGGL(k_mac_spectra, dim3(blocks(total, thr)), dim3(thr), 0, st, acc, D,
                           K + (long)b * total, total, b == 0 ? 1 : 0);
        check_launch("block spectra");
      }
      fft_full(Pd, d, acc, 1, st);
      hipLaunchKernelGGL(k_take_interior, dim3(blocks(nd, thr)), dim3(thr), 0, st, acc, d, N, P,
                         0, nd, scale, tail ? tail + (long)o * nd : nullptr, c, b + (long)o * nd);
      check_launch("interior restriction");
    }
    return;
  }
  if (!khat_ready) {
    hipLaunchKernelGGL(k_wrap_generator, dim3(blocks(total, thr)), dim3(thr), 0, st, G, d, N, P,
                       total, K);
    check_launch("wrap generator");
    fft_full(Pd, d, K, -1, st);
  }
  for (int o = 0; o < nrhs; ++o) {
    hipLaunchKernelGGL(k_place_exterior, dim3(blocks(total, thr)), dim3(thr), 0, st,
                       g_lat + (long)o * Ld, d, N, P, total, D);
    check_launch("place exterior data");
    fft_full(Pd, d, D, -1, st);
    hipLaunchKernelGGL(k_mul_spectra, dim3(blocks(total, thr)), dim3(thr), 0, st, D, K, total);
    check_launch("spectra product");
    fft_full(Pd, d, D, 1, st);
    hipLaunchKernelGGL(k_take_interior, dim3(blocks(nd, thr)), dim3(thr), 0, st, D, d, N, P, N,
                       nd, scale, tail ? tail + (long)o * nd : nullptr, c, b + (long)o * nd);
    check_launch("interior restriction");
  }
}

}  // namespace fl
