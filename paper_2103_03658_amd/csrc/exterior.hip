// Exterior-data term of the scheme with nonhomogeneous data u = g outside
// Omega (Sec. 2.1 eq. (1D-scheme), Sec. 2.2 eq. (2D-scheme) and the terms b
// of their matrix forms):
//   b_i = sum over exterior lattice nodes j, |j - i|_inf <= N, of G_{|j-i|} g(x_j)
//         - c_{d,alpha} tail_i
// Axis s of the grid has Na_s intervals (Na_s = N on the cube), interior
// nodes 1..Na_s - 1 and the node lattice [-N, Na_s + N] (length L_s =
// Na_s + 2N + 1); the lattice sum is a multilevel Toeplitz product of G with
// g on that lattice (zero on the interior nodes).
//
// Direct form (2D, 3D): circular embedding in P_s >= L_s points per axis,
// data at j + N, G wrapped to k mod P_s for |k| <= N.  Every offset i - j of
// an interior i and a lattice j lies in [1 - Na_s - N, Na_s + N - 1], and
// those with |i - j| > N land in the zero band (N, P_s - N) of the wrapped
// generator, so the circular product restricted to the interior is the sum.
//
// Block form (2D, when some L_s would need more than 2048 points): each axis
// of the lattice is cut into [-N, -1], [0, Na_s] and [Na_s + 1, Na_s + N].
// For an interior i and the nodes j of a block from lo to hi, the offsets
// i - j take fewer than P_s >= max(2 Na_s, Na_s + N) distinct values, so with
// the block's data placed from position 0 and G at (i - j + lo) mod P_s (for
// the block's offsets with |i - j| <= N, zero elsewhere) a circular product
// of length P_s is exact at positions i; the 3^d block products are summed
// as spectra and transformed back once.
//
// In 1D the sum over the 2N + 1 offsets is taken directly.

#include <hip/hip_runtime.h>

#include "passes_impl.h"

namespace fl {
namespace {

struct ExtGeom {
  int d, N;
  int Na[3];   // intervals per axis
  int L[3];    // lattice length per axis, Na + 2N + 1
  int P[3];    // transform length per axis
};

__device__ inline void split_index(long e, const ExtGeom& x, int* q) {
  for (int s = x.d - 1; s >= 0; --s) {
    q[s] = (int)(e % x.P[s]);
    e /= x.P[s];
  }
}

// Direct form: wrapped generator K[q] = G_{|k|}, k_s = q_s or q_s - P_s, |k_s| <= N.
__global__ void k_wrap_generator(const double* G, ExtGeom x, long total, cx<double>* K) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int q[3] = {0, 0, 0};
  split_index(e, x, q);
  long gi = 0;
  bool inside = true;
  for (int s = 0; s < x.d; ++s) {
    const int P = x.P[s], N = x.N;
    const int k = q[s] <= N ? q[s] : (q[s] >= P - N ? P - q[s] : -1);
    if (k < 0) inside = false;
    gi = gi * (N + 1) + (k < 0 ? 0 : k);
  }
  K[e] = {inside ? G[gi] : 0.0, 0.0};
}

// Direct form: exterior lattice data at position j + N, zero on interior
// nodes (1 <= j_s <= Na_s - 1 for every s) and beyond the lattice.
__global__ void k_place_exterior(const double* g, ExtGeom x, long total, cx<double>* D) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int q[3] = {0, 0, 0};
  split_index(e, x, q);
  long gi = 0;
  bool inlat = true, interior = true;
  for (int s = 0; s < x.d; ++s) {
    if (q[s] >= x.L[s]) inlat = false;
    const int j = q[s] - x.N;
    if (j < 1 || j > x.Na[s] - 1) interior = false;
    gi = gi * x.L[s] + (q[s] < x.L[s] ? q[s] : 0);
  }
  D[e] = {(inlat && !interior) ? g[gi] : 0.0, 0.0};
}

// Block form: block a_s of axis s covers nodes [lo, hi].
__device__ inline void block_range(const ExtGeom& x, int s, int a, int& lo, int& hi) {
  const int N = x.N, Na = x.Na[s];
  lo = a == 0 ? -N : (a == 1 ? 0 : Na + 1);
  hi = a == 0 ? -1 : (a == 1 ? Na : Na + N);
}

__device__ inline void block_axes(int blk, int d, int* a) {
  for (int s = d - 1; s >= 0; --s) {
    a[s] = blk % 3;
    blk /= 3;
  }
}

// Block form: generator of block blk; position q_s holds the offset
// k_s = v_s - lo_s, v_s = q_s (q_s <= Na_s - 1) or q_s - P_s, for the offsets
// of interior nodes and the block's nodes with |k_s| <= N; zero elsewhere.
__global__ void k_block_generator(const double* G, ExtGeom x, int blk, long total,
                                  cx<double>* K) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int q[3] = {0, 0, 0}, a[3] = {0, 0, 0};
  split_index(e, x, q);
  block_axes(blk, x.d, a);
  const int N = x.N;
  long gi = 0;
  bool ok = true;
  for (int s = 0; s < x.d; ++s) {
    int lo, hi;
    block_range(x, s, a[s], lo, hi);
    const int v = q[s] <= x.Na[s] - 1 ? q[s] : q[s] - x.P[s];
    const int k = v - lo;
    if (k < 1 - hi || k > x.Na[s] - 1 - lo || k < -N || k > N) ok = false;
    gi = gi * (N + 1) + (ok ? (k < 0 ? -k : k) : 0);
  }
  K[e] = {ok ? G[gi] : 0.0, 0.0};
}

// Block form: exterior data of block blk, position q_s holding node lo_s + q_s
// for q_s <= hi_s - lo_s; interior nodes are zero.
__global__ void k_place_block(const double* g, ExtGeom x, int blk, long total, cx<double>* D) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int q[3] = {0, 0, 0}, a[3] = {0, 0, 0};
  split_index(e, x, q);
  block_axes(blk, x.d, a);
  long gi = 0;
  bool in = true, interior = true;
  for (int s = 0; s < x.d; ++s) {
    int lo, hi;
    block_range(x, s, a[s], lo, hi);
    const int j = lo + q[s];
    if (j > hi) in = false;
    if (j < 1 || j > x.Na[s] - 1) interior = false;
    gi = gi * x.L[s] + (j <= hi ? j + x.N : 0);
  }
  D[e] = {(in && !interior) ? g[gi] : 0.0, 0.0};
}

__global__ void k_mul_spectra(cx<double>* D, const cx<double>* K, long total) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) D[e] = cmul(D[e], K[e]);
}

// acc (+)= D * K
__global__ void k_mac_spectra(cx<double>* acc, const cx<double>* D, const cx<double>* K,
                              long total, int first) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const cx<double> t = cmul(D[e], K[e]);
  acc[e] = first ? t : cx<double>{acc[e].x + t.x, acc[e].y + t.y};
}

// b_i = Re D[i + shift] / prod P - c tail_i over the interior nodes.
__global__ void k_take_interior(const cx<double>* D, ExtGeom x, int shift, long nd,
                                double scale, const double* tail, double c, double* b) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nd) return;
  long rem = e, pi = 0;
  int i[3] = {0, 0, 0};
  for (int s = x.d - 1; s >= 0; --s) {
    const int n = x.Na[s] - 1;
    i[s] = (int)(rem % n) + 1;
    rem /= n;
  }
  for (int s = 0; s < x.d; ++s) pi = pi * x.P[s] + (i[s] + shift);
  b[e] = D[pi].x * scale - (tail ? c * tail[e] : 0.0);
}

// 1D: b_i = sum_{j in [i-N, 0] u [Na, i+N]} G_{|j-i|} g_j - c tail_i.
__global__ void k_exterior_1d(const double* G, const double* g, int N, int Na,
                              const double* tail, double c, double* b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (i > Na - 1) return;
  double s = 0.0;
  for (int j = i - N; j <= 0; ++j) s += G[i - j] * g[j + N];
  for (int j = Na; j <= i + N; ++j) s += G[j - i] * g[j + N];
  b[i - 1] = s - (tail ? c * tail[i - 1] : 0.0);
}

__global__ void k_difference(const double* a, const double* b, double* out, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = a[e] - b[e];
}

inline unsigned blocks(long n, int thr) { return (unsigned)((n + thr - 1) / thr); }

inline int pow2_at_least(long v) {
  int p = 8;
  while (p < v) p *= 2;
  return p;
}

// Transform lengths of the direct form, or of the block form when a direct
// axis would need more than 2048 points (2D only).
ExtGeom ext_geom(const Geometry& g, bool* blocked) {
  ExtGeom x{};
  x.d = g.d;
  x.N = g.N;
  bool blk = false;
  for (int s = 0; s < 3; ++s) {
    x.Na[s] = s < g.d ? g.Na[s] : 2;
    x.L[s] = s < g.d ? g.Na[s] + 2 * g.N + 1 : 1;
    x.P[s] = s < g.d ? pow2_at_least(x.L[s]) : 1;
    if (s < g.d && x.P[s] > 2048) blk = true;
  }
  if (blk)
    for (int s = 0; s < g.d; ++s)
      x.P[s] = pow2_at_least(std::max(2L * g.Na[s], (long)g.Na[s] + g.N));
  if (blocked) *blocked = blk;
  return x;
}

long ext_points(const ExtGeom& x) {
  long t = 1;
  for (int s = 0; s < x.d; ++s) t *= x.P[s];
  return t;
}

}  // namespace

void difference(const double* a, const double* b, double* out, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_difference, dim3(blocks(n, 256)), dim3(256), 0, st, a, b, out, n);
  check_launch("difference");
}

bool exterior_supported(const Geometry& g) {
  if (g.d == 1) return true;
  bool blk = false;
  const ExtGeom x = ext_geom(g, &blk);
  // the block form is built for 2D; in 3D the direct form with at most
  // 1024^3 points keeps the two transform buffers at 17 GB each
  if (g.d == 3) return !blk && ext_points(x) <= 1024L * 1024 * 1024;
  return true;
}

size_t exterior_khat_bytes(const Geometry& g) {
  if (g.d == 1) return 0;
  bool blk = false;
  const ExtGeom x = ext_geom(g, &blk);
  return (size_t)(blk ? 9 : 1) * ext_points(x) * sizeof(cx<double>);
}

size_t exterior_work_bytes(const Geometry& g) {
  if (g.d == 1) return 0;
  bool blk = false;
  const ExtGeom x = ext_geom(g, &blk);
  return (size_t)(blk ? 2 : 1) * ext_points(x) * sizeof(cx<double>);
}

void exterior_term(const Geometry& g, const double* G, double c, const double* g_lat,
                   const double* tail, double* b, int nrhs, void* khat, bool khat_ready,
                   void* work, hipStream_t st) {
  const int N = g.N, d = g.d, thr = 256;
  const long nd = g.nd;
  if (d == 1) {
    const int Na = g.Na[0];
    const long L = Na + 2L * N + 1;
    for (int o = 0; o < nrhs; ++o) {
      hipLaunchKernelGGL(k_exterior_1d, dim3(blocks(Na - 1, thr)), dim3(thr), 0, st, G,
                         g_lat + (long)o * L, N, Na, tail ? tail + (long)o * nd : nullptr, c,
                         b + (long)o * nd);
      check_launch("exterior 1D");
    }
    return;
  }
  bool blk = false;
  const ExtGeom x = ext_geom(g, &blk);
  const int Pd[3] = {x.P[0], x.P[1], x.P[2]};
  const long total = ext_points(x);
  long Ld = 1;
  for (int s = 0; s < d; ++s) Ld *= x.L[s];
  cx<double>* K = reinterpret_cast<cx<double>*>(khat);
  cx<double>* D = reinterpret_cast<cx<double>*>(work);
  const double scale = 1.0 / (double)total;
  if (blk) {
    int nb = 1;
    for (int s = 0; s < d; ++s) nb *= 3;
    if (!khat_ready) {
      for (int bi = 0; bi < nb; ++bi) {
        hipLaunchKernelGGL(k_block_generator, dim3(blocks(total, thr)), dim3(thr), 0, st, G, x,
                           bi, total, K + (long)bi * total);
        check_launch("block generator");
        fft_full(Pd, d, K + (long)bi * total, -1, st);
      }
    }
    cx<double>* acc = D + total;
    for (int o = 0; o < nrhs; ++o) {
      for (int bi = 0; bi < nb; ++bi) {
        hipLaunchKernelGGL(k_place_block, dim3(blocks(total, thr)), dim3(thr), 0, st,
                           g_lat + (long)o * Ld, x, bi, total, D);
        check_launch("place block");
        fft_full(Pd, d, D, -1, st);
        hipLaunchKernelGGL(k_mac_spectra, dim3(blocks(total, thr)), dim3(thr), 0, st, acc, D,
                           K + (long)bi * total, total, bi == 0 ? 1 : 0);
        check_launch("block spectra");
      }
      fft_full(Pd, d, acc, 1, st);
      hipLaunchKernelGGL(k_take_interior, dim3(blocks(nd, thr)), dim3(thr), 0, st, acc, x, 0, nd,
                         scale, tail ? tail + (long)o * nd : nullptr, c, b + (long)o * nd);
      check_launch("interior restriction");
    }
    return;
  }
  if (!khat_ready) {
    hipLaunchKernelGGL(k_wrap_generator, dim3(blocks(total, thr)), dim3(thr), 0, st, G, x, total,
                       K);
    check_launch("wrap generator");
    fft_full(Pd, d, K, -1, st);
  }
  for (int o = 0; o < nrhs; ++o) {
    hipLaunchKernelGGL(k_place_exterior, dim3(blocks(total, thr)), dim3(thr), 0, st,
                       g_lat + (long)o * Ld, x, total, D);
    check_launch("place exterior data");
    fft_full(Pd, d, D, -1, st);
    hipLaunchKernelGGL(k_mul_spectra, dim3(blocks(total, thr)), dim3(thr), 0, st, D, K, total);
    check_launch("spectra product");
    fft_full(Pd, d, D, 1, st);
    hipLaunchKernelGGL(k_take_interior, dim3(blocks(nd, thr)), dim3(thr), 0, st, D, x, N, nd,
                       scale, tail ? tail + (long)o * nd : nullptr, c, b + (long)o * nd);
    check_launch("interior restriction");
  }
}

}  // namespace fl
