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
// circular product restricted to the interior is the lattice sum.  In 1D the
// sum over the 2N + 1 offsets is taken directly.

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

// b_i = Re D[i + N] / P^d - c tail_i over the interior i in [1, N-1]^d.
__global__ void k_take_interior(const cx<double>* D, int d, int N, int P, long nd, double scale,
                                const double* tail, double c, double* b) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nd) return;
  const int n = N - 1;
  long rem = e, pi = 0;
  int i[3] = {0, 0, 0};
  for (int s = d - 1; s >= 0; --s) {
    i[s] = (int)(rem % n) + 1;
    rem /= n;
  }
  for (int s = 0; s < d; ++s) pi = pi * P + (i[s] + N);
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

bool exterior_supported(const Geometry& g) {
  // the cube only (the exterior lattice of a box is not built); the
  // transforms take P <= 2048 per axis, and in 3D P <= 1024 keeps the two
  // P^3 complex buffers at 17 GB each
  if (!g.cube()) return false;
  const int P = 2 * g.Ma[0];
  return g.d == 1 || (g.d == 2 && P <= 2048) || (g.d == 3 && P <= 1024);
}

size_t exterior_khat_bytes(const Geometry& g) {
  if (g.d == 1) return 0;
  const long P = 2L * g.Ma[0];
  long total = 1;
  for (int s = 0; s < g.d; ++s) total *= P;
  return (size_t)total * sizeof(cx<double>);
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
  const int P = 2 * g.Ma[0];
  const int Pd[3] = {P, P, P};
  long total = 1, Ld = 1;
  for (int s = 0; s < d; ++s) {
    total *= P;
    Ld *= L;
  }
  cx<double>* K = reinterpret_cast<cx<double>*>(khat);
  cx<double>* D = reinterpret_cast<cx<double>*>(work);
  if (!khat_ready) {
    hipLaunchKernelGGL(k_wrap_generator, dim3(blocks(total, thr)), dim3(thr), 0, st, G, d, N, P,
                       total, K);
    check_launch("wrap generator");
    fft_full(Pd, d, K, -1, st);
  }
  const double scale = 1.0 / (double)total;
  for (int o = 0; o < nrhs; ++o) {
    hipLaunchKernelGGL(k_place_exterior, dim3(blocks(total, thr)), dim3(thr), 0, st,
                       g_lat + (long)o * Ld, d, N, P, total, D);
    check_launch("place exterior data");
    fft_full(Pd, d, D, -1, st);
    hipLaunchKernelGGL(k_mul_spectra, dim3(blocks(total, thr)), dim3(thr), 0, st, D, K, total);
    check_launch("spectra product");
    fft_full(Pd, d, D, 1, st);
    hipLaunchKernelGGL(k_take_interior, dim3(blocks(nd, thr)), dim3(thr), 0, st, D, d, N, P, nd,
                       scale, tail ? tail + (long)o * nd : nullptr, c, b + (long)o * nd);
    check_launch("interior restriction");
  }
}

}  // namespace fl
