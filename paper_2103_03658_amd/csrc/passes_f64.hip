// Double-precision instantiation of the FFT passes, the twiddle tables and
// the symbol construction (lambda-hat = DFT of the embedded generator / M^d).
#include <map>
#include <mutex>

#include "passes_host.h"

namespace fl {

template <>
void apply_passes<double>(const Geometry& g, const Schedule& sc, const double* lam,
                          const void* tw, const double* u, double* y, int nrhs, void* ws,
                          hipStream_t st, int mode, const double* rvec, double* pvec,
                          const double* fvec, const CgScalars* cg, const int* active,
                          hipEvent_t* ev, int only, bool odd) {
  apply_passes_t<double>(g, sc, lam, tw, u, y, nrhs, ws, st, mode, rvec, pvec, fvec, cg, active, ev, only, odd);
}

size_t apply_workspace_bytes(const Geometry& g, int nrhs, bool fp32) {
  return fp32 ? ws_bytes_t<float>(g, nrhs) : ws_bytes_t<double>(g, nrhs);
}

int last_pass_blocks(const Geometry& g, const Schedule& sc) {
  if (g.d == 1) return 1;
  const long C0 = g.d == 2 ? (long)g.n : (long)g.n * g.n;
  return (int)pair_tiles(C0, sc.W_first);
}

const void* twiddles(int M, bool fp32, hipStream_t st) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, bool>, void*> cache;
  int dev = 0;
  FL_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(dev, M, fp32);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  void* p = nullptr;
  const size_t bytes = (size_t)M * (fp32 ? sizeof(cx<float>) : sizeof(cx<double>));
  FL_HIP(hipMalloc(&p, bytes));
  const int thr = 256, blk = (M + thr - 1) / thr;
  if (fp32)
    hipLaunchKernelGGL(k_twiddle<float>, dim3(blk), dim3(thr), 0, st, (cx<float>*)p, M);
  else
    hipLaunchKernelGGL(k_twiddle<double>, dim3(blk), dim3(thr), 0, st, (cx<double>*)p, M);
  check_launch("twiddles");
  FL_HIP(hipStreamSynchronize(st));
  cache[key] = p;
  return p;
}

// c[j] = G[m(j)] with m(j_s) = min(j_s, M - j_s); zero where some m(j_s) > N-2.
__device__ __forceinline__ double embed_value(const double* G, int d, int N, int M, long j) {
  long rem = j;
  long gi = 0;
  bool keep = true;
  int idx[3] = {0, 0, 0};
  for (int s = d - 1; s >= 0; --s) {  // last index fastest
    idx[s] = (int)(rem % M);
    rem /= M;
  }
  for (int s = 0; s < d; ++s) {
    const int m = idx[s] <= M - idx[s] ? idx[s] : M - idx[s];
    keep = keep && (m <= N - 2);
    gi = gi * (N + 1) + m;
  }
  return keep ? G[gi] : 0.0;
}

__global__ void k_embed(cx<double>* c, const double* G, int d, int N, int M, long total) {
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < total) c[j] = {embed_value(G, d, N, M, j), 0.0};
}

__global__ void k_embed_real(double* c, const double* G, int d, int N, int M, long total) {
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < total) c[j] = embed_value(G, d, N, M, j);
}

void embed_generator(const Geometry& g, const double* G, double* out, hipStream_t st) {
  long total = 1;
  for (int s = 0; s < g.d; ++s) total *= g.M;
  hipLaunchKernelGGL(k_embed_real, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, out,
                     G, g.d, g.N, g.M, total);
  check_launch("embed");
}

// lambda-hat folded to k in [0, M/2]^d (H = M/2 + 1 per axis): Re(c_hat[k]) / M^d,
// plus an FP32 copy.
__global__ void k_fold(const cx<double>* chat, double* l64, float* l32, int d, int H, int M,
                       long total, double inv) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= total) return;
  long rem = k;
  int idx[3] = {0, 0, 0};
  for (int s = d - 1; s >= 0; --s) {
    idx[s] = (int)(rem % H);
    rem /= H;
  }
  long ci = 0;
  for (int s = 0; s < d; ++s) ci = ci * M + idx[s];
  const double v = chat[ci].x * inv;
  l64[k] = v;
  l32[k] = (float)v;
}

// Preconditioner multiplier s / max(lambda-hat, 1e-12 max lambda-hat): with
// zero-padded passes the restricted inverse R C^{-1} R^T of the embedding
// circulant C; with odd-extended passes the inverse of the natural tau
// approximation of A (T minus its Hankel part on every level), whose
// eigenvalues t_0 + 2 sum_j t_j cos(j pi k / N) per axis are M^d lambda-hat(k)
// at the interior frequencies k in [1, n]^d (the embedding keeps offsets up
// to N - 2, the tau first column's range).  Floored so that both stay
// positive definite even if some lambda-hat is not.  The transforms are
// unnormalised and lambda-hat carries one 1/M^d, so s = 1/M^(2d).
__global__ void __launch_bounds__(1024) k_symbol_max(const double* l, long n, double* out) {
  __shared__ double sh[16];
  double m = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, l[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t = fmax(t, sh[w]);
    *out = t;
  }
}

__global__ void k_symbol_inv(const double* l, long n, const double* lmax, double s,
                             double* i64, float* i32) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double fl = 1e-12 * lmax[0];
  const double v = s / fmax(l[k], fl);
  i64[k] = v;
  i32[k] = (float)v;
}

void build_inverse_symbol(const Geometry& g, const double* lam64, long nf, double* inv64,
                          float* inv32, double* scratch, hipStream_t st) {
  double s = 1.0;
  for (int k = 0; k < 2 * g.d; ++k) s /= (double)g.M;
  hipLaunchKernelGGL(k_symbol_max, dim3(1), dim3(1024), 0, st, lam64, nf, scratch);
  check_launch("symbol max");
  hipLaunchKernelGGL(k_symbol_inv, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, lam64,
                     nf, scratch, s, inv64, inv32);
  check_launch("symbol inverse");
}

void fft_full(int P, int d, void* cv, int dir, hipStream_t st) {
  cx<double>* c = reinterpret_cast<cx<double>*>(cv);
  const cx<double>* tw = reinterpret_cast<const cx<double>*>(twiddles(P, false, st));
  long total = 1;
  for (int s = 0; s < d; ++s) total *= P;
  const int E = P >= 16 ? 16 : 8;
  const int TPL = P / E;
  const size_t lb = line_lds_bytes<double>(P, E);
  int W = 256 / TPL;
  if (W < 1) W = 1;
  while (W > 1 && tile_lds(P, E, W, sizeof(double)).bytes > 65536) W /= 2;
  const long Pd1 = total / P;  // lines per axis
  if (d >= 2) {
    // axis 0: columns = P^(d-1), row stride P^(d-1)
    C2CArgs<double> a0{c, c, nullptr, Pd1, 0, Pd1, 0, Pd1, 0, 1, P, P, W, 0, 0, 0, tw};
    launch_c2c<double>(P, E, dir, a0, 1, st);
  }
  if (d == 3) {
    // axis 1: slices k0 (stride P*P), rows stride P, columns P
    C2CArgs<double> a1{c, c, nullptr, P, (long)P * P, P, (long)P * P, P, 0, 1, P, P, W, 0, 0, 0,
                       tw};
    launch_c2c<double>(P, E, dir, a1, P, st);
  }
  int LPB = 256 / TPL;
  if (LPB < 1) LPB = 1;
  while (LPB > 1 && lb * LPB > 65536) LPB /= 2;
  launch_rows<double>(P, E, dir, c, Pd1, LPB, tw, st);
}

void build_symbol(const Geometry& g, const double* G, double* lam64, float* lam32,
                  hipStream_t st) {
  const int M = g.M, d = g.d;
  long total = 1;
  for (int s = 0; s < d; ++s) total *= M;
  cx<double>* c = nullptr;
  FL_HIP(hipMalloc(&c, (size_t)total * sizeof(cx<double>)));
  const int thr = 256;
  hipLaunchKernelGGL(k_embed, dim3((unsigned)((total + thr - 1) / thr)), dim3(thr), 0, st, c, G,
                     d, g.N, M, total);
  check_launch("embed");
  fft_full(M, d, c, -1, st);
  long nf = 1;
  for (int s = 0; s < d; ++s) nf *= g.H;
  hipLaunchKernelGGL(k_fold, dim3((unsigned)((nf + thr - 1) / thr)), dim3(thr), 0, st, c, lam64,
                     lam32, d, g.H, M, nf, 1.0 / (double)total);
  check_launch("fold");
  FL_HIP(hipStreamSynchronize(st));
  FL_HIP(hipFree(c));
}

}  // namespace fl
