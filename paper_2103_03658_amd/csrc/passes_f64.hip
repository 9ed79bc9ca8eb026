// Double-precision instantiation of the FFT passes, the twiddle tables and
// the symbol construction (lambda-hat = DFT of the embedded generator / M^d).
#include <map>
#include <mutex>

#include "passes_host.h"

namespace fl {

template <>
void apply_passes<double>(const Geometry& g, const Schedule& sc, const double* lam,
                          const Twiddles& tw, const double* u, double* y, int nrhs, void* ws,
                          hipStream_t st, int mode, const double* rvec, double* pvec,
                          const double* fvec, const CgScalars* cg, const int* active,
                          hipEvent_t* ev, int only, bool odd, bool first_done) {
  apply_passes_t<double>(g, sc, lam, tw, u, y, nrhs, ws, st, mode, rvec, pvec, fvec, cg, active, ev,
                    only, odd, first_done);
}

template <>
void tau_front<double>(const Geometry& g, const Schedule& sc, const double* m, const Twiddles& tw,
                     const double* r, double* S1, int nrhs, hipStream_t st, const CgScalars& cg,
                     const int* active, bool stop_test) {
  tau_front_t<double>(g, sc, m, tw, r, S1, nrhs, st, cg, active, stop_test);
}

template <>
void tau_back_direction<double>(const Geometry& g, const Schedule& sc, const Schedule& sp,
                              const Twiddles& tw, double* S1, double* p, void* T1, int nrhs,
                              hipStream_t st, const CgScalars& cg) {
  tau_back_direction_t<double>(g, sc, sp, tw, S1, p, T1, nrhs, st, cg);
}

size_t apply_workspace_bytes(const Geometry& g, int nrhs, bool fp32) {
  return fp32 ? ws_bytes_t<float>(g, nrhs) : ws_bytes_t<double>(g, nrhs);
}

int last_pass_blocks(const Geometry& g, const Schedule& sc) {
  if (g.d == 1) return 1;
  const long C0 = (long)g.na[1] * g.na[2];   // columns of the axis-0 passes
  return (int)pair_tiles(C0, sc.W_first);
}

void cg1d_solve(const Geometry& g, int E, const double* f, double* x, const double* lam,
                const double* pcs, bool pc_odd, const CgScalars& cg, int nrhs, int maxiter,
                double tol, const void* tw, hipStream_t st) {
  if (g.d != 1) throw Error(2, "one-launch solve: d = 1 only");
  Cg1Args a{f, x, lam, pcs, pc_odd ? 1 : 0, cg, g.na[0], maxiter, tol * tol,
            reinterpret_cast<const cx<double>*>(tw)};
  launch_cg1d(g.Ma[0], E, a, nrhs, st);
}

long sine_mid_blocks(const Geometry& g, const Schedule& sc) {
  const long rows = g.nd / g.na[g.d - 1];     // lines of the last axis
  const long pairs = (rows + 1) / 2;
  return (pairs + sc.LPB_mid - 1) / sc.LPB_mid;
}

int tau_dot_blocks(const Geometry& g, const Schedule& sc, int max_blocks) {
  if (g.d == 1) return 1;
  if (!g.sine_ok()) return tau_dot_blocks_any(g, max_blocks);
  const long mb = sine_mid_blocks(g, sc);
  return mb <= max_blocks ? (int)mb : last_pass_blocks(g, sc);
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

// Sizes of the embedding: per axis the length Ma and the largest kept
// offset Na - 2; the generator is indexed on {0..N}^d.
struct EmbedDims {
  int d, N;
  int Na[3], Ma[3];
};

// c[j] = G[m(j)] with m(j_s) = min(j_s, Ma_s - j_s); zero where some
// m(j_s) > Na_s - 2 (the interior product never reads those offsets).
__device__ __forceinline__ double embed_value(const double* G, const EmbedDims& e, long j) {
  long rem = j;
  long gi = 0;
  bool keep = true;
  int idx[3] = {0, 0, 0};
  for (int s = e.d - 1; s >= 0; --s) {  // last index fastest
    idx[s] = (int)(rem % e.Ma[s]);
    rem /= e.Ma[s];
  }
  for (int s = 0; s < e.d; ++s) {
    const int m = idx[s] <= e.Ma[s] - idx[s] ? idx[s] : e.Ma[s] - idx[s];
    keep = keep && (m <= e.Na[s] - 2);
    gi = gi * (e.N + 1) + (m <= e.N ? m : 0);
  }
  return keep ? G[gi] : 0.0;
}

__global__ void k_embed(cx<double>* c, const double* G, EmbedDims e, long total) {
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < total) c[j] = {embed_value(G, e, j), 0.0};
}

__global__ void k_embed_real(double* c, const double* G, EmbedDims e, long total) {
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < total) c[j] = embed_value(G, e, j);
}

inline EmbedDims embed_dims(const Geometry& g) {
  EmbedDims e{g.d, g.N, {1, 1, 1}, {1, 1, 1}};
  for (int s = 0; s < g.d; ++s) {
    e.Na[s] = g.Na[s];
    e.Ma[s] = g.Ma[s];
  }
  return e;
}

void embed_generator(const Geometry& g, const double* G, double* out, hipStream_t st) {
  const long total = g.nm();
  hipLaunchKernelGGL(k_embed_real, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, out,
                     G, embed_dims(g), total);
  check_launch("embed");
}

// lambda-hat folded to k_s in [0, Ma_s/2] (Ha_s = Ma_s/2 + 1 per axis):
// Re(c_hat[k]) / prod Ma, plus an FP32 copy.
__global__ void k_fold(const cx<double>* chat, double* l64, float* l32, EmbedDims e, long total,
                       double inv) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= total) return;
  long rem = k;
  int idx[3] = {0, 0, 0};
  for (int s = e.d - 1; s >= 0; --s) {
    const int H = e.Ma[s] / 2 + 1;
    idx[s] = (int)(rem % H);
    rem /= H;
  }
  long ci = 0;
  for (int s = 0; s < e.d; ++s) ci = ci * e.Ma[s] + idx[s];
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
  for (int k = 0; k < g.d; ++k) s /= (double)g.Ma[k] * (double)g.Ma[k];
  hipLaunchKernelGGL(k_symbol_max, dim3(1), dim3(1024), 0, st, lam64, nf, scratch);
  check_launch("symbol max");
  hipLaunchKernelGGL(k_symbol_inv, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, lam64,
                     nf, scratch, s, inv64, inv32);
  check_launch("symbol inverse");
}

// One axis transform of the in-place P[0] x .. x P[d-1] array.
static void fft_axis(const int* P, int d, int axis, cx<double>* c, int dir, hipStream_t st) {
  const int L = P[axis];
  const cx<double>* tw = reinterpret_cast<const cx<double>*>(twiddles(L, false, st));
  const int E = L >= 16 ? 16 : 8;
  const int TPL = L / E;
  long outer = 1, inner = 1;
  for (int s = 0; s < axis; ++s) outer *= P[s];
  for (int s = axis + 1; s < d; ++s) inner *= P[s];
  if (axis == d - 1) {
    // contiguous lines
    const size_t lb = line_lds_bytes<double>(L, E);
    int LPB = 256 / TPL;
    if (LPB < 1) LPB = 1;
    while (LPB > 1 && lb * LPB > 65536) LPB /= 2;
    launch_rows<double>(L, E, dir, c, outer, LPB, tw, st);
    return;
  }
  // strided: per outer slice, L rows of `inner` columns
  int W = 256 / TPL;
  if (W < 1) W = 1;
  while (W > 1 && tile_lds(L, E, W, sizeof(double)).bytes > 65536) W /= 2;
  const long os = (long)L * inner;
  C2CArgs<double> a{c, c, nullptr, inner, os, inner, os, inner, 0, 1, L, L, W, 0, 0, 0, tw};
  launch_c2c<double>(L, E, dir, a, outer, st);
}

void fft_full(const int* P, int d, void* cv, int dir, hipStream_t st) {
  cx<double>* c = reinterpret_cast<cx<double>*>(cv);
  for (int axis = 0; axis < d; ++axis) fft_axis(P, d, axis, c, dir, st);
}

void build_symbol(const Geometry& g, const double* G, double* lam64, float* lam32,
                  hipStream_t st) {
  const int d = g.d;
  const long total = g.nm();
  const EmbedDims e = embed_dims(g);
  SetupScratch scr((size_t)total * sizeof(cx<double>), st);
  cx<double>* c = (cx<double>*)scr.take((size_t)total * sizeof(cx<double>));
  const int thr = 256;
  hipLaunchKernelGGL(k_embed, dim3((unsigned)((total + thr - 1) / thr)), dim3(thr), 0, st, c, G,
                     e, total);
  check_launch("embed");
  fft_full(g.Ma, d, c, -1, st);
  const long nf = g.nh();
  hipLaunchKernelGGL(k_fold, dim3((unsigned)((nf + thr - 1) / thr)), dim3(thr), 0, st, c, lam64,
                     lam32, e, nf, 1.0 / (double)total);
  check_launch("fold");
  FL_HIP(hipStreamSynchronize(st));
}

}  // namespace fl

namespace fl {

// ---------------------------------------------------------------------------
// The tau preconditioner where some 2 N_s is not a power of two.  The
// embedding symbol then samples other frequencies, so the eigenvalues of the
// tau approximation are summed directly as the truncated cosine series
//   lam(k) = sum_{j_s <= N_s - 2} G_j prod_s w(j_s) cos(pi j_s k_s / N_s),
// w(0) = 1, w(j) = 2 (the first column of tau(T) on each level), one axis at
// a time, on k in [0, N_s]^d.  The multiplier is then the one the
// power-of-two path stores, 1 / (prod_s 2 N_s  max(lam, 1e-12 max lam)),
// with the maximum over the interior frequencies k_s in [1, N_s - 1], and
// zero elsewhere (those slots multiply zeros).
// ---------------------------------------------------------------------------
bool Geometry::sine_any_ok() const {
  for (int s = 0; s < d; ++s) {
    RadixPlan p;
    if (!radix_plan(La[s], p)) return false;
  }
  return true;
}

int tau_dot_blocks_any(const Geometry& g, int max_blocks) {
  const long mb = sine_any_mid_blocks(g);
  return mb <= max_blocks ? (int)mb : (int)sine_any_last_blocks(g);
}

namespace {

// cos(pi m / Ns), m < 2 Ns
__global__ void k_cos_table(double* t, int Ns) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < 2 * Ns) t[m] = cospi((double)m / (double)Ns);
}

// out[.., k, ..] = sum_{j = 0}^{Ns - 2} w(j) cos(pi j k / Ns) in[.., j, ..]
// along `axis` of the row-major arrays in (dims I) and out (dims O, O[axis] =
// Ns + 1, the others equal to I's).
__global__ void k_tau_axis(const double* in, double* out, int I0, int I1, int I2, int O0,
                           int O1, int O2, int axis, int Ns, const double* ctab) {
  const long total = (long)O0 * O1 * O2;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int o2 = (int)(e % O2), o1 = (int)((e / O2) % O1), o0 = (int)(e / ((long)O1 * O2));
  const int k = axis == 0 ? o0 : axis == 1 ? o1 : o2;
  const long sin0 = (long)I1 * I2, sin1 = I2;
  const long stride = axis == 0 ? sin0 : axis == 1 ? sin1 : 1;
  long base = (axis == 0 ? 0 : (long)o0 * sin0) + (axis == 1 ? 0 : (long)o1 * sin1) +
              (axis == 2 ? 0 : o2);
  double acc = 0.0;
  int m = 0;   // (j k) mod 2 Ns
  for (int j = 0; j <= Ns - 2; ++j) {
    const double w = j == 0 ? 1.0 : 2.0;
    acc += w * ctab[m] * in[base + (long)j * stride];
    m += k;
    if (m >= 2 * Ns) m -= 2 * Ns;
  }
  out[e] = acc;
}

// zero lam outside the interior frequencies k_s in [1, Ns - 1] (in place)
__global__ void k_tau_interior(double* lam, int H0, int H1, int H2, int d) {
  const long total = (long)H0 * H1 * H2;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int k2 = (int)(e % H2), k1 = (int)((e / H2) % H1), k0 = (int)(e / ((long)H1 * H2));
  bool in = k0 >= 1 && k0 <= H0 - 2;
  if (d >= 2) in = in && k1 >= 1 && k1 <= H1 - 2;
  if (d >= 3) in = in && k2 >= 1 && k2 <= H2 - 2;
  if (!in) lam[e] = 0.0;
}

__global__ void k_tau_mult(const double* lam, long n, const double* lmax, double s, double* m64,
                           float* m32) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double l = lam[k];
  const double v = l == 0.0 ? 0.0 : s / fmax(l, 1e-12 * lmax[0]);
  m64[k] = v;
  m32[k] = (float)v;
}

}  // namespace

long tau_any_entries(const Geometry& g) {
  long n = 1;
  for (int s = 0; s < g.d; ++s) n *= g.Na[s] + 1;
  return n;
}

void build_tau_multiplier(const Geometry& g, const double* G, double* m64, float* m32,
                          hipStream_t st) {
  int I[3] = {1, 1, 1};
  for (int s = 0; s < g.d; ++s) I[s] = g.N + 1;
  long cap = 1;
  for (int s = 0; s < g.d; ++s) cap *= g.N + 1;
  int maxN = 0;
  for (int s = 0; s < g.d; ++s) maxN = g.Na[s] > maxN ? g.Na[s] : maxN;
  SetupScratch scr(2 * scratch_round((size_t)cap * sizeof(double)) +
                       scratch_round((size_t)2 * maxN * sizeof(double)) + 256,
                   st);
  double* a = (double*)scr.take((size_t)cap * sizeof(double));
  double* b = (double*)scr.take((size_t)cap * sizeof(double));
  double* ctab = (double*)scr.take((size_t)2 * maxN * sizeof(double));
  double* lmax = (double*)scr.take(sizeof(double));
  const double* src = G;
  double* dst = a;
  for (int ax = 0; ax < g.d; ++ax) {
    const int Ns = g.Na[ax];
    hipLaunchKernelGGL(k_cos_table, dim3((2 * Ns + 255) / 256), dim3(256), 0, st, ctab, Ns);
    check_launch("cosine table");
    int O[3] = {I[0], I[1], I[2]};
    O[ax] = Ns + 1;
    // dims as three axes (trailing ones for d = 2)
    const long tot = (long)O[0] * O[1] * O[2];
    hipLaunchKernelGGL(k_tau_axis, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, src,
                       dst, I[0], I[1], I[2], O[0], O[1], O[2], ax, Ns, ctab);
    check_launch("tau eigenvalues");
    I[ax] = O[ax];
    src = dst;
    dst = dst == a ? b : a;
  }
  double* lam = const_cast<double*>(src);
  const long n = (long)I[0] * I[1] * I[2];
  hipLaunchKernelGGL(k_tau_interior, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lam,
                     I[0], I[1], I[2], g.d);
  check_launch("tau interior");
  hipLaunchKernelGGL(k_symbol_max, dim3(1), dim3(1024), 0, st, lam, n, lmax);
  check_launch("tau max");
  double s = 1.0;
  for (int ax = 0; ax < g.d; ++ax) s /= 2.0 * (double)g.Na[ax];
  hipLaunchKernelGGL(k_tau_mult, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lam, n, lmax,
                     s, m64, m32);
  check_launch("tau multiplier");
  FL_HIP(hipStreamSynchronize(st));
}

}  // namespace fl
