// Operator setup on the GPU in FP64: weight integrals, origin rule,
// coefficients a_k, diagonal a_0 and the generator G = -c a.
//
// Weight integrals (Sec. 2.1 eq. (wi-1D), Sec. 2.2 eq. (2D-scheme0),
// Remark 2.2 for a kernel K):  omega_k = int_{[0,L]^d} phi_k K(|xi|)
// |xi|^{gamma-d-alpha} dxi, gamma in (alpha, 2] the splitting parameter
// (sigma = gamma - alpha below), evaluated element by element:
//  * every element away from xi = 0 by tensor Gauss-Legendre (16 points per
//    axis within four elements of the origin, 8 beyond, where the nearest
//    singularity is far outside the element's Bernstein ellipse);
//  * the element at the origin in cone coordinates xi = r e(w): the radial
//    factor r^{sigma-1} times a polynomial (times exp(-lambda h rho r)) is
//    integrated exactly (power moments, or the all-positive series of the
//    lower incomplete gamma function), the cone coordinates w by
//    Gauss-Legendre.  No closed form with cancellation is used.
// For K = 1 the integrals are taken on the unit lattice and scaled by
// h^{sigma}.  Nodes gather their elements in a fixed order and a_0 is a
// fixed-order tree sum, so the generator is deterministic.
#include <cmath>
#include <vector>

#include "fl_internal.h"

namespace fl {

namespace {

constexpr int NA = 32;   // cone-coordinate points per axis (origin element, far field)
constexpr int QN = 16;   // element points per axis near the origin
constexpr int QF = 8;    // element points per axis elsewhere
constexpr int QP = 16;   // points per panel, far-field radial integral

struct GLTables {
  double xa[NA], wa[NA];   // [0,1]
  double xn[QN], wn[QN];   // [-1,1]
  double xf[QF], wf[QF];
  double xp[QP], wp[QP];   // [-1,1]
};

void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    long double z = std::cos(M_PI * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    x[i] = (double)z;
    w[i] = (double)(2.0L / ((1 - z * z) * dp * dp));
  }
}

// Lagrange basis of the element in local coordinates tau (lattice units):
// coefficient i of tau^i for local basis a.
__device__ __forceinline__ double basis_coef(int p, int a, int i) {
  if (p == 0) return i == 0 ? 1.0 : 0.0;
  if (p == 1) {
    if (a == 0) return i == 0 ? 1.0 : (i == 1 ? -1.0 : 0.0);
    return i == 1 ? 1.0 : 0.0;
  }
  // p = 2 on [0, 2]: (t-1)(t-2)/2, t(2-t), t(t-1)/2
  const double c[3][3] = {{1.0, -1.5, 0.5}, {0.0, 2.0, -1.0}, {0.0, -0.5, 0.5}};
  return i < 3 ? c[a][i] : 0.0;
}

__device__ __forceinline__ double basis_val(int p, int a, double tau) {
  if (p == 0) return 1.0;
  if (p == 1) return a == 0 ? 1.0 - tau : tau;
  if (a == 0) return 0.5 * (tau - 1.0) * (tau - 2.0);
  if (a == 1) return tau * (2.0 - tau);
  return 0.5 * tau * (tau - 1.0);
}

// int_0^H r^{s-1} exp(-c r) dr, s > 0, c >= 0: H^s e^{-cH} sum_k (cH)^k / (s (s+1) .. (s+k))
__device__ double radial_moment(double s, double c, double H) {
  const double Hs = pow(H, s);
  if (c == 0.0) return Hs / s;
  const double x = c * H;
  double term = 1.0 / s, sum = term;
  for (int k = 1; k < 400; ++k) {
    term *= x / (s + k);
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return Hs * exp(-x) * sum;
}

__device__ __forceinline__ double bsum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < 64) {
    s = threadIdx.x < (blockDim.x + 63) / 64 ? sh[threadIdx.x] : 0.0;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  }
  return s;
}

// ---------------------------------------------------------------------------
// origin element: out[a] for local multi-index a (nb^d values), lattice units
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_origin(int d, int p, double sig, double lamh,
                                                const GLTables* tb, double* out) {
  __shared__ double sh[8];
  const int nb = p + 1;
  const double H = p == 0 ? 0.5 : (p == 1 ? 1.0 : 2.0);
  int nout = 1;
  for (int s = 0; s < d; ++s) nout *= nb;
  const int nang = d == 1 ? 1 : (d == 2 ? NA : NA * NA);
  const int npts = d * nang;
  double acc[27];
  for (int i = 0; i < 27; ++i) acc[i] = 0.0;
  for (int pt = threadIdx.x; pt < npts; pt += blockDim.x) {
    const int s = pt / nang, ia = pt % nang;
    double e[3], wang = 1.0;
    int j = 0;
    for (int dd = 0; dd < d; ++dd) {
      if (dd == s) {
        e[dd] = 1.0;
      } else {
        const int q = j == 0 ? ia % NA : ia / NA;
        e[dd] = tb->xa[q];
        wang *= tb->wa[q];
        ++j;
      }
    }
    double rho2 = 0.0;
    for (int dd = 0; dd < d; ++dd) rho2 += e[dd] * e[dd];
    const double rho = sqrt(rho2);
    const double ang = wang * pow(rho, sig - d);
    // radial moments r^{sigma-1+m}, m = 0 .. d*p
    double mom[7];
    for (int m = 0; m <= d * p; ++m) mom[m] = radial_moment(sig + m, lamh * rho, H);
    for (int o = 0; o < nout; ++o) {
      // polynomial in r of prod_dd phi_{a_dd}(r e_dd)
      double poly[7] = {1, 0, 0, 0, 0, 0, 0};
      int deg = 0, rem = o;
      int aidx[3];
      for (int dd = d - 1; dd >= 0; --dd) {
        aidx[dd] = rem % nb;
        rem /= nb;
      }
      for (int dd = 0; dd < d; ++dd) {
        double f[3];
        double ep = 1.0;
        for (int i = 0; i <= p; ++i) {
          f[i] = basis_coef(p, aidx[dd], i) * ep;
          ep *= e[dd];
        }
        double np[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int i = 0; i <= deg; ++i)
          for (int k = 0; k <= p; ++k) np[i + k] += poly[i] * f[k];
        deg += p;
        for (int i = 0; i <= deg; ++i) poly[i] = np[i];
      }
      double v = 0.0;
      for (int m = 0; m <= deg; ++m) v += poly[m] * mom[m];
      acc[o] += ang * v;
    }
  }
  for (int o = 0; o < nout; ++o) {
    const double t = bsum(acc[o], sh);
    if (threadIdx.x == 0) out[o] = t;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// all other elements: out[e][a] (nb^d values per element), lattice units
// ---------------------------------------------------------------------------
__device__ __forceinline__ void elem_bounds(int p, int N, int e, double& lo, double& hi,
                                            double& org) {
  if (p == 0) {
    lo = fmax(e - 0.5, 0.0);
    hi = fmin(e + 0.5, (double)N);
    org = 0.0;
  } else if (p == 1) {
    lo = e;
    hi = e + 1.0;
    org = e;
  } else {
    lo = 2.0 * e;
    hi = 2.0 * e + 2.0;
    org = 2.0 * e;
  }
}

template <int Q>
__device__ void elem_quad(int d, int p, int N, const int* ev, double sig, double lamh,
                          const double* xq, const double* wq, double* acc) {
  const int nb = p + 1;
  double X[3][Q], Wt[3][Q], B[3][3][Q];
  for (int s = 0; s < d; ++s) {
    double lo, hi, org;
    elem_bounds(p, N, ev[s], lo, hi, org);
    for (int q = 0; q < Q; ++q) {
      const double x = lo + (hi - lo) * 0.5 * (xq[q] + 1.0);
      X[s][q] = x;
      Wt[s][q] = wq[q] * (hi - lo) * 0.5;
      for (int a = 0; a < nb; ++a) B[s][a][q] = basis_val(p, a, x - org);
    }
  }
  const double ex = 0.5 * (sig - d);
  int nout = 1;
  for (int s = 0; s < d; ++s) nout *= nb;
  for (int o = 0; o < nout; ++o) acc[o] = 0.0;
  if (d == 1) {
    for (int q = 0; q < Q; ++q) {
      const double r2 = X[0][q] * X[0][q];
      double g = pow(r2, ex) * Wt[0][q];
      if (lamh != 0.0) g *= exp(-lamh * sqrt(r2));
      for (int a = 0; a < nb; ++a) acc[a] += g * B[0][a][q];
    }
  } else if (d == 2) {
    for (int q0 = 0; q0 < Q; ++q0)
      for (int q1 = 0; q1 < Q; ++q1) {
        const double r2 = X[0][q0] * X[0][q0] + X[1][q1] * X[1][q1];
        double g = pow(r2, ex) * Wt[0][q0] * Wt[1][q1];
        if (lamh != 0.0) g *= exp(-lamh * sqrt(r2));
        for (int a = 0; a < nb; ++a) {
          const double ga = g * B[0][a][q0];
          for (int b = 0; b < nb; ++b) acc[a * nb + b] += ga * B[1][b][q1];
        }
      }
  } else {
    for (int q0 = 0; q0 < Q; ++q0)
      for (int q1 = 0; q1 < Q; ++q1) {
        const double r01 = X[0][q0] * X[0][q0] + X[1][q1] * X[1][q1];
        const double w01 = Wt[0][q0] * Wt[1][q1];
        for (int q2 = 0; q2 < Q; ++q2) {
          const double r2 = r01 + X[2][q2] * X[2][q2];
          double g = pow(r2, ex) * w01 * Wt[2][q2];
          if (lamh != 0.0) g *= exp(-lamh * sqrt(r2));
          for (int a = 0; a < nb; ++a) {
            const double ga = g * B[0][a][q0];
            for (int b = 0; b < nb; ++b) {
              const double gab = ga * B[1][b][q1];
              for (int c = 0; c < nb; ++c) acc[(a * nb + b) * nb + c] += gab * B[2][c][q2];
            }
          }
        }
      }
  }
}

__global__ void __launch_bounds__(128) k_elements(int d, int p, int N, int Eel, long total,
                                                  double sig, double lamh,
                                                  const GLTables* tb, double* out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int nb = p + 1;
  int nout = 1;
  for (int s = 0; s < d; ++s) nout *= nb;
  int ev[3] = {0, 0, 0};
  long rem = e;
  int emax = 0;
  for (int s = d - 1; s >= 0; --s) {
    ev[s] = (int)(rem % Eel);
    rem /= Eel;
    emax = ev[s] > emax ? ev[s] : emax;
  }
  double acc[27];
  if (e == 0) {
    for (int o = 0; o < nout; ++o) out[o] = 0.0;  // origin element handled by k_origin
    return;
  }
  if (emax < 4)
    elem_quad<QN>(d, p, N, ev, sig, lamh, tb->xn, tb->wn, acc);
  else
    elem_quad<QF>(d, p, N, ev, sig, lamh, tb->xf, tb->wf, acc);
  for (int o = 0; o < nout; ++o) out[e * nout + o] = acc[o];
}

// node k gathers its elements in a fixed order; omega_k = scale * sum
__global__ void k_gather(int d, int p, int N, int Eel, long total, const double* elem,
                         const double* orig, double scale, int accumulate, double* omega) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= total) return;
  const int nb = p + 1;
  int nout = 1;
  for (int s = 0; s < d; ++s) nout *= nb;
  int kv[3] = {0, 0, 0};
  long rem = k;
  for (int s = d - 1; s >= 0; --s) {
    kv[s] = (int)(rem % (N + 1));
    rem /= (N + 1);
  }
  // per axis: up to two (element, local) pairs
  int ne[3], el[3][2], lo[3][2];
  for (int s = 0; s < d; ++s) {
    const int ks = kv[s];
    int c = 0;
    if (p == 0) {
      el[s][c] = ks; lo[s][c] = 0; ++c;
    } else if (p == 1) {
      if (ks - 1 >= 0) { el[s][c] = ks - 1; lo[s][c] = 1; ++c; }
      if (ks <= N - 1) { el[s][c] = ks; lo[s][c] = 0; ++c; }
    } else {
      if (ks % 2 == 0) {
        if (ks / 2 - 1 >= 0) { el[s][c] = ks / 2 - 1; lo[s][c] = 2; ++c; }
        if (ks / 2 <= N / 2 - 1) { el[s][c] = ks / 2; lo[s][c] = 0; ++c; }
      } else {
        el[s][c] = (ks - 1) / 2; lo[s][c] = 1; ++c;
      }
    }
    ne[s] = c;
  }
  double sum = 0.0;
  const int c0 = ne[0], c1 = d > 1 ? ne[1] : 1, c2 = d > 2 ? ne[2] : 1;
  for (int i0 = 0; i0 < c0; ++i0)
    for (int i1 = 0; i1 < c1; ++i1)
      for (int i2 = 0; i2 < c2; ++i2) {
        const int ii[3] = {i0, i1, i2};
        long eidx = 0;
        int lidx = 0;
        bool origin = true;
        for (int s = 0; s < d; ++s) {
          eidx = eidx * Eel + el[s][ii[s]];
          lidx = lidx * nb + lo[s][ii[s]];
          origin = origin && el[s][ii[s]] == 0;
        }
        sum += origin ? orig[lidx] : elem[eidx * nout + lidx];
      }
  omega[k] = accumulate ? omega[k] + scale * sum : scale * sum;
}

// far-field constant T_d = int over R^d_+ minus [0,L]^d of K |xi|^{-d-alpha},
// in cone coordinates: T_d = d int_{[0,1]^{d-1}} rho^{-d} F(L rho) dw,
// F(R) = int_R^inf K(r) r^{-1-alpha} dr = R^{-alpha} int_0^inf K(R e^s) e^{-alpha s} ds.
__device__ double far_F(double R, double alpha, double lam, const GLTables* tb) {
  const double Ra = pow(R, -alpha);
  if (lam == 0.0) return Ra / alpha;
  const double lr = lam * R;
  const double U = fmax(1.0, log(45.0 / lr) + 1.0);
  const double width = fmin(0.25, 0.5 / lr);
  int np = (int)ceil(U / width);
  if (np > 4096) np = 4096;
  const double hw = U / np;
  double sum = 0.0;
  for (int ip = 0; ip < np; ++ip) {
    const double a = ip * hw;
    double ps = 0.0;
    for (int q = 0; q < QP; ++q) {
      const double s = a + 0.5 * hw * (tb->xp[q] + 1.0);
      ps += tb->wp[q] * exp(-lr * exp(s) - alpha * s);
    }
    sum += ps * 0.5 * hw;
  }
  return Ra * sum;
}

__global__ void __launch_bounds__(256) k_far(int d, double alpha, double lam, double L,
                                             double wt, int accumulate, const GLTables* tb,
                                             double* T) {
  __shared__ double sh[8];
  const int npts = d == 1 ? 1 : (d == 2 ? NA : NA * NA);
  double acc = 0.0;
  for (int pt = threadIdx.x; pt < npts; pt += blockDim.x) {
    double w = 1.0, rho2 = 1.0;
    if (d >= 2) {
      w *= tb->wa[pt % NA];
      rho2 += tb->xa[pt % NA] * tb->xa[pt % NA];
    }
    if (d == 3) {
      w *= tb->wa[pt / NA];
      rho2 += tb->xa[pt / NA] * tb->xa[pt / NA];
    }
    const double rho = sqrt(rho2);
    acc += w * d * pow(rho, -(double)d) * far_F(L * rho, alpha, lam, tb);
  }
  const double t = wt * bsum(acc, sh);
  if (threadIdx.x == 0) *T = accumulate ? *T + t : t;
}

// a_k = 2^{z(k)} W_k / |xi_k|^gamma (W: origin rule applied for gamma = 2;
// for gamma < 2 Phi(x, 0) = 0 and omega_0 drops out), G_k = -c a_k for
// k != 0; per-block partial of sum 2^{d-z(k)} a_k for the diagonal.
__global__ void __launch_bounds__(256) k_coeff(int d, int p, int N, double h, double c,
                                               double gamma, long total, const double* omega,
                                               double* G, double* part) {
  __shared__ double sh[8];
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double term = 0.0;
  if (k < total && k > 0) {
    int kv[3] = {0, 0, 0};
    long rem = k;
    for (int s = d - 1; s >= 0; --s) {
      kv[s] = (int)(rem % (N + 1));
      rem /= (N + 1);
    }
    int z = 0, nz = -1;
    long k2 = 0;
    for (int s = 0; s < d; ++s) {
      z += kv[s] == 0;
      if (kv[s] != 0) nz = s;
      k2 += (long)kv[s] * kv[s];
    }
    double W = omega[k];
    if (gamma == 2.0 && z == d - 1) {  // on an axis: origin rule
      const double w0 = omega[0];
      const int m = kv[nz];
      const double c1 = p <= 1 ? 1.0 : 4.0 / 3.0;
      const double c2 = p <= 1 ? 0.0 : -1.0 / 3.0;
      if (m == 1) W += w0 * c1 / d;
      if (m == 2) W += w0 * c2 / d;
    }
    const double r2 = h * h * (double)k2;
    const double a = (double)(1 << z) * W / (gamma == 2.0 ? r2 : pow(r2, 0.5 * gamma));
    G[k] = -c * a;
    term = (double)(1 << (d - z)) * a;
  }
  const double t = bsum(term, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// G_0 = -c a_0 = c (sum_k 2^{d-z} a_k + 2^d T)
__global__ void __launch_bounds__(256) k_diag(int d, double c, int nparts, const double* part,
                                              const double* T, double* G) {
  __shared__ double sh[8];
  double v = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += part[i];
  v = bsum(v, sh);
  if (threadIdx.x == 0) G[0] = c * (v + (double)(1 << d) * T[0]);
}

}  // namespace

void build_generator(const GenParams& gp, double* G, hipStream_t st) {
  const int d = gp.d, p = gp.p, N = gp.N;
  GLTables tb;
  gauss_legendre(NA, tb.xa, tb.wa);
  for (int i = 0; i < NA; ++i) {
    tb.xa[i] = 0.5 * (tb.xa[i] + 1.0);
    tb.wa[i] *= 0.5;
  }
  gauss_legendre(QN, tb.xn, tb.wn);
  gauss_legendre(QF, tb.xf, tb.wf);
  gauss_legendre(QP, tb.xp, tb.wp);
  const double sig = gp.gamma - gp.alpha;
  const double scale = std::pow(gp.h, sig);
  const int nb = p + 1;
  const int Eel = p == 0 ? N + 1 : (p == 1 ? N : N / 2);
  long nelem = 1, nnode = 1;
  int nout = 1;
  for (int s = 0; s < d; ++s) {
    nelem *= Eel;
    nnode *= (N + 1);
    nout *= nb;
  }
  const int thr = 256;
  const long nblk = (nnode + thr - 1) / thr;
  const size_t b_elem = (size_t)nelem * nout * sizeof(double);
  SetupScratch scr(scratch_round(sizeof(GLTables)) + scratch_round(b_elem) +
                       scratch_round(32 * sizeof(double)) +
                       scratch_round((size_t)nnode * sizeof(double)) +
                       scratch_round((size_t)nblk * sizeof(double)) + scratch_round(sizeof(double)),
                   st);
  GLTables* dtb = (GLTables*)scr.take(sizeof(GLTables));
  double* elem = (double*)scr.take(b_elem);
  double* orig = (double*)scr.take(32 * sizeof(double));
  double* omega = (double*)scr.take((size_t)nnode * sizeof(double));
  double* part = (double*)scr.take((size_t)nblk * sizeof(double));
  double* T = (double*)scr.take(sizeof(double));
  FL_HIP(hipMemcpyAsync(dtb, &tb, sizeof(GLTables), hipMemcpyHostToDevice, st));
  // one pass per kernel term: omega and T accumulate coef * (that term's);
  // the lattice-unit rate is rate * h (K = 1 integrates on the unit lattice)
  for (int i = 0; i < gp.nterm; ++i) {
    const double lamh = gp.rate[i] * gp.h;
    hipLaunchKernelGGL(k_origin, dim3(1), dim3(256), 0, st, d, p, sig, lamh, dtb, orig);
    hipLaunchKernelGGL(k_elements, dim3((unsigned)((nelem + 127) / 128)), dim3(128), 0, st, d, p,
                       N, Eel, nelem, sig, lamh, dtb, elem);
    hipLaunchKernelGGL(k_gather, dim3((unsigned)nblk), dim3(thr), 0, st, d, p, N, Eel, nnode,
                       elem, orig, scale * gp.coef[i], i > 0 ? 1 : 0, omega);
    hipLaunchKernelGGL(k_far, dim3(1), dim3(256), 0, st, d, gp.alpha, gp.rate[i], 2.0,
                       gp.coef[i], i > 0 ? 1 : 0, dtb, T);
  }
  hipLaunchKernelGGL(k_coeff, dim3((unsigned)nblk), dim3(thr), 0, st, d, p, N, gp.h, gp.c,
                     gp.gamma, nnode, omega, G, part);
  hipLaunchKernelGGL(k_diag, dim3(1), dim3(256), 0, st, d, gp.c, (int)nblk, part, T, G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(4, std::string("generator kernels: ") + hipGetErrorString(e));
  // the host tables are read by the copy above: wait before they go
  FL_HIP(hipStreamSynchronize(st));
}

}  // namespace fl
