/*
 * fl.h -- C ABI of the MI355X (gfx950) library for the operator-factorization
 * discretization of the integral fractional Laplacian (-Delta)^{alpha/2} and
 * its tempered generalization (Wu & Zhang, arXiv 2103.03658).
 *
 * Problem (Sec. 1, eq. (Poisson) and (BC)):  (-Delta)^{alpha/2} u = f on
 * Omega = (-1,1)^d, u = g on the complement, d = 1, 2, 3, alpha in (0,2).
 * Discretization (Sec. 2, eq. (1D-scheme), (2D-scheme); Remark 2.2):
 * (-Delta)^{alpha/2}_h u = A u + b, A the symmetric (multilevel) Toeplitz
 * matrix with generator G_k = -c_{d,alpha} a_k, k in {0..N}^d, h = 2/N,
 * splitting parameter gamma = 2, Lagrange basis of degree 0, 1 or 2 in xi.
 * The product A u is computed by circulant embedding of size M per axis, the
 * smallest power of two >= 2N (any M >= 2N - 3 holds the Toeplitz offsets
 * -(N-2)..N-2 without wrap-around), and FFT (Sec. 2.1: the Toeplitz
 * structure admits FFT products).
 *
 * Conventions for every entry point:
 *  - Vectors live in device memory owned by the caller, contiguous,
 *    row-major over the n^d interior points (n = N-1, last index fastest),
 *    right-hand sides stored one after another: element (r, i) at
 *    r * n^d + i.  Interior point i_s corresponds to x = -1 + (i_s+1) h.
 *  - `stream` is a hipStream_t passed as void* (NULL: the default stream).
 *    Work is enqueued on it; fl_apply returns without waiting, fl_solve
 *    waits for its result.
 *  - No C++ exception crosses the boundary.  A non-FL_OK status leaves a
 *    thread-local message readable with fl_last_error().  Argument checks
 *    happen before any device work.
 *  - An operator handle is immutable after creation apart from its
 *    schedule and solver settings; it owns its device buffers (transform
 *    workspaces, CG state) and reuses them across calls.  Calls on one
 *    handle are serialised by a lock of the handle: a call that needs its
 *    buffers or settings (fl_apply, fl_apply_precond, fl_exterior,
 *    fl_profile_*, fl_set_*, fl_solve) waits while another call of the same
 *    handle, including the solve of an fl_solve_async request, is inside
 *    the library.  Handles do not share buffers; calls on different handles
 *    run concurrently.
 */
#ifndef FL_H
#define FL_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fl_op_s *fl_op;

typedef enum {
  FL_OK = 0,
  FL_E_INVAL = 1,       /* invalid argument */
  FL_E_UNSUPPORTED = 2, /* valid but outside what is built (e.g. N > 1024) */
  FL_E_NOMEM = 3,       /* device allocation failed */
  FL_E_DEVICE = 4,      /* a HIP call failed */
  FL_E_NOCONV = 5,      /* maxiter reached before the tolerance */
  FL_E_BREAKDOWN = 6    /* non-finite values or p.Ap <= 0 in CG */
} fl_status;

enum { FL_KERNEL_FRACTIONAL = 0, FL_KERNEL_TEMPERED = 1 };

/* Caller-provided device allocator (fl_set_allocator). */
typedef void *(*fl_alloc_fn)(size_t bytes, void *ctx);
typedef void (*fl_release_fn)(void *ptr, void *ctx);

/* Most exponential terms a kernel of fl_weights_expsum may have. */
#define FL_MAX_KERNEL_TERMS 16

/* Per right-hand-side result of fl_solve. */
typedef struct {
  int iters;          /* CG iterations (FP32 iterations for the mixed paths, summed) */
  int outer_iters;    /* FP64 residual replacements (mixed = 1) or refinement steps
                         (mixed = 2); 0 for mixed = 0 */
  int converged;      /* 1 if the stopping rule was met */
  int status;         /* fl_status of this right-hand side */
  double relres_rec;  /* recursive ||r||_2 / ||f - b||_2 at exit (mixed: the FP64 residual) */
  double relres_true; /* ||f - b - A u||_2 / ||f - b||_2 recomputed with an FP64 product at
                         exit (b = 0 without exterior data) */
} fl_info;

/*
 * fl_weights -- build the operator (-Delta)^{alpha/2}_h (or the tempered
 * operator with kernel K(r) = exp(-lambda r), Remark 2.2) on (-1,1)^d.
 * Computes on the GPU in FP64: the weight integrals omega_k^p (Sec. 2.1
 * eq. (wi-1D), Sec. 2.2 eq. (2D-scheme0)), the origin rule, the
 * coefficients a_k, the diagonal a_0 (with the far-field integral of
 * eq. (L2)), the generator G = -c a, and the symbol lambda-hat = DFT of the
 * circulant embedding of G divided by M^d (FP64 and an FP32 copy).
 *   d       1, 2 or 3
 *   alpha   in (0, 2)
 *   degree  Lagrange degree p in {0, 1, 2}; p = 2 needs N even
 *   h       mesh size; N = 2/h must be an integer (to 1e-12 relative),
 *           4 <= N <= 1024 (embedding M = the smallest power of two
 *           >= 2N, at most 2048)
 *   kernel  FL_KERNEL_FRACTIONAL (lambda ignored) or FL_KERNEL_TEMPERED
 *   lambda  tempering rate >= 0 (normalisation constant c_{d,alpha})
 *   stream  HIP stream for the setup kernels
 *   out     receives the handle; unchanged on error
 * Errors: FL_E_INVAL (argument), FL_E_UNSUPPORTED (size), FL_E_NOMEM,
 * FL_E_DEVICE.  Synchronous: the handle is ready on return.
 */
fl_status fl_weights(int d, double alpha, int degree, double h, int kernel, double lambda,
                     void *stream, fl_op *out);

/*
 * fl_weights_gamma -- as fl_weights with the splitting parameter gamma of
 * the operator factorization (Sec. 2.1: Phi = second difference over
 * |xi|^gamma, weights omega_k = int phi_k K(|xi|) |xi|^{gamma-d-alpha}),
 * gamma in (alpha, 2].  gamma = 2 is fl_weights.  For gamma < 2 the origin
 * value Phi(x, 0) is 0 (eq. (gamma2)): no origin term, a_k = 2^{z(k)}
 * omega_k / |xi_k|^gamma.  FL_E_INVAL for gamma outside (alpha, 2].
 */
fl_status fl_weights_gamma(int d, double alpha, int degree, double h, int kernel, double lambda,
                           double gamma, void *stream, fl_op *out);

/*
 * fl_weights_box -- the operator on a box (Sec. 2.2: Omega a product of
 * intervals, Upsilon = [0, L]^d with L the longest side; N_1 = N on the
 * longest axis and N_s the smallest integer whose N_s h covers side s).
 * The longest axis spans (-1, 1), h = 2/N with N = max_s intervals[s],
 * axis s spans (-1, -1 + intervals[s] h) and has intervals[s] - 1 interior
 * points.  The weights, generator and far-field constant are those of the
 * cube of side 2 (they depend on Upsilon, not on Omega); the matrix is the
 * cube's restricted to the box's interior points.
 *   intervals  host array of d ints, each in [2, N]; N = max in [4, 1024]
 *   gamma      splitting parameter in (alpha, 2] (2: fl_weights)
 * Other arguments and errors as fl_weights_gamma.  Vectors are row-major
 * over n_0 x .. x n_{d-1} (n_s = intervals[s] - 1, last index fastest).
 * The tau preconditioner needs every 2 intervals[s] to be a power of two
 * (otherwise the default is kind 1).  fl_exterior takes the box's node
 * lattice [-N, N_s + N] along axis s.
 */
fl_status fl_weights_box(int d, double alpha, int degree, const int *intervals, int kernel,
                         double lambda, double gamma, void *stream, fl_op *out);

/*
 * fl_weights_expsum -- the operator of Remark 2.2 (kernel K(|x - y|) beside
 * the hypersingular factor, normalisation c_{d,alpha}) for
 *     K(r) = sum_{i < nterm} coef[i] exp(-rate[i] r).
 * Only the weight integrals omega_k (K enters mu_gamma) and the far-field
 * constant of a_0 depend on K, and both are linear in it: each term's are
 * computed as for the tempered kernel, scaled by coef[i] and summed; the
 * origin rule and a_k, a_0 then follow as for any kernel.  rate 0 is K = 1,
 * so {coef 1, rate 0} is fl_weights_box with FL_KERNEL_FRACTIONAL and
 * {coef 1, rate lambda} the tempered operator.  Non-negative sums of
 * exponentials are dense in the completely monotone kernels (those are
 * Laplace transforms of non-negative measures), e.g. quadratures of
 * (1 + r)^{-beta} = int_0^inf t^{beta-1} e^{-t} e^{-t r} dt / Gamma(beta).
 *   intervals  host array of d ints as in fl_weights_box (all equal: the cube)
 *   nterm      1 .. FL_MAX_KERNEL_TERMS
 *   coef       host array of nterm finite values >= 0, not all zero (K >= 0
 *              keeps the matrix symmetric positive definite)
 *   rate       host array of nterm finite rates >= 0
 *   gamma      splitting parameter in (alpha, 2]
 * Other arguments, layout and errors as fl_weights_box; FL_E_INVAL for a
 * bad term.  Setup cost grows linearly with nterm.
 */
fl_status fl_weights_expsum(int d, double alpha, int degree, const int *intervals, int nterm,
                            const double *coef, const double *rate, double gamma, void *stream,
                            fl_op *out);

/* Copy the FP64 generator G_k = -c_{d,alpha} a_k, k in {0..N}^d (row-major,
 * (N+1)^d values), to host memory: the entries of the symmetric (multilevel)
 * Toeplitz matrix, A_{ij} = G_{|i-j|} (Sec. 2.1, the matrix A^(1) after
 * eq. (1D-scheme); Sec. 2.2, the block matrix A^(2) after eq. (2D-scheme)).
 * count must be >= (N+1)^d.  Synchronises the device.  Test hook. */
fl_status fl_generator(fl_op A, double *host_out, size_t count);

/* Copy the folded FP64 symbol lambda-hat_k, k_s in {0..M_s/2} (prod_s
 * (M_s/2 + 1) values; N + 1 per axis when M = 2N): the eigenvalues of the
 * circulant that embeds A^(1) / A^(2) (Sec. 2.1 and 2.2: the Toeplitz
 * structure admits products by FFT), lambda-hat = DFT(c) / prod M_s.  The
 * full symbol on prod {0..M_s-1} is even: lambda-hat_j =
 * lambda-hat_{min(j_s, M_s-j_s)}.  count >= prod (M_s/2 + 1).  Synchronises
 * the device.  Test hook. */
fl_status fl_symbol(fl_op A, double *host_out, size_t count);

/* Copy the circulant embedding c_j, j_s in {0..M_s-1}, of the generator
 * (the first column of a circulant whose leading block is A^(1) / A^(2),
 * Sec. 2.1 and 2.2) as laid out on the device: c_j = G_{m(j)},
 * m(j_s) = min(j_s, M_s - j_s), zero where some m(j_s) > N_s - 2.
 * count >= prod M_s.  Allocates a temporary of prod M_s doubles.  Test hook
 * for the index maps. */
fl_status fl_embedding(fl_op A, double *host_out, size_t count);

/* Geometry of A: dimension, intervals N, interior points per axis n = N-1,
 * embedding length M (the smallest power of two >= 2N).  Any pointer may
 * be NULL. */
fl_status fl_query(fl_op A, int *d, int *N, int *n, int *M);

/* Per-axis geometry of A (d entries each): intervals N_s, interior points
 * n_s = N_s - 1, embedding lengths M_s (the smallest power of two >= 2 N_s).
 * fl_query reports axis 0.  Any pointer may be NULL. */
fl_status fl_query_axes(fl_op A, int *intervals, int *n, int *M);

/*
 * fl_apply -- y = A u for nrhs right-hand sides: the differentiation matrix
 * of the scheme, A^(1) of Sec. 2.1 (after eq. (1D-scheme)) and A^(2) of
 * Sec. 2.2 (after eq. (2D-scheme)) and its 3-level analogue, applied by
 * circulant embedding and FFT (the g = 0 operator; the exterior-data term b
 * is not added).
 *   u, y    device arrays of nrhs * n^d doubles (fp32 = 0) or floats
 *           (fp32 = 1), distinct, caller-owned
 *   nrhs    >= 1
 *   fp32    0: FP64 transforms and FP64 symbol; 1: FP32 transforms and symbol
 * Asynchronous on `stream`.  Errors: FL_E_INVAL, FL_E_NOMEM, FL_E_DEVICE.
 */
fl_status fl_apply(fl_op A, const void *u, void *y, int nrhs, int fp32, void *stream);

/* Size of the fixed scratch area of fl_apply_noalloc, in MiB. */
#define FL_NOALLOC_SCRATCH_MIB 128

/*
 * fl_apply_noalloc -- fl_apply for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same product, kernels and launch schedule, so the
 * same bits as fl_apply, with the transform intermediates in a fixed area of
 * the library (FL_NOALLOC_SCRATCH_MIB, one copy per device, held from the
 * library's first use on that device until the process ends) instead of the
 * handle's workspace.  No call of it allocates device memory or calls
 * hipMalloc / hipFree.
 *   Intermediates needed, s = 8 (FP64) or 4 (FP32) bytes, h0 = M_0/2 + 1:
 *     d = 1: none;  d = 2: nrhs * h0 * n_1 * 2s;
 *     d = 3: nrhs * (h0 * n_1 * n_2 + h0 * M_1 * n_2) * 2s
 *   (e.g. 2D N = 512 FP64: 4.19 MB per right-hand side, 32 fit).
 * Every call on a device uses that device's one area: calls that overlap on
 * one device (on different streams, from different threads or handles)
 * race and give wrong results; the caller orders them.  The area keeps the
 * last call's contents.  Arguments, layout and stream rules as fl_apply.
 * Errors as fl_apply; FL_E_UNSUPPORTED (nothing launched) when the
 * intermediates exceed the area.
 */
fl_status fl_apply_noalloc(fl_op A, const void *u, void *y, int nrhs, int fp32, void *stream);

/*
 * fl_solve -- solve A u = f - b for nrhs right-hand sides by conjugate
 * gradients (the discrete equation A u + b = f of Sec. 2.1 eq. (1D-scheme)
 * and Sec. 2.2 eq. (2D-scheme); A is symmetric positive definite, Sec. 2.2),
 * preconditioned by default (fl_set_preconditioner).
 *   f       device, nrhs * n^d doubles
 *   b       device, nrhs * n^d doubles: the exterior-data term of the scheme
 *           (from fl_exterior, for data u = g outside Omega), or NULL for
 *           g = 0 (b = 0).  Must not alias u.  With b given, the right-hand
 *           side of the system is f - b, and the tolerance and the relres_*
 *           results of fl_info are relative to ||f - b||_2.
 *   tol     stop when ||r||_2 <= tol ||f - b||_2 (per right-hand side),
 *           tol > 0
 *   maxiter CG iteration cap (mixed = 0, 1) / inner iteration cap per
 *           refinement step (mixed = 2), >= 1
 *   mixed   0: FP64 CG; stops on the recursive residual.
 *           1: FP32 CG with FP64 reliable updates: the FP32 recursion runs on
 *           a correction; whenever its residual norm has dropped by the factor
 *           delta (fl_set_refinement) since the last update, the
 *           correction is added to the FP64 iterate and the residual is
 *           recomputed as r = f - A u with an FP64 product; stops when that
 *           FP64 residual meets tol.  The drop is tested at every iteration
 *           start on the device (a right-hand side that reaches it waits);
 *           the update runs after the current chunk of iterations.
 *           Preconditioned, the search direction restarts from the new
 *           residual at each update.
 *           2: iterative refinement with restarts: FP32 CG solves A d = r to
 *           the relative tolerance inner_tol, u += d in FP64, r = f - A u in
 *           FP64, until the FP64 residual meets tol.
 *   u       device, nrhs * n^d doubles, output (x0 = 0)
 *   info    host array of nrhs fl_info, or NULL
 * Blocks until done.  Returns FL_OK if every right-hand side converged,
 * otherwise the first failing status (FL_E_NOCONV, FL_E_BREAKDOWN); u then
 * holds the last iterate.  A right-hand side f = 0 gives u = 0.
 */
fl_status fl_solve(fl_op A, const double *f, const double *b, double tol, int maxiter, int mixed,
                   double *u, int nrhs, fl_info *info, void *stream);

/*
 * fl_solve_async -- fl_solve without blocking the calling thread, for
 * serving loops that keep submitting while solves run.  The solve runs on a
 * host thread of its own with the same arguments, semantics and results as
 * fl_solve, after the work queued on `stream` so far; solves of one operator
 * run one at a time (not necessarily in submission order), solves of
 * different operators concurrently on their own streams.  f, b and u belong
 * to the caller and must stay valid, f and b unchanged, until the request
 * is finished, and the operator must not be destroyed before; `stream` does
 * not wait for the result.  The solve holds the operator's lock while it
 * runs: other calls on the same operator (fl_apply, fl_exterior, fl_set_*,
 * ...) wait until it has finished, so they never share its workspaces.
 *   out  receives the request; every request must be finished with fl_wait
 * Errors: argument errors as fl_solve, returned here (no request is made).
 */
typedef struct fl_request_s *fl_request;
fl_status fl_solve_async(fl_op A, const double *f, const double *b, double tol, int maxiter,
                         int mixed, double *u, int nrhs, void *stream, fl_request *out);

/* fl_poll -- *done = 1 once the request's solve has finished (u and the
 * results are then final), else 0.  Does not block. */
fl_status fl_poll(fl_request r, int *done);

/* fl_wait -- block until the request's solve has finished, copy its per-RHS
 * results into info (nrhs entries, or NULL) and free the request.  Returns
 * the solve's status (as fl_solve would have; fl_last_error then holds its
 * text). */
fl_status fl_wait(fl_request r, fl_info *info);

/*
 * fl_exterior -- the exterior-data term b of the scheme with nonhomogeneous
 * data u = g outside Omega (Sec. 2.1 eq. (1D-scheme) and Sec. 2.2
 * eq. (2D-scheme), the terms of the discrete operator that involve values of
 * g; with them the discrete equation reads A u + b = f):
 *   b_i = sum over lattice nodes j outside the interior with |j - i|_inf <= N
 *           of G_{|j - i|} g(x_j)  -  c_{d,alpha} tail_i,
 *   tail_i = sum over the 2^d sign patterns m of the integral over the far
 *            field (xi >= 0 outside the box [0, L]^d, L = 2) of
 *            g(x_i + (-1)^m o xi) K(|xi|) |xi|^{-d-alpha} d xi.
 * On a box (fl_weights_box) axis s has the interior nodes 1 .. N_s - 1 and
 * the node lattice [-N, N_s + N] (N_s = N on the cube).  The lattice sum runs
 * on the GPU (a multilevel Toeplitz product of G with g on the node lattice:
 * for d = 2, 3 by circulant embedding in P_s >= N_s + 2N + 1 points per axis,
 * or for d = 2 beyond 2048 points by 3 x 3 lattice blocks whose circular
 * products of length P_s >= max(2 N_s, N_s + N) are summed as spectra;
 * directly for d = 1).  The far-field integrals need g beyond the lattice,
 * which the library cannot evaluate: the caller supplies them.
 *   g_lat  device, nrhs * prod_s (N_s + 2N + 1) doubles: g(x_j), x_j = -1 +
 *          j h for j_s in [-N, N_s + N], row-major, last index fastest
 *          (entries at interior nodes are ignored)
 *   tail   device, nrhs * n^d doubles (interior layout), or NULL (tail = 0)
 *   b      device, nrhs * n^d doubles, output
 * FL_E_UNSUPPORTED for d = 3 beyond 1024^3 transform points (N <= 256 on
 * the cube).  Same stream rules as fl_apply; allocates its transform
 * buffers on first use and keeps them with the operator: 2 prod P_s complex
 * doubles (4.3 GB at d = 3, N = 128), 11 prod P_s for the 2D block form
 * (0.74 GB at N = 1024).
 */
fl_status fl_exterior(fl_op A, const double *g_lat, const double *tail, double *b, int nrhs,
                      void *stream);

/* Mixed-precision settings.  delta (default 1e-5): a reliable update
 * (mixed = 1) happens at the first FP32 iteration whose residual norm has
 * dropped below delta times its value at the previous update (or below the
 * tolerance); that right-hand side waits there for the FP64 residual.  inner_tol (default 1e-4):
 * relative tolerance of each FP32 inner solve of mixed = 2.  max_outer
 * (default 40): refinement step cap of mixed = 2.  delta, inner_tol in
 * (0, 1), max_outer >= 1, else FL_E_INVAL and nothing changes. */
fl_status fl_set_refinement(fl_op A, double delta, double inner_tol, int max_outer);

/*
 * Launch schedule of the transform passes (elements per thread E and lines
 * per block) for FP64 (fp32 = 0) or FP32 transforms.  E in {8, 16, 32},
 * E <= M; lines per block >= 1 with (lines * M / E) <= 512 threads and
 * lines * 2 (M + M/E) * sizeof(real) <= 160 KiB of LDS (the contiguous
 * middle pass uses half of that).  Values <= 0 keep
 * the current setting; FL_E_INVAL leaves it unchanged.  Used by the
 * schedule tuner; results do not depend on the schedule beyond rounding.
 */
fl_status fl_set_schedule(fl_op A, int fp32, int e_first, int e_mid, int e_c2c, int w_first,
                          int w_c2c, int lpb_mid);
fl_status fl_get_schedule(fl_op A, int fp32, int *sched6);

/*
 * The same for the preconditioner's passes (fl_apply_precond and the
 * preconditioned solves), which have a schedule of their own: the tau
 * preconditioner's sine passes move half the bytes of the product's
 * complex passes and prefer other shapes.  Starts equal to the product's
 * default schedule.  Same ranges and errors as fl_set_schedule.
 */
fl_status fl_set_precond_schedule(fl_op A, int fp32, int e_first, int e_mid, int e_c2c,
                                  int w_first, int w_c2c, int lpb_mid);
fl_status fl_get_precond_schedule(fl_op A, int fp32, int *sched6);

/*
 * fl_profile_apply -- measurement hook: run fl_apply's kernel sequence once
 * on `stream` (so every kernel's input is in place), then each kernel alone
 * `reps` times back to back between two HIP events, and return the mean
 * duration per launch of each kernel in milliseconds; a last whole sequence
 * leaves y = A u.  If max_passes >= 2 * n_passes, each kernel is then also
 * launched `reps` times with an event pair around every launch, and the mean
 * of those single-dispatch durations (what a kernel trace reports per
 * dispatch; it includes each dispatch's start-up and completion, which
 * back-to-back launches overlap) goes to ms_per_pass[n_passes + k].
 * The kernels are the transform passes in launch order: 1 for d = 1 (the
 * whole product), 3 for d = 2 (axis 0 forward, last axis forward * symbol *
 * inverse, axis 0 inverse), 5 for d = 3 (axis 0, axis 1, last axis, axis 1
 * inverse, axis 0 inverse).  Same arguments as fl_apply plus
 *   reps          >= 1
 *   ms_per_pass   host array of at least max_passes doubles (output)
 *   n_passes      host int (output): number of kernels per application
 * Blocks until done.  Errors as fl_apply; FL_E_INVAL if max_passes is too small.
 */
fl_status fl_profile_apply(fl_op A, const void *u, void *y, int nrhs, int fp32, int reps,
                           void *stream, double *ms_per_pass, int max_passes, int *n_passes);

/*
 * fl_profile_precond -- the same measurement for the preconditioner y = P u
 * of fl_apply_precond (kind 2: the sine passes of the tau inverse, 1 kernel
 * for d = 1, 3 for d = 2, 5 for d = 3; kind 1: the zero-padded passes of
 * fl_profile_apply with the inverse multiplier).  Same arguments and errors
 * as fl_profile_apply; FL_E_INVAL with preconditioner kind 0.
 */
fl_status fl_profile_precond(fl_op A, const void *u, void *y, int nrhs, int fp32, int reps,
                             void *stream, double *ms_per_pass, int max_passes, int *n_passes);

/*
 * Preconditioning of fl_solve (the paper names no solver; A is SPD, Sec. 2.2):
 *   kind 2 (the default where available): P = tau(A)^{-1}, the inverse of
 *     the natural tau approximation of the multilevel Toeplitz matrix (A
 *     minus its Hankel part on every level), diagonalised by the sine
 *     transform of each axis and applied by real sine passes (DST-I of every
 *     axis through the length-2 N_s transform of odd-extended line pairs).
 *     Available when every 2 N_s is a power of two (radix-8/16/32 passes),
 *     and also when every 2 N_s has no prime factor above 7 (mixed-radix
 *     8/4/2/3/5/7 passes, lines held in LDS, eigenvalues summed as the
 *     cosine series of the generator); FL_E_UNSUPPORTED otherwise;
 *   kind 1 (default otherwise): P = R C^{-1} R^T, the restriction to the
 *     n^d interior of the inverse of the embedding circulant C (symbol
 *     1 / max(lambda-hat, 1e-12 max lambda-hat));
 *   kind 0: plain CG.
 * Both preconditioners are symmetric positive definite (eigenvalues floored
 * at 1e-12 of the largest).  The stopping rule is the relative residual
 * ||r||_2 <= tol ||f||_2 either way.  FL_E_INVAL for other kinds.
 */
fl_status fl_set_preconditioner(fl_op A, int kind);

/* The preconditioner kind fl_solve uses now (the default chosen at creation,
 * or the last fl_set_preconditioner).  FL_E_INVAL for a null handle or
 * pointer. */
fl_status fl_get_preconditioner(fl_op A, int *kind);

/* y = P u for nrhs right-hand sides with the selected preconditioner (same
 * layout, precision and stream rules as fl_apply).  FL_E_INVAL with kind 0.
 * Test hook for the preconditioners. */
fl_status fl_apply_precond(fl_op A, const void *u, void *y, int nrhs, int fp32, void *stream);

/* Replay CG iteration chunks from captured HIP graphs or launch every
 * kernel directly: enable = 1 (the default) captures a chunk the first time
 * it runs; enable = 2 runs it directly the first time and captures it when
 * the same launch sequence comes again (for operators that are solved once
 * or twice, e.g. in a serving stream: no capture and instantiation cost on
 * their first solve); enable = 0 never captures.  Results are the same every
 * way; graphs cut host launch cost.  FL_E_INVAL for other values.  fl_solve
 * runs its work on a stream owned by the handle, ordered after `stream` and
 * before later work on `stream` by events. */
fl_status fl_set_graphs(fl_op A, int enable);

/*
 * fl_set_allocator -- route the library's device allocations through the
 * caller's allocator (a memory pool, a framework's caching allocator), for
 * callers that manage device memory themselves.  Every buffer of an operator
 * (generator, symbols, workspaces, CG state, exterior-data buffers) allocated
 * after this call comes from alloc(bytes, ctx) on the current device; the
 * library returns it with release(ptr, ctx) once the device has finished
 * with it (fl_destroy, or a workspace that grows).  Setup temporaries (the
 * weight integrals, the embedded generator being transformed) use a scratch
 * area that each device keeps for the life of the process, grown with
 * hipMalloc to the largest setup so far up to 256 MiB, so that setup frees
 * nothing; a larger one comes from alloc and goes back through release.
 * Blocks keep the allocator that made them: a later call changes only new
 * allocations.  alloc must return memory aligned to 256 bytes, or NULL
 * (FL_E_NOMEM from the call that needed it).  alloc = release = NULL
 * restores hipMalloc / hipFree.  Twiddle tables, cached per device for the
 * life of the process, always use hipMalloc.  Process-wide; do not call it
 * while another thread is inside the library.
 * FL_E_INVAL if exactly one of alloc and release is NULL.
 */
fl_status fl_set_allocator(fl_alloc_fn alloc, fl_release_fn release, void *ctx);

/* Release the handle and its device memory.  NULL is accepted.  Freeing
 * device memory waits for all work on the device (hipFree, or an explicit
 * device synchronisation before a registered allocator's release), so a
 * server should destroy handles outside its latency-critical locks. */
void fl_destroy(fl_op A);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *fl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FL_H */
