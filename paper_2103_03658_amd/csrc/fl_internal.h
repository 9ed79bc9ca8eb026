// Host-side interfaces between the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <stdexcept>
#include <string>

struct fl_op_s;   // the operator handle (include/fl.h)

namespace fl {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define FL_HIP(call)                                                             \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      throw ::fl::Error(4, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

// ---------------------------------------------------------------------------
// Per-RHS CG state on the device (arrays of length nrhs unless noted).
//
// Reductions never use atomics or device-scope fences: each block of a kernel
// writes its partial sum to part_a / part_b, and every block of the kernel
// that consumes the sum re-adds the partials itself in a fixed order.  Each
// scalar is written by block 0 of one kernel and read only by later kernels:
//   first pass  reads part_b (rho), part_c (r.r, preconditioned), rr_prev,
//               iters, thresh2; writes rr_cur (rho), res2, thresh2 (first
//               iteration), and on exit active/status/n_active
//   last pass   writes part_a (p.q)
//   update      reads part_a, rr_cur; writes the r.r partials (part_b, or
//               part_c when preconditioned), rr_prev <- rr_cur, iters += 1
//   precond.    z = P r: its last pass writes part_b (r.z)
// so no kernel reads a value that a concurrently running block may change.
// ---------------------------------------------------------------------------
struct CgScalars {
  double* rr_cur;    // ||r_k||^2 of the current iteration
  double* rr_prev;   // ||r_{k-1}||^2
  double* thresh2;   // stop when ||r||^2 <= thresh2 (= tol^2 ||r_0||^2)
  double* alpha;     // last step length (diagnostics)
  int* active;       // 1 while iterating
  int* iters;        // completed updates
  int* status;       // 0 converged/running, 5 no convergence, 6 breakdown
  int* n_active;     // single int: number of active RHS (host polls it)
  double* part_a;    // p.q partials, nrhs * max_blocks
  double* part_b;    // rho partials: r.r (CG) or r.z (preconditioned), nrhs * max_blocks
  double* part_c;    // r.r partials when preconditioned, nrhs * max_blocks
  double* res2;      // ||r_k||^2 of the current iteration (stopping test, reports)
  int nb_a;          // valid partials per RHS in part_a (last-pass blocks)
  int nb_b;          // valid partials per RHS in part_b
  int nb_c;          // valid partials per RHS in part_c (update / init blocks)
  int max_blocks;
  int maxiter;
  int precond;       // 1: z = P r (preconditioned CG), rho = r.z
  double tol2;
  // FP32 recursion of the mixed path (null otherwise): at an iteration start
  // whose r.r fell below rel_delta2 * rel_last[o] or rel_tol2 * rel_f2[o],
  // RHS o stops and waits (rel_trig[o] = 1) for the reliable step
  const double* rel_last;
  const double* rel_f2;
  int* rel_trig;
  double rel_delta2, rel_tol2;
};

// Epilogue/prologue selection of the first and last FFT passes.
enum PassMode {
  PM_PLAIN = 0,     // y = A u
  PM_CG = 1,        // d = 1: beta, convergence, p = r + beta p, q = A p, p.q partials
  PM_RESID = 2,     // last pass: y = f - A u and partials of ||y||^2 (FP64 only)
  PM_DOT = 3,       // y = A u and partials of u.y into `part` (preconditioner r.z)
  PM_PQ = 4,        // d >= 2: q = A p with p.q partials (after cg_direction)
};

// Geometry of one operator application.  The generator lives on the cube
// {0..N}^d (h = 2/N, the longest axis spans (-1, 1)); axis s of the grid has
// Na[s] <= N intervals (a box; Na[s] = N for the cube) and n_s = Na[s] - 1
// interior points.  Entries beyond d are 1 (na, Ma, Ha) so products over all
// three axes hold.
struct Geometry {
  int d;       // 1, 2, 3
  int N;       // generator intervals per axis
  int Na[3];   // intervals of axis s
  int na[3];   // interior points of axis s = Na[s] - 1
  int Ma[3];   // embedding length of axis s: the smallest power of two >= 2 Na[s]
  int Ha[3];   // folded symbol length of axis s = Ma[s]/2 + 1
  int La[3];   // sine transform length of axis s (tau preconditioner) = 2 Na[s]
  long nd;     // prod_s na[s]
  bool cube() const {
    for (int s = 1; s < d; ++s)
      if (Na[s] != Na[0]) return false;
    return true;
  }
  // the power-of-two sine passes of the tau preconditioner need Ma[s] = 2 Na[s]
  bool sine_ok() const {
    for (int s = 0; s < d; ++s)
      if (Ma[s] != 2 * Na[s]) return false;
    return true;
  }
  // otherwise the mixed-radix sine passes take every La[s] whose prime
  // factors are 2, 3, 5 and 7
  bool sine_any_ok() const;
  bool tau_ok() const { return sine_ok() || sine_any_ok(); }
  long nh() const { return (long)Ha[0] * Ha[1] * Ha[2]; }
  long nm() const { return (long)Ma[0] * Ma[1] * Ma[2]; }
};

// Twiddle tables of one precision, one per axis (the axes' embedding lengths
// may differ).
struct Twiddles {
  const void* ax[3];   // exp(-2 pi i j / Ma[s]), j < Ma[s]
  const void* sx[3];   // exp(-2 pi i j / La[s]): the mixed-radix sine passes
};

// Launch schedule (tunable).
struct Schedule {
  int E_first;   // elements per thread, strided passes along axis 0
  int E_mid;     // elements per thread, contiguous middle pass
  int E_c2c;     // elements per thread, 3D axis-1 passes
  int W_first;   // lines per block in the axis-0 passes
  int W_c2c;     // lines per block in the 3D axis-1 passes
  int LPB_mid;   // lines per block in the middle pass
};

constexpr size_t kMaxLds = 160 * 1024;   // LDS per workgroup on gfx950

// LDS layout of a strided-pass block of W lines (W a power of two): line l
// owns [l*LS, (l+1)*LS) elements of the element type, its real plane at 0
// and its imaginary plane at PO, each M + M/E long (padded index).  In the
// cooperative row-segment phases a half wave touches 32/(2W) rows of the
// 2W planes of the tile; with PO = R and LS = 2R (mod the bank count, in
// elements), R = banks/(2W), those accesses land in distinct banks.
struct TileLds {
  int PO, LS;
  size_t bytes;
};
inline TileLds tile_lds(int M, int E, int W, size_t elem) {
  const int ldsn = M + M / E;
  const int banks = elem == 8 ? 16 : 32;   // 4-byte banks, in elements
  int R = banks / (2 * W);
  if (R < 1) R = 1;
  auto up = [&](int x, int res) { return x + (((res - x) % banks) + banks) % banks; };
  const int PO = up(ldsn, R % banks);
  const int LS = up(PO + ldsn, (2 * R) % banks);
  return {PO, LS, (size_t)W * LS * elem};
}
// The sine passes that keep only the lower half of each line (the odd
// extension's mirror is formed in registers, and only outputs below M/2 are
// read) hold a line's real and imaginary lower halves in one plane of
// M + M/E (the real half at 0, the imaginary half at PO), which is also the
// transform's exchange plane: half the LDS of tile_lds.
inline TileLds tile_lds_half(int M, int E, int W, size_t elem) {
  const int ldsn = M + M / E;
  const int half = M / 2 + M / (2 * E);   // padded index of row M/2
  const int banks = elem == 8 ? 16 : 32;
  int R = banks / (2 * W);
  if (R < 1) R = 1;
  auto up = [&](int x, int res) { return x + (((res - x) % banks) + banks) % banks; };
  const int PO = up(half, R % banks);
  const int LS = up(PO + half > ldsn ? PO + half : ldsn, (2 * R) % banks);
  return {PO, LS, (size_t)W * LS * elem};
}
inline bool pow2(int w) { return w >= 1 && (w & (w - 1)) == 0; }
inline int ilog2i(int w) {
  int l = 0;
  while ((1 << l) < w) ++l;
  return l;
}

Schedule default_schedule(const Geometry& g, bool fp32);
bool schedule_ok(const Geometry& g, const Schedule& s, bool fp32);

// Workspace bytes for nrhs right-hand sides (FFT intermediates).
size_t apply_workspace_bytes(const Geometry& g, int nrhs, bool fp32);

// Number of blocks per RHS of the last pass (= partials it writes).
int last_pass_blocks(const Geometry& g, const Schedule& sc);
// d = 1, FP64: the whole PCG solve in one launch, one workgroup per RHS
// (x, r, p, z in LDS).  pcs: preconditioner multiplier or null (plain CG);
// pc_odd: the tau preconditioner.  Writes x and cg.iters / status / res2 /
// active (0) per RHS; stops like the multi-kernel solve.
void cg1d_solve(const Geometry& g, int E, const double* f, double* x, const double* lam,
                const double* pcs, bool pc_odd, const CgScalars& cg, int nrhs, int maxiter,
                double tol, const void* tw, hipStream_t st);
// Blocks per RHS of the tau preconditioner's middle pass, and the number of
// r.z partials its PM_DOT application writes: the middle pass's blocks when
// they fit max_blocks (the dot is taken there, from the transformed values),
// else the last pass's.
long sine_mid_blocks(const Geometry& g, const Schedule& sc);
int tau_dot_blocks(const Geometry& g, const Schedule& sc, int max_blocks);
// The same for the mixed-radix sine passes (some 2 N_s not a power of two).
int tau_dot_blocks_any(const Geometry& g, int max_blocks);
// Multiplier of the tau preconditioner for the mixed-radix sine passes:
// tau_any_entries() = prod_s (N_s + 1) values (folded frequencies k_s in
// [0, N_s]), FP64 and FP32, from the generator G on {0..N}^d.
long tau_any_entries(const Geometry& g);
void build_tau_multiplier(const Geometry& g, const double* G, double* m64, float* m32,
                          hipStream_t st);
// Blocks per RHS of the vector kernels (update, init, sums).
int vec_blocks(long nd, int nrhs);

// y = A u (mode PM_PLAIN), CG product (d = 1, PM_CG: iteration start,
// p <- r + beta p from rvec/pvec, q = A p into y; d >= 2, PM_PQ: q = A u
// with u = p, p.q partials into cg->part_a), or FP64 residual (PM_RESID:
// y = f - A u).  PM_DOT writes its partials to cg->part_b.  ev (optional): npasses + 1
// events recorded around the passes; only >= 0 launches that pass alone.
// odd: every axis is odd-extended instead of zero-padded (positions 1..n and
// their negated reflections), which with a real even symbol applies
// S diag(.) S with S the sine transform of each axis (not with PM_CG).
template <typename T>
void apply_passes(const Geometry& g, const Schedule& sc, const T* lam, const Twiddles& tw,
                  const T* u, T* y, int nrhs, void* ws, hipStream_t st, int mode,
                  const T* rvec, T* pvec, const double* fvec, const CgScalars* cg,
                  const int* active, hipEvent_t* ev = nullptr, int only = -1,
                  bool odd = false, bool first_done = false);

// The tau preconditioner (d >= 2) split around the CG iteration start, for
// preconditioned CG: tau_front applies the sine passes of r up to the middle
// pass (into S1, nrhs * n^d values of T, with the r.z partials of the middle
// pass in cg.part_b); tau_back_direction finishes z = P r from S1 and, in
// the same pass, starts the next iteration: stopping test and beta
// (cg_begin), then p = z + beta p; given T1 (the product's workspace) that
// pass also runs the product's axis-0 forward pass of p on its tile (on the
// product's schedule sc; sp is the preconditioner's), so the product follows
// with apply_passes(..., first_done = true).  Only when sine_mid_blocks <=
// max_blocks.
// stop_test: tau_front's first pass begins with the end-of-iteration tests
// on r.r (tolerance, maxiter, non-finite, the reliable-update trigger), and
// tau_back_direction then tests r.z and forms beta; without it (after a
// reliable update) no test runs before the next iteration.
template <typename T>
void tau_front(const Geometry& g, const Schedule& sc, const T* m, const Twiddles& tw, const T* r,
               T* S1, int nrhs, hipStream_t st, const CgScalars& cg, const int* active,
               bool stop_test);
template <typename T>
void tau_back_direction(const Geometry& g, const Schedule& sc, const Schedule& sp,
                        const Twiddles& tw, T* S1, T* p, void* T1, int nrhs, hipStream_t st,
                        const CgScalars& cg);

// Number of kernel launches (passes) of one application: 1, 3 or 5 for d = 1, 2, 3.
inline int apply_npasses(int d) { return d == 1 ? 1 : (d == 2 ? 3 : 5); }

// Device memory for operator buffers and setup temporaries: the allocator
// registered with fl_set_allocator, else hipMalloc.  dev_free returns a block
// to the allocator that made it (after the device has finished with it).
void* dev_alloc(size_t bytes);
void dev_free(void* p);

// Scratch memory of operator setup on the current device.  Each device keeps
// one area (hipMalloc) for the life of the process; it grows to the largest
// lease up to kSetupScratchCap, so that a setup after the first frees
// nothing (hipFree waits for the whole device, stalling other streams' work).
// A larger lease takes a block of its own from dev_alloc.  The lease holds
// the device's area until it ends and synchronises `st` first, so every use
// of the memory must be queued on `st`.
constexpr size_t kSetupScratchCap = size_t(256) << 20;
class SetupScratch {
 public:
  SetupScratch(size_t bytes, hipStream_t st);
  ~SetupScratch();
  SetupScratch(const SetupScratch&) = delete;
  SetupScratch& operator=(const SetupScratch&) = delete;
  // Next `bytes` of the lease, 256-byte aligned; throws past its size.
  void* take(size_t bytes);
  struct Area;

 private:
  Area* area_ = nullptr;      // the device's area (locked), or null for a block of its own
  char* base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  hipStream_t st_;
};
inline size_t scratch_round(size_t b) { return (b + 255) & ~size_t(255); }

// Twiddle table exp(-2 pi i j / M), j < M (cx<T> array), cached per device
// for the life of the process (hipMalloc, not the registered allocator).
const void* twiddles(int M, bool fp32, hipStream_t st);

// Generator, symbol: see weights unit.
// Kernel K(r) = sum_i coef[i] exp(-rate[i] r) (rate 0: K = 1).  The weight
// integrals and the far-field constant are linear in K, so each term's are
// built as for one exponential and summed with its coefficient.
constexpr int kMaxKernelTerms = 16;
struct GenParams {
  int d, p, N;
  double alpha, h, c;
  double gamma;   // splitting parameter in (alpha, 2]
  int nterm;
  double coef[kMaxKernelTerms], rate[kMaxKernelTerms];
};
void build_generator(const GenParams& gp, double* G, hipStream_t st);
void build_symbol(const Geometry& g, const double* G, double* lam64, float* lam32,
                  hipStream_t st);
void embed_generator(const Geometry& g, const double* G, double* out, hipStream_t st);
// Exterior-data term (exterior unit): b = lattice sum of G with g on
// [-N, 2N]^d minus c * tail (tail may be null).  khat: the transformed
// wrapped generator(s) (exterior_khat_bytes), filled when !khat_ready; work:
// exterior_work_bytes.  Supported for d = 1, 2 and for d = 3 up to 1024^3
// transform points (cubes and boxes).
bool exterior_supported(const Geometry& g);
void difference(const double* a, const double* b, double* out, long n, hipStream_t st);
size_t exterior_khat_bytes(const Geometry& g);
size_t exterior_work_bytes(const Geometry& g);
void exterior_term(const Geometry& g, const double* G, double c, const double* g_lat,
                   const double* tail, double* b, int nrhs, void* khat, bool khat_ready,
                   void* work, hipStream_t st);

// In-place unnormalised DFT (dir -1) or inverse (dir +1) of a complex FP64
// array of P[0] x .. x P[d-1] points (interleaved re, im, last index
// fastest), each P[s] a supported power of two.
void fft_full(const int* P, int d, void* c, int dir, hipStream_t st);
void build_inverse_symbol(const Geometry& g, const double* lam64, long nf, double* inv64,
                          float* inv32, double* scratch, hipStream_t st);

// CG kernels (cg unit).  The vector kernels run cg.nb_c = vec_blocks(g.nd, nrhs)
// blocks per RHS and write that many r.r partials.
template <typename T>
void cg_init(const Geometry& g, const T* rhs, T* x, T* r, T* p, int nrhs, const CgScalars& cg,
             const int* outer_active, hipStream_t st);
// d >= 2: iteration start (stopping test, beta) and p = zr + beta p as a
// streaming pass; the product then runs with PM_PQ.
template <typename T>
void cg_direction(const Geometry& g, T* p, const T* zr, int nrhs, const CgScalars& cg,
                  hipStream_t st);
template <typename T>
void cg_update(const Geometry& g, T* x, T* r, const T* p, const T* q, int nrhs,
               const CgScalars& cg, hipStream_t st);
void fill_int(int* p, int v, int n, hipStream_t st);
// out[0] = n_active; out[1 + POLL_STRIDE o ..] = res2, thresh2, active, iters,
// r.r now, rr_last[o], f2[o], nupd[o] of RHS o (the last three 0 if null).
constexpr int POLL_STRIDE = 8;   // doubles per RHS in the poll record
void pack_poll(const CgScalars& cg, int nrhs, const double* rr_last, const double* f2,
               const int* nupd, double* out, hipStream_t st);
// Results of a finished solve for the host, RESULT_STRIDE doubles per RHS:
// iterations, status, reliable updates, recursive r.r, FP64 residual r.r,
// ||f||^2 (nupd and res2 may be null: 0).
constexpr int RESULT_STRIDE = 6;
void pack_results(int nrhs, const int* iters, const int* status, const int* nupd,
                  const double* res2, const double* rro, const double* f2, double* out,
                  hipStream_t st);
void fill_zero_bytes(void* p, size_t bytes, hipStream_t st);
// out[o] = sum_{b < nb} part[o * max_blocks + b] (fixed order)
void reduce_parts(const double* part, int nb, int max_blocks, int nrhs, double* out,
                  const int* active, hipStream_t st);
// refinement helpers
void refine_scale(const double* r64, float* r32, const double* rr, double* scale, long nd,
                  int nrhs, const int* active, hipStream_t st);
void refine_axpy(double* u, const float* d32, const double* scale, long nd, int nrhs,
                 const int* active, hipStream_t st);
// FP32 CG with FP64 reliable updates (see cg unit)
void to_float(const double* src, float* dst, long n, hipStream_t st);
void reliable_accum(const Geometry& g, double* xhi, float* xlo, int nrhs, const CgScalars& cg,
                    const int* trig, bool force, hipStream_t st);
void reliable_final(const int* status, const double* rr_last, int* mask, double* rr_true,
                    int nrhs, hipStream_t st);
void reliable_replace(const Geometry& g, const double* r64, float* r32, int nrhs,
                      const CgScalars& cg, const double* part64, int nb64, int mb64,
                      double* rr_last, const double* f2, double tol2, int* trig,
                      int* nupd, hipStream_t st);
// partials of sum v^2 per RHS into part (vec_blocks per RHS)
void sum_squares_parts(const double* v, long nd, int nrhs, double* part, int max_blocks,
                       hipStream_t st);

// The body of fl_apply_noalloc: fl_apply's checks and passes, with the
// transform intermediates in a fixed area of area_bytes instead of the
// handle's workspace.  area_of_device(dev) returns the area's address on
// device dev and is called with that device current (only when the product
// needs intermediates, d >= 2).  Allocates nothing; FL_E_UNSUPPORTED when
// the product needs more than area_bytes.  Returns an fl_status and sets the
// thread's error text like every entry point.
int apply_in_area(::fl_op_s* A, const void* u, void* y, int nrhs, int fp32, void* stream,
                  void* (*area_of_device)(int dev), size_t area_bytes);

}  // namespace fl
