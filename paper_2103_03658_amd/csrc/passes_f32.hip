// Single-precision instantiation of the FFT passes (inner solves).
#include "passes_host.h"

namespace fl {

template <>
void apply_passes<float>(const Geometry& g, const Schedule& sc, const float* lam,
                         const Twiddles& tw, const float* u, float* y, int nrhs, void* ws,
                         hipStream_t st, int mode, const float* rvec, float* pvec,
                         const double* fvec, const CgScalars* cg, const int* active,
                          hipEvent_t* ev, int only, bool odd, bool first_done) {
  apply_passes_t<float>(g, sc, lam, tw, u, y, nrhs, ws, st, mode, rvec, pvec, fvec, cg, active, ev,
                    only, odd, first_done);
}

template <>
void tau_front<float>(const Geometry& g, const Schedule& sc, const float* m, const Twiddles& tw,
                     const float* r, float* S1, int nrhs, hipStream_t st, const CgScalars& cg,
                     const int* active, bool stop_test) {
  tau_front_t<float>(g, sc, m, tw, r, S1, nrhs, st, cg, active, stop_test);
}

template <>
void tau_back_direction<float>(const Geometry& g, const Schedule& sc, const Schedule& sp,
                              const Twiddles& tw, float* S1, float* p, void* T1, int nrhs,
                              hipStream_t st, const CgScalars& cg) {
  tau_back_direction_t<float>(g, sc, sp, tw, S1, p, T1, nrhs, st, cg);
}

}  // namespace fl
