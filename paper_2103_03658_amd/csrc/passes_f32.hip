// Single-precision instantiation of the FFT passes (inner solves).
#include "passes_host.h"

namespace fl {

template <>
void apply_passes<float>(const Geometry& g, const Schedule& sc, const float* lam,
                         const Twiddles& tw, const float* u, float* y, int nrhs, void* ws,
                         hipStream_t st, int mode, const float* rvec, float* pvec,
                         const double* fvec, const CgScalars* cg, const int* active,
                          hipEvent_t* ev, int only, bool odd) {
  apply_passes_t<float>(g, sc, lam, tw, u, y, nrhs, ws, st, mode, rvec, pvec, fvec, cg, active, ev, only, odd);
}

}  // namespace fl
