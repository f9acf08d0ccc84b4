// Depth-2 temporally blocked wave sweep with an absorbing layer (radius 4,
// FP32 storage): the damped leapfrog in both stages.
#include "zmarch_tb.hpp"

namespace stn {

hipError_t tb2_wave_damp_f32(const TBView& v, const Coefs& w, int arow, int trow_u, int trow_p, hipStream_t s) {
    return tb2_launch<MODE_WAVE_DAMP, 4, float>(v, w, arow, trow_u, trow_p, s);
}

}  // namespace stn
