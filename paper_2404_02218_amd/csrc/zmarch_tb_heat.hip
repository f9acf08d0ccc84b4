// Depth-2 temporally blocked heat sweep, FP32 storage, radius 1..4.
#include "zmarch_tb.hpp"

namespace stn {

hipError_t tb2_heat_f32(int radius, const TBView& v, const Coefs& w, hipStream_t s) {
    switch (radius) {
        case 1: return tb2_launch<MODE_HEAT, 1, float>(v, w, 0, -1, -1, s);
        case 2: return tb2_launch<MODE_HEAT, 2, float>(v, w, 0, -1, -1, s);
        case 3: return tb2_launch<MODE_HEAT, 3, float>(v, w, 0, -1, -1, s);
        case 4: return tb2_launch<MODE_HEAT, 4, float>(v, w, 0, -1, -1, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace stn
