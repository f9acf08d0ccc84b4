// Depth-2 temporally blocked wave sweep, one instantiation per storage type.
#include "zmarch_tb.hpp"

namespace stn {

hipError_t tb2_f32(const TBView& v, const Coefs& w, int arow, int trow_u, int trow_p, hipStream_t s) {
    return tb2_launch<float>(v, w, arow, trow_u, trow_p, s);
}

hipError_t tb2_bf16(const TBView& v, const Coefs& w, int arow, int trow_u, int trow_p, hipStream_t s) {
    return tb2_launch<bf16>(v, w, arow, trow_u, trow_p, s);
}

hipError_t tb2_f16(const TBView& v, const Coefs& w, int arow, int trow_u, int trow_p, hipStream_t s) {
    return tb2_launch<f16>(v, w, arow, trow_u, trow_p, s);
}

}  // namespace stn
