// Depth-2 temporally blocked wave sweep (radius 4; single field set and
// batched shots), one instantiation per storage type.
#include "zmarch_tb.hpp"

namespace stn {

hipError_t tb2_wave(int dtype, const TBView& v, const Coefs& w, int arow, int trow_u, int trow_p, hipStream_t s) {
    switch (dtype) {
        case DT_F32: return tb2_launch<MODE_WAVE, 4, float>(v, w, arow, trow_u, trow_p, s);
        case DT_BF16: return tb2_launch<MODE_WAVE, 4, bf16>(v, w, arow, trow_u, trow_p, s);
        case DT_F16: return tb2_launch<MODE_WAVE, 4, f16>(v, w, arow, trow_u, trow_p, s);
    }
    return hipErrorInvalidValue;
}

hipError_t tb2_batch(int dtype, const TBView* views, const int* bmap, int nblocks, const Coefs& w, int arow,
                     int trow_u, int trow_p, hipStream_t s) {
    switch (dtype) {
        case DT_F32: return tb2_batch_launch<float>(views, bmap, nblocks, w, arow, trow_u, trow_p, s);
        case DT_BF16: return tb2_batch_launch<bf16>(views, bmap, nblocks, w, arow, trow_u, trow_p, s);
        case DT_F16: return tb2_batch_launch<f16>(views, bmap, nblocks, w, arow, trow_u, trow_p, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace stn
