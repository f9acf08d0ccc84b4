// Heat and wave z-marching sweeps, f32 storage, and the batched-shot sweep.
#include "zmarch.hpp"

namespace stn {

hipError_t zmarch_fwd_f32(int mode, int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow,
                          int trow, hipStream_t s) {
    return zmarch_modes<float>(mode, radius, cfg, v, w, parity, arow, trow, s);
}

hipError_t zmarch_batch_f32(int radius, int cfg, const ZView* views, const int* bmap, int nblocks,
                            const Coefs& w, int parity, int arow, int trow, hipStream_t s) {
    return zb_cfg<float>(radius, cfg, views, bmap, nblocks, w, parity, arow, trow, s);
}

}  // namespace stn
