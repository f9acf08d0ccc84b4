// Heat and wave z-marching sweeps, f16 storage, and the batched-shot sweep.
#include "zmarch.hpp"

namespace stn {

hipError_t zmarch_fwd_f16(int mode, int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow,
                          int trow, hipStream_t s) {
    return zmarch_modes<f16>(mode, radius, cfg, v, w, parity, arow, trow, s);
}

hipError_t zmarch_batch_f16(int radius, int cfg, const ZView* views, const int* bmap, int nblocks,
                            const Coefs& w, int parity, int arow, int trow, hipStream_t s) {
    return zb_cfg<f16>(radius, cfg, views, bmap, nblocks, w, parity, arow, trow, s);
}

}  // namespace stn
