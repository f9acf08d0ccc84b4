// Heat and wave z-marching sweeps, bf16 storage, and the batched-shot sweep.
#include "zmarch.hpp"

namespace stn {

hipError_t zmarch_fwd_bf16(int mode, int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow,
                          int trow, hipStream_t s) {
    return zmarch_modes<bf16>(mode, radius, cfg, v, w, parity, arow, trow, s);
}

hipError_t zmarch_batch_bf16(int radius, int cfg, const ZView* views, const int* bmap, int nblocks,
                            const Coefs& w, int parity, int arow, int trow, hipStream_t s) {
    return zb_cfg<bf16>(radius, cfg, views, bmap, nblocks, w, parity, arow, trow, s);
}

hipError_t zmarch_batch_persistent_bf16(int radius, int cfg, const ZView* views, const int* list, const int* off, int grid,
                                      const Coefs& w, int t0, int t1, int rec_on, int pmask, unsigned long long* sync,
                                      int spin_limit, hipStream_t s) {
    return zbp_launch<bf16>(radius, cfg, views, list, off, grid, w, t0, t1, rec_on, pmask, sync, spin_limit, s);
}

hipError_t zmarch_batch_persistent_per_cu_bf16(int radius, int cfg, int* per_cu) {
    return zbp_per_cu<bf16>(radius, cfg, *per_cu);
}

}  // namespace stn
