// FP32-only z-marching sweeps: the adjoint path's forward recompute writing
// second differences and adjoint with imaging (one or two levels per
// launch), and the wave with an absorbing layer.
#include "zmarch.hpp"

namespace stn {

hipError_t zmarch_adj_f32(int mode, int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow,
                         int trow, hipStream_t s) {
    if (mode == MODE_WAVE_D) return zm_r<MODE_WAVE_D, float>(radius, cfg, v, w, parity, arow, trow, s);
    if (mode == MODE_WAVE_ADJ) return zm_r<MODE_WAVE_ADJ, float>(radius, cfg, v, w, parity, arow, trow, s);
    if (mode == MODE_WAVE_ADJ2) return zm_r<MODE_WAVE_ADJ2, float>(radius, cfg, v, w, parity, arow, trow, s);
    if (mode == MODE_WAVE_DAMP) return zm_r<MODE_WAVE_DAMP, float>(radius, cfg, v, w, parity, arow, trow, s);
    return hipErrorInvalidValue;
}

}  // namespace stn
