// float32 screen kernels: the instantiations of screen_core.h for each
// compiled factor-chunk count.
#include "screen_core.h"

namespace mips {

hipError_t launch_screen_fp32(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    switch (p.NCH) {
        case 8: return screen_km<PREC_FP32, 8>(p, a, s);
        case 16: return screen_km<PREC_FP32, 16>(p, a, s);
        case 25: return screen_km<PREC_FP32, 25>(p, a, s);
        case 32: return screen_km<PREC_FP32, 32>(p, a, s);
        case 50: return screen_km<PREC_FP32, 50>(p, a, s);
        default: return screen_km<PREC_FP32, 64>(p, a, s);
    }
}

}  // namespace mips
