// E4M3 screen kernels: the instantiations of screen_core.h for each
// compiled factor-chunk count.
#include "screen_core.h"

namespace mips {

hipError_t launch_screen_fp8(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    switch (p.NCH) {
        case 1: return screen_km<PREC_FP8, 1>(p, a, s);
        default: return screen_km<PREC_FP8, 2>(p, a, s);
    }
}

}  // namespace mips
