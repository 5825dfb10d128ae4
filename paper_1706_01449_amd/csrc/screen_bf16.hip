// bfloat16 screen kernels: the instantiations of screen_core.h for each
// compiled factor-chunk count.
#include "screen_core.h"

namespace mips {

hipError_t launch_screen_bf16(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s) {
    switch (p.NCH) {
        case 1: return screen_km<PREC_BF16, 1>(p, a, s);
        case 2: return screen_km<PREC_BF16, 2>(p, a, s);
        case 4: return screen_km<PREC_BF16, 4>(p, a, s);
        default: return screen_km<PREC_BF16, 8>(p, a, s);
    }
}

}  // namespace mips
