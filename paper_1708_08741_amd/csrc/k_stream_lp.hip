// k_stream_lp.hip -- FP32 and FP16 deviation-storage instantiations of the
// fused sweep (sweep_impl.h), FP32 arithmetic with FMA contraction, and the
// precision dispatch of the sweep launch.
#include "sweep_impl.h"

namespace lbmep {

hipError_t launch_sweep_f64(int mode, int force_mode, const SweepArgs &a, int block_x,
                            hipStream_t s);

hipError_t launch_sweep(int precision, int mode, int force_mode, const SweepArgs &a, int block_x,
                        hipStream_t s) {
    if (precision == LBMEP_FP64) return launch_sweep_f64(mode, force_mode, a, block_x, s);
    if (precision == LBMEP_FP32DEV)
        return sweep::launch_typed<float>(mode, force_mode, a, block_x, s);
    return sweep::launch_typed<__half>(mode, force_mode, a, block_x, s);
}

}  // namespace lbmep
