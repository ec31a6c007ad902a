// k_stream_lp.hip -- FP32 and FP16 deviation-storage instantiations of the
// fused sweep (sweep_impl.h), FP32 arithmetic, and the precision dispatch of
// the sweep launch.
#include "near_impl.h"

namespace lbmep {

hipError_t launch_sweep_f64(int mode, int force_mode, const SweepArgs &a, int block_x,
                            int cpt, hipStream_t s);

hipError_t launch_sweep(int precision, int mode, int force_mode, const SweepArgs &a, int block_x,
                        int cpt, hipStream_t s) {
    if (precision == LBMEP_FP64) return launch_sweep_f64(mode, force_mode, a, block_x, cpt, s);
    if (precision == LBMEP_FP32DEV)
        return sweep::launch_typed<float>(mode, force_mode, a, block_x, cpt, s);
    return sweep::launch_typed<__half>(mode, force_mode, a, block_x, cpt, s);
}

hipError_t launch_near_f64(const SweepArgs &a, int wall_blocks, hipStream_t s);

hipError_t launch_near(int precision, const SweepArgs &a, int wall_blocks, hipStream_t s) {
    if (precision == LBMEP_FP64) return launch_near_f64(a, wall_blocks, s);
    if (precision == LBMEP_FP32DEV) return sweep::launch_near_typed<float>(a, wall_blocks, s);
    return sweep::launch_near_typed<__half>(a, wall_blocks, s);
}

hipError_t launch_sweep_packed_f64(int force_mode, const PackTable &t, hipStream_t s);
hipError_t launch_near_packed_f64(const PackTable &t, hipStream_t s);

hipError_t launch_sweep_packed(int precision, int force_mode, const PackTable &t, hipStream_t s) {
    if (precision == LBMEP_FP64) return launch_sweep_packed_f64(force_mode, t, s);
    if (precision == LBMEP_FP32DEV) return sweep::launch_sweep_packed_typed<float>(force_mode, t, s);
    return sweep::launch_sweep_packed_typed<__half>(force_mode, t, s);
}

hipError_t launch_near_packed(int precision, const PackTable &t, hipStream_t s) {
    if (precision == LBMEP_FP64) return launch_near_packed_f64(t, s);
    if (precision == LBMEP_FP32DEV) return sweep::launch_near_packed_typed<float>(t, s);
    return sweep::launch_near_packed_typed<__half>(t, s);
}

}  // namespace lbmep
