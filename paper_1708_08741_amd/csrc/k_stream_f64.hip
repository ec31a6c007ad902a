// k_stream_f64.hip -- FP64 instantiation of the fused sweep (sweep_impl.h).
// Built without floating-point contraction: the collision, forcing and
// bounce-back evaluate the same operation sequence as a plain FP64 CPU
// implementation of Sec. 3.1-3.2 of arXiv:1708.08741.
#include "near_impl.h"

namespace lbmep {

hipError_t launch_sweep_f64(int mode, int force_mode, const SweepArgs &a, int block_x,
                            int cpt, hipStream_t s) {
    return sweep::launch_typed<double>(mode, force_mode, a, block_x, cpt, s);
}

hipError_t launch_near_f64(const SweepArgs &a, int wall_blocks, hipStream_t s) {
    return sweep::launch_near_typed<double>(a, wall_blocks, s);
}

hipError_t launch_sweep_packed_f64(int force_mode, const PackTable &t, hipStream_t s) {
    return sweep::launch_sweep_packed_typed<double>(force_mode, t, s);
}

hipError_t launch_near_packed_f64(const PackTable &t, hipStream_t s) {
    return sweep::launch_near_packed_typed<double>(t, s);
}

int near_wall_blocks(const Grid &g, bool walls) { return sweep::near_wall_blocks(g.N, walls); }
int near_blocks(int np, const Grid &g, bool walls) {
    return (int)sweep::near_particle_blocks(np) + sweep::near_wall_blocks(g.N, walls);
}

}  // namespace lbmep
