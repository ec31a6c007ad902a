// near_impl.h -- velocity bounce-back and momentum exchange at the fluid
// cells next to solid cells (arXiv:1708.08741, Sec. 3.2: Eq. LBMMovWall and
// Eq. LBMhydrodynForce with the torque about the particle centre).
//
// Runs after the sweep on the post-collision state f* it wrote.  For every
// blocked link (fluid cell x, direction q, solid neighbour s = x + e_q) the
// value that returns to x as population q-bar at the next gather,
//     f*_q(x) - 2 w_q rho0 c_q.u_s / c_s^2,
// is written into slot q-bar of s (solid cells are not updated, so their
// slots are free); a link to an obstacle cell of particle p adds
// [2 f*_q - 2 w_q rho0 c_q.u_s / c_s^2] c_q to F_p and r x (that) to M_p.
//
// Work distribution: one workgroup per particle walks the particle's link
// list (written by the classification: the fluid cells next to the particle
// with the directions that hit it), one link per lane in direction-major
// order, so the particle's position and velocities are uniform, no owner
// look-up is needed, and force and torque are summed over each wavefront in
// a fixed order (DPP row butterflies), the wavefronts' sums are combined in
// wavefront order through LDS after one barrier, and the result is stored
// without atomics.  Links to wall cells come from a list built when the
// walls are set.
#pragma once
#include "sweep_impl.h"

namespace lbmep {
namespace sweep {

// per-particle sums: F_dev[3], M_dev[3], K[3], T[3]
constexpr int kAcc = 12;

// v of the lane selected by a DPP control inside each row of 16 lanes (the
// two 32-bit halves moved separately)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) |
                                            (unsigned long long)(uint32_t)lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// sum of v over the wavefront (all 64 lanes active): butterfly inside each
// row of 16 by DPP (xor 1 and 2 by quad permutes, then the half-row and row
// mirrors), then the four row sums read from lanes 0, 16, 32, 48
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// the D3Q19 velocity components as 2-bit fields (value + 1), for directions
// known only at run time
constexpr uint64_t pack_dir(const int (&v)[Q]) {
    uint64_t r = 0;
    for (int q = 0; q < Q; ++q) r |= (uint64_t)(v[q] + 1) << (2 * q);
    return r;
}
constexpr uint64_t kPackCx = pack_dir(kCx), kPackCy = pack_dir(kCy), kPackCz = pack_dir(kCz);

__device__ __forceinline__ int dir_comp(uint64_t packed, int q) {
    return (int)((packed >> (2 * q)) & 3u) - 1;
}

// wrap one coordinate of a neighbour on a periodic axis; false beyond the
// edge of a non-periodic axis
__device__ __forceinline__ bool wrap_axis(int &v, int len, int periodic) {
    if (v < 0 || v >= len) {
        if (!periodic) return false;
        v = v < 0 ? v + len : v - len;
    }
    return true;
}

// the value bounced into slot opp(q) of the solid neighbour s
template <typename ST, typename OFF>
__device__ __forceinline__ void store_slot(const SweepArgs &a, int q, OFF s,
                                           typename Storage<ST>::CT fq, double mw) {
    using T = Storage<ST>;
    using CT = typename T::CT;
    // population base in 64 bits (q Ns can exceed 4 GiB), cell offset in OFF
    void *slot_base = static_cast<char *>(a.dst) + (size_t)opp(q) * a.g.Ns * sizeof(ST);
    ST *slot = at<ST>(slot_base, s * (OFF)sizeof(ST));
    if constexpr (sizeof(CT) == 8) {
        T::store(slot, fq - mw);
    } else {
        T::store(slot, (CT)((double)fq - mw));
    }
}

// post-collision value of population q of cell c
template <typename ST, typename OFF>
__device__ __forceinline__ typename Storage<ST>::CT load_fstar(const SweepArgs &a, int q,
                                                               uint32_t c) {
    const void *base = static_cast<const char *>(a.dst) + (size_t)q * a.g.Ns * sizeof(ST);
    return Storage<ST>::load(at<ST>(base, (OFF)c * (OFF)sizeof(ST)));
}

// One link of particle p in direction q (1..18, known at run time): the
// bounce-back slot and the momentum exchange into the lane's sums.
template <typename ST, typename OFF>
__device__ __forceinline__ void particle_link(const SweepArgs &a, uint32_t c, int q,
                                              const double Xp[3], const double Up[3],
                                              const double Wp[3], double acc[kAcc]) {
    using T = Storage<ST>;
    using CT = typename T::CT;
    const Grid &g = a.g;
    const int nx = g.nx, ny = g.ny;
    const int cx = dir_comp(kPackCx, q), cy = dir_comp(kPackCy, q), cz = dir_comp(kPackCz, q);
    int sx = (int)(c % (uint32_t)nx) + cx;
    int sy = (int)((c / (uint32_t)nx) % (uint32_t)ny) + cy;
    int sz = (int)(c / ((uint32_t)nx * (uint32_t)ny)) + cz;
    wrap_axis(sx, g.nx, g.per[0]);  // an obstacle cell: always inside
    wrap_axis(sy, g.ny, g.per[1]);
    wrap_axis(sz, g.nz, g.per[2]);
    const CT fq = load_fstar<ST, OFF>(a, q, c);
    // lever arm r = x_s - x_C (minimum image) and u_s = U + W x r
    const double r0 = min_image(((double)sx + 0.5) - Xp[0], g.nx, g.per[0]);
    const double r1 = min_image(((double)sy + 0.5) - Xp[1], g.ny, g.per[1]);
    const double r2 = min_image(((double)sz + 0.5) - Xp[2], g.nz, g.per[2]);
    const double us0 = Up[0] + (Wp[1] * r2 - Wp[2] * r1);
    const double us1 = Up[1] + (Wp[2] * r0 - Wp[0] * r2);
    const double us2 = Up[2] + (Wp[0] * r1 - Wp[1] * r0);
    // c_q . u_s with unit components: the zero terms add exact zeros
    const double cus = ((double)cx * us0 + (double)cy * us1) + (double)cz * us2;
    const double w = q <= 6 ? wq(1) : wq(7);
    // 2 (w_q / c_s^2) rho0 c_q . u_s (Eq. LBMMovWall)
    const double mw = 2.0 * w * 3.0 * cus;
    // [2 f*_q - 2 (w_q/c_s^2) rho0 c_q . u_s] c_q (Eq. LBMhydrodynForce),
    // summed as [2 (f*_q - w_q) - ...] c_q plus the rest-weight part
    // 2 w_q c_q = (k/18) c_q (k = 2 axis, 1 diagonal), whose sum cancels
    // over a closed body and is accumulated exactly as integers:
    // K = sum k c_q, T = sum k x_s x c_q (x_s the exact half-integer image
    // of the cell centre)
    const double gm = 2.0 * T::devval(fq, q) - mw;
    const double g0 = cx == 0 ? 0.0 : (cx > 0 ? gm : -gm);
    const double g1 = cy == 0 ? 0.0 : (cy > 0 ? gm : -gm);
    const double g2 = cz == 0 ? 0.0 : (cz > 0 ? gm : -gm);
    const double k = q <= 6 ? 2.0 : 1.0;
    const double xs0 = image_coord((double)sx + 0.5, Xp[0], g.nx, g.per[0]);
    const double xs1 = image_coord((double)sy + 0.5, Xp[1], g.ny, g.per[1]);
    const double xs2 = image_coord((double)sz + 0.5, Xp[2], g.nz, g.per[2]);
    acc[0] += g0;
    acc[1] += g1;
    acc[2] += g2;
    acc[3] += r1 * g2 - r2 * g1;
    acc[4] += r2 * g0 - r0 * g2;
    acc[5] += r0 * g1 - r1 * g0;
    acc[6] += k * (double)cx;
    acc[7] += k * (double)cy;
    acc[8] += k * (double)cz;
    acc[9] += k * (xs1 * (double)cz - xs2 * (double)cy);
    acc[10] += k * (xs2 * (double)cx - xs0 * (double)cz);
    acc[11] += k * (xs0 * (double)cy - xs1 * (double)cx);
    const OFF s = (OFF)sx + (OFF)g.nx * ((OFF)sy + (OFF)g.ny * (OFF)sz);
    store_slot<ST, OFF>(a, q, s, fq, mw);
}

// waves per particle in the exchange kernel (a 256-thread workgroup)
constexpr int kNearWaves = 4;
constexpr int kNearThreads = 64 * kNearWaves;
// list entries per pass: their links (at most 18 each) are staged in LDS
constexpr int kNearEntries = 128;

// All links of particle p (its list from the classification: cells with the
// directions whose neighbour is an obstacle cell of p), one workgroup: the
// bounce-back slots and the momentum exchange, summed in a fixed order and
// stored (no atomics: the result does not depend on scheduling).  The
// workgroup takes 128 list entries per pass and lays their links out
// direction by direction (per direction in list order, i.e. neighbouring
// cells along x), then works through them 256 at a time, one link per lane:
// every lane does useful work whatever the links per cell, and neighbouring
// lanes load and store neighbouring values of one population.
template <typename ST, typename OFF>
__device__ __forceinline__ void near_particle(const SweepArgs &a, uint32_t p) {
    __shared__ uint32_t lcell[kNearEntries * (Q - 1)];
    __shared__ uint8_t lq[kNearEntries * (Q - 1)];
    __shared__ uint32_t qcnt[2][Q];  // per direction: links of each half of the pass
    __shared__ double part[kNearWaves][kAcc];
    const int tid = (int)threadIdx.x, lane = (int)__lane_id(), wave = tid / 64;
    const uint2 *list = a.plist + (size_t)p * a.pcap;
    const uint32_t n = a.pcount[p];
    const double Xp[3] = {a.Xc[3 * (size_t)p], a.Xc[3 * (size_t)p + 1], a.Xc[3 * (size_t)p + 2]};
    const double Up[3] = {a.U[3 * (size_t)p], a.U[3 * (size_t)p + 1], a.U[3 * (size_t)p + 2]};
    const double Wp[3] = {a.W[3 * (size_t)p], a.W[3 * (size_t)p + 1], a.W[3 * (size_t)p + 2]};
    double acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (uint32_t e0 = 0; e0 < n; e0 += kNearEntries) {
        // waves 0 and 1 hold the pass's entries (one per lane); per direction
        // a ballot gives each lane its rank and each wave its count
        const uint32_t i = e0 + (uint32_t)tid;
        const bool mine = wave < 2 && i < n;
        const uint2 e = mine ? list[i] : make_uint2(0u, 0u);
        uint32_t rank[Q - 1];
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            const unsigned long long b = __ballot((e.y >> (q - 1)) & 1u);
            rank[q - 1] = (uint32_t)__popcll(b & below);
            if (lane == 0 && wave < 2) qcnt[wave][q] = (uint32_t)__popcll(b);
        }
        __syncthreads();
        // links in direction-major order: direction q starts after all links
        // of the lower directions, wave 1's after wave 0's
        uint32_t start = 0, total = 0;
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            const uint32_t off = start + (wave == 1 ? qcnt[0][q] : 0u);
            if (mine && ((e.y >> (q - 1)) & 1u)) {
                lcell[off + rank[q - 1]] = e.x;
                lq[off + rank[q - 1]] = (uint8_t)q;
            }
            start += qcnt[0][q] + qcnt[1][q];
        }
        total = start;
        __syncthreads();
        for (uint32_t k = (uint32_t)tid; k < total; k += kNearThreads)
            particle_link<ST, OFF>(a, lcell[k], (int)lq[k], Xp, Up, Wp, acc);
        __syncthreads();  // lcell, lq and qcnt are rewritten by the next pass
    }
    // wave sums, then the waves' sums in wave order: a fixed order
#pragma unroll
    for (int k = 0; k < kAcc; ++k) {
        const double t = wave_sum_f64(acc[k]);
        if (lane == 0) part[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < kAcc && a.FM) {
        double t = part[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < kNearWaves; ++w) t += part[w][threadIdx.x];
        a.FM[kAcc * (size_t)p + threadIdx.x] = t;
    }
}

// Links to wall cells (a list fixed while the walls are): plain bounce-back
// from a resting wall, grid-stride over the listed cells with their
// wall-link masks.
template <typename ST, typename OFF>
__device__ __forceinline__ void near_walls(const SweepArgs &a, uint32_t blk, uint32_t nblk) {
    using CT = typename Storage<ST>::CT;
    const uint32_t n = *a.wcount;
    const Grid &g = a.g;
    const int nx = g.nx, ny = g.ny;
    for (uint32_t i = blk * blockDim.x + threadIdx.x; i < n; i += nblk * blockDim.x) {
        const uint32_t c = a.wlist[i];
        uint32_t mask = a.nearmask[c];
        const int x = (int)(c % (uint32_t)nx);
        const int y = (int)((c / (uint32_t)nx) % (uint32_t)ny);
        const int z = (int)(c / ((uint32_t)nx * (uint32_t)ny));
        while (mask) {
            const int q = __ffs((int)mask);
            mask &= mask - 1u;
            int sx = x + dir_comp(kPackCx, q), sy = y + dir_comp(kPackCy, q),
                sz = z + dir_comp(kPackCz, q);
            wrap_axis(sx, nx, g.per[0]);  // a wall cell: always inside
            wrap_axis(sy, ny, g.per[1]);
            wrap_axis(sz, g.nz, g.per[2]);
            const CT fq = load_fstar<ST, OFF>(a, q, c);
            const OFF s = (OFF)sx + (OFF)nx * ((OFF)sy + (OFF)ny * (OFF)sz);
            store_slot<ST, OFF>(a, q, s, fq, 0.0);
        }
    }
}

// one particle per workgroup of the exchange kernel
__host__ __device__ inline uint32_t near_particle_blocks(int np) { return (uint32_t)np; }

// workgroups [0, np): one particle each; the rest: the wall links
template <typename ST, typename OFF>
__device__ __forceinline__ void near_block(const SweepArgs &a, uint32_t blk, uint32_t nblk) {
    const uint32_t pb = near_particle_blocks(a.np);
    if (blk < pb) {
        near_particle<ST, OFF>(a, blk);
    } else {
        near_walls<ST, OFF>(a, blk - pb, nblk - pb);
    }
}

template <typename ST, typename OFF>
__global__ void __launch_bounds__(256) k_near(SweepArgs a) {
    near_block<ST, OFF>(a, blockIdx.x, gridDim.x);
}

template <typename ST>
__global__ void __launch_bounds__(256) k_near_packed(PackTable t) {
    const int e = pack_find(t, blockIdx.x);
    const LatticeDev *d = t.d[e];
    const SweepArgs a = d->sweep[t.state[e]];
    near_block<ST, uint32_t>(a, blockIdx.x - t.start[e], t.start[e + 1] - t.start[e]);
}

// workgroups of the wall pass (0 without wall cells)
inline int near_wall_blocks(size_t N, bool walls) {
    if (!walls) return 0;
    size_t b = (N / 256 + 255) / 256;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

template <typename ST>
hipError_t launch_near_packed_typed(const PackTable &t, hipStream_t s) {
    const uint32_t total = t.start[t.n];
    if (t.n == 0 || total == 0) return hipSuccess;
    hipLaunchKernelGGL((k_near_packed<ST>), dim3(total), dim3(256), 0, s, t);
    return hipGetLastError();
}

template <typename ST>
hipError_t launch_near_typed(const SweepArgs &a, int wall_blocks, hipStream_t s) {
    const unsigned blocks = near_particle_blocks(a.np) + (unsigned)wall_blocks;
    if (blocks == 0) return hipSuccess;
    const bool small = 2 * a.g.Ns * sizeof(ST) < (size_t(1) << 32) && 4 * a.g.Ns < (size_t(1) << 32);
    if (small)
        hipLaunchKernelGGL((k_near<ST, uint32_t>), dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_near<ST, uint64_t>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sweep
}  // namespace lbmep
