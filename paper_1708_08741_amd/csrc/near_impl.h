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
// Work distribution: each wavefront takes 64 consecutive entries of the list
// of NEAR cells, scans the popcounts of their blocked-direction masks, and
// then lets every lane handle one link per iteration (the link's cell and
// direction decoded from the scan by a fixed-length binary search over the
// lanes), so lanes do not idle on cells with few blocked links.  Each lane
// takes a contiguous run of links (mostly of one cell, hence one particle);
// force and torque are summed per lane, then per particle across the
// wavefront by shuffles after each chunk, with one FP64 atomic per particle,
// chunk and component (the wavefront sums by DPP row butterflies).
#pragma once
#include "sweep_impl.h"

namespace lbmep {
namespace sweep {

// per-particle accumulators: F_dev[3], M_dev[3], K[3], T[3]
constexpr int kAcc = 12;

__device__ __forceinline__ void flush_particle(double *FM, uint32_t p, const double acc[kAcc]) {
#pragma unroll
    for (int k = 0; k < kAcc; ++k) unsafeAtomicAdd(&FM[kAcc * (size_t)p + k], acc[k]);
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

// c . a with the zero terms of ((c_x a_x + c_y a_y) + c_z a_z) dropped, in
// the same order and rounding as cdot<q>
__device__ __forceinline__ double cdot_rt(int cx, int cy, int cz, double ax, double ay,
                                          double az) {
    double r = 0.0;
    if (cx != 0 && cy != 0)
        r = (cx > 0 ? ax : -ax) + (cy > 0 ? ay : -ay);
    else if (cx != 0)
        r = cx > 0 ? ax : -ax;
    else if (cy != 0)
        r = cy > 0 ? ay : -ay;
    if (cz != 0) r = (cx != 0 || cy != 0) ? r + (cz > 0 ? az : -az) : (cz > 0 ? az : -az);
    return r;
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

// one blocked link: the bounce-back slot and, for an obstacle cell of
// particle p, the momentum exchange into the lane's accumulators
template <typename ST, typename OFF>
__device__ __forceinline__ void bounce_link(const SweepArgs &a, int q, int cx, int cy, int cz,
                                            int sx, int sy, int sz,
                                            typename Storage<ST>::CT fq, uint32_t p,
                                            uint32_t &pp, double acc[kAcc]) {
    using T = Storage<ST>;
    using CT = typename T::CT;
    const Grid &g = a.g;
    const OFF s = (OFF)sx + (OFF)g.nx * ((OFF)sy + (OFF)g.ny * (OFF)sz);
    const double w = q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0;
    double mw = 0.0;
    if (p != kNone) {
        const double *X = a.Xc + 3 * (size_t)p;
        const double *U = a.U + 3 * (size_t)p;
        const double *W = a.W + 3 * (size_t)p;
        // lever arm r = x_s - x_C (minimum image) and u_s = U + W x r
        const double r0 = min_image(((double)sx + 0.5) - X[0], g.nx, g.per[0]);
        const double r1 = min_image(((double)sy + 0.5) - X[1], g.ny, g.per[1]);
        const double r2 = min_image(((double)sz + 0.5) - X[2], g.nz, g.per[2]);
        const double us0 = U[0] + (W[1] * r2 - W[2] * r1);
        const double us1 = U[1] + (W[2] * r0 - W[0] * r2);
        const double us2 = U[2] + (W[0] * r1 - W[1] * r0);
        const double cus = cdot_rt(cx, cy, cz, us0, us1, us2);
        // 2 (w_q / c_s^2) rho0 c_q . u_s (Eq. LBMMovWall)
        mw = 2.0 * w * 3.0 * cus;
        // [2 f*_q - 2 (w_q/c_s^2) rho0 c_q . u_s] c_q (Eq. LBMhydrodynForce),
        // summed as [2 (f*_q - w_q) - ...] c_q plus the rest-weight part
        // 2 w_q c_q = (k/18) c_q (k = 2 axis, 1 diagonal), whose sum cancels
        // over a closed body and is accumulated exactly as integers:
        // K = sum k c_q, T = sum k x_s x c_q (x_s the exact half-integer
        // image of the cell centre)
        const double gm = 2.0 * T::devval(fq, q) - mw;
        const double g0 = cx == 0 ? 0.0 : (cx > 0 ? gm : -gm);
        const double g1 = cy == 0 ? 0.0 : (cy > 0 ? gm : -gm);
        const double g2 = cz == 0 ? 0.0 : (cz > 0 ? gm : -gm);
        const double k = q <= 6 ? 2.0 : 1.0;
        const double xs0 = image_coord((double)sx + 0.5, X[0], g.nx, g.per[0]);
        const double xs1 = image_coord((double)sy + 0.5, X[1], g.ny, g.per[1]);
        const double xs2 = image_coord((double)sz + 0.5, X[2], g.nz, g.per[2]);
        if (pp != p) {
            if (pp != kNone) flush_particle(a.FM, pp, acc);
            pp = p;
#pragma unroll
            for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
        }
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
    }
    // population base in 64 bits (q Ns can exceed 4 GiB), cell offset in OFF
    const int qb = opp(q);
    void *slot_base = static_cast<char *>(a.dst) + (size_t)qb * g.Ns * sizeof(ST);
    ST *slot = at<ST>(slot_base, s * (OFF)sizeof(ST));
    if constexpr (sizeof(CT) == 8) {
        T::store(slot, fq - mw);
    } else {
        T::store(slot, (CT)((double)fq - mw));
    }
}

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

// sum the lanes' accumulators per particle across the wavefront (every lane
// takes part) and add them with one FP64 atomic per particle and component;
// clears the lanes' accumulators
__device__ __forceinline__ void wave_flush(double *FM, uint32_t &pp, double acc[kAcc]) {
    const int lane = (int)__lane_id();
    unsigned long long pend = __ballot(pp != kNone);
    while (pend) {
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const uint32_t lp = (uint32_t)__builtin_amdgcn_readlane((int)pp, leader);
        const bool mine = pp == lp;
        // one component at a time (keeps the register footprint low)
#pragma unroll
        for (int k = 0; k < kAcc; ++k) {
            const double t = wave_sum_f64(mine ? acc[k] : 0.0);
            if (lane == leader) unsafeAtomicAdd(&FM[kAcc * (size_t)lp + k], t);
        }
        if (mine) pp = kNone;
        pend = __ballot(pp != kNone);
    }
#pragma unroll
    for (int k = 0; k < kAcc; ++k) acc[k] = 0.0;
}

template <typename ST, typename OFF>
__device__ __forceinline__ void near_range(const SweepArgs &a, const uint32_t *list,
                                           const uint32_t *count, uint32_t blk, uint32_t nblk) {
    using T = Storage<ST>;
    using CT = typename T::CT;
    const uint32_t n = *count;
    const Grid &g = a.g;
    const int nx = g.nx, ny = g.ny;
    const int lane = (int)__lane_id();
    const uint32_t wpb = blockDim.x / 64;
    const uint32_t wave = blk * wpb + threadIdx.x / 64, nwaves = nblk * wpb;
    uint32_t pp = kNone;
    double acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;
    for (uint32_t base = wave * 64u; base < n; base += nwaves * 64u) {
        const uint32_t i = base + (uint32_t)lane;
        uint32_t c = 0, mask = 0;
        if (i < n) {
            c = list[i];
            mask = a.nearmask[c];
        }
        // inclusive scan of the link counts over the wavefront
        uint32_t incl = (uint32_t)__popc(mask);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
            if (lane >= off) incl += t;
        }
        const uint32_t total = (uint32_t)__shfl((int)incl, 63);
        // lane l takes the contiguous links [l len, (l+1) len): mostly links
        // of one cell, so of one particle
        const uint32_t len = (total + 63u) / 64u;
        for (uint32_t it = 0; it < len; ++it) {
            const uint32_t k = (uint32_t)lane * len + it;
            // owning lane: the number of lanes whose inclusive count is <= k
            int j = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                const uint32_t v = (uint32_t)__shfl((int)incl, j + step - 1);
                if (v <= k) j += step;
            }
            const uint32_t cj = (uint32_t)__shfl((int)c, j);
            uint32_t mj = (uint32_t)__shfl((int)mask, j);
            const uint32_t ej = (uint32_t)__shfl((int)incl, j) - (uint32_t)__popc(mj);
            if (k >= total) continue;
            // the (k - ej)-th blocked direction of cell cj
            for (uint32_t r = k - ej; r > 0; --r) mj &= mj - 1u;
            const int q = __ffs((int)mj);  // bit q-1 <-> direction q
            const int x = (int)(cj % (uint32_t)nx);
            const int y = (int)((cj / (uint32_t)nx) % (uint32_t)ny);
            const int z = (int)(cj / ((uint32_t)nx * (uint32_t)ny));
            const int cx = dir_comp(kPackCx, q), cy = dir_comp(kPackCy, q),
                      cz = dir_comp(kPackCz, q);
            int sx = x + cx, sy = y + cy, sz = z + cz;
            // beyond a non-periodic edge the sweep bounces from the cell itself
            if (!(wrap_axis(sx, nx, g.per[0]) && wrap_axis(sy, ny, g.per[1]) &&
                  wrap_axis(sz, g.nz, g.per[2])))
                continue;
            const void *fq_base = static_cast<const char *>(a.dst) + (size_t)q * g.Ns * sizeof(ST);
            const CT fq = T::load(at<ST>(fq_base, (OFF)cj * (OFF)sizeof(ST)));
            uint32_t p = kNone;
            if (a.owner)
                p = a.owner[(size_t)sx + (size_t)nx * ((size_t)sy + (size_t)ny * (size_t)sz)];
            bounce_link<ST, OFF>(a, q, cx, cy, cz, sx, sy, sz, fq, p, pp, acc);
        }
        if (a.FM) wave_flush(a.FM, pp, acc);
    }
}

template <typename ST, typename OFF>
__global__ void __launch_bounds__(256) k_near(SweepArgs a, const uint32_t *list,
                                              const uint32_t *count) {
    near_range<ST, OFF>(a, list, count, blockIdx.x, gridDim.x);
}

template <typename ST>
__global__ void __launch_bounds__(256) k_near_packed(PackTable t) {
    const int e = pack_find(t, blockIdx.x);
    const LatticeDev *d = t.d[e];
    const SweepArgs a = d->sweep[t.state[e]];
    near_range<ST, uint32_t>(a, d->near_list, d->near_count, blockIdx.x - t.start[e],
                             t.start[e + 1] - t.start[e]);
}

// workgroups of the exchange kernel for a grid of N cells: a NEAR list of a
// few per cent of the cells, a few list chunks per wavefront, at most enough
// workgroups to fill the GPU several times
inline int near_blocks_for(size_t N) {
    size_t blocks = (N / 64 + 1023) / 1024;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}

template <typename ST>
hipError_t launch_near_packed_typed(const PackTable &t, hipStream_t s) {
    const uint32_t total = t.start[t.n];
    if (t.n == 0 || total == 0) return hipSuccess;
    hipLaunchKernelGGL((k_near_packed<ST>), dim3(total), dim3(256), 0, s, t);
    return hipGetLastError();
}

template <typename ST>
hipError_t launch_near_typed(const SweepArgs &a, const uint32_t *list, const uint32_t *count,
                             hipStream_t s) {
    const size_t blocks = (size_t)near_blocks_for(a.g.N);
    const bool small = 2 * a.g.Ns * sizeof(ST) < (size_t(1) << 32) && 4 * a.g.Ns < (size_t(1) << 32);
    if (small)
        hipLaunchKernelGGL((k_near<ST, uint32_t>), dim3((unsigned)blocks), dim3(256), 0, s, a,
                           list, count);
    else
        hipLaunchKernelGGL((k_near<ST, uint64_t>), dim3((unsigned)blocks), dim3(256), 0, s, a,
                           list, count);
    return hipGetLastError();
}

}  // namespace sweep
}  // namespace lbmep
