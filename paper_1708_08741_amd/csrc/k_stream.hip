// k_stream.hip -- fused collide + push-stream sweep of the D3Q19 TRT lattice
// Boltzmann method with a body force and moving-obstacle bounce-back
// (arXiv:1708.08741, Sec. 3.1 Eq. LBMcollideStep / Eq. LBMstreamStep with
// Eq. LBE_forcetermLuo and Eq. modified_velocity; Sec. 3.2 Eq. LBMMovWall and
// Eq. LBMhydrodynForce).
//
// One thread per cell, one block per (part of an) x-row.  Populations are SoA
// f[q][z][y][x]; a thread loads its own 19 values (aligned, coalesced), does
// the TRT collision with the forcing term, and pushes f*_q to x + e_q
// (writes shifted by at most one element along x, so a row's cache lines are
// completed inside its block).  The bulk path has no neighbour look-ups.
// Cells next to a wall, an obstacle or the edge of a non-periodic axis carry
// the NEAR flag and an 18-bit mask of blocked directions; for them the
// blocked pushes are replaced by the (velocity) bounce-back into the cell's
// own slot of the opposite population, and the momentum-exchange terms are
// summed per particle in FP64 (per lane, then across the wavefront by
// shuffles, then one FP64 atomic per particle and wavefront).
#include "lbmep_internal.h"

namespace lbmep {
namespace {

template <typename ST>
struct Storage;

// FP64: absolute populations
template <>
struct Storage<double> {
    using CT = double;
    static __device__ __forceinline__ double load(const double *p) { return *p; }
    static __device__ __forceinline__ void store(double *p, double v) { *p = v; }
    // deviation f - w_q of a computed population q, in FP64
    static __device__ __forceinline__ double devval(double v, int q) { return v - wq(q); }
};

// FP32: deviations f - w_q
template <>
struct Storage<float> {
    using CT = float;
    static __device__ __forceinline__ float load(const float *p) { return *p; }
    static __device__ __forceinline__ void store(float *p, float v) { *p = v; }
    static __device__ __forceinline__ double devval(float v, int q) { return (double)v; }
};

// FP16: deviations scaled by 2^24
template <>
struct Storage<__half> {
    using CT = float;
    static __device__ __forceinline__ float load(const __half *p) {
        return __half2float(*p) * kHalfInvScale;
    }
    static __device__ __forceinline__ void store(__half *p, float v) {
        *p = __float2half_rn(v * kHalfScale);
    }
    static __device__ __forceinline__ double devval(float v, int q) { return (double)v; }
};

// a . c_q for a lattice direction, with the zero terms of
// ((c_x a_x + c_y a_y) + c_z a_z) dropped (same value, same rounding)
template <int q, typename T>
__device__ __forceinline__ T cdot(T ax, T ay, T az) {
    constexpr int a = kCx[q], b = kCy[q], c = kCz[q];
    T r = T(0);
    if constexpr (a != 0 && b != 0) {
        r = (a > 0 ? ax : -ax) + (b > 0 ? ay : -ay);
    } else if constexpr (a != 0) {
        r = (a > 0 ? ax : -ax);
    } else if constexpr (b != 0) {
        r = (b > 0 ? ay : -ay);
    }
    if constexpr (c != 0) {
        if constexpr (a != 0 || b != 0)
            r = r + (c > 0 ? az : -az);
        else
            r = (c > 0 ? az : -az);
    }
    return r;
}

__device__ __forceinline__ double min_image(double d, int len, int periodic) {
    if (periodic) {
        const double h = 0.5 * (double)len;
        if (d > h)
            d -= (double)len;
        else if (d < -h)
            d += (double)len;
    }
    return d;
}

// nearest periodic image of the half-integer cell coordinate c to X (exact)
__device__ __forceinline__ double image_coord(double c, double X, int len, int periodic) {
    if (periodic) {
        const double d = c - X, h = 0.5 * (double)len;
        if (d > h)
            c -= (double)len;
        else if (d < -h)
            c += (double)len;
    }
    return c;
}

// per-particle accumulators: F_dev[3], M_dev[3], K[3], T[3]
constexpr int kAcc = 12;

__device__ __forceinline__ void flush_particle(double *FM, uint32_t p, const double acc[kAcc]) {
#pragma unroll
    for (int k = 0; k < kAcc; ++k) unsafeAtomicAdd(&FM[kAcc * (size_t)p + k], acc[k]);
}

// Velocity bounce-back of population q (blocked: x + e_q is solid or out of
// the domain) and its momentum-exchange contribution.
template <int q, typename ST>
__device__ __forceinline__ void bounce(const SweepArgs &a, ST *__restrict__ dst, size_t c, int x,
                                       int y, int z, typename Storage<ST>::CT fq, uint32_t &pp,
                                       double acc[kAcc]) {
    using T = Storage<ST>;
    using CT = typename T::CT;
    constexpr int cx = kCx[q], cy = kCy[q], cz = kCz[q];
    const Grid &g = a.g;
    int sx = x + cx, sy = y + cy, sz = z + cz;
    bool inside = true;
    if (sx < 0 || sx >= g.nx) {
        if (g.per[0]) sx = sx < 0 ? sx + g.nx : sx - g.nx; else inside = false;
    }
    if (sy < 0 || sy >= g.ny) {
        if (g.per[1]) sy = sy < 0 ? sy + g.ny : sy - g.ny; else inside = false;
    }
    if (sz < 0 || sz >= g.nz) {
        if (g.per[2]) sz = sz < 0 ? sz + g.nz : sz - g.nz; else inside = false;
    }
    double mw = 0.0;
    if (inside && a.owner) {
        const size_t s = (size_t)sx + (size_t)g.nx * ((size_t)sy + (size_t)g.ny * (size_t)sz);
        const uint32_t p = a.owner[s];
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
            const double cus = cdot<q>(us0, us1, us2);
            // 2 (w_q / c_s^2) rho0 c_q . u_s (Eq. LBMMovWall)
            mw = 2.0 * wq(q) * 3.0 * cus;
            // [2 f*_q - 2 (w_q/c_s^2) rho0 c_q . u_s] c_q (Eq. LBMhydrodynForce),
            // summed as [2 (f*_q - w_q) - ...] c_q plus the rest-weight part
            // 2 w_q c_q = (k/18) c_q (k = 2 axis, 1 diagonal), whose sum
            // cancels over a closed body and is accumulated exactly as
            // integers: K = sum k c_q, T = sum k x_s x c_q (x_s the exact
            // half-integer image of the cell centre)
            const double gm = 2.0 * T::devval(fq, q) - mw;
            const double g0 = cx == 0 ? 0.0 : (cx > 0 ? gm : -gm);
            const double g1 = cy == 0 ? 0.0 : (cy > 0 ? gm : -gm);
            const double g2 = cz == 0 ? 0.0 : (cz > 0 ? gm : -gm);
            constexpr double k = q <= 6 ? 2.0 : 1.0;
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
    }
    constexpr int qb = opp(q);
    if constexpr (sizeof(CT) == 8) {
        T::store(dst + (size_t)qb * g.Ns + c, fq - mw);
    } else {
        T::store(dst + (size_t)qb * g.Ns + c, (CT)((double)fq - mw));
    }
}

template <int q, typename ST>
__device__ __forceinline__ void push(ST *__restrict__ dst, size_t Ns, const size_t rows[3][3],
                                     const int xs[3], typename Storage<ST>::CT v, uint32_t mask) {
    if (!(mask & (1u << (q - 1)))) {
        const size_t i = (size_t)xs[kCx[q] + 1] + rows[kCy[q] + 1][kCz[q] + 1];
        Storage<ST>::store(dst + (size_t)q * Ns + i, v);
    }
}

template <int q, typename ST>
__device__ __forceinline__ void maybe_bounce(const SweepArgs &a, ST *__restrict__ dst, size_t c,
                                             int x, int y, int z, typename Storage<ST>::CT v,
                                             uint32_t mask, uint32_t &pp, double acc[kAcc]) {
    if (mask & (1u << (q - 1))) bounce<q, ST>(a, dst, c, x, y, z, v, pp, acc);
}

// the TRT collision of one opposite pair (q, q+1) with the forcing term
template <int q, typename CT>
__device__ __forceinline__ void collide_pair(CT (&v)[Q], CT rho, CT ux, CT uy, CT uz, CT uu,
                                             CT ufb, CT fb0, CT fb1, CT fb2, CT le, CT lo, CT ae,
                                             CT ao, bool forced) {
    constexpr int qb = q + 1;
    const CT w = (CT)wq(q);
    const CT cu = cdot<q>(ux, uy, uz);
    // equilibrium halves (Eq. EqPDF_TRT), rho0 = 1, 1/c_s^2 = 3, 1/c_s^4 = 9
    const CT feq_e = w * ((rho - uu * CT(1.5)) + (cu * cu) * CT(4.5));
    const CT feq_o = w * (CT(3.0) * cu);
    const CT fe = CT(0.5) * (v[q] + v[qb]);
    const CT fo = CT(0.5) * (v[q] - v[qb]);
    const CT A = le * (fe - feq_e);
    const CT B = lo * (fo - feq_o);
    CT fq = (v[q] + A) + B;
    CT fqb = (v[qb] + A) - B;
    if (forced) {
        // Luo term split into even / odd parts, weighted (1 + lambda/2)
        const CT cf = cdot<q>(fb0, fb1, fb2);
        const CT Fe = w * ((-ufb * CT(3.0)) + (cu * cf) * CT(9.0));
        const CT Fo = w * (cf * CT(3.0));
        fq = (fq + ae * Fe) + ao * Fo;
        fqb = (fqb + ae * Fe) - ao * Fo;
    }
    v[q] = fq;
    v[qb] = fqb;
}

template <typename ST, int FMODE>
__global__ void __launch_bounds__(512) k_stream_collide(SweepArgs a) {
    using T = Storage<ST>;
    using CT = typename T::CT;
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const size_t Ns = a.g.Ns;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    const ST *__restrict__ src = static_cast<const ST *>(a.src);
    ST *__restrict__ dst = static_cast<ST *>(a.dst);

    bool act = x < nx;
    const size_t c = (size_t)(act ? x : 0) + (size_t)nx * ((size_t)y + (size_t)ny * (size_t)z);
    const uint8_t fl = act ? a.flag[c] : kWall;
    act = act && !(fl & (kWall | kObst));

    uint32_t pp = kNone;
    double acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = 0.0;

    if (act) {
        const uint32_t mask = (fl & kNear) ? a.nearmask[c] : 0u;
        CT v[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) v[q] = T::load(src + (size_t)q * Ns + c);

        CT fb0 = CT(0), fb1 = CT(0), fb2 = CT(0);
        if constexpr (FMODE == kForceDense) {
            const CT *F = static_cast<const CT *>(a.force);
            fb0 = F[c];
            fb1 = F[Ns + c];
            fb2 = F[2 * Ns + c];
        } else if constexpr (FMODE == kForceCharge) {
            const CT re = static_cast<const CT *>(a.force)[c];
            fb0 = re * (CT)a.E[0];
            fb1 = re * (CT)a.E[1];
            fb2 = re * (CT)a.E[2];
        }

        // moments (Eq. MacroscopVel), in q order
        CT rho = CT(0), jx = CT(0), jy = CT(0), jz = CT(0);
#pragma unroll
        for (int q = 0; q < Q; ++q) rho += v[q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (kCx[q] > 0) jx += v[q];
            if (kCx[q] < 0) jx -= v[q];
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (kCy[q] > 0) jy += v[q];
            if (kCy[q] < 0) jy -= v[q];
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (kCz[q] > 0) jz += v[q];
            if (kCz[q] < 0) jz -= v[q];
        }
        // Eq. modified_velocity: u = (sum c f + f_b / 2) / rho0
        const bool forced = FMODE != kForceNone;
        const CT ux = forced ? jx + CT(0.5) * fb0 : jx;
        const CT uy = forced ? jy + CT(0.5) * fb1 : jy;
        const CT uz = forced ? jz + CT(0.5) * fb2 : jz;
        const CT uu = (ux * ux + uy * uy) + uz * uz;
        const CT ufb = forced ? (ux * fb0 + uy * fb1) + uz * fb2 : CT(0);
        const CT le = (CT)a.le, lo = (CT)a.lo, ae = (CT)a.ae, ao = (CT)a.ao;

        // rest population
        {
            const CT w0 = (CT)wq(0);
            const CT feq_e = w0 * (rho - uu * CT(1.5));
            CT f0 = v[0] + le * (v[0] - feq_e);
            if (forced) f0 = f0 + ae * (w0 * (-ufb * CT(3.0)));
            v[0] = f0;
        }
        collide_pair<1>(v, rho, ux, uy, uz, uu, ufb, fb0, fb1, fb2, le, lo, ae, ao, forced);
        collide_pair<3>(v, rho, ux, uy, uz, uu, ufb, fb0, fb1, fb2, le, lo, ae, ao, forced);
        collide_pair<5>(v, rho, ux, uy, uz, uu, ufb, fb0, fb1, fb2, le, lo, ae, ao, forced);
        collide_pair<7>(v, rho, ux, uy, uz, uu, ufb, fb0, fb1, fb2, le, lo, ae, ao, forced);
        collide_pair<9>(v, rho, ux, uy, uz, uu, ufb, fb0, fb1, fb2, le, lo, ae, ao, forced);
        collide_pair<11>(v, rho, ux, uy, uz, uu, ufb, fb0, fb1, fb2, le, lo, ae, ao, forced);
        collide_pair<13>(v, rho, ux, uy, uz, uu, ufb, fb0, fb1, fb2, le, lo, ae, ao, forced);
        collide_pair<15>(v, rho, ux, uy, uz, uu, ufb, fb0, fb1, fb2, le, lo, ae, ao, forced);
        collide_pair<17>(v, rho, ux, uy, uz, uu, ufb, fb0, fb1, fb2, le, lo, ae, ao, forced);

        // push-stream (Eq. LBMstreamStep) with periodic wrap
        const int xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
        const int ys[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
        const int zs[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
        size_t rows[3][3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                rows[j][k] = (size_t)nx * ((size_t)ys[j] + (size_t)ny * (size_t)zs[k]);
        T::store(dst + c, v[0]);
        push<1>(dst, Ns, rows, xs, v[1], mask);
        push<2>(dst, Ns, rows, xs, v[2], mask);
        push<3>(dst, Ns, rows, xs, v[3], mask);
        push<4>(dst, Ns, rows, xs, v[4], mask);
        push<5>(dst, Ns, rows, xs, v[5], mask);
        push<6>(dst, Ns, rows, xs, v[6], mask);
        push<7>(dst, Ns, rows, xs, v[7], mask);
        push<8>(dst, Ns, rows, xs, v[8], mask);
        push<9>(dst, Ns, rows, xs, v[9], mask);
        push<10>(dst, Ns, rows, xs, v[10], mask);
        push<11>(dst, Ns, rows, xs, v[11], mask);
        push<12>(dst, Ns, rows, xs, v[12], mask);
        push<13>(dst, Ns, rows, xs, v[13], mask);
        push<14>(dst, Ns, rows, xs, v[14], mask);
        push<15>(dst, Ns, rows, xs, v[15], mask);
        push<16>(dst, Ns, rows, xs, v[16], mask);
        push<17>(dst, Ns, rows, xs, v[17], mask);
        push<18>(dst, Ns, rows, xs, v[18], mask);

        if (mask) {
            maybe_bounce<1>(a, dst, c, x, y, z, v[1], mask, pp, acc);
            maybe_bounce<2>(a, dst, c, x, y, z, v[2], mask, pp, acc);
            maybe_bounce<3>(a, dst, c, x, y, z, v[3], mask, pp, acc);
            maybe_bounce<4>(a, dst, c, x, y, z, v[4], mask, pp, acc);
            maybe_bounce<5>(a, dst, c, x, y, z, v[5], mask, pp, acc);
            maybe_bounce<6>(a, dst, c, x, y, z, v[6], mask, pp, acc);
            maybe_bounce<7>(a, dst, c, x, y, z, v[7], mask, pp, acc);
            maybe_bounce<8>(a, dst, c, x, y, z, v[8], mask, pp, acc);
            maybe_bounce<9>(a, dst, c, x, y, z, v[9], mask, pp, acc);
            maybe_bounce<10>(a, dst, c, x, y, z, v[10], mask, pp, acc);
            maybe_bounce<11>(a, dst, c, x, y, z, v[11], mask, pp, acc);
            maybe_bounce<12>(a, dst, c, x, y, z, v[12], mask, pp, acc);
            maybe_bounce<13>(a, dst, c, x, y, z, v[13], mask, pp, acc);
            maybe_bounce<14>(a, dst, c, x, y, z, v[14], mask, pp, acc);
            maybe_bounce<15>(a, dst, c, x, y, z, v[15], mask, pp, acc);
            maybe_bounce<16>(a, dst, c, x, y, z, v[16], mask, pp, acc);
            maybe_bounce<17>(a, dst, c, x, y, z, v[17], mask, pp, acc);
            maybe_bounce<18>(a, dst, c, x, y, z, v[18], mask, pp, acc);
        }
    }

    // per-particle sums across the wavefront: one FP64 atomic per particle,
    // component and wavefront (every lane of the wave takes part)
    if (a.FM) {
        unsigned long long pend = __ballot(pp != kNone);
        while (pend) {
            const int leader = __ffsll((unsigned long long)pend) - 1;
            const uint32_t lp = (uint32_t)__shfl((int)pp, leader);
            const bool mine = pp == lp;
            double t[kAcc];
#pragma unroll
            for (int k = 0; k < kAcc; ++k) t[k] = mine ? acc[k] : 0.0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
                for (int k = 0; k < kAcc; ++k) t[k] += __shfl_xor(t[k], off);
            }
            if ((int)__lane_id() == leader) flush_particle(a.FM, lp, t);
            if (mine) pp = kNone;
            pend = __ballot(pp != kNone);
        }
    }
}

template <typename ST>
hipError_t launch_typed(int force_mode, const SweepArgs &a, int block_x, hipStream_t s) {
    const dim3 block(block_x, 1, 1);
    const dim3 grid((a.g.nx + block_x - 1) / block_x, a.g.ny, a.g.nz);
    switch (force_mode) {
    case kForceNone:
        hipLaunchKernelGGL((k_stream_collide<ST, kForceNone>), grid, block, 0, s, a);
        break;
    case kForceDense:
        hipLaunchKernelGGL((k_stream_collide<ST, kForceDense>), grid, block, 0, s, a);
        break;
    default:
        hipLaunchKernelGGL((k_stream_collide<ST, kForceCharge>), grid, block, 0, s, a);
        break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stream_collide(int precision, int force_mode, const SweepArgs &a, int block_x,
                                 hipStream_t s) {
    if (precision == LBMEP_FP64) return launch_typed<double>(force_mode, a, block_x, s);
    if (precision == LBMEP_FP32DEV) return launch_typed<float>(force_mode, a, block_x, s);
    return launch_typed<__half>(force_mode, a, block_x, s);
}

}  // namespace lbmep
