// sweep_impl.h -- fused gather-stream + collide sweep of the D3Q19 TRT lattice
// Boltzmann method with a body force and moving-obstacle bounce-back
// (arXiv:1708.08741, Sec. 3.1 Eq. LBMcollideStep / Eq. LBMstreamStep with
// Eq. LBE_forcetermLuo and Eq. modified_velocity; Sec. 3.2 Eq. LBMMovWall and
// Eq. LBMhydrodynForce).
//
// Pull scheme with post-collision storage.  The grid holds f*, the
// post-collision populations (with the forcing term) of the previous time
// level.  One thread per cell; a workgroup covers a segment of an x-row and
// consecutive segments are dealt onto one XCD.  A thread gathers f*_q from
// x - e_q (reads shifted by at most one element along x; this completes the
// stream of Eq. LBMstreamStep), refills the cell if it has just been
// uncovered, collides, and writes its 19 new values aligned to its own cell.
// Bounce-back needs no look-up at gather time: after the sweep, the kernel
// of near_impl.h writes the bounced value of every blocked link into a slot
// of the solid neighbour that the fluid cell gathers from at the next step.
// Only the edge of a non-periodic axis is resolved at gather time, from the
// cell coordinates.
//
// The template is instantiated in two translation units, k_stream_f64.hip
// (FP64) and k_stream_lp.hip (FP32 / FP16 deviation storage), both compiled
// without floating-point contraction: the FP64 sweep evaluates exactly the
// operation sequence of a plain CPU implementation; the FP32-compute sweep
// (FP32 and FP16 storage) uses the rearranged collision of collide_f32 with
// explicit FMAs; either way every sweep mode rounds identically.
// Byte offsets are 32-bit (global loads/stores with a scalar base) whenever a
// population array is smaller than 4 GiB.
#pragma once
#include "potential_impl.h"

namespace lbmep {
namespace sweep {

template <typename ST>
struct Storage;

// FP64: absolute populations
template <>
struct Storage<double> {
    using CT = double;
    static __device__ __forceinline__ double load(const double *p) { return *p; }
    static __device__ __forceinline__ void store(double *p, double v) { *p = v; }
    // streaming forms (non-temporal hint: each value is read or written once)
    static __device__ __forceinline__ double load_nt(const double *p) {
        return __builtin_nontemporal_load(p);
    }
    static __device__ __forceinline__ void store_nt(double *p, double v) {
        __builtin_nontemporal_store(v, p);
    }
    // deviation f - w_q of a computed population q, in FP64
    static __device__ __forceinline__ double devval(double v, int q) { return v - wq(q); }
    // f^eq(rho0 = 1, u) of population q (Eq. fequ_Incompr_SRT) as stored
    static __device__ __forceinline__ double feq(int q, double d) { return wq(q) * (1.0 + 1.0 * d); }
    // the sweep's compute units are the stored values themselves
    static __device__ __forceinline__ double lc(const double *p) { return load(p); }
    static __device__ __forceinline__ double lc_nt(const double *p) { return load_nt(p); }
    static __device__ __forceinline__ void sc(double *p, double v) { store(p, v); }
    static __device__ __forceinline__ void sc_nt(double *p, double v) { store_nt(p, v); }
    static __device__ __forceinline__ double feq_c(int q, double d) { return feq(q, d); }
};

// FP32: deviations f - w_q
template <>
struct Storage<float> {
    using CT = float;
    static __device__ __forceinline__ float load(const float *p) { return *p; }
    static __device__ __forceinline__ void store(float *p, float v) { *p = v; }
    static __device__ __forceinline__ float load_nt(const float *p) {
        return __builtin_nontemporal_load(p);
    }
    static __device__ __forceinline__ void store_nt(float *p, float v) {
        __builtin_nontemporal_store(v, p);
    }
    static __device__ __forceinline__ double devval(float v, int q) { return (double)v; }
    static __device__ __forceinline__ float feq(int q, double d) { return (float)(wq(q) * d); }
    // compute units: the deviations themselves
    static __device__ __forceinline__ float lc(const float *p) { return load(p); }
    static __device__ __forceinline__ float lc_nt(const float *p) { return load_nt(p); }
    static __device__ __forceinline__ void sc(float *p, float v) { store(p, v); }
    static __device__ __forceinline__ void sc_nt(float *p, float v) { store_nt(p, v); }
    static __device__ __forceinline__ float feq_c(int q, double d) { return feq(q, d); }
};

// FP16: deviations scaled by 2^22
template <>
struct Storage<__half> {
    using CT = float;
    static __device__ __forceinline__ float load(const __half *p) {
        return __half2float(*p) * kHalfInvScale;
    }
    static __device__ __forceinline__ void store(__half *p, float v) {
        *p = __float2half_rn(v * kHalfScale);
    }
    static __device__ __forceinline__ float load_nt(const __half *p) {
        const unsigned short b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p));
        return __half2float(__ushort_as_half(b)) * kHalfInvScale;
    }
    static __device__ __forceinline__ void store_nt(__half *p, float v) {
        __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v * kHalfScale)),
                                    reinterpret_cast<unsigned short *>(p));
    }
    static __device__ __forceinline__ double devval(float v, int q) { return (double)v; }
    // rounded to the storage format, as a stored and re-loaded value would be
    static __device__ __forceinline__ float feq(int q, double d) {
        return __half2float(__float2half_rn((float)(wq(q) * d) * kHalfScale)) * kHalfInvScale;
    }
    // compute units: deviations times 2^22, the stored half values widened
    // (loads and stores convert only; the power-of-two scale is exact)
    static __device__ __forceinline__ float lc(const __half *p) { return __half2float(*p); }
    static __device__ __forceinline__ float lc_nt(const __half *p) {
        const unsigned short b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p));
        return __half2float(__ushort_as_half(b));
    }
    static __device__ __forceinline__ void sc(__half *p, float v) { *p = __float2half_rn(v); }
    static __device__ __forceinline__ void sc_nt(__half *p, float v) {
        __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(v)),
                                    reinterpret_cast<unsigned short *>(p));
    }
    static __device__ __forceinline__ float feq_c(int q, double d) {
        return __half2float(__float2half_rn((float)(wq(q) * d) * kHalfScale));
    }
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

// address of element `off` (bytes) of the array starting at the uniform
// `base`; with OFF = uint32_t this becomes a global access with a scalar base
// register and a 32-bit vector offset
template <typename ST, typename OFF>
__device__ __forceinline__ ST *at(void *base, OFF off) {
    return reinterpret_cast<ST *>(static_cast<char *>(base) + off);
}
template <typename ST, typename OFF>
__device__ __forceinline__ const ST *at(const void *base, OFF off) {
    return reinterpret_cast<const ST *>(static_cast<const char *>(base) + off);
}

// sweep modes
enum { kPull = 0,     // gather f* of the previous level, refill, collide
       kLocal = 1,    // collide the post-stream state held in the grid
       kReadout = 2,  // gather and refill only: write the post-stream state
       kPullNT = 3,   // as kPull, loads and stores with streaming hints
       kPullNTS = 4   // as kPull, stores with streaming hints
};

// load / store of one stored population in compute units, with the
// streaming hint in kPullNT
template <int MODE, typename ST>
__device__ __forceinline__ typename Storage<ST>::CT pop_load(const ST *p) {
    if constexpr (MODE == kPullNT)
        return Storage<ST>::lc_nt(p);
    else
        return Storage<ST>::lc(p);
}
template <int MODE, typename ST>
__device__ __forceinline__ void pop_store(ST *p, typename Storage<ST>::CT v) {
    if constexpr (MODE == kPullNT || MODE == kPullNTS)
        Storage<ST>::sc_nt(p, v);
    else
        Storage<ST>::sc(p, v);
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

// FP32 compute (FP32 and FP16 storage): the TRT collision with the Luo
// forcing term (Eq. LBMcollideStep with Eq. EqPDF_TRT, Eq. LBE_forcetermLuo
// and Eq. modified_velocity) rearranged to fewer operations.  With the pair
// sum s = f_q + f_qbar and difference d = f_q - f_qbar, the update of an
// opposite pair is f_q <- f_q + (E + O), f_qbar <- f_qbar + (E - O) with
//   E = le/2 s - G_k - (c.u)(9/2 le w (c.u) - 9 ae w (c.F))
//   O = le/2 d - 3 lo w (c.u) + 3 ao w (c.F)
//     = lo/6 (3 d - c.u) + ao/6 (c.F)      (axis, w = 1/18)
//     = lo/12 (6 d - c.u) + ao/12 (c.F)    (diagonal, w = 1/36)
// and G_k = le w (rho - 3/2 u.u) + 3 ae w u.F per weight class; the rest
// population becomes f_0 + (le f_0 - G_0).  The increments are added to the
// loaded values (the unit part of the update stays exact), and in the odd
// part d and c.u enter with exact integer weights, so the momentum the
// collision changes, lo (j - u) + ao F, has no bias from the rounding of the
// rates.  Algebraically the textbook form; the rounding differs (FMA,
// regrouped sums).  rho and j = sum c f come from the same pair sums and
// differences.  Values are in compute units (see TrtF32).
template <int q, bool FORCED>
__device__ __forceinline__ void trt_pair_f32(float (&v)[Q], const TrtF32 &t, float s, float d,
                                             float ux, float uy, float uz, float fx, float fy,
                                             float fz, float G) {
    constexpr int qb = q + 1;
    constexpr int k = q <= 6 ? 0 : 1;  // weight class: axis / diagonal
    const float cu = cdot<q>(ux, uy, uz);
    const float D = __builtin_fmaf(k == 0 ? 3.0f : 6.0f, d, -cu);
    float E, O;
    if constexpr (FORCED) {
        const float cf = cdot<q>(fx, fy, fz);
        const float h = __builtin_fmaf(t.k1[k], cu, -(t.k3[k] * cf));
        E = __builtin_fmaf(t.hle, s, -__builtin_fmaf(cu, h, G));
        O = __builtin_fmaf(t.hlo[k], D, t.k4[k] * cf);
    } else {
        E = __builtin_fmaf(t.hle, s, -__builtin_fmaf(cu, t.k1[k] * cu, G));
        O = t.hlo[k] * D;
    }
    v[q] = v[q] + (E + O);
    v[qb] = v[qb] + (E - O);
}

template <bool FORCED>
__device__ __forceinline__ void collide_f32(float (&v)[Q], const TrtF32 &t, float fx, float fy,
                                            float fz) {
    // directions 2p+1, 2p+2 are opposite; the first of each pair points
    // along +x for p = 0, 3, 4, 5, 6, along +y for p = 1, 3, 7, 8 and -y for
    // p = 4, along +z for p = 2, 5, 7 and -z for p = 6, 8
    static_assert(kCx[1] == 1 && kCx[7] == 1 && kCx[9] == 1 && kCx[11] == 1 && kCx[13] == 1 &&
                  kCx[3] == 0 && kCx[5] == 0 && kCx[15] == 0 && kCx[17] == 0, "x layout");
    static_assert(kCy[3] == 1 && kCy[7] == 1 && kCy[9] == -1 && kCy[15] == 1 && kCy[17] == 1 &&
                  kCy[1] == 0 && kCy[5] == 0 && kCy[11] == 0 && kCy[13] == 0, "y layout");
    static_assert(kCz[5] == 1 && kCz[11] == 1 && kCz[13] == -1 && kCz[15] == 1 && kCz[17] == -1 &&
                  kCz[1] == 0 && kCz[3] == 0 && kCz[7] == 0 && kCz[9] == 0, "z layout");
    static_assert(opp(1) == 2 && opp(7) == 8 && opp(17) == 18, "pairs");
    float s[9], d[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        s[p] = v[2 * p + 1] + v[2 * p + 2];
        d[p] = v[2 * p + 1] - v[2 * p + 2];
    }
    float rho = v[0];
#pragma unroll
    for (int p = 0; p < 9; ++p) rho += s[p];
    const float jx = (((d[0] + d[3]) + d[4]) + d[5]) + d[6];
    const float jy = (((d[1] + d[3]) - d[4]) + d[7]) + d[8];
    const float jz = (((d[2] + d[5]) - d[6]) + d[7]) - d[8];
    // Eq. modified_velocity: u = j + F/2 (rho0 = 1)
    const float ux = FORCED ? __builtin_fmaf(0.5f, fx, jx) : jx;
    const float uy = FORCED ? __builtin_fmaf(0.5f, fy, jy) : jy;
    const float uz = FORCED ? __builtin_fmaf(0.5f, fz, jz) : jz;
    const float uu = __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
    const float base = __builtin_fmaf(-t.b15, uu, rho);
    float G0, G1, G2;
    if constexpr (FORCED) {
        const float ufb = __builtin_fmaf(ux, fx, __builtin_fmaf(uy, fy, uz * fz));
        G0 = __builtin_fmaf(t.m0, ufb, t.lw0 * base);
        G1 = __builtin_fmaf(t.m[0], ufb, t.lw[0] * base);
        G2 = __builtin_fmaf(t.m[1], ufb, t.lw[1] * base);
    } else {
        G0 = t.lw0 * base;
        G1 = t.lw[0] * base;
        G2 = t.lw[1] * base;
    }
    v[0] = v[0] + __builtin_fmaf(t.le, v[0], -G0);
    trt_pair_f32<1, FORCED>(v, t, s[0], d[0], ux, uy, uz, fx, fy, fz, G1);
    trt_pair_f32<3, FORCED>(v, t, s[1], d[1], ux, uy, uz, fx, fy, fz, G1);
    trt_pair_f32<5, FORCED>(v, t, s[2], d[2], ux, uy, uz, fx, fy, fz, G1);
    trt_pair_f32<7, FORCED>(v, t, s[3], d[3], ux, uy, uz, fx, fy, fz, G2);
    trt_pair_f32<9, FORCED>(v, t, s[4], d[4], ux, uy, uz, fx, fy, fz, G2);
    trt_pair_f32<11, FORCED>(v, t, s[5], d[5], ux, uy, uz, fx, fy, fz, G2);
    trt_pair_f32<13, FORCED>(v, t, s[6], d[6], ux, uy, uz, fx, fy, fz, G2);
    trt_pair_f32<15, FORCED>(v, t, s[7], d[7], ux, uy, uz, fx, fy, fz, G2);
    trt_pair_f32<17, FORCED>(v, t, s[8], d[8], ux, uy, uz, fx, fy, fz, G2);
}

#define LBMEP_FOR_Q18(M) \
    M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16) M(17) M(18)

// gather population q of the cell from x - e_q; beyond the edge of a
// non-periodic axis the population bounces at the (resting) edge: it is the
// cell's own opposite population
template <int q, typename ST, typename OFF, int MODE>
__device__ __forceinline__ typename Storage<ST>::CT gather(const void *src, OFF pst, OFF es,
                                                           OFF cb, const OFF rows[3][3],
                                                           const bool rok[3][3], const OFF xs[3],
                                                           const bool xok[3]) {
    constexpr int qb = opp(q);
    constexpr int lo = q < qb ? q : qb;
    const void *base = static_cast<const char *>(src) + (size_t)lo * pst;
    const bool ok = rok[kCy[q] + 1][kCz[q] + 1] && xok[kCx[q] + 1];
    const OFF nb = (OFF)(q - lo) * pst + xs[kCx[q] + 1] + rows[kCy[q] + 1][kCz[q] + 1];
    const OFF own = (OFF)(qb - lo) * pst + cb;
    return pop_load<MODE, ST>(at<ST>(base, ok ? nb : own));
}

// Free-slip faces: a population that a face cell x gathers from beyond a
// free-slip face (direction q, source x - c_q outside along the axes of
// mask) comes from the tangential neighbour s' (x - c_q with those
// components set back to x's) in the direction p = q mirrored across the
// crossed axes, unless s' is a wall or obstacle cell or a crossed face is
// no-slip (then the half-way bounce-back stands).  Beyond a non-periodic
// edge the gather reads slot q-bar of x itself, which no other gather reads;
// slot p of s' is likewise read only through the reflection of (s', q2),
// q2 = q-bar mirrored across the same axes, whose partner is (x, q).  So the
// reflection is a swap of the two slots, made once per pair before a gather
// of the state by a pass over the face cells; the gather itself keeps no
// branch for it.
template <int q, typename ST>
__device__ __forceinline__ void slip_pair(const SweepArgs &a, const int (&o)[3], size_t c,
                                          int ax, int side) {
    constexpr int cq[3] = {kCx[q], kCy[q], kCz[q]};
    // the pass of face (ax, side) takes the directions that cross it
    if (cq[ax] == 0 || (side == 0) != (cq[ax] > 0)) return;
    const int len[3] = {a.g.nx, a.g.ny, a.g.nz};
    int s[3] = {o[0] - cq[0], o[1] - cq[1], o[2] - cq[2]};
    int mask = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (s[k] >= 0 && s[k] < len[k]) continue;
        if (a.g.per[k]) {
            s[k] = s[k] < 0 ? s[k] + len[k] : s[k] - len[k];
            continue;
        }
        if (!(a.slip & (1 << (2 * k + (s[k] < 0 ? 0 : 1))))) return;  // no-slip face
        mask |= 1 << k;
        s[k] = o[k];
    }
    // a pair that crosses an edge or corner is taken by its lowest axis
    if (mask & ((1 << ax) - 1)) return;
    int p = q, q2 = q;
    switch (mask) {
        case 1: p = mirror_dir(q, 1); q2 = mirror_dir(opp(q), 1); break;
        case 2: p = mirror_dir(q, 2); q2 = mirror_dir(opp(q), 2); break;
        case 3: p = mirror_dir(q, 3); q2 = mirror_dir(opp(q), 3); break;
        case 4: p = mirror_dir(q, 4); q2 = mirror_dir(opp(q), 4); break;
        case 5: p = mirror_dir(q, 5); q2 = mirror_dir(opp(q), 5); break;
        case 6: p = mirror_dir(q, 6); q2 = mirror_dir(opp(q), 6); break;
        default: p = mirror_dir(q, 7); q2 = mirror_dir(opp(q), 7); break;
    }
    const size_t sc = (size_t)s[0] + (size_t)a.g.nx * ((size_t)s[1] + (size_t)a.g.ny * (size_t)s[2]);
    // normal incidence (s' = x, p = q-bar): the bounce-back is the reflection;
    // otherwise the pair is swapped by its smaller (cell, direction)
    if (sc * Q + (size_t)q2 <= c * Q + (size_t)q) return;
    if ((a.flag[c] | a.flag[sc]) & (kWall | kObst)) return;
    ST *f = static_cast<ST *>(const_cast<void *>(a.src));
    ST *u = f + (size_t)opp(q) * a.g.Ns + c;
    ST *v = f + (size_t)p * a.g.Ns + sc;
    const ST t = *u;
    *u = *v;
    *v = t;
}

// one thread per cell of free-slip face (ax, side)
template <typename ST>
__global__ void __launch_bounds__(256) k_slip_swap(SweepArgs a, int ax, int side) {
    const int len[3] = {a.g.nx, a.g.ny, a.g.nz};
    const int a1 = ax == 0 ? 1 : 0, a2 = ax == 2 ? 1 : 2;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)len[a1] * (size_t)len[a2]) return;
    int o[3];
    o[ax] = side ? len[ax] - 1 : 0;
    o[a1] = (int)(i % (size_t)len[a1]);
    o[a2] = (int)(i / (size_t)len[a1]);
    const size_t c = (size_t)o[0] + (size_t)a.g.nx * ((size_t)o[1] + (size_t)a.g.ny * (size_t)o[2]);
#define LBMEP_SLIP(q) slip_pair<q, ST>(a, o, c, ax, side);
    LBMEP_FOR_Q18(LBMEP_SLIP)
#undef LBMEP_SLIP
}

// store population q of a cell at byte offset cb; addressed from the base of
// its opposite pair like the gather (a uniform base plus a 32-bit offset)
template <int q, int MODE, typename ST, typename OFF>
__device__ __forceinline__ void store_pop(void *dst, OFF pst, OFF cb, typename Storage<ST>::CT v) {
    constexpr int lo = q == 0 ? 0 : (q < opp(q) ? q : opp(q));
    char *base = static_cast<char *>(dst) + (size_t)lo * pst;
    pop_store<MODE, ST>(at<ST>(base, (OFF)(q - lo) * pst + cb), v);
}

// loaded inputs of one cell
template <typename CT>
struct CellIn {
    CT v[Q];
    CT fb0, fb1, fb2;
    uint8_t fl;
};

// issue every load of cell (x, y, z) (solid cells and cells beyond the grid
// load in-range values and drop them), so that the flag and the populations
// share one memory latency
template <typename ST, int FMODE, typename OFF, int MODE>
__device__ __forceinline__ void load_cell(const SweepArgs &a, int x, int y, int z, bool valid,
                                          CellIn<typename Storage<ST>::CT> &c) {
    using T = Storage<ST>;
    using CT = typename T::CT;
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const OFF es = (OFF)sizeof(ST);
    const OFF pst = (OFF)a.g.Ns * es;
    const int xc = valid ? x : 0, yc = valid ? y : 0;
    const OFF ci = (OFF)xc + (OFF)nx * ((OFF)yc + (OFF)ny * (OFF)z);
    const OFF cb = ci * es;
    const uint8_t *flp = at<uint8_t>((const void *)a.flag, ci);
    uint8_t fl;
    if constexpr (MODE == kPullNT)
        fl = __builtin_nontemporal_load(flp);
    else
        fl = *flp;
    c.fl = valid ? fl : kWall;
    // source rows (y - c_y, z - c_z) and columns x - c_x, wrapped on
    // periodic axes; beyond a non-periodic edge: not ok (pull modes)
    OFF rows[3][3];
    bool rok[3][3];
    OFF xs[3];
    bool xok[3];
    if constexpr (MODE == kLocal) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            c.v[q] = T::lc(at<ST>(static_cast<const char *>(a.src) + (size_t)q * pst, cb));
    } else {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                int ys = yc - (j - 1), zs = z - (k - 1);
                bool ok = true;
                if (ys < 0 || ys >= ny) {
                    if (a.g.per[1]) ys = ys < 0 ? ys + ny : ys - ny; else { ok = false; ys = yc; }
                }
                if (zs < 0 || zs >= nz) {
                    if (a.g.per[2]) zs = zs < 0 ? zs + nz : zs - nz; else { ok = false; zs = z; }
                }
                rows[j][k] = (OFF)nx * ((OFF)ys + (OFF)ny * (OFF)zs) * es;
                rok[j][k] = ok;
            }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            int xq = xc - (i - 1);
            bool ok = true;
            if (xq < 0 || xq >= nx) {
                if (a.g.per[0]) xq = xq < 0 ? xq + nx : xq - nx; else { ok = false; xq = xc; }
            }
            xs[i] = (OFF)xq * es;
            xok[i] = ok;
        }
        c.v[0] = pop_load<MODE, ST>(at<ST>(a.src, cb));
#define LBMEP_GATHER(q) c.v[q] = gather<q, ST, OFF, MODE>(a.src, pst, es, cb, rows, rok, xs, xok);
        LBMEP_FOR_Q18(LBMEP_GATHER)
#undef LBMEP_GATHER
    }
    c.fb0 = c.fb1 = c.fb2 = CT(0);
    if constexpr (MODE != kReadout) {
        if constexpr (FMODE == kForceDense) {
            const OFF fo = ci * (OFF)sizeof(CT), fs = (OFF)a.g.Ns * (OFF)sizeof(CT);
            c.fb0 = *at<CT>(a.force, fo);
            c.fb1 = *at<CT>(a.force, fo + fs);
            c.fb2 = *at<CT>(a.force, fo + 2 * fs);
        } else if constexpr (FMODE == kForcePotential) {
            // colour-split psi (even nx) with even extents along the
            // periodic y and z axes, so a neighbour across a wrap keeps the
            // colour parity of its unwrapped place
            const bool split_even = psi_split(a.g) && (!a.g.per[1] || a.g.ny % 2 == 0) &&
                                    (!a.g.per[2] || a.g.nz % 2 == 0);
            if (MODE != kLocal && split_even && valid && !(fl & (kWall | kObst | kNear))) {
                // every neighbour a fluid cell inside the grid: the
                // stencil's slots from the gather's wrapped rows and columns
                // (row (y', z') starts at entry nx / 2 (y' + ny z'), column
                // x' is entry x' / 2, the colour-1 half at Ns / 2); the
                // colour of the neighbour (x, y, z) + (dx, dy, dz) is the
                // cell's own xor the parity of dx + dy + dz
                const OFF half = (OFF)(a.g.Ns >> 1) * (OFF)sizeof(CT);
                const OFF cs = (OFF)(((xc + yc + z) & 1) ? half : 0), co = half - cs;
                auto val = [&](int dx, int dy, int dz) -> CT {
                    const OFF ob = rows[1 - dy][1 - dz] / (2 * es) * (OFF)sizeof(CT) +
                                   xs[1 - dx] / (2 * es) * (OFF)sizeof(CT) +
                                   (((dx + dy + dz) & 1) ? co : cs);
                    return *at<CT>(a.force, ob);
                };
                CT pc, g0, g1, g2;
                psi_grad_inner<CT>(val, pc, g0, g1, g2);
                edl_force<CT>(pc, g0, g1, g2, (CT)a.keps, (CT)a.E[0], (CT)a.E[1], (CT)a.E[2],
                              c.fb0, c.fb1, c.fb2);
            } else if (valid && !(fl & (kWall | kObst))) {
                potential_force<CT>(a.g, x, y, z, fl, static_cast<const CT *>(a.force), a.flag,
                                    a.owner, a.zeta, (CT)a.keps, (CT)a.E[0], (CT)a.E[1],
                                    (CT)a.E[2], c.fb0, c.fb1, c.fb2);
            }
        } else if constexpr (FMODE == kForceCharge) {
            const CT *rp = at<CT>(a.force, ci * (OFF)sizeof(CT));
            CT re;
            if constexpr (MODE == kPullNT)
                re = __builtin_nontemporal_load(rp);
            else
                re = *rp;
            if constexpr (sizeof(CT) == 4) {
                // the field in compute units (exact power-of-two scale)
                c.fb0 = re * a.tf.Ec[0];
                c.fb1 = re * a.tf.Ec[1];
                c.fb2 = re * a.tf.Ec[2];
            } else {
                c.fb0 = re * (CT)a.E[0];
                c.fb1 = re * (CT)a.E[1];
                c.fb2 = re * (CT)a.E[2];
            }
        }
        if constexpr (sizeof(ST) == 2 && (FMODE == kForceDense || FMODE == kForcePotential)) {
            c.fb0 *= a.tf.fscale;
            c.fb1 *= a.tf.fscale;
            c.fb2 *= a.tf.fscale;
        }
    }
}

// refill (if uncovered), collide and store one loaded cell
template <typename ST, int FMODE, typename OFF, int MODE>
__device__ __forceinline__ void finish_cell(const SweepArgs &a, int x, int y, int z,
                                            CellIn<typename Storage<ST>::CT> &c) {
    using T = Storage<ST>;
    using CT = typename T::CT;
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const OFF es = (OFF)sizeof(ST);
    const OFF pst = (OFF)a.g.Ns * es;
    const bool act = !(c.fl & (kWall | kObst));
    const OFF ci = act ? (OFF)x + (OFF)nx * ((OFF)y + (OFF)ny * (OFF)z) : (OFF)0;
    const OFF cb = ci * es;
    CT(&v)[Q] = c.v;

    // refill of a cell uncovered at this level: f^eq(rho0, u_s) with the
    // surface velocity of its previous owner at its previous place (Sec. 3.2)
    if constexpr (MODE != kLocal) {
        if (act && (c.fl & kUncov)) {
            const uint32_t po = a.owner_old[ci];
            const double *Xp = a.Xold + 3 * (size_t)po;
            const double *U = a.U + 3 * (size_t)po;
            const double *W = a.W + 3 * (size_t)po;
            const double r0 = min_image(((double)x + 0.5) - Xp[0], nx, a.g.per[0]);
            const double r1 = min_image(((double)y + 0.5) - Xp[1], ny, a.g.per[1]);
            const double r2 = min_image(((double)z + 0.5) - Xp[2], nz, a.g.per[2]);
            const double u0 = U[0] + (W[1] * r2 - W[2] * r1);
            const double u1 = U[1] + (W[2] * r0 - W[0] * r2);
            const double u2 = U[2] + (W[0] * r1 - W[1] * r0);
            const double uu = (u0 * u0 + u1 * u1) + u2 * u2;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const double cu = ((double)kCx[q] * u0 + (double)kCy[q] * u1) + (double)kCz[q] * u2;
                v[q] = (CT)T::feq_c(q, (cu * 3.0 + (cu * cu) * 4.5) - uu * 1.5);
            }
        }
    }

    if constexpr (MODE == kReadout) {
        // solid cells get defined values: the rest state at walls and
        // f^eq(rho0, u_s) of the owning particle at obstacle cells
        if (!act && (c.fl & (kWall | kObst)) && x < nx && y < ny) {
            const OFF si = (OFF)x + (OFF)nx * ((OFF)y + (OFF)ny * (OFF)z);
            double u0 = 0.0, u1 = 0.0, u2 = 0.0;
            if (!(c.fl & kWall)) {
                const uint32_t po = a.owner[si];
                const double *Xp = a.Xc + 3 * (size_t)po;
                const double *U = a.U + 3 * (size_t)po;
                const double *W = a.W + 3 * (size_t)po;
                const double r0 = min_image(((double)x + 0.5) - Xp[0], nx, a.g.per[0]);
                const double r1 = min_image(((double)y + 0.5) - Xp[1], ny, a.g.per[1]);
                const double r2 = min_image(((double)z + 0.5) - Xp[2], nz, a.g.per[2]);
                u0 = U[0] + (W[1] * r2 - W[2] * r1);
                u1 = U[1] + (W[2] * r0 - W[0] * r2);
                u2 = U[2] + (W[0] * r1 - W[1] * r0);
            }
            const double uu = (u0 * u0 + u1 * u1) + u2 * u2;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const double cu = ((double)kCx[q] * u0 + (double)kCy[q] * u1) + (double)kCz[q] * u2;
                T::sc(at<ST>(static_cast<char *>(a.dst) + (size_t)q * pst, si * es),
                      (CT)T::feq_c(q, (cu * 3.0 + (cu * cu) * 4.5) - uu * 1.5));
            }
        }
        if (act) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                T::sc(at<ST>(static_cast<char *>(a.dst) + (size_t)q * pst, cb), v[q]);
        }
    } else {
        // the collision runs on every lane; only the stores are restricted
        // to fluid cells
        if constexpr (sizeof(CT) == 4) {
            collide_f32<FMODE != kForceNone>(v, a.tf, c.fb0, c.fb1, c.fb2);
        } else {
        const CT fb0 = c.fb0, fb1 = c.fb1, fb2 = c.fb2;

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
        }

        if (act) {
            // aligned store of the post-collision state
#define LBMEP_STORE(q) store_pop<q, MODE, ST, OFF>(a.dst, pst, cb, v[q]);
            LBMEP_STORE(0)
            LBMEP_FOR_Q18(LBMEP_STORE)
#undef LBMEP_STORE
        }
    }
}


// one workgroup's x-segment of a 1-D grid of segments: CPT cells per
// thread, on consecutive rows y (their loads are all issued before the first
// collision, for more memory-level parallelism per wave)
template <typename ST, int FMODE, typename OFF, int MODE, int CPT>
__device__ __forceinline__ void sweep_segment(const SweepArgs &a, uint32_t lb) {
    using T = Storage<ST>;
    using CT = typename T::CT;
    const int nx = a.g.nx, ny = a.g.ny;
    const uint32_t nyb = (uint32_t)((ny + CPT - 1) / CPT);
    const uint32_t xb = lb % (uint32_t)a.nxb, row = lb / (uint32_t)a.nxb;
    const int y0 = (int)(row % nyb) * CPT, z = (int)(row / nyb);
    const int x = (int)xb * blockDim.x + threadIdx.x;

    CellIn<CT> c[CPT];
#pragma unroll
    for (int r = 0; r < CPT; ++r)
        load_cell<ST, FMODE, OFF, MODE>(a, x, y0 + r, z, x < nx && y0 + r < ny, c[r]);
#pragma unroll
    for (int r = 0; r < CPT; ++r) finish_cell<ST, FMODE, OFF, MODE>(a, x, y0 + r, z, c[r]);
}

template <typename ST, int FMODE, typename OFF, int MODE, int CPT>
__global__ void __launch_bounds__(512) k_sweep(SweepArgs a) {
    const uint32_t lb = a.xcd_swizzle ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    sweep_segment<ST, FMODE, OFF, MODE, CPT>(a, lb);
}

// the gather sweep of several lattices in one dispatch
template <typename ST, int FMODE>
__global__ void __launch_bounds__(kPackBlockX) k_sweep_packed(PackTable t) {
    const uint32_t gb = t.xcd_swizzle ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const int e = pack_find(t, gb);
    const SweepArgs a = t.d[e]->sweep[t.state[e]];
    // streaming hints as in the single-lattice default: stores only
    constexpr int MODE = kPullNTS;
    sweep_segment<ST, FMODE, uint32_t, MODE, 1>(a, gb - t.start[e]);
}

template <typename ST>
hipError_t launch_sweep_packed_typed(int force_mode, const PackTable &t, hipStream_t s) {
    const uint32_t total = t.start[t.n];
    if (t.n == 0 || total == 0) return hipSuccess;
    if (force_mode == kForceNone)
        hipLaunchKernelGGL((k_sweep_packed<ST, kForceNone>), dim3(total), dim3(kPackBlockX), 0, s, t);
    else if (force_mode == kForceDense)
        hipLaunchKernelGGL((k_sweep_packed<ST, kForceDense>), dim3(total), dim3(kPackBlockX), 0, s, t);
    else if (force_mode == kForceCharge)
        hipLaunchKernelGGL((k_sweep_packed<ST, kForceCharge>), dim3(total), dim3(kPackBlockX), 0, s, t);
    else
        return hipErrorInvalidValue;  // served requests carry no potential force
    return hipGetLastError();
}

// host launcher for one storage type; cpt = cells per thread (1 or 2)
template <typename ST>
hipError_t launch_typed(int mode, int force_mode, SweepArgs a, int block_x, int cpt,
                        hipStream_t s) {
    // 32-bit byte offsets when two population arrays fit in 4 GiB (the
    // gather addresses an opposite pair from one base)
    const bool small = 2 * a.g.Ns * sizeof(ST) < (size_t(1) << 32) && 4 * a.g.Ns < (size_t(1) << 32);
    if (a.slip && mode != kLocal) {
        // free-slip faces: the reflected values into the slots the gather
        // reads beyond those faces
        const int len[3] = {a.g.nx, a.g.ny, a.g.nz};
        for (int f = 0; f < 6; ++f) {
            if (!(a.slip & (1 << f))) continue;
            const int ax = f / 2;
            const size_t cells = (size_t)len[ax == 0 ? 1 : 0] * (size_t)len[ax == 2 ? 1 : 2];
            hipLaunchKernelGGL((k_slip_swap<ST>), dim3((unsigned)((cells + 255) / 256)), dim3(256), 0,
                               s, a, ax, f & 1);
        }
    }
    if (!small || mode == kReadout) cpt = 1;
    // the workgroups-per-CU cap was measured on the 32-bit-offset kernel;
    // the 64-bit one runs faster without it (864 x 1248 x 864 FP32: 24.6
    // against 27.5 ms)
    if (!small) a.lds = 0;
    a.nxb = (a.g.nx + block_x - 1) / block_x;
    const size_t nblocks = (size_t)a.nxb * ((a.g.ny + cpt - 1) / cpt) * a.g.nz;
    const dim3 block(block_x, 1, 1);
    const dim3 grid((unsigned)nblocks, 1, 1);
#define LBMEP_LAUNCH(MD, FM, OFF, C) \
    hipLaunchKernelGGL((k_sweep<ST, FM, OFF, MD, C>), grid, block, a.lds, s, a)
#define LBMEP_BY_FORCE(MD, OFF, C)                                           \
    do {                                                                     \
        if (force_mode == kForceNone) LBMEP_LAUNCH(MD, kForceNone, OFF, C);      \
        else if (force_mode == kForceDense) LBMEP_LAUNCH(MD, kForceDense, OFF, C); \
        else if (force_mode == kForceCharge) LBMEP_LAUNCH(MD, kForceCharge, OFF, C); \
        else LBMEP_LAUNCH(MD, kForcePotential, OFF, C);                        \
    } while (0)
#define LBMEP_BY_CPT(MD)                                    \
    do {                                                    \
        if (cpt == 2) LBMEP_BY_FORCE(MD, uint32_t, 2);      \
        else LBMEP_BY_FORCE(MD, uint32_t, 1);               \
    } while (0)
    if (small) {
        if (mode == kPull) LBMEP_BY_CPT(kPull);
        else if (mode == kPullNT) LBMEP_BY_CPT(kPullNT);
        else if (mode == kPullNTS) LBMEP_BY_CPT(kPullNTS);
        else if (mode == kLocal) LBMEP_BY_CPT(kLocal);
        else LBMEP_LAUNCH(kReadout, kForceNone, uint32_t, 1);
    } else {
        if (mode == kPull || mode == kPullNT || mode == kPullNTS) LBMEP_BY_FORCE(kPull, uint64_t, 1);
        else if (mode == kLocal) LBMEP_BY_FORCE(kLocal, uint64_t, 1);
        else LBMEP_LAUNCH(kReadout, kForceNone, uint64_t, 1);
    }
#undef LBMEP_BY_CPT
#undef LBMEP_BY_FORCE
#undef LBMEP_LAUNCH
    return hipGetLastError();
}

}  // namespace sweep
}  // namespace lbmep
