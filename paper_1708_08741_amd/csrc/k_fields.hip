// k_fields.hip -- field kernels around the sweep: fills, equilibrium
// initialisation, conversion between absolute FP64 populations and the
// storage formats, force conversion, macroscopic read-out (Eq. MacroscopVel
// with the velocity of Eq. modified_velocity, arXiv:1708.08741 Sec. 3.1) and
// deterministic FP64 global sums (mass and momentum over fluid cells).
#include "potential_impl.h"

namespace lbmep {
namespace {

constexpr int kThreads = 256;

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f64(double *p, double v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int grid_for(size_t n) {
    size_t b = (n + kThreads - 1) / kThreads;
    if (b > 65536) b = 65536;
    if (b == 0) b = 1;
    return (int)b;
}

// storage <-> deviation / absolute value helpers
template <typename ST>
__device__ __forceinline__ double to_abs(ST v, int q);
template <>
__device__ __forceinline__ double to_abs<double>(double v, int q) { return v; }
template <>
__device__ __forceinline__ double to_abs<float>(float v, int q) { return (double)v + wq(q); }
template <>
__device__ __forceinline__ double to_abs<__half>(__half v, int q) {
    return (double)(__half2float(v) * kHalfInvScale) + wq(q);
}

template <typename ST>
__device__ __forceinline__ ST from_abs(double f, int q);
template <>
__device__ __forceinline__ double from_abs<double>(double f, int q) { return f; }
template <>
__device__ __forceinline__ float from_abs<float>(double f, int q) { return (float)(f - wq(q)); }
template <>
__device__ __forceinline__ __half from_abs<__half>(double f, int q) {
    return __float2half_rn((float)(f - wq(q)) * kHalfScale);
}

// deviation value (compute precision) of a stored population
template <typename ST>
__device__ __forceinline__ double dev_value(ST v);
template <>
__device__ __forceinline__ double dev_value<float>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double dev_value<__half>(__half v) {
    return (double)(__half2float(v) * kHalfInvScale);
}

template <typename ST>
__global__ void k_init_eq(Grid g, ST *f, double rho, double u0, double u1, double u2) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    const double uu = (u0 * u0 + u1 * u1) + u2 * u2;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const double cu = ((double)kCx[q] * u0 + (double)kCy[q] * u1) + (double)kCz[q] * u2;
        const double w = wq(q);
        // Eq. fequ_Incompr_SRT with rho0 = 1
        const double d = (cu * 3.0 + (cu * cu) * 4.5) - uu * 1.5;
        if constexpr (sizeof(ST) == 8) {
            f[(size_t)q * g.Ns + c] = w * (rho + 1.0 * d);
        } else if constexpr (sizeof(ST) == 4) {
            f[(size_t)q * g.Ns + c] = (float)(w * ((rho - 1.0) + d));
        } else {
            f[(size_t)q * g.Ns + c] = __float2half_rn((float)(w * ((rho - 1.0) + d)) * kHalfScale);
        }
    }
}

// one population q: absolute FP64 in[c] -> storage f[c]
template <typename ST>
__global__ void k_pdfs_from(size_t N, int q, const double *in, ST *f) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    f[c] = from_abs<ST>(in[c], q);
}

// one population q: storage f[c] -> absolute FP64 out[c]
template <typename ST>
__global__ void k_pdfs_to(size_t N, int q, const ST *f, double *out) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    out[c] = to_abs<ST>(f[c], q);
}

template <typename TI, typename TO>
__global__ void k_convert(const TI *in, TO *out, size_t n, size_t si, size_t so, int ncomp) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        for (int k = 0; k < ncomp; ++k) out[k * so + i] = (TO)in[k * si + i];
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

template <typename ST, typename CT>
__global__ void k_macro(Grid g, int force_mode, const ST *f, const uint8_t *flag,
                        const uint32_t *owner, const double *Xc, const double *U, const double *W,
                        const CT *force, double E0, double E1, double E2, double keps,
                        const double *zeta, double *rho, double *u) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const size_t c = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
    const uint8_t fl = flag[c];
    if (fl & kWall) {
        rho[c] = 1.0;
        u[c] = u[g.N + c] = u[2 * g.N + c] = 0.0;
        return;
    }
    if (fl & kObst) {
        const uint32_t p = owner[c];
        const double *Xp = Xc + 3 * (size_t)p;
        const double r0 = min_image(((double)x + 0.5) - Xp[0], g.nx, g.per[0]);
        const double r1 = min_image(((double)y + 0.5) - Xp[1], g.ny, g.per[1]);
        const double r2 = min_image(((double)z + 0.5) - Xp[2], g.nz, g.per[2]);
        const double *Up = U + 3 * (size_t)p, *Wp = W + 3 * (size_t)p;
        rho[c] = 1.0;
        u[c] = Up[0] + (Wp[1] * r2 - Wp[2] * r1);
        u[g.N + c] = Up[1] + (Wp[2] * r0 - Wp[0] * r2);
        u[2 * g.N + c] = Up[2] + (Wp[0] * r1 - Wp[1] * r0);
        return;
    }
    double fb[3] = {0.0, 0.0, 0.0};
    if (force_mode == kForceDense) {
        fb[0] = (double)force[c];
        fb[1] = (double)force[g.Ns + c];
        fb[2] = (double)force[2 * g.Ns + c];
    } else if (force_mode == kForceCharge) {
        const double re = (double)force[c];
        fb[0] = re * E0;
        fb[1] = re * E1;
        fb[2] = re * E2;
    } else if (force_mode == kForcePotential) {
        // the force of the sweep, in its compute precision
        CT f0, f1, f2;
        potential_force<CT>(g, x, y, z, fl, force, flag, owner, zeta, (CT)keps, (CT)E0, (CT)E1,
                            (CT)E2, f0, f1, f2);
        fb[0] = (double)f0;
        fb[1] = (double)f1;
        fb[2] = (double)f2;
    }
    double s = 0.0, j[3] = {0.0, 0.0, 0.0};
    if constexpr (sizeof(ST) == 8) {
#pragma unroll
        for (int q = 0; q < Q; ++q) s += (double)f[(size_t)q * g.Ns + c];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double v = (double)f[(size_t)q * g.Ns + c];
            j[0] += (double)kCx[q] * v;
            j[1] += (double)kCy[q] * v;
            j[2] += (double)kCz[q] * v;
        }
        rho[c] = s;
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double v = dev_value<ST>(f[(size_t)q * g.Ns + c]);
            s += v;
            j[0] += (double)kCx[q] * v;
            j[1] += (double)kCy[q] * v;
            j[2] += (double)kCz[q] * v;
        }
        rho[c] = 1.0 + s;
    }
    // Eq. modified_velocity
    u[c] = j[0] + 0.5 * fb[0];
    u[g.N + c] = j[1] + 0.5 * fb[1];
    u[2 * g.N + c] = j[2] + 0.5 * fb[2];
}

// block-level sums of (rho or rho - 1, j) over fluid cells; the block sums
// are reduced by one block in a fixed order -> deterministic result
template <typename ST>
__global__ void __launch_bounds__(kThreads)
    k_invariants(Grid g, const ST *f, const uint8_t *flag, double *partials) {
    __shared__ double sh[4][kThreads];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.N;
         c += (size_t)gridDim.x * blockDim.x) {
        if (flag[c] & (kWall | kObst)) continue;
        double s = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double v;
            if constexpr (sizeof(ST) == 8)
                v = (double)f[(size_t)q * g.Ns + c];
            else
                v = dev_value<ST>(f[(size_t)q * g.Ns + c]);
            s += v;
            j0 += (double)kCx[q] * v;
            j1 += (double)kCy[q] * v;
            j2 += (double)kCz[q] * v;
        }
        if constexpr (sizeof(ST) == 8) s -= 1.0;  // accumulate rho - 1 (exact sums of counts)
        acc[0] += s;
        acc[1] += j0;
        acc[2] += j1;
        acc[3] += j2;
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) partials[4 * (size_t)blockIdx.x + k] = sh[k][0];
}

// count of fluid cells per block, same decomposition
__global__ void __launch_bounds__(kThreads)
    k_fluid_count(Grid g, const uint8_t *flag, double *partials) {
    __shared__ double sh[kThreads];
    double n = 0.0;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < g.N;
         c += (size_t)gridDim.x * blockDim.x)
        if (!(flag[c] & (kWall | kObst))) n += 1.0;
    sh[threadIdx.x] = n;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(kThreads)
    k_reduce_partials(const double *partials, const double *counts, int nblocks, double *out) {
    __shared__ double sh[5][kThreads];
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        for (int k = 0; k < 4; ++k) acc[k] += partials[4 * (size_t)b + k];
        acc[4] += counts[b];
    }
    for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // mass = (number of fluid cells) + sum (rho - 1)
        out[0] = sh[4][0] + sh[0][0];
        out[1] = sh[1][0];
        out[2] = sh[2][0];
        out[3] = sh[3][0];
    }
}

__global__ void k_export_flags(Grid g, const uint8_t *flag, uint8_t *out) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    const uint8_t f = flag[c];
    out[c] = (f & kWall) ? LBMEP_WALL : (f & kObst) ? LBMEP_OBST : (f & kNear) ? LBMEP_NEAR
                                                                                : LBMEP_FLUID;
}

__global__ void k_import_flags(Grid g, const uint8_t *in, uint8_t *flag) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    flag[c] = in[c] == LBMEP_WALL ? kWall : 0;
}

}  // namespace

int invariants_blocks(const Grid &g) {
    size_t b = (g.N + kThreads * 8 - 1) / (kThreads * 8);
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kThreads), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(kThreads), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_init_equilibrium(int precision, const Grid &g, void *f, double rho,
                                   const double u[3], hipStream_t s) {
    const dim3 grid((unsigned)((g.N + kThreads - 1) / kThreads)), block(kThreads);
    if (precision == LBMEP_FP64)
        hipLaunchKernelGGL(k_init_eq<double>, grid, block, 0, s, g, (double *)f, rho, u[0], u[1],
                           u[2]);
    else if (precision == LBMEP_FP32DEV)
        hipLaunchKernelGGL(k_init_eq<float>, grid, block, 0, s, g, (float *)f, rho, u[0], u[1],
                           u[2]);
    else
        hipLaunchKernelGGL(k_init_eq<__half>, grid, block, 0, s, g, (__half *)f, rho, u[0], u[1],
                           u[2]);
    return hipGetLastError();
}

hipError_t launch_pdfs_from_f64(int precision, const Grid &g, int q, const double *in, void *f,
                                hipStream_t s) {
    const dim3 grid((unsigned)((g.N + kThreads - 1) / kThreads)), block(kThreads);
    const size_t off = (size_t)q * g.Ns;
    if (precision == LBMEP_FP64)
        hipLaunchKernelGGL(k_pdfs_from<double>, grid, block, 0, s, g.N, q, in, (double *)f + off);
    else if (precision == LBMEP_FP32DEV)
        hipLaunchKernelGGL(k_pdfs_from<float>, grid, block, 0, s, g.N, q, in, (float *)f + off);
    else
        hipLaunchKernelGGL(k_pdfs_from<__half>, grid, block, 0, s, g.N, q, in, (__half *)f + off);
    return hipGetLastError();
}

hipError_t launch_pdfs_to_f64(int precision, const Grid &g, int q, const void *f, double *out,
                              hipStream_t s) {
    const dim3 grid((unsigned)((g.N + kThreads - 1) / kThreads)), block(kThreads);
    const size_t off = (size_t)q * g.Ns;
    if (precision == LBMEP_FP64)
        hipLaunchKernelGGL(k_pdfs_to<double>, grid, block, 0, s, g.N, q, (const double *)f + off,
                           out);
    else if (precision == LBMEP_FP32DEV)
        hipLaunchKernelGGL(k_pdfs_to<float>, grid, block, 0, s, g.N, q, (const float *)f + off,
                           out);
    else
        hipLaunchKernelGGL(k_pdfs_to<__half>, grid, block, 0, s, g.N, q, (const __half *)f + off,
                           out);
    return hipGetLastError();
}

hipError_t launch_convert_force(int precision, const void *in, int in_dtype, void *out, size_t n,
                                size_t in_stride, size_t out_stride, int ncomp, hipStream_t s) {
    const dim3 grid(grid_for(n)), block(kThreads);
    const bool out64 = precision == LBMEP_FP64;
    if (in_dtype == LBMEP_DTYPE_F64 && out64)
        hipLaunchKernelGGL((k_convert<double, double>), grid, block, 0, s, (const double *)in,
                           (double *)out, n, in_stride, out_stride, ncomp);
    else if (in_dtype == LBMEP_DTYPE_F64)
        hipLaunchKernelGGL((k_convert<double, float>), grid, block, 0, s, (const double *)in,
                           (float *)out, n, in_stride, out_stride, ncomp);
    else if (out64)
        hipLaunchKernelGGL((k_convert<float, double>), grid, block, 0, s, (const float *)in,
                           (double *)out, n, in_stride, out_stride, ncomp);
    else
        hipLaunchKernelGGL((k_convert<float, float>), grid, block, 0, s, (const float *)in,
                           (float *)out, n, in_stride, out_stride, ncomp);
    return hipGetLastError();
}

hipError_t launch_macro(int precision, int force_mode, const Grid &g, const void *f,
                        const uint8_t *flag, const uint32_t *owner, const double *Xc,
                        const double *U, const double *W, const void *force, const double E[3],
                        double keps, const double *zeta, double *rho, double *u, hipStream_t s) {
    const int bx = 64;
    const dim3 grid((g.nx + bx - 1) / bx, g.ny, g.nz), block(bx);
    if (precision == LBMEP_FP64)
        hipLaunchKernelGGL((k_macro<double, double>), grid, block, 0, s, g, force_mode,
                           (const double *)f, flag, owner, Xc, U, W, (const double *)force, E[0],
                           E[1], E[2], keps, zeta, rho, u);
    else if (precision == LBMEP_FP32DEV)
        hipLaunchKernelGGL((k_macro<float, float>), grid, block, 0, s, g, force_mode,
                           (const float *)f, flag, owner, Xc, U, W, (const float *)force, E[0],
                           E[1], E[2], keps, zeta, rho, u);
    else
        hipLaunchKernelGGL((k_macro<__half, float>), grid, block, 0, s, g, force_mode,
                           (const __half *)f, flag, owner, Xc, U, W, (const float *)force, E[0],
                           E[1], E[2], keps, zeta, rho, u);
    return hipGetLastError();
}

hipError_t launch_invariants(int precision, const Grid &g, const void *f, const uint8_t *flag,
                             double *partials, int nblocks, double *out, hipStream_t s) {
    double *counts = partials + 4 * (size_t)nblocks;
    if (precision == LBMEP_FP64)
        hipLaunchKernelGGL(k_invariants<double>, dim3(nblocks), dim3(kThreads), 0, s, g,
                           (const double *)f, flag, partials);
    else if (precision == LBMEP_FP32DEV)
        hipLaunchKernelGGL(k_invariants<float>, dim3(nblocks), dim3(kThreads), 0, s, g,
                           (const float *)f, flag, partials);
    else
        hipLaunchKernelGGL(k_invariants<__half>, dim3(nblocks), dim3(kThreads), 0, s, g,
                           (const __half *)f, flag, partials);
    hipLaunchKernelGGL(k_fluid_count, dim3(nblocks), dim3(kThreads), 0, s, g, flag, counts);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kThreads), 0, s, partials, counts,
                       nblocks, out);
    return hipGetLastError();
}

// the achievable-bandwidth reference: a plain copy in 16-byte lanes with
// streaming (non-temporal) stores, one element per thread (measured faster
// than a grid-strided loop over fewer workgroups: 6.3 against 5.2 TB/s)
__global__ void __launch_bounds__(256) k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                size_t n, size_t base) {
    const size_t i = base + (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint4 v = src[i];
    __builtin_nontemporal_store(v.x, &dst[i].x);
    __builtin_nontemporal_store(v.y, &dst[i].y);
    __builtin_nontemporal_store(v.z, &dst[i].z);
    __builtin_nontemporal_store(v.w, &dst[i].w);
}

hipError_t launch_copy16(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    // at most 2^31 - 1 workgroups per launch
    const size_t per = (size_t)0x7FFFFFFF * 256;
    for (size_t base = 0; base < n; base += per) {
        const size_t m = n - base < per ? n - base : per;
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                           static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n, base);
    }
    return hipGetLastError();
}

hipError_t launch_export_flags(const Grid &g, const uint8_t *flag, uint8_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_export_flags, dim3((unsigned)((g.N + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, g, flag, out);
    return hipGetLastError();
}

hipError_t launch_import_flags(const Grid &g, const uint8_t *in, uint8_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_import_flags, dim3((unsigned)((g.N + kThreads - 1) / kThreads)),
                       dim3(kThreads), 0, s, g, in, flag);
    return hipGetLastError();
}

}  // namespace lbmep
