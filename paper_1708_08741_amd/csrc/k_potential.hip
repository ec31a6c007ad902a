// k_potential.hip -- the Debye-Hueckel equation of the EDL potential solved
// by SOR in red-black order (arXiv:1708.08741, Sec. "Finite Volume
// Discretization for Electric Potential Equations", Sec. "Solver for Linear
// Elliptic PDEs with Moving Boundaries", Sec. "Boundary Condition Handling
// for Solver Module").
//
// Unknowns are the cells that are neither wall nor obstacle cells.  With
// dx = 1 the seven-point finite-volume row of unknown i is
//     diag_i psi_i - sum_{unknown q} psi(x_i + e_q) = rhs_i,
//     diag_i = 6 + kappa^2 + n_D - n_N,   rhs_i = 2 sum_{obstacle q} b_p,
// where a neighbour that is an obstacle cell of particle p is a Dirichlet
// boundary on the shared face (value b_p = zeta_p, or the field's value at
// that cell without zeta; linear extrapolation to the cell gives
// 2 b_p - psi_i) and a wall or beyond-edge neighbour is a homogeneous
// Neumann boundary (it counts psi_i).  A half-sweep relaxes every unknown of
// one colour ((x + y + z) & 1) with
//     psi_i <- (1 - omega) psi_i + omega (rhs_i + sum) / diag_i;
// same-coloured cells are never neighbours (even extents along periodic
// axes), so a half-sweep is order-free and each cell is written by one
// thread.  Terms are formed in the order x-, x+, y-, y+, z-, z+, so the
// FP64 kernel rounds like a plain CPU evaluation of the same rows.
//
// Two implementations of an iteration, bitwise identical:
//   * k_sor_half: one launch per colour, in place (each colour streams psi
//     through HBM once);
//   * k_sor_fused (default): one launch per iteration from psi into a second
//     buffer.  A workgroup owns a 64 x 16 tile of (x, y) and a chunk of z
//     planes and marches through its planes with rings of planes in LDS:
//     the old values of a plane with a two-cell halo, then the new red
//     values of that plane on a one-cell halo ring (from old black
//     neighbours), then the new black values of the plane behind it (from
//     the new red values around it).  Halo values are recomputed from the
//     same old values by every workgroup that needs them, so the result is
//     the red-black sweep exactly, read once and written once per
//     iteration.
//
// The residual's L2 norm is the root mean square over the unknowns, summed
// in a fixed order (per-thread strided sums, a block tree, one block over
// the blocks), so it is reproducible run to run.
#include "lbmep_internal.h"

namespace lbmep {
namespace {

constexpr int kSorBlock = 256;
constexpr int kResBlock = 256;

// row of unknown cell (x, y, z) with flag fl: diag, rhs and the sum over
// unknown neighbours
template <typename CT>
__device__ __forceinline__ void dha_row(const Grid &g, int x, int y, int z, uint8_t fl,
                                        const CT *psi, const uint8_t *flag,
                                        const uint32_t *owner, const double *zeta, CT kappa2,
                                        CT &diag, CT &rhs, CT &sum) {
    diag = CT(6.0) + kappa2;
    rhs = CT(0);
    sum = CT(0);
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    const size_t nx = (size_t)g.nx, nxy = (size_t)g.nx * (size_t)g.ny;
    const size_t row = nx * (size_t)y + nxy * (size_t)z;
    if (!(fl & kNear)) {
        // every neighbour is an unknown inside the grid (periodic wrap)
        sum = sum + psi[(size_t)xm + row];
        sum = sum + psi[(size_t)xp + row];
        sum = sum + psi[(size_t)x + nx * (size_t)ym + nxy * (size_t)z];
        sum = sum + psi[(size_t)x + nx * (size_t)yp + nxy * (size_t)z];
        sum = sum + psi[(size_t)x + nx * (size_t)y + nxy * (size_t)zm];
        sum = sum + psi[(size_t)x + nx * (size_t)y + nxy * (size_t)zp];
        return;
    }
    const int lo[3] = {x == 0, y == 0, z == 0};
    const int hi[3] = {x == g.nx - 1, y == g.ny - 1, z == g.nz - 1};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int a = k >> 1;
        const bool up = k & 1;
        if ((up ? hi[a] : lo[a]) && !g.per[a]) {
            diag = diag - CT(1.0);  // homogeneous Neumann (edge)
            continue;
        }
        const int vx = a == 0 ? (up ? xp : xm) : x;
        const int vy = a == 1 ? (up ? yp : ym) : y;
        const int vz = a == 2 ? (up ? zp : zm) : z;
        const size_t s = (size_t)vx + nx * (size_t)vy + nxy * (size_t)vz;
        const uint8_t fs = flag[s];
        if (fs & kWall) {
            diag = diag - CT(1.0);  // homogeneous Neumann (wall)
        } else if (fs & kObst) {
            const CT b = zeta ? (CT)zeta[owner[s]] : psi[s];
            diag = diag + CT(1.0);  // Dirichlet on the shared face
            rhs = rhs + CT(2.0) * b;
        } else {
            sum = sum + psi[s];
        }
    }
}

__global__ void k_sor_begin(SorCtl *ctl) {
    if (threadIdx.x == 0) {
        ctl->done = 0;
        ctl->iters = 0;
        ctl->res0 = -1.0;
        ctl->res = -1.0;
    }
}

// one half-sweep: the unknowns of one colour, one per thread; rows of
// (nx + 1) / 2 slots
template <typename CT>
__global__ void __launch_bounds__(kSorBlock) k_sor_half(SorArgs a, int colour, int count) {
    if (a.ctl->done) return;
    if (count && blockIdx.x == 0 && threadIdx.x == 0) a.ctl->iters += 1;
    const Grid &g = a.g;
    const uint32_t lb = a.xcd_swizzle ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const size_t t = (size_t)lb * kSorBlock + threadIdx.x;
    const size_t hx = (size_t)((g.nx + 1) / 2);
    const size_t r = t / hx;
    if (r >= (size_t)g.ny * (size_t)g.nz) return;
    const int y = (int)(r % (size_t)g.ny), z = (int)(r / (size_t)g.ny);
    const int x = 2 * (int)(t - r * hx) + ((colour + y + z) & 1);
    if (x >= g.nx) return;
    const size_t c = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
    const uint8_t fl = a.flag[c];
    if (fl & (kWall | kObst)) return;
    CT *psi = static_cast<CT *>(a.psi);
    CT diag, rhs, sum;
    dha_row<CT>(g, x, y, z, fl, psi, a.flag, a.owner, a.zeta, (CT)a.kappa2, diag, rhs, sum);
    const CT om = (CT)a.omega;
    psi[c] = (CT(1.0) - om) * psi[c] + om * ((rhs + sum) / diag);
}

// residual: per-thread strided sums of r^2 and of the unknowns, a block tree,
// one FP64 pair per block
template <typename CT>
__global__ void __launch_bounds__(kResBlock) k_dha_residual(SorArgs a) {
    if (a.ctl->done) return;
    const Grid &g = a.g;
    const CT *psi = static_cast<const CT *>(a.psi);
    double ss = 0.0, n = 0.0;
    const size_t stride = (size_t)gridDim.x * kResBlock;
    for (size_t c = (size_t)blockIdx.x * kResBlock + threadIdx.x; c < g.N; c += stride) {
        const uint8_t fl = a.flag[c];
        if (fl & (kWall | kObst)) continue;
        const int x = (int)(c % (size_t)g.nx);
        const size_t yz = c / (size_t)g.nx;
        const int y = (int)(yz % (size_t)g.ny), z = (int)(yz / (size_t)g.ny);
        CT diag, rhs, sum;
        dha_row<CT>(g, x, y, z, fl, psi, a.flag, a.owner, a.zeta, (CT)a.kappa2, diag, rhs, sum);
        const double r = (double)(rhs + sum - diag * psi[c]);
        ss += r * r;
        n += 1.0;
    }
    __shared__ double s_ss[kResBlock], s_n[kResBlock];
    s_ss[threadIdx.x] = ss;
    s_n[threadIdx.x] = n;
    __syncthreads();
    for (int h = kResBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s_ss[threadIdx.x] += s_ss[threadIdx.x + h];
            s_n[threadIdx.x] += s_n[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.partial[2 * blockIdx.x] = s_ss[0];
        a.partial[2 * blockIdx.x + 1] = s_n[0];
    }
}

// one block: the norm from the partials; first = the initial residual
__global__ void __launch_bounds__(kResBlock) k_dha_finalize(SorArgs a, int nparts, int first) {
    if (a.ctl->done) return;
    double ss = 0.0, n = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kResBlock) {
        ss += a.partial[2 * i];
        n += a.partial[2 * i + 1];
    }
    __shared__ double s_ss[kResBlock], s_n[kResBlock];
    s_ss[threadIdx.x] = ss;
    s_n[threadIdx.x] = n;
    __syncthreads();
    for (int h = kResBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s_ss[threadIdx.x] += s_ss[threadIdx.x + h];
            s_n[threadIdx.x] += s_n[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double res = s_n[0] > 0.0 ? sqrt(s_ss[0] / s_n[0]) : 0.0;
        a.ctl->res = res;
        if (first) {
            a.ctl->res0 = res;
            if (res == 0.0) a.ctl->done = 1;
        } else if (res < a.rf * a.ctl->res0) {
            a.ctl->done = 1;
        }
    }
}

// relaxation of unknown cell (x, y, z) with flag fl and old value own;
// get(k) is the current value of the unknown neighbour in direction k
// (x-, x+, y-, y+, z-, z+).  Same terms in the same order as dha_row.
template <typename CT, typename Get>
__device__ __forceinline__ CT relax(const SorArgs &a, int x, int y, int z, uint8_t fl, CT own,
                                    const CT *psi_old, Get get) {
    const Grid &g = a.g;
    CT diag = CT(6.0) + (CT)a.kappa2, rhs = CT(0), sum = CT(0);
    if (!(fl & kNear)) {
#pragma unroll
        for (int k = 0; k < 6; ++k) sum = sum + get(k);
    } else {
        const int lo[3] = {x == 0, y == 0, z == 0};
        const int hi[3] = {x == g.nx - 1, y == g.ny - 1, z == g.nz - 1};
        const size_t nx = (size_t)g.nx, nxy = (size_t)g.nx * (size_t)g.ny;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int ax = k >> 1;
            const bool up = k & 1;
            if ((up ? hi[ax] : lo[ax]) && !g.per[ax]) {
                diag = diag - CT(1.0);
                continue;
            }
            int v[3] = {x, y, z};
            const int len[3] = {g.nx, g.ny, g.nz};
            v[ax] += up ? 1 : -1;
            if (v[ax] < 0) v[ax] += len[ax];
            if (v[ax] >= len[ax]) v[ax] -= len[ax];
            const size_t s = (size_t)v[0] + nx * (size_t)v[1] + nxy * (size_t)v[2];
            const uint8_t fs = a.flag[s];
            if (fs & kWall) {
                diag = diag - CT(1.0);
            } else if (fs & kObst) {
                // obstacle cells never change: the old buffer holds b
                const CT b = a.zeta ? (CT)a.zeta[a.owner[s]] : psi_old[s];
                diag = diag + CT(1.0);
                rhs = rhs + CT(2.0) * b;
            } else {
                sum = sum + get(k);
            }
        }
    }
    const CT om = (CT)a.omega;
    return (CT(1.0) - om) * own + om * ((rhs + sum) / diag);
}

constexpr int kFTX = 64, kFTY = 16, kFZC = 32, kFBlock = 256;

__device__ __forceinline__ int wrap_axis_or(int v, int len, int per, bool &ok) {
    if (v < 0 || v >= len) {
        if (!per) {
            ok = false;
            return 0;
        }
        v = v < 0 ? v + len : v - len;
    }
    ok = true;
    return v;
}

template <typename CT>
__global__ void __launch_bounds__(kFBlock) k_sor_fused(SorArgs a, const CT *src, CT *dst,
                                                        int ntx, int nty) {
    if (a.ctl->done) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->iters += 1;
    constexpr int OW = kFTX + 4, OH = kFTY + 4;  // old planes: two-cell halo
    constexpr int RW = kFTX + 2, RH = kFTY + 2;  // new red values: one-cell halo
    __shared__ CT s_old[4][OH][OW];
    __shared__ CT s_rn[3][RH][RW];
    const Grid &g = a.g;
    const uint32_t lb = a.xcd_swizzle ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tx = (int)(lb % (uint32_t)ntx);
    const int ty = (int)((lb / (uint32_t)ntx) % (uint32_t)nty);
    const int tz = (int)(lb / ((uint32_t)ntx * (uint32_t)nty));
    const int X0 = tx * kFTX, Y0 = ty * kFTY, Z0 = tz * kFZC;
    const int Z1 = min(Z0 + kFZC, g.nz);
    const size_t nx = (size_t)g.nx, nxy = (size_t)g.nx * (size_t)g.ny;
    const int tid = threadIdx.x;

    // plane j (unwrapped) exists and its wrapped index
    auto plane = [&](int j, int &jw) {
        bool ok;
        jw = wrap_axis_or(j, g.nz, g.per[2], ok);
        return ok;
    };
    auto load_old = [&](int j) {
        int jw;
        if (!plane(j, jw)) return;
        CT(*o)[OW] = s_old[(j - Z0 + 8) & 3];
        for (int i = tid; i < OH * OW; i += kFBlock) {
            const int r = i / OW, c = i - r * OW;
            bool okx, oky;
            const int gx = wrap_axis_or(X0 - 2 + c, g.nx, g.per[0], okx);
            const int gy = wrap_axis_or(Y0 - 2 + r, g.ny, g.per[1], oky);
            if (okx && oky) o[r][c] = src[(size_t)gx + nx * (size_t)gy + nxy * (size_t)jw];
        }
    };

    load_old(Z0 - 2);
    load_old(Z0 - 1);
    load_old(Z0);
    for (int j = Z0 - 1; j <= Z1; ++j) {
        load_old(j + 1);
        __syncthreads();
        // new red values of plane j on the tile and a one-cell ring
        int jw;
        if (plane(j, jw)) {
            CT(*om)[OW] = s_old[(j - 1 - Z0 + 8) & 3];
            CT(*o0)[OW] = s_old[(j - Z0 + 8) & 3];
            CT(*op)[OW] = s_old[(j + 1 - Z0 + 8) & 3];
            CT(*rn)[RW] = s_rn[(j - Z0 + 6) % 3];
            for (int i = tid; i < RH * (RW / 2); i += kFBlock) {
                const int r = i / (RW / 2), k = i - r * (RW / 2);
                const int c = 2 * k + ((X0 + Y0 + r + j) & 1);  // (x + y + z) even
                bool okx, oky;
                const int gx = wrap_axis_or(X0 - 1 + c, g.nx, g.per[0], okx);
                const int gy = wrap_axis_or(Y0 - 1 + r, g.ny, g.per[1], oky);
                if (!okx || !oky) continue;
                const size_t cell = (size_t)gx + nx * (size_t)gy + nxy * (size_t)jw;
                const uint8_t fl = a.flag[cell];
                if (fl & (kWall | kObst)) continue;
                const int R = r + 1, C = c + 1;  // in the old planes
                rn[r][c] = relax<CT>(a, gx, gy, jw, fl, o0[R][C], src, [&](int d) {
                    switch (d) {
                        case 0: return o0[R][C - 1];
                        case 1: return o0[R][C + 1];
                        case 2: return o0[R - 1][C];
                        case 3: return o0[R + 1][C];
                        case 4: return om[R][C];
                        default: return op[R][C];
                    }
                });
            }
        }
        __syncthreads();
        // plane j - 1 of the tile: new black values from the new red ones,
        // new red values, unchanged boundary cells; written in x pairs
        const int jj = j - 1;
        if (jj >= Z0) {
            int jjw;
            plane(jj, jjw);
            CT(*o0)[OW] = s_old[(jj - Z0 + 8) & 3];
            CT(*rm)[RW] = s_rn[(jj - 1 - Z0 + 6) % 3];
            CT(*r0)[RW] = s_rn[(jj - Z0 + 6) % 3];
            CT(*rp)[RW] = s_rn[(jj + 1 - Z0 + 6) % 3];
            for (int i = tid; i < kFTY * kFTX; i += kFBlock) {
                const int r = i / kFTX, c = i - r * kFTX;
                const int gx = X0 + c, gy = Y0 + r;
                if (gx >= g.nx || gy >= g.ny) continue;
                const size_t cell = (size_t)gx + nx * (size_t)gy + nxy * (size_t)jjw;
                const uint8_t fl = a.flag[cell];
                const int R = r + 1, C = c + 1;  // in the red planes
                CT out;
                if (fl & (kWall | kObst)) {
                    out = o0[r + 2][c + 2];
                } else if (((gx + gy + jjw) & 1) == 0) {
                    out = r0[R][C];
                } else {
                    out = relax<CT>(a, gx, gy, jjw, fl, o0[r + 2][c + 2], src, [&](int d) {
                        switch (d) {
                            case 0: return r0[R][C - 1];
                            case 1: return r0[R][C + 1];
                            case 2: return r0[R - 1][C];
                            case 3: return r0[R + 1][C];
                            case 4: return rm[R][C];
                            default: return rp[R][C];
                        }
                    });
                }
                dst[cell] = out;
            }
        }
    }
}

template <typename CT>
__global__ void k_to_f64(Grid g, const CT *psi, double *out) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < g.N) out[c] = (double)psi[c];
}

template <typename CT>
hipError_t sor_solve_typed(const SorArgs &a0, int max_iter, int check_every, bool fused,
                           hipStream_t s, int *swapped) {
    const Grid &g = a0.g;
    const size_t hx = (size_t)((g.nx + 1) / 2);
    const size_t slots = hx * (size_t)g.ny * (size_t)g.nz;
    const uint32_t nblk = (uint32_t)((slots + kSorBlock - 1) / kSorBlock);
    const int ntx = (g.nx + kFTX - 1) / kFTX, nty = (g.ny + kFTY - 1) / kFTY;
    const int ntz = (g.nz + kFZC - 1) / kFZC;
    const uint32_t nfused = (uint32_t)ntx * (uint32_t)nty * (uint32_t)ntz;
    const size_t rblk = (g.N + kResBlock - 1) / kResBlock;
    const int nres = (int)(rblk < (size_t)(kSorPartials / 2) ? rblk : (size_t)(kSorPartials / 2));
    const bool with_res = a0.rf > 0.0;
    SorArgs a = a0;  // a.psi: the buffer holding the current iterate
    hipLaunchKernelGGL(k_sor_begin, dim3(1), dim3(64), 0, s, a.ctl);
    if (with_res) {
        hipLaunchKernelGGL((k_dha_residual<CT>), dim3(nres), dim3(kResBlock), 0, s, a);
        hipLaunchKernelGGL(k_dha_finalize, dim3(1), dim3(kResBlock), 0, s, a, nres, 1);
    }
    for (int it = 1; it <= max_iter; ++it) {
        if (fused) {
            void *next = a.psi == a0.psi ? a0.psi2 : a0.psi;
            hipLaunchKernelGGL((k_sor_fused<CT>), dim3(nfused), dim3(kFBlock), 0, s, a,
                               static_cast<const CT *>(a.psi), static_cast<CT *>(next), ntx, nty);
            a.psi = next;
        } else {
            hipLaunchKernelGGL((k_sor_half<CT>), dim3(nblk), dim3(kSorBlock), 0, s, a, 0, 0);
            hipLaunchKernelGGL((k_sor_half<CT>), dim3(nblk), dim3(kSorBlock), 0, s, a, 1, 1);
        }
        if (with_res && (it % check_every == 0 || it == max_iter)) {
            hipLaunchKernelGGL((k_dha_residual<CT>), dim3(nres), dim3(kResBlock), 0, s, a);
            hipLaunchKernelGGL(k_dha_finalize, dim3(1), dim3(kResBlock), 0, s, a, nres, 0);
        }
        if (with_res && it % 64 == 0 && it < max_iter) {
            int32_t done = 0;
            hipError_t e = hipMemcpyAsync(&done, &a.ctl->done, sizeof done, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
            if (done) break;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the fused iterations alternate buffers: which one holds the result
    *swapped = 0;
    if (fused) {
        int32_t iters = max_iter;
        if (with_res) {
            e = hipMemcpyAsync(&iters, &a.ctl->iters, sizeof iters, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return e;
        }
        *swapped = iters & 1;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_sor_solve(int precision, const SorArgs &a, int max_iter, int check_every,
                            bool fused, hipStream_t s, int *swapped) {
    *swapped = 0;
    if (a.g.N == 0) return hipSuccess;
    if (fused && !a.psi2) return hipErrorInvalidValue;
    if (precision == LBMEP_FP64)
        return sor_solve_typed<double>(a, max_iter, check_every, fused, s, swapped);
    return sor_solve_typed<float>(a, max_iter, check_every, fused, s, swapped);
}

hipError_t launch_potential_to_f64(int precision, const Grid &g, const void *psi, double *out,
                                   hipStream_t s) {
    if (g.N == 0) return hipSuccess;
    const uint32_t nb = (uint32_t)((g.N + 255) / 256);
    if (precision == LBMEP_FP64)
        hipLaunchKernelGGL((k_to_f64<double>), dim3(nb), dim3(256), 0, s, g,
                           static_cast<const double *>(psi), out);
    else
        hipLaunchKernelGGL((k_to_f64<float>), dim3(nb), dim3(256), 0, s, g,
                           static_cast<const float *>(psi), out);
    return hipGetLastError();
}

}  // namespace lbmep
