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
// psi is stored colour-split for even nx (psi_slot: colour k's cells at
// [k Ns / 2, k Ns / 2 + N / 2), cell c at c >> 1), in cell order for odd nx.
//
// Two implementations of an iteration, bitwise identical:
//   * in use: one launch per colour, in place: for even nx k_sor_half_vec,
//     whose workgroups march through chunks of z planes with the other
//     colour's three-plane window in registers (the other colour read once,
//     the own colour read and written once) and relax the listed boundary
//     cells in the same grid; for odd nx k_sor_half, then k_sor_near for the
//     listed cells;
//   * k_sor_fused (switched off, see launch_sor_solve): one launch per
//     iteration from psi into a second buffer.  A workgroup owns a 64 x 16 tile of (x, y) and a chunk of z
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
// unknown neighbours.  Next to boundaries, the six neighbour flags and
// values are loaded together (then owner and zeta for obstacle neighbours),
// so a boundary cell costs a few round trips, not one per direction; the
// terms are then formed in the fixed order.
template <typename CT>
__device__ __forceinline__ void dha_row(const Grid &g, int x, int y, int z, uint8_t fl,
                                        const CT *psi, const uint8_t *flag,
                                        const uint32_t *owner, const double *zeta, CT kappa2,
                                        CT &diag, CT &rhs, CT &sum, uint8_t *unknown = nullptr) {
    diag = CT(6.0) + kappa2;
    rhs = CT(0);
    sum = CT(0);
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    const size_t nx = (size_t)g.nx, nxy = (size_t)g.nx * (size_t)g.ny;
    const size_t row = nx * (size_t)y + nxy * (size_t)z;
    size_t s[6];
    s[0] = (size_t)xm + row;
    s[1] = (size_t)xp + row;
    s[2] = (size_t)x + nx * (size_t)ym + nxy * (size_t)z;
    s[3] = (size_t)x + nx * (size_t)yp + nxy * (size_t)z;
    s[4] = (size_t)x + nx * (size_t)y + nxy * (size_t)zm;
    s[5] = (size_t)x + nx * (size_t)y + nxy * (size_t)zp;
    // the six neighbours have the other colour (even extents along periodic
    // axes; a neighbour beyond a non-periodic edge is never read)
    const uint32_t oc = (uint32_t)((x + y + z + 1) & 1);
    if (!(fl & kNear)) {
        // every neighbour is an unknown inside the grid (periodic wrap)
#pragma unroll
        for (int k = 0; k < 6; ++k) sum = sum + psi[psi_slot(g, s[k], oc)];
        if (unknown) *unknown = 63;
        return;
    }
    // a neighbour beyond a non-periodic edge: homogeneous Neumann
    bool edge[6];
    edge[0] = x == 0 && !g.per[0];
    edge[1] = x == g.nx - 1 && !g.per[0];
    edge[2] = y == 0 && !g.per[1];
    edge[3] = y == g.ny - 1 && !g.per[1];
    edge[4] = z == 0 && !g.per[2];
    edge[5] = z == g.nz - 1 && !g.per[2];
    uint8_t fs[6];
    CT pv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        fs[k] = edge[k] ? (uint8_t)kWall : flag[s[k]];
        pv[k] = edge[k] ? CT(0) : psi[psi_slot(g, s[k], oc)];
    }
    CT bv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        // Dirichlet value of an obstacle neighbour: zeta of its particle,
        // or psi's value there
        bv[k] = pv[k];
        if (zeta && !edge[k] && (fs[k] & kObst) && !(fs[k] & kWall)) bv[k] = (CT)zeta[owner[s[k]]];
    }
    uint8_t um = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (edge[k] || (fs[k] & kWall)) {
            diag = diag - CT(1.0);  // homogeneous Neumann (edge or wall)
        } else if (fs[k] & kObst) {
            diag = diag + CT(1.0);  // Dirichlet on the shared face
            rhs = rhs + CT(2.0) * bv[k];
        } else {
            sum = sum + pv[k];
            um |= (uint8_t)(1u << k);
        }
    }
    if (unknown) *unknown = um;
}

__global__ void k_sor_begin(SorCtl *ctl) {
    if (threadIdx.x == 0) {
        ctl->done = 0;
        ctl->iters = 0;
        ctl->res0 = -1.0;
        ctl->res = -1.0;
    }
}

// one half-sweep: the interior unknowns of one colour.  A workgroup covers
// 2 kSorBlock cells of kSorRows consecutive rows (y) of one plane; thread t
// owns the pair x = 2t, 2t + 1 of each row and relaxes the one of this
// colour.  It writes the whole pair back (the other cell unchanged: no
// thread changes it in this half-sweep), so every cache line is written
// in full.  Rows are addressed through workgroup-uniform row pointers and a
// per-lane x, so loads take a scalar base and a 32-bit offset.  The flags
// of all its rows are loaded first, then every neighbour value of its
// interior cells, so a wave keeps many loads in flight.
constexpr int kSorRows = 4;

template <typename CT>
__global__ void __launch_bounds__(kSorBlock) k_sor_half(SorArgs a, int colour, int count,
                                                        uint32_t nxb, uint32_t nyb) {
    if (a.ctl->done) return;
    if (count && blockIdx.x == 0 && threadIdx.x == 0) a.ctl->iters += 1;
    const Grid &g = a.g;
    const uint32_t lb = a.xcd_swizzle ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t row = lb / nxb, xb = lb - row * nxb;
    const int y0 = (int)(row % nyb) * kSorRows, z = (int)(row / nyb);
    const int x2 = (int)(xb * (2 * kSorBlock) + 2 * threadIdx.x);
    if (x2 >= g.nx) return;
    const bool two = x2 + 1 < g.nx;  // the pair's second cell exists
    const size_t nx = (size_t)g.nx, nxy = (size_t)g.nx * (size_t)g.ny;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    CT *psi = static_cast<CT *>(a.psi);
    const CT *pz_m = psi + nxy * (size_t)zm, *pz_p = psi + nxy * (size_t)zp;
    CT *pz = psi + nxy * (size_t)z;
    const uint8_t *fz = a.flag + nxy * (size_t)z;
    uint32_t xs[kSorRows];
    uint8_t fl[kSorRows];
    CT pair[kSorRows][2];
#pragma unroll
    for (int r = 0; r < kSorRows; ++r) {
        const int y = y0 + r;
        const uint32_t p = (uint32_t)((colour + y + z) & 1);  // the pair's cell of this colour
        xs[r] = (uint32_t)x2 + p;
        fl[r] = kWall;
        if (y < g.ny) {
            const CT *pr = pz + nx * (size_t)y;
            pair[r][0] = pr[x2];
            if (two) pair[r][1] = pr[x2 + 1];
            if (xs[r] < (uint32_t)g.nx) fl[r] = fz[nx * (size_t)y + xs[r]];
        }
    }
    // interior cells: the six neighbours in the row order x-, x+, y-, y+,
    // z-, z+ (every neighbour an unknown inside the grid)
    CT v[kSorRows][6];
#pragma unroll
    for (int r = 0; r < kSorRows; ++r) {
        if (fl[r] & (kWall | kObst | kNear)) continue;
        const uint32_t x = xs[r];
        const int y = y0 + r;
        const uint32_t xm = x == 0 ? (uint32_t)g.nx - 1 : x - 1;
        const uint32_t xp = x == (uint32_t)g.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
        const CT *pr = pz + nx * (size_t)y;
        v[r][0] = pr[xm];
        v[r][1] = pr[xp];
        v[r][2] = (pz + nx * (size_t)ym)[x];
        v[r][3] = (pz + nx * (size_t)yp)[x];
        v[r][4] = (pz_m + nx * (size_t)y)[x];
        v[r][5] = (pz_p + nx * (size_t)y)[x];
    }
    const CT om = (CT)a.omega;
#pragma unroll
    for (int r = 0; r < kSorRows; ++r) {
        const int y = y0 + r;
        if (y >= g.ny) continue;
        const uint32_t p = xs[r] - (uint32_t)x2;
        if (!(fl[r] & (kWall | kObst | kNear))) {
            // interior cell; boundary cells are relaxed from the list
            const CT diag = CT(6.0) + (CT)a.kappa2, rhs = CT(0);
            CT sum = CT(0);
#pragma unroll
            for (int k = 0; k < 6; ++k) sum = sum + v[r][k];
            const CT old = p ? pair[r][1] : pair[r][0];
            const CT nw = (CT(1.0) - om) * old + om * ((rhs + sum) / diag);
            if (p) pair[r][1] = nw;
            else pair[r][0] = nw;
        }
        CT *pr = pz + nx * (size_t)y;
        pr[x2] = pair[r][0];
        if (two) pr[x2 + 1] = pair[r][1];
    }
}

template <typename CT>
__device__ __forceinline__ CT lane_shift(CT v, int delta) {
    // value of lane (lane + delta) of the wave
    return __shfl(v, (int)(threadIdx.x & 63) + delta, 64);
}

template <typename CT>
__device__ void sor_near_part(const SorArgs &a, int colour, uint32_t b0, uint32_t nb);

// a wave-uniform global pointer, made opaque to the optimiser: loads then
// take it as a scalar base plus the lane's 32-bit offset, instead of a
// per-lane 64-bit address kept in vector registers across the plane loop
template <typename T>
using GlobalPtr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ GlobalPtr<T> uniform_ptr(T *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (GlobalPtr<T>)(((uint64_t)hi << 32) | lo);
}

// the interior half-sweep for even nx, on the colour-split storage of psi,
// marching along z.  Entry i of the row (y, z) of colour k is the cell
// x = 2i + p, p = (k + y + z) & 1; its neighbours all have the other colour:
// x - 1 and x + 1 are entries i - 1 + p and i + p of the other colour's row
// (y, z), and y -+ 1 and z -+ 1 are entry i of the other colour's rows
// (y -+ 1, z) and (y, z -+ 1).  A workgroup is four waves, WX along x and
// 4 / WX along y; lane l of a wave owns entry i of a 64-entry segment (128
// cells) in kSorRows consecutive rows, and the workgroup walks a.zc
// consecutive planes.  Per thread the window of three planes of the other
// colour stays in registers (rows y0 - 1 .. y0 + kSorRows of the plane,
// kSorRows rows of each neighbour plane); moving to the next plane loads
// kSorRows rows of the new plane ahead, the two y-halo rows of the new
// centre plane and the thread's own entries.  The second x-neighbour comes
// from the neighbouring lane (the wave's end lanes load theirs).  The other
// colour is not written in this half-sweep, so reading it early changes
// nothing: every cell gets the same operands, in the same order, as in a
// plane-at-a-time sweep; a half-sweep reads the other colour once and reads
// and writes its own once.
constexpr int kSorWaves = kSorBlock / 64;
constexpr int kSorWaveX = 64;  // entries (of one colour) of a wave's row segment
// workgroup tile: WX waves along x, kSorWaves / WX along y
template <int WX>
constexpr int sor_tile_x() { return WX * kSorWaveX; }
template <int WX, int RW>
constexpr int sor_tile_y() { return (kSorWaves / WX) * RW; }

// RW: rows per thread (4 or 8)
template <typename CT, int WX, int RW>
__global__ void __launch_bounds__(kSorBlock) k_sor_half_vec(SorArgs a, int colour, int count,
                                                            uint32_t nxb, uint32_t nyb,
                                                            uint32_t ninterior) {
    static_assert(kSorWaves % WX == 0, "whole waves along y");
    if (a.ctl->done) return;
    if (count && blockIdx.x == 0 && threadIdx.x == 0) a.ctl->iters += 1;
    // the grid's first blocks (dispatched first, so they overlap the
    // streaming) relax the colour's listed boundary cells: the interior
    // blocks write no boundary cell, and both read only cells of the other
    // colour
    const uint32_t nnb = gridDim.x - ninterior;
    if (blockIdx.x < nnb) {
        sor_near_part<CT>(a, colour, blockIdx.x, nnb);
        return;
    }
    const Grid &g = a.g;
    // tiles in x, then y, then z-chunk order; with the XCD-contiguous order
    // neighbouring tiles (whose halo lines a tile reads) share an L2
    const uint32_t hb = blockIdx.x - nnb;  // nnb % 8 == 0: same XCD as blockIdx.x
    const uint32_t lb = a.xcd_swizzle ? xcd_remap(hb, ninterior) : hb;
    const uint32_t t = lb / nxb, xb = lb - t * nxb;
    const uint32_t zb = t / nyb, yb = t - zb * nyb;
    const int lane = (int)(threadIdx.x & 63);
    // wave-uniform (scalar): rows and planes are addressed by scalar bases
    // plus the lane's 32-bit entry offset
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wx = w % WX, wy = w / WX;
    const int y0 = (int)yb * sor_tile_y<WX, RW>() + wy * RW;
    const int zs = (int)zb * (int)a.zc;
    const int ze = min(zs + (int)a.zc, g.nz);
    const int hx = g.nx >> 1;  // entries of one colour per row
    const int i = (int)xb * sor_tile_x<WX>() + wx * kSorWaveX + lane;
    const bool act = i < hx;  // lanes past the row take part in the shuffles only
    const uint32_t ic = act ? (uint32_t)i : 0u;  // a valid entry for lanes past the row
    const uint32_t il = i == 0 ? (uint32_t)(hx - 1) : (uint32_t)(i - 1);
    const uint32_t ir = i + 1 >= hx ? (uint32_t)(i + 1 - hx) : (uint32_t)(i + 1);
    const size_t hxs = (size_t)hx, hxy = (size_t)hx * (size_t)g.ny;
    CT *psi = static_cast<CT *>(a.psi);
    CT *own = psi + (size_t)colour * (g.Ns >> 1);
    const CT *oth = psi + (size_t)(colour ^ 1) * (g.Ns >> 1);
    const uint32_t *bits_c = a.ibits + (size_t)colour * sor_ibits_words_per_colour(g.N);
    // rows y0 .. y0 + RW - 1 and the two halo rows (in entries),
    // wrapped into the grid (rows a cell needs wrap once; the rows past ny of
    // the last workgroup are the wrapped y + 1 neighbours of its last valid
    // row after the window slides, so they wrap too)
    size_t ro[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) ro[r] = hxs * (size_t)((y0 + r) % g.ny);
    const size_t rlo = hxs * (size_t)(((y0 - 1) % g.ny + g.ny) % g.ny);
    const size_t rhi = hxs * (size_t)((y0 + RW) % g.ny);
    auto plane = [&](const CT *base, int z) -> const CT * {
        const int zw = z < 0 ? z + g.nz : (z >= g.nz ? z - g.nz : z);
        return base + hxy * (size_t)zw;
    };
    // byte offsets of the lane's entries (32-bit: a row is < 4 GiB)
    const uint32_t io = ic * (uint32_t)sizeof(CT), ilo = il * (uint32_t)sizeof(CT),
                   iro = ir * (uint32_t)sizeof(CT);
    auto ld = [&](const CT *row, uint32_t off) -> CT {
        return *reinterpret_cast<GlobalPtr<const CT>>(
            uniform_ptr(reinterpret_cast<const char *>(row)) + off);
    };
    // interior bit of the lane's entry in row r of plane z
    auto bit = [&](int z, int r) -> uint32_t {
        const uint32_t e = (uint32_t)(hxy * (size_t)z + ro[r]) + ic;
        return (bits_c[e >> 5] >> (e & 31)) & 1u;
    };
    // window at the first plane
    CT C[RW + 2], M[RW], P[RW], O[RW];
    uint32_t F = 0;  // bit r: row r's entry is an interior unknown
    {
        const CT *pz = plane(oth, zs), *pm = plane(oth, zs - 1), *pp = plane(oth, zs + 1);
        const CT *qz = plane(own, zs);
        C[0] = ld(pz + rlo, io);
        C[RW + 1] = ld(pz + rhi, io);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            C[r + 1] = ld(pz + ro[r], io);
            M[r] = ld(pm + ro[r], io);
            P[r] = ld(pp + ro[r], io);
            O[r] = ld(qz + ro[r], io);
            F |= bit(zs, r) << r;
        }
    }
    const CT om = (CT)a.omega;
    const CT diag = CT(6.0) + (CT)a.kappa2;
    for (int z = zs; z < ze; ++z) {
        if (z > zs) {
            // slide the window one plane up: the plane behind is the old
            // centre, the centre is the old plane ahead plus its two halo
            // rows, and the new plane ahead and the own entries are loaded
            const CT *pz = plane(oth, z), *pp = plane(oth, z + 1), *qz = plane(own, z);
            C[0] = ld(pz + rlo, io);
            C[RW + 1] = ld(pz + rhi, io);
            F = 0;
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                M[r] = C[r + 1];
                C[r + 1] = P[r];
                P[r] = ld(pp + ro[r], io);
                O[r] = ld(qz + ro[r], io);
                F |= bit(z, r) << r;
            }
        }
        const CT *pz = oth + hxy * (size_t)z;
        CT *qz = own + hxy * (size_t)z;
        // the two x-neighbours: entries i - 1 + p and i + p of the other
        // colour's row; one is the lane's own, the other the neighbouring
        // lane's (p is uniform per row), or a load at the wave's ends
        CT xm[RW], xp[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int p = (colour + y0 + r + z) & 1;
            if (p) {
                xm[r] = C[r + 1];
                xp[r] = lane_shift(C[r + 1], 1);
                if (act && (lane == 63 || i + 1 >= hx)) xp[r] = ld(pz + ro[r], iro);
            } else {
                xp[r] = C[r + 1];
                xm[r] = lane_shift(C[r + 1], -1);
                if (act && (lane == 0 || i == 0)) xm[r] = ld(pz + ro[r], ilo);
            }
        }
        if (act) {
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                if (y0 + r >= g.ny || !((F >> r) & 1u)) continue;
                // interior cell: x-, x+, y-, y+, z-, z+
                const CT nb[6] = {xm[r], xp[r], C[r], C[r + 2], M[r], P[r]};
                CT sum = CT(0);
#pragma unroll
                for (int k = 0; k < 6; ++k) sum = sum + nb[k];
                const CT rhs = CT(0);
                const CT nw = (CT(1.0) - om) * O[r] + om * ((rhs + sum) / diag);
                *reinterpret_cast<GlobalPtr<CT>>(
                    uniform_ptr(reinterpret_cast<char *>(qz + ro[r])) + io) = nw;
            }
        }
    }
}

// a boundary unknown: a NEAR cell that is neither wall nor obstacle
__device__ __forceinline__ bool near_unknown(uint8_t f) {
    return (f & kNear) && !(f & (kWall | kObst));
}

// once per solve (even nx): bit e of colour k's interior bitmap = the cell of
// colour k at entry e is an interior unknown (neither wall, obstacle nor
// NEAR); of its boundary bitmap = that cell is a boundary unknown.  A thread
// covers the 64 cells of 32 entries of each colour, read as four 16-byte
// loads (the flag buffer is padded to 4096 cells; entries past N/2 are not
// taken); a pair (x even, x + 1) has the colours (y + z) & 1 and its flip,
// and the row parity is recomputed only where the pairs cross into a new row.
__global__ void __launch_bounds__(256) k_interior_bits_split(Grid g, const uint8_t *flag,
                                                             uint32_t *ibits) {
    const size_t W = sor_ibits_words_per_colour(g.N);
    const size_t w = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (w >= W) return;
    const size_t e0 = w * 32, half = g.N / 2, c0 = 2 * e0;
    const uint4 *fp = reinterpret_cast<const uint4 *>(flag + c0);
    const uint4 q0 = fp[0], q1 = fp[1], q2 = fp[2], q3 = fp[3];
    const uint32_t fw[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                             q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
    const size_t nx = (size_t)g.nx, ny = (size_t)g.ny;
    size_t yz = c0 / nx, x = c0 - yz * nx;
    uint32_t rp = (uint32_t)((yz % ny + yz / ny) & 1);  // colour of the pair's first cell
    uint32_t b[2] = {0, 0}, nb[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (e0 + k >= half) break;
        const uint32_t f0 = (fw[k >> 1] >> (16 * (k & 1))) & 0xffu;
        const uint32_t f1 = (fw[k >> 1] >> (16 * (k & 1) + 8)) & 0xffu;
        if (!(f0 & (kWall | kObst | kNear))) b[rp] |= 1u << k;
        if (!(f1 & (kWall | kObst | kNear))) b[rp ^ 1] |= 1u << k;
        if (near_unknown((uint8_t)f0)) nb[rp] |= 1u << k;
        if (near_unknown((uint8_t)f1)) nb[rp ^ 1] |= 1u << k;
        x += 2;
        if (x >= nx) {  // nx even: the pairs end exactly at the row end
            x = 0;
            ++yz;
            rp = (uint32_t)((yz % ny + yz / ny) & 1);
        }
    }
    ibits[w] = b[0];
    ibits[W + w] = b[1];
    ibits[2 * W + w] = nb[0];
    ibits[3 * W + w] = nb[1];
}

// even nx: the boundary lists from the boundary bitmaps.  A list segment of
// kNearSeg cells is kNearSeg / 64 words of each colour; one workgroup per
// segment, one thread per word.
constexpr int kWordsPerSeg = kNearSeg / 64;
static_assert(kNearSeg % 64 == 0, "segments of whole words");

// counts of one segment per colour: scratch[2 s + colour]
__global__ void __launch_bounds__(kWordsPerSeg) k_nlist_count_bits(Grid g, const uint32_t *ibits,
                                                                   uint32_t *scratch) {
    const size_t W = sor_ibits_words_per_colour(g.N);
    const size_t w = (size_t)blockIdx.x * kWordsPerSeg + threadIdx.x;
    __shared__ uint32_t t[2][kWordsPerSeg];
#pragma unroll
    for (int k = 0; k < 2; ++k)
        t[k][threadIdx.x] = w < W ? (uint32_t)__popc(ibits[(2 + k) * W + w]) : 0u;
    __syncthreads();
    for (int h = kWordsPerSeg / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            t[0][threadIdx.x] += t[0][threadIdx.x + h];
            t[1][threadIdx.x] += t[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scratch[2 * blockIdx.x] = t[0][0];
        scratch[2 * blockIdx.x + 1] = t[1][0];
    }
}

// each segment writes its boundary unknowns of both colours in increasing
// cell order: the segment's offset (k_nlist_scan), the set bits of the
// words before this one, the set bits below each bit
__global__ void __launch_bounds__(kWordsPerSeg) k_nlist_write_bits(Grid g, const uint32_t *ibits,
                                                                   const uint32_t *scratch,
                                                                   uint32_t nseg, uint32_t *list) {
    const size_t W = sor_ibits_words_per_colour(g.N);
    const size_t half = g.N / 2 + 1;
    const uint32_t s = blockIdx.x;
    const size_t w = (size_t)s * kWordsPerSeg + threadIdx.x;
    uint32_t word[2];
    __shared__ uint32_t t[2][kWordsPerSeg];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        word[k] = w < W ? ibits[(2 + k) * W + w] : 0u;
        t[k][threadIdx.x] = (uint32_t)__popc(word[k]);
    }
    __syncthreads();
    // inclusive Hillis-Steele scan of both colours' counts
    for (int d = 1; d < kWordsPerSeg; d <<= 1) {
        const uint32_t v0 = threadIdx.x >= (unsigned)d ? t[0][threadIdx.x - d] : 0u;
        const uint32_t v1 = threadIdx.x >= (unsigned)d ? t[1][threadIdx.x - d] : 0u;
        __syncthreads();
        t[0][threadIdx.x] += v0;
        t[1][threadIdx.x] += v1;
        __syncthreads();
    }
    const size_t nx = (size_t)g.nx, ny = (size_t)g.ny;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        uint32_t pos = scratch[2 * nseg + 2 * s + k] + t[k][threadIdx.x] - (uint32_t)__popc(word[k]);
        uint32_t m = word[k];
        while (m) {
            const int bit = __ffs(m) - 1;
            m &= m - 1u;
            const size_t ce = 2 * (w * 32 + (size_t)bit);  // the entry's even-x cell
            const size_t yz = ce / nx;
            const uint32_t rp = (uint32_t)((yz % ny + yz / ny) & 1);
            list[(k ? half : 0) + pos] = (uint32_t)(rp == (uint32_t)k ? ce : ce + 1);
            ++pos;
        }
    }
}

// the boundary unknowns (NEAR cells) of each colour, listed once per solve
// (the map is fixed during a solve): counts per segment of kNearSeg cells,
// an exclusive scan over the segments, then each segment writes its cells
// in increasing order
// (the solver requires N < 2^32 - 2, so cell indices fit 32 bits)
__device__ __forceinline__ uint32_t cell_colour(const Grid &g, uint32_t c) {
    const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
    const uint32_t yz = c / nx, x = c - yz * nx;
    const uint32_t z = yz / ny, y = yz - z * ny;
    return (x + y + z) & 1u;
}

constexpr int kNearBlock = 256;
static_assert(kNearSeg % kNearBlock == 0, "segment = whole block passes");


// counts of one segment per colour: scratch[2 s + colour]
__global__ void __launch_bounds__(kNearBlock) k_nlist_count(Grid g, const uint8_t *flag,
                                                            uint32_t *scratch) {
    const size_t c0 = (size_t)blockIdx.x * kNearSeg;
    uint32_t n[2] = {0, 0};
    for (int k = 0; k < kNearSeg / kNearBlock; ++k) {
        const size_t c = c0 + (size_t)k * kNearBlock + threadIdx.x;
        if (c < g.N && near_unknown(flag[c])) n[cell_colour(g, (uint32_t)c)] += 1;
    }
    __shared__ uint32_t s0[kNearBlock], s1[kNearBlock];
    s0[threadIdx.x] = n[0];
    s1[threadIdx.x] = n[1];
    __syncthreads();
    for (int h = kNearBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        scratch[2 * blockIdx.x] = s0[0];
        scratch[2 * blockIdx.x + 1] = s1[0];
    }
}

// one block: exclusive scan of the segment counts of both colours into
// scratch[2 nseg + 2 s + colour]; the totals into the control block
__global__ void __launch_bounds__(1024) k_nlist_scan(uint32_t *scratch, uint32_t nseg, SorCtl *ctl) {
    __shared__ uint32_t t0[1024], t1[1024];
    const uint32_t per = (nseg + 1023) / 1024;
    const uint32_t b = threadIdx.x * per, e = min(b + per, nseg);
    uint32_t a0 = 0, a1 = 0;
    for (uint32_t s = b; s < e; ++s) {
        a0 += scratch[2 * s];
        a1 += scratch[2 * s + 1];
    }
    t0[threadIdx.x] = a0;
    t1[threadIdx.x] = a1;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread sums
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v0 = threadIdx.x >= (unsigned)d ? t0[threadIdx.x - d] : 0;
        const uint32_t v1 = threadIdx.x >= (unsigned)d ? t1[threadIdx.x - d] : 0;
        __syncthreads();
        t0[threadIdx.x] += v0;
        t1[threadIdx.x] += v1;
        __syncthreads();
    }
    uint32_t o0 = t0[threadIdx.x] - a0, o1 = t1[threadIdx.x] - a1;
    for (uint32_t s = b; s < e; ++s) {
        const uint32_t n0 = scratch[2 * s], n1 = scratch[2 * s + 1];
        scratch[2 * nseg + 2 * s] = o0;
        scratch[2 * nseg + 2 * s + 1] = o1;
        o0 += n0;
        o1 += n1;
    }
    if (threadIdx.x == 1023) {
        ctl->nnear[0] = t0[1023];
        ctl->nnear[1] = t1[1023];
    }
}

// each segment writes its boundary unknowns of both colours, in order
__global__ void __launch_bounds__(kNearBlock) k_nlist_write(Grid g, const uint8_t *flag,
                                                            const uint32_t *scratch, uint32_t nseg,
                                                            uint32_t *list) {
    const size_t c0 = (size_t)blockIdx.x * kNearSeg;
    const size_t half = g.N / 2 + 1;
    uint32_t off[2] = {scratch[2 * nseg + 2 * blockIdx.x], scratch[2 * nseg + 2 * blockIdx.x + 1]};
    __shared__ uint32_t w0[kNearBlock / 64], w1[kNearBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = 0; k < kNearSeg / kNearBlock; ++k) {
        const size_t c = c0 + (size_t)k * kNearBlock + threadIdx.x;
        const bool nu = c < g.N && near_unknown(flag[c]);
        const uint32_t col = nu ? cell_colour(g, (uint32_t)c) : 0;
        const uint64_t b0 = __ballot(nu && col == 0), b1 = __ballot(nu && col == 1);
        if (lane == 0) {
            w0[wv] = (uint32_t)__popcll(b0);
            w1[wv] = (uint32_t)__popcll(b1);
        }
        __syncthreads();
        uint32_t p0 = off[0], p1 = off[1];
        for (int v = 0; v < wv; ++v) {
            p0 += w0[v];
            p1 += w1[v];
        }
        const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
        if (nu) {
            if (col == 0) list[p0 + (uint32_t)__popcll(b0 & below)] = (uint32_t)c;
            else list[half + p1 + (uint32_t)__popcll(b1 & below)] = (uint32_t)c;
        }
        for (int v = 0; v < kNearBlock / 64; ++v) {
            off[0] += w0[v];
            off[1] += w1[v];
        }
        __syncthreads();
    }
}

// the boundary unknowns of one colour, from its list (fixed grid, strided)
constexpr int kNearGrid = 2048;
// list blocks in a vector half-sweep (default; measured at 512^3 with 4096
// spheres: 64 / 128 / 256 / 1024 / 8192 blocks -> 0.449 / 0.442 / 0.422 /
// 0.433 / 0.445 ms per iteration)
constexpr int kNearInVec = 256;

// global indices of the six D3Q7 neighbours (periodic wrap; a neighbour
// beyond a non-periodic edge gets the cell itself, never used)
__device__ __forceinline__ void d3q7_neighbours(const Grid &g, uint32_t c, uint32_t s[6]) {
    const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny, nz = (uint32_t)g.nz;
    const uint32_t yz = c / nx, x = c - yz * nx;
    const uint32_t z = yz / ny, y = yz - z * ny;
    const uint32_t row = c - x, plane = nx * ny;
    s[0] = row + (x == 0 ? nx - 1 : x - 1);
    s[1] = row + (x == nx - 1 ? 0 : x + 1);
    s[2] = c - (y == 0 ? 0 : nx) + (y == 0 ? (ny - 1) * nx : 0);
    s[3] = y == ny - 1 ? c - (ny - 1) * nx : c + nx;
    s[4] = z == 0 ? c + (nz - 1) * plane : c - plane;
    s[5] = z == nz - 1 ? c - (nz - 1) * plane : c + plane;
}

// once per solve: the boundary rows of both lists, diag, rhs and the mask of
// unknown neighbours, formed as dha_row forms them (the map and the
// obstacle cells' values are fixed during a solve)
template <typename CT>
__global__ void __launch_bounds__(kNearBlock) k_nlist_rows(SorArgs a) {
    const Grid &g = a.g;
    const size_t half = g.N / 2 + 1;
    const CT *psi = static_cast<const CT *>(a.psi);
    CT *rows = static_cast<CT *>(a.nrow);
    for (int colour = 0; colour < 2; ++colour) {
        const uint32_t n = a.ctl->nnear[colour];
        const size_t base = colour ? half : 0;
        for (uint32_t i = blockIdx.x * kNearBlock + threadIdx.x; i < n;
             i += kNearGrid * kNearBlock) {
            const uint32_t c = a.nlist[base + i];
            const uint32_t yz = c / (uint32_t)g.nx;
            const int x = (int)(c - yz * (uint32_t)g.nx);
            const int z = (int)(yz / (uint32_t)g.ny), y = (int)(yz - (uint32_t)z * (uint32_t)g.ny);
            CT diag, rhs, sum;
            uint8_t mask;
            dha_row<CT>(g, x, y, z, kNear, psi, a.flag, a.owner, a.zeta, (CT)a.kappa2, diag, rhs,
                        sum, &mask);
            rows[2 * (base + i)] = diag;
            rows[2 * (base + i) + 1] = rhs;
            a.nmask[base + i] = mask;
        }
    }
}

// the colour's listed boundary cells, entries strided over nb blocks of
// kNearBlock threads (this block: b0)
template <typename CT>
__device__ void sor_near_part(const SorArgs &a, int colour, uint32_t b0, uint32_t nb) {
    const Grid &g = a.g;
    const uint32_t n = a.ctl->nnear[colour];
    const size_t base = colour ? g.N / 2 + 1 : 0;
    const CT *rows = static_cast<const CT *>(a.nrow);
    CT *psi = static_cast<CT *>(a.psi);
    const CT om = (CT)a.omega;
    for (uint32_t i = b0 * kNearBlock + threadIdx.x; i < n; i += nb * kNearBlock) {
        const uint32_t c = a.nlist[base + i];
        const uint8_t mask = a.nmask[base + i];
        const CT diag = rows[2 * (base + i)], rhs = rows[2 * (base + i) + 1];
        uint32_t s[6];
        d3q7_neighbours(g, c, s);
        // the neighbours have the other colour (even periodic extents)
        CT v[6];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            v[k] = (mask >> k) & 1 ? psi[psi_slot(g, s[k], (uint32_t)colour ^ 1u)] : CT(0);
        const size_t pc = psi_slot(g, c, (uint32_t)colour);
        const CT own = psi[pc];
        CT sum = CT(0);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if ((mask >> k) & 1) sum = sum + v[k];
        psi[pc] = (CT(1.0) - om) * own + om * ((rhs + sum) / diag);
    }
}

template <typename CT>
__global__ void __launch_bounds__(kNearBlock) k_sor_near(SorArgs a, int colour) {
    if (a.ctl->done) return;
    sor_near_part<CT>(a, colour, blockIdx.x, gridDim.x);
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
        const double r = (double)(rhs + sum - diag * psi[psi_slot(g, c, (uint32_t)((x + y + z) & 1))]);
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

// relaxation of unknown cell (x, y, z) with flag fl and old value own.
// get(k) is the current value and flg(k) the flag of the neighbour in
// direction k (x-, x+, y-, y+, z-, z+); at(k) its global index (only taken
// for an obstacle neighbour).  Same terms in the same order as dha_row.
template <typename CT, typename Get, typename Flg, typename At>
__device__ __forceinline__ CT relax(const SorArgs &a, int x, int y, int z, uint8_t fl, CT own,
                                    const CT *psi_old, Get get, Flg flg, At at) {
    const Grid &g = a.g;
    CT diag = CT(6.0) + (CT)a.kappa2, rhs = CT(0), sum = CT(0);
    if (!(fl & kNear)) {
#pragma unroll
        for (int k = 0; k < 6; ++k) sum = sum + get(k);
    } else {
        const int lo[3] = {x == 0, y == 0, z == 0};
        const int hi[3] = {x == g.nx - 1, y == g.ny - 1, z == g.nz - 1};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int ax = k >> 1;
            const bool up = k & 1;
            if ((up ? hi[ax] : lo[ax]) && !g.per[ax]) {
                diag = diag - CT(1.0);
                continue;
            }
            const uint8_t fs = flg(k);
            if (fs & kWall) {
                diag = diag - CT(1.0);
            } else if (fs & kObst) {
                // obstacle cells never change: the old buffer holds b
                const size_t s = at(k);
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
constexpr int kOW = kFTX + 4, kOH = kFTY + 4;  // old planes: two-cell halo
constexpr int kRW = kFTX + 2, kRH = kFTY + 2;  // new red values: one-cell halo
constexpr int kNLoad = (kOH * kOW + kFBlock - 1) / kFBlock;              // 6
constexpr int kNRed = (kRH * (kRW / 2) + kFBlock - 1) / kFBlock;         // 3
constexpr int kNBlack = kFTY * kFTX / kFBlock;                           // 4
static_assert(kFTX == 64 && kFBlock % kFTX == 0, "black phase: one row of 64 per 64 threads");

// v wrapped once into [0, len) on a periodic axis; ok = false outside a
// non-periodic edge and for positions more than one period away (halo
// slots of a tile wider than the grid, which no cell needs)
__device__ __forceinline__ int wrap_axis_or(int v, int len, int per, bool &ok) {
    if (v < 0 || v >= len) {
        if (!per) {
            ok = false;
            return 0;
        }
        v = v < 0 ? v + len : v - len;
        if (v < 0 || v >= len) {
            ok = false;
            return 0;
        }
    }
    ok = true;
    return v;
}

// global index of the neighbour in direction k of in-grid cell (x, y, z)
__device__ __forceinline__ size_t neighbour_index(const Grid &g, int x, int y, int z, int k) {
    int v[3] = {x, y, z};
    const int len[3] = {g.nx, g.ny, g.nz};
    const int ax = k >> 1;
    v[ax] += (k & 1) ? 1 : -1;
    if (v[ax] < 0) v[ax] += len[ax];
    if (v[ax] >= len[ax]) v[ax] -= len[ax];
    return (size_t)v[0] + (size_t)g.nx * ((size_t)v[1] + (size_t)g.ny * (size_t)v[2]);
}

// one red-black iteration src -> dst (see the file comment).  Per-thread
// in-plane offsets are fixed for the whole column of planes; plane j + 2 is
// fetched into registers while plane j is relaxed.  In-plane offsets are
// 32-bit (nx ny < 2^31, checked by the launcher).
template <typename CT>
__global__ void __launch_bounds__(kFBlock) k_sor_fused(SorArgs a, const CT *src, CT *dst,
                                                        int ntx, int nty) {
    if (a.ctl->done) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->iters += 1;
    __shared__ CT s_old[4][kOH * kOW];
    __shared__ uint8_t s_fl[5][kOH * kOW];  // the black phase still reads plane j - 2's
    __shared__ CT s_rn[3][kRH * kRW];
    const Grid &g = a.g;
    const uint32_t lb = a.xcd_swizzle ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const int tx = (int)(lb % (uint32_t)ntx);
    const int ty = (int)((lb / (uint32_t)ntx) % (uint32_t)nty);
    const int tz = (int)(lb / ((uint32_t)ntx * (uint32_t)nty));
    const int X0 = tx * kFTX, Y0 = ty * kFTY, Z0 = tz * kFZC;
    const int Z1 = min(Z0 + kFZC, g.nz);
    const int nx = g.nx;
    const size_t nxy = (size_t)g.nx * (size_t)g.ny;
    const int tid = threadIdx.x;

    // load slots: in-plane offset (-1: outside a non-periodic edge)
    int loff[kNLoad];
#pragma unroll
    for (int m = 0; m < kNLoad; ++m) {
        const int i = tid + m * kFBlock;
        loff[m] = -1;
        if (i < kOH * kOW) {
            const int r = i / kOW, c = i - r * kOW;
            bool okx, oky;
            const int gx = wrap_axis_or(X0 - 2 + c, g.nx, g.per[0], okx);
            const int gy = wrap_axis_or(Y0 - 2 + r, g.ny, g.per[1], oky);
            if (okx && oky) loff[m] = gx + nx * gy;
        }
    }
    auto exists = [&](int j, int &jw) {
        bool ok;
        jw = wrap_axis_or(j, g.nz, g.per[2], ok);
        return ok;
    };
    // plane j of the old values and flags, through registers into its LDS
    // slot (cells outside a non-periodic edge read as walls: never relaxed,
    // never taken as neighbour values)
    CT pv[kNLoad];
    uint8_t fv[kNLoad];
    bool pok = false;
    auto fetch = [&](int j) {
        int jw;
        pok = exists(j, jw);
        const size_t base = nxy * (size_t)jw;
#pragma unroll
        for (int m = 0; m < kNLoad; ++m) {
            pv[m] = CT(0);
            fv[m] = kWall;
            if (pok && loff[m] >= 0) {
                pv[m] = src[base + (size_t)loff[m]];
                fv[m] = a.flag[base + (size_t)loff[m]];
            }
        }
    };
    auto fslot = [&](int j) { return (j - Z0 + 10) % 5; };
    auto stash = [&](int j) {
        const int sl = (j - Z0 + 8) & 3, sf = fslot(j);
#pragma unroll
        for (int m = 0; m < kNLoad; ++m) {
            const int i = tid + m * kFBlock;
            if (i < kOH * kOW) {
                s_old[sl][i] = pv[m];
                s_fl[sf][i] = fv[m];
            }
        }
    };

    fetch(Z0 - 2);
    stash(Z0 - 2);
    fetch(Z0 - 1);
    stash(Z0 - 1);
    fetch(Z0);
    stash(Z0);
    __syncthreads();
    // step j: fetch plane j + 2, relax the red cells of plane j (old planes
    // j - 1 .. j + 1), put plane j + 2 into the value slot plane j - 2 held
    // and into the flag slot of plane j - 3 (the black phase reads the flags
    // of planes j - 2 .. j), then relax the black cells of plane j - 1 (new
    // red planes j - 2 .. j)
    for (int j = Z0 - 1; j <= Z1; ++j) {
        const bool ahead = j + 2 <= Z1 + 1;
        if (ahead) fetch(j + 2);
        // new red values of plane j on the tile and a one-cell ring
        int jw;
        if (exists(j, jw)) {
            const CT *om = s_old[(j - 1 - Z0 + 8) & 3], *o0 = s_old[(j - Z0 + 8) & 3],
                     *op = s_old[(j + 1 - Z0 + 8) & 3];
            const uint8_t *fm = s_fl[fslot(j - 1)], *f0 = s_fl[fslot(j)], *fp = s_fl[fslot(j + 1)];
            CT *rn = s_rn[(j - Z0 + 6) % 3];
#pragma unroll
            for (int m = 0; m < kNRed; ++m) {
                const int i = tid + m * kFBlock;
                if (i >= kRH * (kRW / 2)) break;
                const int r = i / (kRW / 2), k = i - r * (kRW / 2);
                const int c = 2 * k + ((X0 + Y0 + r + j) & 1);  // (x + y + z) even
                const int O = (r + 1) * kOW + (c + 1);          // in the old planes
                const uint8_t fl = f0[O];
                if (fl & (kWall | kObst)) continue;  // also outside a non-periodic edge
                const int gx = X0 - 1 + c < 0 ? X0 - 1 + c + g.nx
                               : X0 - 1 + c >= g.nx ? X0 - 1 + c - g.nx : X0 - 1 + c;
                const int gy = Y0 - 1 + r < 0 ? Y0 - 1 + r + g.ny
                               : Y0 - 1 + r >= g.ny ? Y0 - 1 + r - g.ny : Y0 - 1 + r;
                const int nb[4] = {O - 1, O + 1, O - kOW, O + kOW};
                rn[r * kRW + c] = relax<CT>(
                    a, gx, gy, jw, fl, o0[O], src,
                    [&](int d) { return d < 4 ? o0[nb[d]] : d == 4 ? om[O] : op[O]; },
                    [&](int d) { return d < 4 ? f0[nb[d]] : d == 4 ? fm[O] : fp[O]; },
                    [&](int d) { return neighbour_index(g, gx, gy, jw, d); });
            }
        }
        if (ahead) stash(j + 2);
        __syncthreads();
        // plane j - 1 of the tile: new black values from the new red ones,
        // new red values, unchanged boundary cells
        const int jj = j - 1;
        if (jj >= Z0) {
            int jjw;
            exists(jj, jjw);
            const CT *o0 = s_old[(jj - Z0 + 8) & 3];
            const uint8_t *fm = s_fl[fslot(jj - 1)], *f0 = s_fl[fslot(jj)],
                          *fp = s_fl[fslot(jj + 1)];
            const CT *rm = s_rn[(jj - 1 - Z0 + 6) % 3], *r0 = s_rn[(jj - Z0 + 6) % 3],
                     *rp = s_rn[(jj + 1 - Z0 + 6) % 3];
            const size_t base = nxy * (size_t)jjw;
            const int c = tid % kFTX;
            const int gx = X0 + c;
#pragma unroll
            for (int m = 0; m < kNBlack; ++m) {
                const int r = tid / kFTX + m * (kFBlock / kFTX);
                const int gy = Y0 + r;
                if (gx >= g.nx || gy >= g.ny) continue;
                const int O = (r + 2) * kOW + (c + 2), Rr = (r + 1) * kRW + (c + 1);
                const uint8_t fl = f0[O];
                CT out;
                if (fl & (kWall | kObst)) {
                    out = o0[O];
                } else if (((gx + gy + jjw) & 1) == 0) {
                    out = r0[Rr];
                } else {
                    const int nr[4] = {Rr - 1, Rr + 1, Rr - kRW, Rr + kRW};
                    const int nb[4] = {O - 1, O + 1, O - kOW, O + kOW};
                    out = relax<CT>(
                        a, gx, gy, jjw, fl, o0[O], src,
                        [&](int d) { return d < 4 ? r0[nr[d]] : d == 4 ? rm[Rr] : rp[Rr]; },
                        [&](int d) { return d < 4 ? f0[nb[d]] : d == 4 ? fm[O] : fp[O]; },
                        [&](int d) { return neighbour_index(g, gx, gy, jjw, d); });
                }
                dst[base + (size_t)(gx + nx * gy)] = out;
            }
        }
        __syncthreads();
    }
}

template <typename CT>
__global__ void k_to_f64(Grid g, const CT *psi, double *out) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    const size_t yz = c / (size_t)g.nx, x = c - yz * (size_t)g.nx;
    const uint32_t col = (uint32_t)((x + yz % (size_t)g.ny + yz / (size_t)g.ny) & 1);
    out[c] = (double)psi[psi_slot(g, c, col)];
}

// psi in cell order (input type TI) into the storage order of the compute type
template <typename TI, typename CT>
__global__ void k_psi_pack(Grid g, const TI *in, CT *psi) {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.N) return;
    const size_t yz = c / (size_t)g.nx, x = c - yz * (size_t)g.nx;
    const uint32_t col = (uint32_t)((x + yz % (size_t)g.ny + yz / (size_t)g.ny) & 1);
    psi[psi_slot(g, c, col)] = (CT)in[c];
}

template <typename CT>
hipError_t sor_solve_typed(const SorArgs &a0, int max_iter, int check_every, bool fused,
                           hipStream_t s, int *swapped) {
    const Grid &g = a0.g;
    const uint32_t nxb = (uint32_t)((g.nx + 2 * kSorBlock - 1) / (2 * kSorBlock));
    const uint32_t nyb = (uint32_t)((g.ny + kSorRows - 1) / kSorRows);
    const uint32_t nblk = nxb * nyb * (uint32_t)g.nz;
    // the z-marching interior half-sweep (even nx): tile of wx waves along x
    const int wx = a0.wx == 2 || a0.wx == 4 ? (int)a0.wx : 1;
    const int rw = a0.rows == 8 ? 8 : 4;
    const int hx = g.nx / 2;  // entries of one colour per row
    const uint32_t vxb = (uint32_t)((hx + wx * kSorWaveX - 1) / (wx * kSorWaveX));
    const int tyr = (kSorWaves / wx) * rw;
    const uint32_t vyb = (uint32_t)((g.ny + tyr - 1) / tyr);
    const uint32_t vblk = vxb * vyb * (uint32_t)((g.nz + (int)a0.zc - 1) / (int)a0.zc);
    // even nx: psi is colour-split, the z-marching tiles relax the interior
    const bool vec = (g.nx % 2) == 0;
    const int ntx = (g.nx + kFTX - 1) / kFTX, nty = (g.ny + kFTY - 1) / kFTY;
    const int ntz = (g.nz + kFZC - 1) / kFZC;
    const uint32_t nfused = (uint32_t)ntx * (uint32_t)nty * (uint32_t)ntz;
    const size_t rblk = (g.N + kResBlock - 1) / kResBlock;
    const int nres = (int)(rblk < (size_t)(kSorPartials / 2) ? rblk : (size_t)(kSorPartials / 2));
    const bool with_res = a0.rf > 0.0;
    SorArgs a = a0;  // a.psi: the buffer holding the current iterate
    hipLaunchKernelGGL(k_sor_begin, dim3(1), dim3(64), 0, s, a.ctl);
    if (!fused) {
        const uint32_t nseg = (uint32_t)((g.N + kNearSeg - 1) / kNearSeg);
        if (vec) {
            // one pass over the flags into the bitmaps; the lists from the
            // boundary bitmaps
            const size_t words = sor_ibits_words_per_colour(g.N);
            hipLaunchKernelGGL(k_interior_bits_split, dim3((uint32_t)((words + 255) / 256)),
                               dim3(256), 0, s, g, a.flag, a.ibits);
            hipLaunchKernelGGL(k_nlist_count_bits, dim3(nseg), dim3(kWordsPerSeg), 0, s, g,
                               a.ibits, a.nscratch);
            hipLaunchKernelGGL(k_nlist_scan, dim3(1), dim3(1024), 0, s, a.nscratch, nseg, a.ctl);
            hipLaunchKernelGGL(k_nlist_write_bits, dim3(nseg), dim3(kWordsPerSeg), 0, s, g,
                               a.ibits, a.nscratch, nseg, a.nlist);
        } else {
            hipLaunchKernelGGL(k_nlist_count, dim3(nseg), dim3(kNearBlock), 0, s, g, a.flag,
                               a.nscratch);
            hipLaunchKernelGGL(k_nlist_scan, dim3(1), dim3(1024), 0, s, a.nscratch, nseg, a.ctl);
            hipLaunchKernelGGL(k_nlist_write, dim3(nseg), dim3(kNearBlock), 0, s, g, a.flag,
                               a.nscratch, nseg, a.nlist);
        }
        hipLaunchKernelGGL((k_nlist_rows<CT>), dim3(kNearGrid), dim3(kNearBlock), 0, s, a);
    }
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
            for (int col = 0; col < 2; ++col) {
                if (vec) {
                    // kNearInVec blocks for the boundary list, then the interior blocks
                    const uint32_t nlb = a0.near_blocks ? a0.near_blocks : (uint32_t)kNearInVec;
                    const dim3 grid(vblk + nlb), blk(kSorBlock);
#define LBMEP_SOR_VEC(WX, RW)                                                              \
    hipLaunchKernelGGL((k_sor_half_vec<CT, WX, RW>), grid, blk, 0, s, a, col, col, vxb, vyb, \
                       vblk)
                    if (rw == 8) {
                        if (wx == 4) LBMEP_SOR_VEC(4, 8);
                        else if (wx == 2) LBMEP_SOR_VEC(2, 8);
                        else LBMEP_SOR_VEC(1, 8);
                    } else {
                        if (wx == 4) LBMEP_SOR_VEC(4, 4);
                        else if (wx == 2) LBMEP_SOR_VEC(2, 4);
                        else LBMEP_SOR_VEC(1, 4);
                    }
#undef LBMEP_SOR_VEC
                } else {
                    hipLaunchKernelGGL((k_sor_half<CT>), dim3(nblk), dim3(kSorBlock), 0, s, a,
                                       col, col, nxb, nyb);
                    hipLaunchKernelGGL((k_sor_near<CT>), dim3(kNearGrid), dim3(kNearBlock), 0, s,
                                       a, col);
                }
            }
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
    // the fused iteration is switched off until its plane-ring fix has run
    // on the device (it is also written for the plain cell order of psi,
    // not the colour-split order of even nx): its flag ring shared 4 slots
    // with the values, so the
    // black phase read the z- flags of a plane already replaced by the
    // prefetch (a stale obstacle flag then indexed zeta with kNone)
    if (fused) return hipErrorNotSupported;
    if (a.zc < 1) return hipErrorInvalidValue;
    if (fused && !a.psi2) return hipErrorInvalidValue;
    // the fused kernel keeps 32-bit in-plane offsets
    if ((size_t)a.g.nx * (size_t)a.g.ny >= ((size_t)1 << 31)) fused = false;
    if (precision == LBMEP_FP64)
        return sor_solve_typed<double>(a, max_iter, check_every, fused, s, swapped);
    return sor_solve_typed<float>(a, max_iter, check_every, fused, s, swapped);
}

hipError_t launch_potential_pack(int precision, const Grid &g, const void *in, int in_dtype,
                                 void *psi, hipStream_t s) {
    if (g.N == 0) return hipSuccess;
    const uint32_t nb = (uint32_t)((g.N + 255) / 256);
    const bool in64 = in_dtype == LBMEP_DTYPE_F64;
    if (precision == LBMEP_FP64) {
        if (in64)
            hipLaunchKernelGGL((k_psi_pack<double, double>), dim3(nb), dim3(256), 0, s, g,
                               static_cast<const double *>(in), static_cast<double *>(psi));
        else
            hipLaunchKernelGGL((k_psi_pack<float, double>), dim3(nb), dim3(256), 0, s, g,
                               static_cast<const float *>(in), static_cast<double *>(psi));
    } else {
        if (in64)
            hipLaunchKernelGGL((k_psi_pack<double, float>), dim3(nb), dim3(256), 0, s, g,
                               static_cast<const double *>(in), static_cast<float *>(psi));
        else
            hipLaunchKernelGGL((k_psi_pack<float, float>), dim3(nb), dim3(256), 0, s, g,
                               static_cast<const float *>(in), static_cast<float *>(psi));
    }
    return hipGetLastError();
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
