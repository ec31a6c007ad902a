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
//     psi_i <- (1 - omega) psi_i + omega (rhs_i + sum) / diag_i
// (in FP32 the quotient as a product with the reciprocal, see sor_quot);
// same-coloured cells are never neighbours (even extents along periodic
// axes), so a half-sweep is order-free and each cell is written by one
// thread.  Terms are formed in the order x-, x+, y-, y+, z-, z+, so the
// FP64 kernel rounds like a plain CPU evaluation of the same rows.
//
// psi is stored colour-split for even nx (psi_slot: colour k's cells at
// [k Ns / 2, k Ns / 2 + N / 2), cell c at c >> 1), in cell order for odd nx.
//
// Two implementations of an iteration, bitwise identical:
//   * one pass per iteration (even nx, rows of up to 2048 cells; the
//     default): k_sor_march from psi into a second buffer, every cell of
//     both colours in one z-march (see k_sor_march);
//   * one launch per colour, in place: for even nx k_sor_half_vec, whose
//     workgroups march through chunks of z planes with the other colour's
//     three-plane window in registers (the other colour read once, the own
//     colour read and written once) and relax the listed boundary cells in
//     the same grid; for odd nx k_sor_half, then k_sor_near for the listed
//     cells.
//
// The residual's L2 norm is the root mean square over the unknowns, summed
// in a fixed order (per-thread strided sums, a block tree, one block over
// the blocks), so it is reproducible run to run.
#include "lbmep_internal.h"

namespace lbmep {
namespace {

constexpr int kSorBlock = 256;
constexpr int kResBlock = 256;

// (rhs + sum) / diag of a relaxation: the exact quotient in FP64 (the
// rounding of a plain CPU evaluation); in FP32 the product with the
// reciprocal, which for the interior rows is a constant of the launch (one
// multiplication instead of a correctly rounded division, within one
// rounding of it).  Every FP32 form of an iteration uses it, so they stay
// bitwise equal to each other.
__device__ __forceinline__ double sor_quot(double x, double diag) { return x / diag; }
__device__ __forceinline__ float sor_quot(float x, float diag) { return x * (1.0f / diag); }

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
    if (!(fl & kNear7)) {
        // every face neighbour is an unknown inside the grid (periodic wrap)
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
        if (zeta && !edge[k] && (fs[k] & kObst) && !(fs[k] & kWall)) {
            const uint32_t po = owner[s[k]];
            if (po != kNone) bv[k] = (CT)zeta[po];
        }
    }
    uint8_t um = 0;
    int nd = 0, nn = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (edge[k] || (fs[k] & kWall)) {
            // homogeneous Neumann (edge or wall)
            if constexpr (sizeof(CT) == 8) diag = diag - CT(1.0);
            ++nn;
        } else if (fs[k] & kObst) {
            // Dirichlet on the shared face
            if constexpr (sizeof(CT) == 8) diag = diag + CT(1.0);
            ++nd;
            rhs = rhs + CT(2.0) * bv[k];
        } else {
            sum = sum + pv[k];
            um |= (uint8_t)(1u << k);
        }
    }
    // FP32: the face count added to 6 + kappa^2 at once (see relax_code)
    if constexpr (sizeof(CT) == 4) diag = diag + (CT)(nd - nn);
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
        if (fl[r] & (kWall | kObst | kNear7)) continue;
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
        if (!(fl[r] & (kWall | kObst | kNear7))) {
            // interior cell; boundary cells are relaxed from the list
            const CT diag = CT(6.0) + (CT)a.kappa2, rhs = CT(0);
            CT sum = CT(0);
#pragma unroll
            for (int k = 0; k < 6; ++k) sum = sum + v[r][k];
            const CT old = p ? pair[r][1] : pair[r][0];
            const CT nw = (CT(1.0) - om) * old + om * sor_quot(rhs + sum, diag);
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
__device__ void sor_near_part(const SorArgs &a, int colour, uint32_t b0, uint32_t nb,
                              const CT *src, CT *dst);

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
        sor_near_part<CT>(a, colour, blockIdx.x, nnb, static_cast<const CT *>(a.psi),
                          static_cast<CT *>(a.psi));
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
                const CT nw = (CT(1.0) - om) * O[r] + om * sor_quot(rhs + sum, diag);
                *reinterpret_cast<GlobalPtr<CT>>(
                    uniform_ptr(reinterpret_cast<char *>(qz + ro[r])) + io) = nw;
            }
        }
    }
}

// a boundary unknown: a cell with a solid face neighbour (kNear7) that is
// neither wall nor obstacle; a NEAR cell whose solid neighbours are all
// diagonal has the interior row (the D3Q7 stencil sees only faces)
__device__ __forceinline__ bool near_unknown(uint8_t f) {
    return (f & kNear7) && !(f & (kWall | kObst));
}

// once per solve (even nx): bit e of colour k's interior bitmap = the cell of
// colour k at entry e is an interior unknown (neither wall, obstacle nor
// next to a solid face neighbour); of its boundary bitmap = that cell is a
// boundary unknown.  A thread
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
        if (!(f0 & (kWall | kObst | kNear7))) b[rp] |= 1u << k;
        if (!(f1 & (kWall | kObst | kNear7))) b[rp ^ 1] |= 1u << k;
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
    // both colours' interior words side by side, for the one-pass iteration
    reinterpret_cast<uint2 *>(ibits + 4 * W)[w] = make_uint2(b[0], b[1]);
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
            dha_row<CT>(g, x, y, z, kNear | kNear7, psi, a.flag, a.owner, a.zeta, (CT)a.kappa2, diag, rhs,
                        sum, &mask);
            rows[2 * (base + i)] = diag;
            rows[2 * (base + i) + 1] = rhs;
            a.nmask[base + i] = mask;
        }
    }
}

// the colour's listed boundary cells, entries strided over nb blocks of
// kNearBlock threads (this block: b0); neighbours and old values from src,
// new values into dst (the same buffer in the in-place half-sweeps)
template <typename CT>
__device__ void sor_near_part(const SorArgs &a, int colour, uint32_t b0, uint32_t nb,
                              const CT *src, CT *dst) {
    const Grid &g = a.g;
    const uint32_t n = a.ctl->nnear[colour];
    const size_t base = colour ? g.N / 2 + 1 : 0;
    const CT *rows = static_cast<const CT *>(a.nrow);
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
            v[k] = (mask >> k) & 1 ? src[psi_slot(g, s[k], (uint32_t)colour ^ 1u)] : CT(0);
        const size_t pc = psi_slot(g, c, (uint32_t)colour);
        const CT own = src[pc];
        CT sum = CT(0);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if ((mask >> k) & 1) sum = sum + v[k];
        dst[pc] = (CT(1.0) - om) * own + om * sor_quot(rhs + sum, diag);
    }
}

template <typename CT>
__global__ void __launch_bounds__(kNearBlock) k_sor_near(SorArgs a, int colour, const CT *src,
                                                         CT *dst) {
    if (a.ctl->done) return;
    sor_near_part<CT>(a, colour, blockIdx.x, gridDim.x, src, dst);
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

// ---------------------------------------------------------------------------
// One red-black iteration in one pass (even nx, rows of at most 2048 cells).
// Buffer A holds iterate n and is only read; buffer B receives iterate
// n + 1, every cell of it.  A workgroup holds whole rows (every entry of both
// colours) of RW consecutive y and marches through a chunk of z planes.  At
// step z it forms the new red values of plane z + 1 on its rows and one halo
// row on each side (from A) and the new black values of plane z on its rows
// from the new red values of planes z - 1, z, z + 1, and writes its rows of
// both into B.  Same-coloured cells are never neighbours, so every value is
// formed from the operands of the in-place red-black sweep, in the same
// order: the result is bitwise that sweep's.  A is read once per iteration
// (the halo rows, re-read by the neighbouring tiles, mostly from L2) and B
// written once.
// Rows are formed from per-solve codes (k_sor_prepare): an interior unknown's
// code is implied by its interior bit (1 bit per cell, always read); the
// 16-bit code of any other cell is read only when its bit is clear.  With
// surface potentials, the obstacle cells hold their particle's zeta during
// the solve (k_sor_prepare / k_dirichlet_restore), so a Dirichlet value is
// the neighbour's value like any other.
// The x-neighbours come from the neighbouring lane (DPP wavefront rotate)
// and, at the ends of a wavefront, from the end values that every wavefront
// leaves in LDS (double-buffered by step parity: one barrier per step).
constexpr int kMarchMaxWaves = 16;  // rows of up to 2048 cells

template <typename CT>
__device__ __forceinline__ CT dpp_rot(CT v, int ctrl);
template <>
__device__ __forceinline__ float dpp_rot<float>(float v, int ctrl) {
    // ctrl is a constant at every call site after inlining; a wavefront
    // rotate has a source lane for every lane, so no old value is needed
    return ctrl == 0x13C ? __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x13C, 0xF, 0xF, false))
                         : __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x134, 0xF, 0xF, false));
}
template <>
__device__ __forceinline__ double dpp_rot<double>(double v, int ctrl) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    int lo, hi;
    if (ctrl == 0x13C) {
        lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x13C, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x13C, 0xF, 0xF, false);
    } else {
        lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x134, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x134, 0xF, 0xF, false);
    }
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) |
                                            (unsigned long long)(uint32_t)lo));
}
// bitwise select: b where the lane's mask m is all ones, a where it is zero
// (a bit operation, so a load feeding b is not moved under a lane branch)
__device__ __forceinline__ float sel_lane(float a, float b, uint32_t m) {
    return __uint_as_float((__float_as_uint(a) & ~m) | (__float_as_uint(b) & m));
}
__device__ __forceinline__ double sel_lane(double a, double b, uint32_t m) {
    const unsigned long long mm = ((unsigned long long)m << 32) | m;
    return __longlong_as_double((long long)(((unsigned long long)__double_as_longlong(a) & ~mm) |
                                            ((unsigned long long)__double_as_longlong(b) & mm)));
}
// value of lane l - 1 (wave_ror:1) and of lane l + 1 (wave_rol:1)
template <typename CT>
__device__ __forceinline__ CT lane_prev(CT v) { return dpp_rot<CT>(v, 0x13C); }
template <typename CT>
__device__ __forceinline__ CT lane_next(CT v) { return dpp_rot<CT>(v, 0x134); }

// code of an interior unknown: an unknown whose six neighbours are unknowns
// (and the word of an entry whose two cells are)
constexpr uint32_t kCodeInterior = 0x8000u;
constexpr uint32_t kCodePairInterior = 0x80008000u;

// the row of a cell from its code (see sor_code), its old value and its
// six neighbours' values in the order x-, x+, y-, y+, z-, z+; the terms in
// dha_row's order (adding 0 where dha_row adds nothing changes no bit)
template <typename CT>
__device__ __forceinline__ CT relax_code(uint32_t code, CT own, const CT (&nb)[6], CT om, CT om1,
                                         CT diag0, const float *rd) {
    // the interior form when every lane of the wavefront holds an interior
    // unknown (a uniform branch); otherwise the general form for all lanes,
    // which for an interior code adds the same terms in the same order
    // (zeros where the interior form adds nothing) and divides by the same
    // diagonal, so the lanes' bits do not depend on their neighbours
    if (__ballot(code != kCodeInterior) == 0ull) {
        CT sum = CT(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) sum = sum + nb[k];
        return om1 * own + om * sor_quot(CT(0) + sum, diag0);
    }
    // diag = 6 + kappa^2 + (Dirichlet faces) - (Neumann faces): in FP64 the
    // +-1 of each face in direction order (a plain CPU evaluation's
    // rounding); in FP32 the face count added at once, as dha_row does for
    // FP32, and sor_quot's reciprocal of it read from the table rd (the 13
    // correctly rounded values, so the same bits as the division); rhs and
    // sum add their terms in direction order (a skipped term adds an exact 0)
    CT diag = diag0, rhs = CT(0), sum = CT(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const uint32_t t = (code >> (2 * k)) & 3u;
        if constexpr (sizeof(CT) == 8) diag = diag + (t == 1u ? CT(-1.0) : (t == 2u ? CT(1.0) : CT(0.0)));
        rhs = rhs + (t == 2u ? CT(2.0) * nb[k] : CT(0.0));
        sum = sum + (t == 0u ? nb[k] : CT(0.0));
    }
    CT nw;
    if constexpr (sizeof(CT) == 4) {
        const int k = 6 + __builtin_popcount(code & 0xAAAu) - __builtin_popcount(code & 0x555u);
        nw = om1 * own + om * ((rhs + sum) * rd[k]);
    } else {
        nw = om1 * own + om * sor_quot(rhs + sum, diag);
    }
    return (code & 0x8000u) ? nw : own;
}

template <typename CT, int RW, int MAXW>
__global__ void __launch_bounds__(64 * MAXW) k_sor_march(SorArgs a, const CT *A, CT *B, uint32_t nyb,
                                                         uint32_t zc) {
    if (a.ctl->done) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->iters += 1;
    // end values of each wavefront's rows: [step parity][row][wavefront][first, last]
    __shared__ CT e_old[2][RW + 2][MAXW][2];  // black, old, plane z + 1
    __shared__ CT e_new[2][RW][MAXW][2];      // red, new, plane z + 1
    __shared__ float rd[16];                  // FP32: the reciprocals of the diagonals
    if (threadIdx.x < 13) rd[threadIdx.x] = a.rdiag[threadIdx.x];  // read after a barrier
    const Grid &g = a.g;
    const uint32_t lb = a.xcd_swizzle ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint32_t zb = lb / nyb, yb = lb - zb * nyb;  // neighbouring y-blocks share an XCD
    const int y0 = (int)yb * RW;
    const int zs = (int)(zb * zc), ze = min(zs + (int)zc, g.nz);
    const int hx = g.nx >> 1;  // entries of one colour per row
    const int nw = (int)(blockDim.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int i = 64 * w + lane;
    const bool act = i < hx;
    const uint32_t ic = act ? (uint32_t)i : (uint32_t)(hx - 1);  // in-range entry for the rest
    const int lw = min(63, hx - 1 - 64 * w);                      // last lane holding an entry
    const int wl = (w + nw - 1) % nw, wr = (w + 1) % nw;          // wavefronts holding i - 1, i + 1
    const uint32_t m_0 = lane == 0 ? ~0u : 0u, m_lw = lane == lw ? ~0u : 0u;  // lane masks
    const size_t hxs = (size_t)hx, hxy = hxs * (size_t)g.ny, half = g.Ns >> 1;
    const CT *Ar = A, *Ab = A + half;  // colour 0 (red) and colour 1 (black)
    CT *Br = B, *Bb = B + half;
    const uint2 *mb = reinterpret_cast<const uint2 *>(a.ibits + 4 * sor_ibits_words_per_colour(g.N));
    const uint32_t *codes = a.codes;
    // rows -2 .. RW + 1 of the tile: wrapped y and entry offset
    int yr[RW + 4];
    size_t ro_[RW + 4];
#pragma unroll
    for (int k = 0; k < RW + 4; ++k) {
        int y = (y0 + k - 2) % g.ny;
        if (y < 0) y += g.ny;
        yr[k] = y;
        ro_[k] = hxs * (size_t)y;
    }
    auto zwrap = [&](int z) {  // z within two planes of the grid: one step
        int v = z;
        if (v < 0) v += g.nz;
        else if (v >= g.nz) v -= g.nz;
        if (v < 0 || v >= g.nz) {
            v %= g.nz;
            if (v < 0) v += g.nz;
        }
        return v;
    };
    const uint32_t io = ic * (uint32_t)sizeof(CT), ico = ic * 4u;
    auto ld = [&](const CT *row) -> CT {
        return *reinterpret_cast<GlobalPtr<const CT>>(
            uniform_ptr(reinterpret_cast<const char *>(row)) + io);
    };
    auto ldc = [&](size_t e0) -> uint32_t {  // the code pair of the lane's entry in row e0
        return *reinterpret_cast<GlobalPtr<const uint32_t>>(
            uniform_ptr(reinterpret_cast<const char *>(codes + e0)) + ico);
    };
    auto st = [&](CT *row, CT v) {
        *reinterpret_cast<GlobalPtr<CT>>(uniform_ptr(reinterpret_cast<char *>(row)) + io) = v;
    };
    // interior bits of the lane's entry in row k of the plane at entry
    // offset pzo: red into bit kr of rb, black into bit kb of bb
    auto bits = [&](size_t pzo, int k, uint32_t &rb, int kr, uint32_t &bb, int kb) {
        const uint32_t e = (uint32_t)(pzo + ro_[k]) + ic;
        const uint2 m = mb[e >> 5];
        rb |= ((m.x >> (e & 31)) & 1u) << kr;
        if (kb >= 0) bb |= ((m.y >> (e & 31)) & 1u) << kb;
    };
    const CT om = (CT)a.omega, om1 = CT(1.0) - om;
    const CT diag0 = CT(6.0) + (CT)a.kappa2;

    // windows: black old of planes z (rows -1..RW), z + 1 (rows -2..RW+1),
    // z + 2 (rows -1..RW); red new of planes z - 1 (rows 0..RW-1), z and
    // z + 1 (rows -1..RW)
    CT Bo0[RW + 2], Bo1[RW + 4], Bo2[RW + 2], Rm[RW], R0[RW + 2], R1[RW + 2];
    // interior bits: red of plane z + 1, black of planes z and z + 1
    uint32_t rb1 = 0, bb0 = 0, bb1 = 0;
    {
        const CT *p0 = Ab + hxy * (size_t)zwrap(zs - 2), *p1 = Ab + hxy * (size_t)zwrap(zs - 1);
#pragma unroll
        for (int r = 0; r < RW + 2; ++r) {
            Bo0[r] = ld(p0 + ro_[r + 1]);
            Bo1[r + 1] = ld(p1 + ro_[r + 1]);
            bits(hxy * (size_t)zwrap(zs - 1), r + 1, rb1, r, bb1, r >= 1 && r <= RW ? r - 1 : -1);
        }
#pragma unroll
        for (int r = 0; r < RW + 2; ++r) R0[r] = CT(0);
#pragma unroll
        for (int r = 0; r < RW; ++r) Rm[r] = CT(0);
    }
    // wrapped planes z, z + 1, z + 2 and their entry offsets, carried from
    // step to step
    int zw = zwrap(zs - 2), zw1 = zwrap(zs - 1), zw2 = zwrap(zs);
    size_t pz = hxy * (size_t)zw, pz1 = hxy * (size_t)zw1, pz2 = hxy * (size_t)zw2;
    for (int z = zs - 2; z < ze; ++z) {
        const int par = (z - zs + 2) & 1;
        // plane z + 2 of the black window, the two outer rows of plane z + 1,
        // the red old values of plane z + 1, the bits of plane z + 2, and the
        // code words of the cells to be relaxed that are not interior
        // unknowns (as loaded: the colour is taken apart at its use, so that
        // the conditional loads need no wait here)
        Bo1[0] = ld(Ab + pz1 + ro_[0]);
        Bo1[RW + 3] = ld(Ab + pz1 + ro_[RW + 3]);
        CT Ro1[RW + 2];
        uint32_t Cr[RW + 2], Cb[RW];
        uint32_t rb2 = 0, bb2 = 0;
#pragma unroll
        for (int r = 0; r < RW + 2; ++r) {
            Bo2[r] = ld(Ab + pz2 + ro_[r + 1]);
            Ro1[r] = ld(Ar + pz1 + ro_[r + 1]);
            Cr[r] = kCodePairInterior;
            if (!((rb1 >> r) & 1u)) Cr[r] = ldc(pz1 + ro_[r + 1]);
            bits(pz2, r + 1, rb2, r, bb2, r >= 1 && r <= RW ? r - 1 : -1);
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            Cb[r] = kCodePairInterior;
            if (z >= zs && !((bb0 >> r) & 1u)) Cb[r] = ldc(pz + ro_[r + 2]);
        }
        // end values of the black rows of plane z + 1 (lane 0 the first, lane
        // lw the last; one lane holds both when the wavefront has one entry)
        if (lw == 0) {
            if (lane == 0) {
#pragma unroll
                for (int r = 0; r < RW + 2; ++r) e_old[par][r][w][0] = e_old[par][r][w][1] = Bo1[r + 1];
            }
        } else if (lane == 0 || lane == lw) {
            const int side = lane == 0 ? 0 : 1;
#pragma unroll
            for (int r = 0; r < RW + 2; ++r) e_old[par][r][w][side] = Bo1[r + 1];
        }
        __syncthreads();
        // new red values of plane z + 1, rows -1 .. RW (index r = row + 1)
#pragma unroll
        for (int r = 0; r < RW + 2; ++r) {
            const int p = (yr[r + 1] + zw1) & 1;  // the red cell of entry i is x = 2i + p
            const CT own = Bo1[r + 1];
            // p is uniform: one rotate, and the value beyond the wavefront's
            // end (one LDS word, read by every lane) for lane 0's x- (p = 0)
            // or lane lw's x+ (p = 1)
            CT xm, xp;
            if (p) {
                xm = own;
                xp = sel_lane(lane_next(own), e_old[par][r][wr][0], m_lw);
            } else {
                xm = sel_lane(lane_prev(own), e_old[par][r][wl][1], m_0);
                xp = own;
            }
            const CT nb[6] = {xm, xp, Bo1[r], Bo1[r + 2], Bo0[r], Bo2[r]};
            R1[r] = relax_code<CT>(Cr[r] & 0xFFFFu, Ro1[r], nb, om, om1, diag0, rd);
        }
        if (act && z + 1 >= zs && z + 1 < ze) {
#pragma unroll
            for (int r = 1; r <= RW; ++r) st(Br + pz1 + ro_[r + 1], R1[r]);
        }
        if (lw == 0) {
            if (lane == 0) {
#pragma unroll
                for (int r = 0; r < RW; ++r) e_new[par][r][w][0] = e_new[par][r][w][1] = R1[r + 1];
            }
        } else if (lane == 0 || lane == lw) {
            const int side = lane == 0 ? 0 : 1;
#pragma unroll
            for (int r = 0; r < RW; ++r) e_new[par][r][w][side] = R1[r + 1];
        }
        // new black values of plane z, rows 0 .. RW - 1, from the new red
        // values of planes z - 1, z, z + 1 (the end values of plane z were
        // left in LDS at the previous step)
        if (z >= zs) {
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const int p = (1 + yr[r + 2] + zw) & 1;  // the black cell of entry i
                const CT own = R0[r + 1];
                CT xm, xp;
                if (p) {
                    xm = own;
                    xp = sel_lane(lane_next(own), e_new[par ^ 1][r][wr][0], m_lw);
                } else {
                    xm = sel_lane(lane_prev(own), e_new[par ^ 1][r][wl][1], m_0);
                    xp = own;
                }
                const CT nb[6] = {xm, xp, R0[r], R0[r + 2], Rm[r], R1[r + 1]};
                const CT v = relax_code<CT>(Cb[r] >> 16, Bo0[r + 1], nb, om, om1, diag0, rd);
                if (act) st(Bb + pz + ro_[r + 2], v);
            }
        }
        // slide the windows one plane up
#pragma unroll
        for (int r = 0; r < RW + 2; ++r) {
            Bo0[r] = Bo1[r + 1];
            Bo1[r + 1] = Bo2[r];
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) Rm[r] = R0[r + 1];
#pragma unroll
        for (int r = 0; r < RW + 2; ++r) R0[r] = R1[r];
        rb1 = rb2;
        bb0 = bb1;
        bb1 = bb2;
        zw = zw1;
        zw1 = zw2;
        pz = pz1;
        pz1 = pz2;
        if (++zw2 == g.nz) zw2 = 0;
        pz2 = hxy * (size_t)zw2;
    }
}

// the code of cell (x, y, z) for the one-pass iteration (both colours of an
// entry share one word, colour 0 low).  Bit 15: the cell is an unknown;
// bits 2k, 2k + 1: how its neighbour in direction k (x-, x+, y-, y+, z-,
// z+) enters its row, as in dha_row: 0 an unknown (its value is summed), 1 a
// wall or beyond a non-periodic edge (homogeneous Neumann: diag - 1), 2 an
// obstacle cell (Dirichlet on the shared face: diag + 1, rhs + 2 b).  Walls
// and obstacle cells: 0.
__device__ __forceinline__ uint32_t sor_code(const Grid &g, const uint8_t *flag, int x, int y,
                                             int z) {
    const size_t nx = (size_t)g.nx, nxy = (size_t)g.nx * (size_t)g.ny;
    if (flag[(size_t)x + nx * (size_t)y + nxy * (size_t)z] & (kWall | kObst)) return 0u;
    uint32_t code = 0x8000u;
    const int len[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int v[3] = {x, y, z};
        const int ax = k >> 1;
        v[ax] += (k & 1) ? 1 : -1;
        if (v[ax] < 0 || v[ax] >= len[ax]) {
            if (!g.per[ax]) {
                code |= 1u << (2 * k);
                continue;
            }
            v[ax] = v[ax] < 0 ? v[ax] + len[ax] : v[ax] - len[ax];
        }
        const uint8_t fs = flag[(size_t)v[0] + nx * (size_t)v[1] + nxy * (size_t)v[2]];
        if (fs & kWall) code |= 1u << (2 * k);
        else if (fs & kObst) code |= 2u << (2 * k);
    }
    return code;
}

// the code of a cell that is an unknown or not, from its own flag and its
// six neighbours' flags in the order x-, x+, y-, y+, z-, z+ (as sor_code)
__device__ __forceinline__ uint32_t code_of_flags(uint32_t self, const uint32_t (&fs)[6]) {
    if (self & (kWall | kObst)) return 0u;
    uint32_t code = 0x8000u;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (fs[k] & kWall) code |= 1u << (2 * k);
        else if (fs[k] & kObst) code |= 2u << (2 * k);
    }
    return code;
}

// once per solve: the code word of every entry (the cells x = 2i, 2i + 1 of
// a row) with a cell that is not an interior unknown (the only words
// k_sor_march reads), and, with surface potentials, zeta into the obstacle
// cells (their own values kept in save and put back by k_dirichlet_restore
// after the solve).  A thread takes one entry in PR consecutive rows
// (grid: entries of a row along x, groups of rows, planes) and issues each
// phase's loads together -- the two flags of every row, the neighbour flags
// of every boundary entry away from the grid faces, the owners, then zeta
// and psi -- so a wavefront waits a few memory round trips, not a few per
// row.  Measured at 512^3 with 4096 spheres (a one-iteration solve): 2 rows
// per thread 0.740 ms, 1 row 0.762, 4 rows 0.745, 8 rows (124 VGPRs)
// 0.871; the restore, with far fewer registers, is fastest with 8 (0.13
// against 0.19 ms with 1); 16 cells per thread with a 64-bit index
// decomposition took 0.53 ms for the prepare alone
constexpr int kPrepareRows = 2;
constexpr int kPrepRows = 8;  // rows per thread of k_dirichlet_restore
template <typename CT, int PR>
__global__ void __launch_bounds__(256) k_sor_prepare(SorArgs a, CT *psi, CT *save, int dirichlet) {
    const Grid &g = a.g;
    const int hx = g.nx >> 1;
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);
    if (i >= hx) return;
    const int y0 = (int)blockIdx.y * PR, z = (int)blockIdx.z;
    const int nr = min(PR, g.ny - y0);  // rows of this thread (>= 1)
    const int x = 2 * i;
    const size_t e0 = ((size_t)z * (size_t)g.ny + (size_t)y0) * (size_t)hx + (size_t)i;
    const uint32_t bnd = kWall | kObst | kNear7;
    uint32_t fp[PR];  // cells x (low byte), x + 1
#pragma unroll
    for (int k = 0; k < PR; ++k)
        fp[k] = k < nr ? *reinterpret_cast<const uint16_t *>(a.flag + 2 * (e0 + (size_t)k * hx)) : 0u;
    // neighbour flags of the boundary entries with no neighbour across a
    // grid face: x - 1, x + 2 (bytes), the pairs in rows y -+ 1 and planes
    // z -+ 1
    const bool xzin = x > 0 && x + 1 < g.nx - 1 && z > 0 && z < g.nz - 1;
    const ptrdiff_t nx = g.nx, nxy = (ptrdiff_t)g.nx * g.ny;
    uint32_t nf[PR][6];
#pragma unroll
    for (int k = 0; k < PR; ++k) {
        const int y = y0 + k;
#pragma unroll
        for (int d = 0; d < 6; ++d) nf[k][d] = 0u;
        if (k < nr && ((fp[k] | (fp[k] >> 8)) & bnd) && xzin && y > 0 && y < g.ny - 1) {
            const uint8_t *c = a.flag + 2 * (e0 + (size_t)k * hx);
            nf[k][0] = c[-1];
            nf[k][1] = c[2];
            nf[k][2] = *reinterpret_cast<const uint16_t *>(c - nx);
            nf[k][3] = *reinterpret_cast<const uint16_t *>(c + nx);
            nf[k][4] = *reinterpret_cast<const uint16_t *>(c - nxy);
            nf[k][5] = *reinterpret_cast<const uint16_t *>(c + nxy);
        }
    }
    // the obstacle cells' owners (surface potentials)
    uint32_t ow[PR][2];
#pragma unroll
    for (int k = 0; k < PR; ++k) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const uint32_t fl = (fp[k] >> (8 * m)) & 0xFFu;
            ow[k][m] = kNone;
            if (dirichlet && k < nr && (fl & kObst) && !(fl & kWall))
                ow[k][m] = a.owner[2 * (e0 + (size_t)k * hx) + (size_t)m];
        }
    }
    // the codes
#pragma unroll
    for (int k = 0; k < PR; ++k) {
        const int y = y0 + k;
        if (k >= nr || !((fp[k] | (fp[k] >> 8)) & bnd)) continue;
        const int pr = (y + z) & 1;  // the red cell of the entry is x + pr
        uint32_t cl, ch;             // codes of cells x and x + 1
        if (xzin && y > 0 && y < g.ny - 1) {
            const uint32_t f0 = fp[k] & 0xFFu, f1 = fp[k] >> 8;
            const uint32_t fs0[6] = {nf[k][0], f1, nf[k][2] & 0xFFu, nf[k][3] & 0xFFu,
                                     nf[k][4] & 0xFFu, nf[k][5] & 0xFFu};
            const uint32_t fs1[6] = {f0, nf[k][1], nf[k][2] >> 8, nf[k][3] >> 8, nf[k][4] >> 8,
                                     nf[k][5] >> 8};
            cl = code_of_flags(f0, fs0);
            ch = code_of_flags(f1, fs1);
        } else {
            cl = sor_code(g, a.flag, x, y, z);
            ch = sor_code(g, a.flag, x + 1, y, z);
        }
        const uint32_t cr = pr ? ch : cl, cb = pr ? cl : ch;
        a.codes[e0 + (size_t)k * hx] = cr | (cb << 16);
    }
    if (!dirichlet) return;
    // zeta into the obstacle cells, their values into save
    CT zv[PR][2], pv[PR][2];
#pragma unroll
    for (int k = 0; k < PR; ++k) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            zv[k][m] = pv[k][m] = CT(0);
            if (ow[k][m] != kNone) {
                const size_t e = e0 + (size_t)k * hx;
                // cell x + m has colour (x + m + y + z) & 1
                const size_t sl = (size_t)((x + m + y0 + k + z) & 1) * (g.Ns >> 1) + e;
                zv[k][m] = (CT)a.zeta[ow[k][m]];
                pv[k][m] = psi[sl];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < PR; ++k) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (ow[k][m] != kNone) {
                const size_t e = e0 + (size_t)k * hx;
                const size_t sl = (size_t)((x + m + y0 + k + z) & 1) * (g.Ns >> 1) + e;
                save[sl] = pv[k][m];
                psi[sl] = zv[k][m];
            }
        }
    }
}

// after the solve: the obstacle cells' own values back into both buffers
// (the result is in either); same grid and phases as k_sor_prepare
template <typename CT>
__global__ void __launch_bounds__(256) k_dirichlet_restore(SorArgs a, CT *p0, CT *p1, const CT *save) {
    const Grid &g = a.g;
    const int hx = g.nx >> 1;
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);
    if (i >= hx) return;
    const int y0 = (int)blockIdx.y * kPrepRows, z = (int)blockIdx.z;
    const int nr = min(kPrepRows, g.ny - y0);
    const int x = 2 * i;
    const size_t e0 = ((size_t)z * (size_t)g.ny + (size_t)y0) * (size_t)hx + (size_t)i;
    uint32_t fp[kPrepRows];
#pragma unroll
    for (int k = 0; k < kPrepRows; ++k)
        fp[k] = k < nr ? *reinterpret_cast<const uint16_t *>(a.flag + 2 * (e0 + (size_t)k * hx)) : 0u;
    uint32_t ow[kPrepRows][2];
#pragma unroll
    for (int k = 0; k < kPrepRows; ++k) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const uint32_t fl = (fp[k] >> (8 * m)) & 0xFFu;
            ow[k][m] = kNone;
            if (k < nr && (fl & kObst) && !(fl & kWall))
                ow[k][m] = a.owner[2 * (e0 + (size_t)k * hx) + (size_t)m];
        }
    }
    CT sv[kPrepRows][2];
#pragma unroll
    for (int k = 0; k < kPrepRows; ++k) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            sv[k][m] = CT(0);
            if (ow[k][m] != kNone) {
                const size_t sl = (size_t)((x + m + y0 + k + z) & 1) * (g.Ns >> 1) + e0 + (size_t)k * hx;
                sv[k][m] = save[sl];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kPrepRows; ++k) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (ow[k][m] != kNone) {
                const size_t sl = (size_t)((x + m + y0 + k + z) & 1) * (g.Ns >> 1) + e0 + (size_t)k * hx;
                p0[sl] = sv[k][m];
                p1[sl] = sv[k][m];
            }
        }
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
    // one pass per iteration: even nx, whole rows in one workgroup, a second
    // buffer; rows per thread: the largest of mrw, mrw / 2, ... dividing ny
    const bool march = fused && vec && hx <= 64 * kMarchMaxWaves && a0.psi2 != nullptr;
    const uint32_t mthreads = 64u * (uint32_t)((hx + 63) / 64);
    // windows of more than 4 rows per thread spill in a kernel bounded for
    // 1024 threads; bounded for 256 (rows of up to 512 cells) 8 rows fit in
    // 130 VGPRs, but at 3 waves per SIMD the march ran slower (512^3 FP32:
    // 0.453 against 0.377 ms per iteration)
    int mrw = a0.mrw >= 4 ? 4 : (a0.mrw >= 2 ? 2 : 1);
    while (g.ny % mrw) mrw >>= 1;
    const uint32_t mzc = a0.mzc >= 1 ? a0.mzc : 16u;
    const uint32_t myb = (uint32_t)(g.ny / mrw);
    const uint32_t mblk = myb * (uint32_t)((g.nz + (int)mzc - 1) / (int)mzc);
    const size_t rblk = (g.N + kResBlock - 1) / kResBlock;
    const int nres = (int)(rblk < (size_t)(kSorPartials / 2) ? rblk : (size_t)(kSorPartials / 2));
    const bool with_res = a0.rf > 0.0;
    SorArgs a = a0;  // a.psi: the buffer holding the current iterate
    {
        // 1 / diag for the 13 diagonals of FP32 rows (IEEE division in
        // single precision, as the kernels' own)
        const float d0 = 6.0f + (float)a0.kappa2;
        for (int k = 0; k < 13; ++k) {
            volatile float d = d0 + (float)(k - 6);
            a.rdiag[k] = 1.0f / d;
        }
    }
    hipLaunchKernelGGL(k_sor_begin, dim3(1), dim3(64), 0, s, a.ctl);
    const bool dirichlet = march && a0.zeta && a0.owner;  // obstacle cells hold zeta meanwhile
    // per-solve passes over the entries: rows of hx entries, then y and z
    const dim3 egrid((uint32_t)((hx + 255) / 256), (uint32_t)((g.ny + kPrepRows - 1) / kPrepRows),
                     (uint32_t)g.nz);
    if (march) {
        // what k_sor_march assumes of its launch: whole rows in one workgroup
        // (at most kMarchMaxWaves wavefronts), rows per thread dividing ny
        if (mthreads > 64u * kMarchMaxWaves || hx < 1 || g.ny % mrw != 0 || myb < 1 || !a0.codes ||
            (dirichlet && !a0.save))
            return hipErrorInvalidValue;
        // the interior bits (one pass over the flags) and the codes of the rows
        const size_t words = sor_ibits_words_per_colour(g.N);
        hipLaunchKernelGGL(k_interior_bits_split, dim3((uint32_t)((words + 255) / 256)), dim3(256),
                           0, s, g, a.flag, a.ibits);
        const dim3 pgrid(egrid.x, (uint32_t)((g.ny + kPrepareRows - 1) / kPrepareRows), egrid.z);
        hipLaunchKernelGGL((k_sor_prepare<CT, kPrepareRows>), pgrid, dim3(256), 0, s, a,
                           static_cast<CT *>(a0.psi), static_cast<CT *>(a0.save), dirichlet ? 1 : 0);
    } else {
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
        if (march) {
            const CT *src = static_cast<const CT *>(a.psi);
            CT *dst = static_cast<CT *>(a.psi == a0.psi ? a0.psi2 : a0.psi);
#define LBMEP_SOR_MARCH(RW, W)                                                                 \
    hipLaunchKernelGGL((k_sor_march<CT, RW, W>), dim3(mblk), dim3(mthreads), 0, s, a, src, dst, \
                       myb, mzc)
            if (mrw == 4) LBMEP_SOR_MARCH(4, kMarchMaxWaves);
            else if (mrw == 2) LBMEP_SOR_MARCH(2, kMarchMaxWaves);
            else LBMEP_SOR_MARCH(1, kMarchMaxWaves);
#undef LBMEP_SOR_MARCH
            a.psi = dst;
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
                                       a, col, static_cast<const CT *>(a.psi),
                                       static_cast<CT *>(a.psi));
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
    // the obstacle cells' own values back, in both buffers (the result is in
    // either)
    if (dirichlet)
        hipLaunchKernelGGL((k_dirichlet_restore<CT>), egrid, dim3(256), 0, s, a,
                           static_cast<CT *>(a0.psi), static_cast<CT *>(a0.psi2),
                           static_cast<const CT *>(a0.save));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the one-pass iterations alternate buffers: which one holds the result
    *swapped = 0;
    if (march) {
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
    if (a.zc < 1) return hipErrorInvalidValue;
    if (fused && !a.psi2) return hipErrorInvalidValue;
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
