// potential_impl.h -- electrostatic body force of the electric double layer
// from the EDL potential psi (arXiv:1708.08741, Sec. "Computing Electrostatic
// Forces on Fluid and Particles"): at a fluid cell
//     f_b = rho_e(psi) (E_ext - grad psi),   rho_e = -kappa^2 eps_e psi
// (Eq. ChrgDensDHA).  grad psi is the w_q-weighted difference over the 18
// D3Q19 neighbours divided by the rest weight (Eq. ElPotGradComp, dx = 1)
// where no neighbour is a wall, obstacle or outside a non-periodic edge (the
// cell is not NEAR), and the central D3Q7 difference otherwise, with the
// value at a boundary cell extrapolated from the boundary value (Sec.
// "Boundary Condition Handling for Solver Module"): particle p holds the
// Dirichlet value b_p (zeta_p, or the field's value at the obstacle cell
// when no zeta is given) on the shared face, so the obstacle cell counts
// 2 b_p - psi_c; walls and non-periodic edges are homogeneous Neumann
// boundaries (they count psi_c).  Shared by the sweep and the macroscopic
// read-out; the operation order is fixed, so the FP64 form rounds like a
// plain CPU evaluation.  psi is addressed through psi_slot (colour-split
// order for even nx), with each cell's colour from its own coordinates.
#pragma once
#include "lbmep_internal.h"

namespace lbmep {

// psi at the neighbour (x, y, z) + (dx, dy, dz) seen from a cell of value
// centre: the boundary-extrapolated value at obstacle, wall and beyond-edge
// cells
template <typename CT>
__device__ __forceinline__ CT psi_bc(const Grid &g, int x, int y, int z, int dx, int dy, int dz,
                                     const CT *psi, const uint8_t *flag, const uint32_t *owner,
                                     const double *zeta, CT centre) {
    int v[3] = {x + dx, y + dy, z + dz};
    const int len[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (v[k] < 0 || v[k] >= len[k]) {
            if (!g.per[k]) return centre;
            v[k] = v[k] < 0 ? v[k] + len[k] : v[k] - len[k];
        }
    }
    const size_t s = (size_t)v[0] + (size_t)g.nx * ((size_t)v[1] + (size_t)g.ny * (size_t)v[2]);
    if (flag[s] & kWall) return centre;
    const size_t ps = psi_slot(g, s, (uint32_t)((v[0] + v[1] + v[2]) & 1));
    if (owner) {
        const uint32_t p = owner[s];
        if (p != kNone) {
            const CT b = zeta ? (CT)zeta[p] : psi[ps];
            return CT(2.0) * b - centre;
        }
    }
    return psi[ps];
}

// grad psi of a cell that is not NEAR (Eq. ElPotGradComp): the centre
// value and the w_q-weighted sums over the 18 neighbours, divided by the
// rest weight 1/3, in the fixed order; val(dx, dy, dz) is psi at the
// neighbour (x + dx, y + dy, z + dz).  Every caller uses this one form.
template <typename CT, typename V>
__device__ __forceinline__ void psi_grad_inner(V &&val, CT &pc, CT &g0, CT &g1, CT &g2) {
    pc = val(0, 0, 0);
    CT s0 = CT(0), s1 = CT(0), s2 = CT(0);
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const CT t = (CT)wq(q) * val(kCx[q], kCy[q], kCz[q]);
        if (kCx[q] > 0) s0 = s0 + t;
        if (kCx[q] < 0) s0 = s0 - t;
        if (kCy[q] > 0) s1 = s1 + t;
        if (kCy[q] < 0) s1 = s1 - t;
        if (kCz[q] > 0) s2 = s2 + t;
        if (kCz[q] < 0) s2 = s2 - t;
    }
    g0 = s0 * CT(3.0);
    g1 = s1 * CT(3.0);
    g2 = s2 * CT(3.0);
}

// f_b = rho_e (E_ext - grad psi), rho_e = -kappa^2 eps_e psi (Eq. ChrgDensDHA)
template <typename CT>
__device__ __forceinline__ void edl_force(CT pc, CT g0, CT g1, CT g2, CT keps, CT E0, CT E1,
                                          CT E2, CT &f0, CT &f1, CT &f2) {
    const CT rho_e = -(keps * pc);
    f0 = rho_e * (E0 - g0);
    f1 = rho_e * (E1 - g1);
    f2 = rho_e * (E2 - g2);
}

// the body force at fluid cell (x, y, z) with flag fl
template <typename CT>
__device__ __forceinline__ void potential_force(const Grid &g, int x, int y, int z, uint8_t fl,
                                                const CT *psi, const uint8_t *flag,
                                                const uint32_t *owner, const double *zeta,
                                                CT keps, CT E0, CT E1, CT E2, CT &f0, CT &f1,
                                                CT &f2) {
    CT pc, g0, g1, g2;
    if (!(fl & kNear)) {
        // every neighbour is a fluid cell inside the grid (periodic wrap)
        const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
        const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
        const int xs[3] = {xm, x, xp}, ys[3] = {ym, y, yp}, zs[3] = {zm, z, zp};
        // storage slots of the neighbours: a base per row (y', z') and an
        // offset per column x' (psi_slot written out for the 3 x 3 x 3 block)
        const bool split = psi_split(g);
        const size_t half = split ? (g.Ns >> 1) : 0;
        const size_t rowlen = split ? (size_t)(g.nx >> 1) : (size_t)g.nx;
        size_t xo[3];
        uint32_t xpar[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            xo[i] = split ? (size_t)(xs[i] >> 1) : (size_t)xs[i];
            xpar[i] = (uint32_t)xs[i] & 1u;
        }
        auto slot = [&](int i, int j, int k) -> size_t {
            const size_t rb = rowlen * ((size_t)ys[j] + (size_t)g.ny * (size_t)zs[k]) + xo[i];
            return split && ((xpar[i] ^ (uint32_t)(ys[j] + zs[k])) & 1u) ? rb + half : rb;
        };
        psi_grad_inner<CT>([&](int dx, int dy, int dz) { return psi[slot(dx + 1, dy + 1, dz + 1)]; },
                           pc, g0, g1, g2);
    } else {
        pc = psi[psi_slot_xyz(g, x, y, z)];
        g0 = (psi_bc(g, x, y, z, 1, 0, 0, psi, flag, owner, zeta, pc) -
              psi_bc(g, x, y, z, -1, 0, 0, psi, flag, owner, zeta, pc)) * CT(0.5);
        g1 = (psi_bc(g, x, y, z, 0, 1, 0, psi, flag, owner, zeta, pc) -
              psi_bc(g, x, y, z, 0, -1, 0, psi, flag, owner, zeta, pc)) * CT(0.5);
        g2 = (psi_bc(g, x, y, z, 0, 0, 1, psi, flag, owner, zeta, pc) -
              psi_bc(g, x, y, z, 0, 0, -1, psi, flag, owner, zeta, pc)) * CT(0.5);
    }
    edl_force<CT>(pc, g0, g1, g2, keps, E0, E1, E2, f0, f1, f2);
}

}  // namespace lbmep
