// lbmep_internal.h -- shared definitions of the gfx950 library (device side
// and host runtime).  Not part of the public ABI (include/lbmep.h).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbmep.h"

namespace lbmep {

constexpr int Q = 19;

// D3Q19 velocity set in the ABI order: q=0 rest, 1..6 axis directions,
// 7..18 diagonals, opposite pairs (2k-1, 2k).  Sec. 3.1 uses Qian et al.'s
// D3Q19 model with weights 1/3, 1/18, 1/36 and c_s^2 = 1/3.
constexpr int kCx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int kCy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int kCz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__host__ __device__ constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
// the direction of q with the components in mask (bit a = axis a) negated
__host__ __device__ constexpr int mirror_dir(int q, int mask) {
    const int wx = (mask & 1) ? -kCx[q] : kCx[q];
    const int wy = (mask & 2) ? -kCy[q] : kCy[q];
    const int wz = (mask & 4) ? -kCz[q] : kCz[q];
    for (int k = 0; k < Q; ++k)
        if (kCx[k] == wx && kCy[k] == wy && kCz[k] == wz) return k;
    return -1;
}
__host__ __device__ constexpr double wq(int q) {
    return q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// cell flag bits (internal encoding of LBMEP_WALL / OBST / NEAR); kUncov
// marks a fluid cell that was an obstacle cell at the previous time level;
// kNear7 (set with kNear) a fluid cell with a face neighbour (q = 1..6)
// that is a wall or obstacle cell or lies beyond a non-periodic edge: the
// cells whose Debye-Hueckel row is not the interior one
constexpr uint8_t kWall = 1, kObst = 2, kNear = 4, kUncov = 8, kNear7 = 16;
// bits q - 1 of a direction mask for the face directions q = 1..6
constexpr uint32_t kFaceDirs = 0x3Fu;
// owner value of a cell no particle covers
constexpr uint32_t kNone = 0xFFFFFFFFu;

// FP16 deviation storage scale: stored h = (f - w) * 2^22.  Deviations
// between 1.5e-11 (smallest normal FP16 / 2^22) and 1.56e-2 (largest FP16 /
// 2^22) keep 11 significant bits; the largest deviations of a flow are the
// moving-wall terms 2 w_q c_q.u_s / c_s^2 (|u_s| / 3 on axis links), so
// velocities up to ~0.04 lattice units fit.
constexpr float kHalfScale = 4194304.0f;
constexpr float kHalfInvScale = 1.0f / 4194304.0f;

// force modes of the sweep
// (dense f_b field; rho_e field times a uniform E; EDL potential psi, with
// f_b = rho_e(psi) (E_ext - grad psi) computed in the sweep)
enum ForceMode { kForceNone = 0, kForceDense = 1, kForceCharge = 2, kForcePotential = 3 };

struct Grid {
    int nx, ny, nz;
    int per[3];
    size_t N;   // nx*ny*nz
    size_t Ns;  // population stride (N rounded up to a multiple of 128)
};

// storage order of the EDL potential psi (Ns values of the compute type).
// For even nx the cells of the two colours of the red-black order
// ((x + y + z) & 1) are kept apart: colour k in [k Ns / 2, k Ns / 2 + N / 2),
// cell c at c >> 1 within its colour (the x-pairs (2i, 2i + 1) of a row hold
// one cell of each colour, so each colour's row is a contiguous run of
// nx / 2 values).  A half-sweep of one colour then reads the other colour's
// array and reads and writes its own, instead of all of psi twice.  For
// odd nx the plain cell order.
__host__ __device__ __forceinline__ bool psi_split(const Grid &g) { return (g.nx & 1) == 0; }
__host__ __device__ __forceinline__ size_t psi_slot(const Grid &g, size_t c, uint32_t colour) {
    return psi_split(g) ? (size_t)colour * (g.Ns >> 1) + (c >> 1) : c;
}
__host__ __device__ __forceinline__ size_t psi_slot_xyz(const Grid &g, int x, int y, int z) {
    const size_t c = (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
    return psi_slot(g, c, (uint32_t)((x + y + z) & 1));
}

// workgroups are dealt to the 8 XCDs round-robin; this remaps them so that
// consecutive segments of a grid (which share cache lines through their
// neighbour reads) run on the same XCD and its L2.  A permutation of
// [0, nblk).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t lb, uint32_t nblk) {
    const uint32_t xcd = lb % 8u, slot = lb / 8u, per = nblk / 8u, rem = nblk % 8u;
    return (xcd < rem ? xcd * (per + 1u) : rem * (per + 1u) + (xcd - rem) * per) + slot;
}

// arguments of the fused stream-collide sweep
// constants of the FP32-compute TRT collision (FP32 and FP16 storage), set
// on the host from lambda_e, lambda_o and the compute unit kC of the storage
// (values are deviations times kC: 1 for FP32, 2^22 for FP16 storage).  Per
// weight class k (w = 1/18 for the axis, 1/36 for the diagonal directions):
//   lw = le w, m = 3 ae w / kC, k1 = 9/2 le w / kC, k3 = 9 ae w / kC,
//   hlo = lo / 6 (axis), lo / 12 (diagonal), k4 = 3 ao w
struct TrtF32 {
    float hle;      // le / 2
    float le;       // le (rest population)
    float b15;      // 3/2 / kC
    float lw0, m0;  // le w_0, 3 ae w_0 / kC
    float lw[2], m[2], k1[2], k3[2], hlo[2], k4[2];
    float fscale;   // kC: a body force in compute units
    float Ec[3];    // charge force: the field times kC
};

struct SweepArgs {
    Grid g;
    const void *src;
    void *dst;
    const uint8_t *flag;
    const uint32_t *nearmask;   // per cell: directions whose neighbour is a wall cell
    const uint32_t *owner;      // map of the current time level
    const uint32_t *owner_old;  // map of the previous time level (refill)
    const double *Xc;  // particle centres of the current time level (3n)
    const double *Xold; // particle centres of the previous time level (3n)
    const double *U;   // 3n
    const double *W;   // 3n
    double *FM;        // 12n accumulators per particle: F_dev, M_dev, K, T; or null
    const void *force; // dense: 3*Ns compute type; charge, potential: Ns compute type
    double E[3];       // charge: the uniform field; potential: E_ext
    double keps;       // potential: kappa^2 eps_e (rho_e = -keps psi)
    const double *zeta; // potential: per-particle boundary value, or null
    double le, lo, ae, ao;  // lambda_e, lambda_o, 1 + lambda_e/2, 1 + lambda_o/2
    TrtF32 tf;              // the same rates for the FP32-compute collision
    int nxb;                // x-segments per row (set by the launcher)
    int xcd_swizzle;        // 1: map consecutive segments onto one XCD
    int slip;               // free-slip faces: bit 2a + side (a = axis, side 1 = high)
    uint32_t lds;           // dynamic LDS bytes per sweep workgroup (caps the waves per CU; 0: none)
    int np;                 // particles
    uint32_t pcap;          // link-list capacity per particle
    const uint2 *plist;     // per particle: (cell, directions into the particle)
    const uint32_t *pcount; // per particle: list length
    const uint32_t *wlist;  // cells with a wall link (fixed while the walls are)
    const uint32_t *wcount; // their number (device)
};

// sweep modes: gather + collide, collide in place, gather only (read-out)
enum SweepMode {
    kSweepPull = 0,     // gather + collide
    kSweepLocal = 1,    // collide in place
    kSweepReadout = 2,  // gather only
    kSweepPullNT = 3,   // gather + collide, streaming hints on loads and stores
    kSweepPullNTS = 4   // gather + collide, streaming hints on stores
};

// particle table of one lattice (device pointers)
struct ParticleArgs {
    Grid g;
    int np;
    int moving;
    int dynamic;       // Newton-Euler dynamics: X0 holds the current positions
    const double *X0, *R, *U, *W;
    uint2 *plist;      // link lists written by the classification
    uint32_t *pcount;
    uint32_t pcap;
    uint32_t halo_cap; // LDS bytes of the classification's staged box (one per cell)
};

// link-list capacity per particle for radii up to r_max: the cells whose
// centre lies within one cell (per axis) of the ball, (2 ceil(R) + 3)^3
uint32_t link_capacity(double r_max);
// LDS bytes that stage the classification box of a particle of radius up to
// r_max moving less than one cell per step, with its halo: (2 ceil(R) + 9)^3,
// at most 32768 (larger boxes are classified from global memory)
uint32_t halo_capacity(double r_max);

// ---------------------------------------------------------------------------
// Packed launches: one dispatch runs a kernel of the step for several
// resident lattices.  Each lattice has a descriptor in device memory; the
// kernel arguments carry a table of entries with the first block of each, and
// every workgroup finds its entry by a binary search over the block starts.
// ---------------------------------------------------------------------------
constexpr int kMaxPack = 64;

struct LatticeDev {
    // sweep arguments by state = cur | cur_owner << 1 (which population grid
    // is the source, which owner map / positions are the current level's)
    SweepArgs sweep[4];
    ParticleArgs pa;
    uint8_t *flag;
    uint32_t *owner[2];
    double *Xheld[2];
    int wall_blocks;  // workgroups of the wall links in the exchange kernel
};

struct PackTable {
    int n;
    int xcd_swizzle;
    uint32_t start[kMaxPack + 1];  // first workgroup of each entry; start[n] = total
    const LatticeDev *d[kMaxPack];
    uint32_t state[kMaxPack];      // cur | cur_owner << 1 before the step
    int64_t level[kMaxPack];       // kinematic level being advanced to (particle kernels)
};

// entry of the workgroup b (the last entry whose first block is <= b)
__device__ __forceinline__ int pack_find(const PackTable &t, uint32_t b) {
    int lo = 0, hi = t.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.start[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// launch shape of the packed sweep (x-segments of 128 cells, one cell per thread)
constexpr int kPackBlockX = 128;

// kernels (host-side launchers); each returns hipError_t of the launch
hipError_t launch_sweep(int precision, int mode, int force_mode, const SweepArgs &a, int block_x,
                        int cpt, hipStream_t s);

// bounce-back slots and momentum exchange after a sweep: one workgroup per
// particle over its link list, then wall_blocks workgroups over the wall list
hipError_t launch_near(int precision, const SweepArgs &a, int wall_blocks, hipStream_t s);
int near_wall_blocks(const Grid &g, bool walls);
// all workgroups of the exchange kernel (particles, then wall links)
int near_blocks(int np, const Grid &g, bool walls);
// compact list, in cell order, of the cells with a wall link (wallmask != 0);
// scratch of wall_list_scratch(g) entries
int wall_list_blocks(const Grid &g);
int wall_list_tiles(const Grid &g);
size_t wall_list_scratch(const Grid &g);
hipError_t launch_wall_list(const Grid &g, const uint32_t *wallmask, uint32_t *list,
                            uint32_t *count, uint32_t *scratch, hipStream_t s);

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s);

// equilibrium everywhere (rho, u)
hipError_t launch_init_equilibrium(int precision, const Grid &g, void *f, double rho,
                                   const double u[3], hipStream_t s);
// absolute FP64 values of population q <-> storage (N values)
hipError_t launch_pdfs_from_f64(int precision, const Grid &g, int q, const double *in, void *f,
                                hipStream_t s);
hipError_t launch_pdfs_to_f64(int precision, const Grid &g, int q, const void *f, double *out,
                              hipStream_t s);
// force conversion into the compute precision
hipError_t launch_convert_force(int precision, const void *in, int in_dtype, void *out,
                                size_t n, size_t in_stride, size_t out_stride, int ncomp,
                                hipStream_t s);
// macroscopic read-out
hipError_t launch_macro(int precision, int force_mode, const Grid &g, const void *f,
                        const uint8_t *flag, const uint32_t *owner, const double *Xc,
                        const double *U, const double *W, const void *force,
                        const double E[3], double keps, const double *zeta, double *rho,
                        double *u, hipStream_t s);
// Debye-Hueckel equation of the EDL potential by red-black SOR: control
// block in device memory (the kernels of a solve stop once done is set)
struct SorCtl {
    int32_t done;
    int32_t iters;   // iterations of the current / last solve
    uint32_t nnear[2];  // boundary unknowns of each colour (lists of the solve)
    double res0;     // L2 norm of the initial residual (-1: not computed)
    double res;      // L2 norm of the last computed residual (-1: none)
};
struct SorArgs {
    Grid g;
    void *psi;                 // Ns values of the compute type (current iterate)
    void *psi2;                // second buffer of the fused iteration
    const uint8_t *flag;       // map of the current time level
    const uint32_t *owner;     // null without particles
    const double *zeta;        // per-particle Dirichlet value, or null
    double kappa2, omega, rf;
    SorCtl *ctl;
    double *partial;           // kSorPartials FP64 partial sums
    uint32_t *nlist;           // boundary unknowns: colour 0 at [0, N/2 + 1),
                               // colour 1 at [N/2 + 1, N + 2)
    uint32_t *nscratch;        // per-segment counts / offsets of the list build
    void *nrow;                // per list entry: diag and rhs of the row (2 compute values)
    uint8_t *nmask;            // per list entry: bit k = neighbour k is an unknown
    uint32_t *ibits;           // 6 arrays of (N/2 + 31)/32 words: the interior bitmaps of the
                               // two colours, their boundary bitmaps, then the two interior
                               // bitmaps interleaved word by word
    uint32_t xcd_swizzle;
    uint32_t zc;               // planes per workgroup of the interior half-sweep (>= 1)
    uint32_t wx;               // waves along x of its workgroup tile (1, 2 or 4)
    uint32_t rows;             // rows per thread of the tile (4 or 8)
    uint32_t near_blocks;      // workgroups of the boundary list part (0: default; % 8 == 0)
    uint32_t *codes;           // one-pass iteration: per entry the codes of its two cells
    void *save;                // one-pass iteration: obstacle cells' values (Ns compute values)
    uint32_t mzc;              // planes per workgroup of the one-pass iteration (>= 1)
    uint32_t mrw;              // rows per thread of the one-pass iteration (1, 2, 4)
    float rdiag[13];           // FP32: 1 / (6 + kappa^2 + k), k = -6 .. 6, correctly rounded
};
constexpr int kSorPartials = 8192;
// the boundary lists are built per segment of kNearSeg cells
constexpr int kNearSeg = 8192;
inline size_t sor_nlist_entries(size_t N) { return N + 2; }
inline size_t sor_nscratch_entries(size_t N) { return 4 * ((N + kNearSeg - 1) / kNearSeg) + 2; }
// interior bitmaps of the two colours (even nx): 32 entries per word
__host__ __device__ inline size_t sor_ibits_words_per_colour(size_t N) { return (N / 2 + 31) / 32; }
// one solve on the current map: max_iter iterations of (red, black), with
// rf > 0 a residual before the first and after every check_every-th (and the
// last) iteration, stopping at res < rf res0 (the host reads the control
// block every 64 iterations and stops launching once it is done).  fused
// (even nx, rows of up to 2048 cells): one pass per iteration from psi into
// psi2 and back; *swapped = 1 when the result ends in psi2 (the caller swaps
// the buffers).  Otherwise one launch per colour in place.
hipError_t launch_sor_solve(int precision, const SorArgs &a, int max_iter, int check_every,
                            bool fused, hipStream_t s, int *swapped);
hipError_t launch_potential_to_f64(int precision, const Grid &g, const void *psi, double *out,
                                   hipStream_t s);
// psi given in cell order (LBMEP_DTYPE_F32 / F64, device memory) into the
// storage order (psi_slot) of the compute type
hipError_t launch_potential_pack(int precision, const Grid &g, const void *in, int in_dtype,
                                 void *psi, hipStream_t s);

// deterministic FP64 invariants: partial sums per block, then one block
hipError_t launch_invariants(int precision, const Grid &g, const void *f, const uint8_t *flag,
                             double *partials, int nblocks, double *out, hipStream_t s);
int invariants_blocks(const Grid &g);

// particles
hipError_t launch_positions(const ParticleArgs &pa, int64_t level, double *X, hipStream_t s);
hipError_t launch_map_clear(const ParticleArgs &pa, const double *X, uint32_t *owner,
                            hipStream_t s);
hipError_t launch_map_set(const ParticleArgs &pa, const double *X, const uint8_t *flag,
                          uint32_t *owner, hipStream_t s);
// classify cells (flags + wall-link masks) over the whole grid
hipError_t launch_classify_all(const Grid &g, uint8_t *flag, uint32_t *wallmask,
                               const uint32_t *owner, hipStream_t s);
// classify around every particle (union of the boxes at Xold and Xnew,
// grown by one cell), marking uncovered cells for the refill in the sweep,
// and write each particle's link list
hipError_t launch_classify_boxes(const ParticleArgs &pa, const double *Xold, const double *Xnew,
                                 uint8_t *flag, const uint32_t *owner_new,
                                 const uint32_t *owner_old, hipStream_t s);
// final force and torque (6n: F then M per particle) from the 12n sweep
// accumulators and the particle centres of the streamed time level
// Newton-Euler update of every particle from the step's accumulators: U, W
// in place, X0 = the next level's positions; *too_fast = 1 when a velocity
// component reaches one cell per step
struct DynArgs {
    Grid g;
    int np;
    const double *acc;   // 12 per particle (F_dev, M_dev, K, T)
    const double *X;     // current positions
    const double *R;
    const double *q;     // charges or null
    double *U, *W, *X0;
    double rho_p;
    double E[3];
    int32_t *too_fast;
};
hipError_t launch_dynamics(const DynArgs &d, hipStream_t s);
hipError_t launch_finalize_ft(int np, const double *acc, const double *X, double *out,
                              hipStream_t s);
// map read-out in the ABI encoding
hipError_t launch_export_flags(const Grid &g, const uint8_t *flag, uint8_t *out, hipStream_t s);
hipError_t launch_copy16(const void *src, void *dst, size_t bytes, hipStream_t s);
// user flags -> internal wall bits (clears OBST/NEAR)
hipError_t launch_import_flags(const Grid &g, const uint8_t *in, uint8_t *flag, hipStream_t s);


// packed launches (tables filled by the host; entries with no work omitted)
hipError_t launch_sweep_packed(int precision, int force_mode, const PackTable &t, hipStream_t s);
hipError_t launch_near_packed(int precision, const PackTable &t, hipStream_t s);
// clear each particle's cells of the map held two levels back, then move it
// to t.level (one workgroup per particle)
hipError_t launch_advance_packed(const PackTable &t, hipStream_t s);
hipError_t launch_map_set_packed(const PackTable &t, hipStream_t s);
hipError_t launch_classify_packed(const PackTable &t, hipStream_t s);
// single-lattice form of the advance kernel
hipError_t launch_advance(const ParticleArgs &pa, int64_t level, double *X, uint32_t *owner,
                          hipStream_t s);

}  // namespace lbmep
