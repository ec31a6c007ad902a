// lattice.h -- the lattice object behind the C ABI and the host-runtime
// helpers shared by the single-lattice API (lbmep_api.hip) and the request
// server (lbmep_server.hip).  Not part of the public ABI.
#pragma once

#include <string>
#include <vector>

#include "lbmep_internal.h"

namespace lbmep {

// source of a lattice's device memory: hipMalloc / hipFree, or a server's
// pre-allocated arena (whose release never synchronises the device)
struct DevHeap {
    virtual ~DevHeap() = default;
    virtual void *alloc(size_t bytes) = 0;  // nullptr when it does not fit
    virtual void release(void *p) = 0;
};

}  // namespace lbmep

struct lbmep_lattice {
    lbmep_config cfg{};
    lbmep::Grid g{};
    hipStream_t stream = nullptr;
    int precision = 0;
    double tau = 0, le = 0, lo = 0, ae = 0, ao = 0;
    void *f[2] = {nullptr, nullptr};
    int cur = 0;
    // false: f[cur] holds the post-stream state of the current level (as set
    // by init / set_pdfs / load); true: f[cur] holds the post-collision
    // populations of the previous level plus the bounce-back slots, from
    // which the sweep (or a read-out) gathers the current state
    bool pmode = false;
    uint8_t *flag = nullptr;
    uint32_t *wallmask = nullptr;     // per cell: directions whose neighbour is a wall
    uint32_t *wall_list = nullptr;    // cells with a wall link
    uint32_t *wall_count = nullptr;   // their number (device)
    uint32_t *wall_scratch = nullptr; // per-block counts of the list scan
    bool has_walls = false;           // any WALL cell (sizes the wall pass)
    // per particle: link lists (and their lengths) of the current level and,
    // with overlapped stepping, of the next level
    uint2 *plist_buf[2] = {nullptr, nullptr};
    uint32_t *pcount_buf[2] = {nullptr, nullptr};
    int lcur = 0;                     // list buffer of the current level
    uint32_t pcap = 0;                // list capacity per particle
    uint32_t halo_cap = 0;            // LDS bytes of the classification's staged box
    size_t plist_entries = 0;         // allocated entries
    uint32_t *owner[2] = {nullptr, nullptr};
    double *Xheld[2] = {nullptr, nullptr};  // positions of the level each map holds
    int cur_owner = 0;
    int ft_buf = 0;  // owner/position buffer of the last streamed time level
    int np = 0;
    size_t np_cap = 0;
    double *X0 = nullptr, *R = nullptr, *U = nullptr, *W = nullptr, *FM = nullptr;
    std::vector<double> hX0, hR, hU, hW;  // host copy of the particle table
    int64_t level = 0;
    int force_mode = lbmep::kForceNone;
    void *force = nullptr;
    size_t force_bytes = 0;
    double E[3] = {0, 0, 0};
    int slip = 0;              // free-slip faces (bit 2a + side)
    // Newton-Euler dynamics of the particles (X0, U, W become state)
    bool dynamic = false;
    double rho_p = 0, Edyn[3] = {0, 0, 0};
    double *q = nullptr;           // device charges (np), or null
    std::vector<double> hq;        // host copy
    int32_t *too_fast = nullptr;   // device flag: a velocity reached 1
    double keps = 0;           // potential force: kappa^2 eps_e
    double *zeta = nullptr;    // potential force: per-particle boundary value (device)
    std::vector<double> hzeta; // host copy (np values, empty: the field's value)
    // red-black SOR for the Debye-Hueckel equation of psi (per-step solve
    // when sor_iters > 0)
    int32_t sor_iters = 0, sor_check = 1;
    double sor_kappa2 = 0, sor_omega = 1.7, sor_rf = 0;
    bool sor_set = false;
    lbmep::SorCtl *sor_ctl = nullptr;
    double *sor_partial = nullptr;
    uint32_t *sor_nlist = nullptr;     // boundary unknowns of each colour
    uint32_t *sor_nscratch = nullptr;  // segment counts / offsets of the list build
    void *sor_nrow = nullptr;          // per list entry: diag, rhs (compute precision)
    uint8_t *sor_nmask = nullptr;      // per list entry: unknown neighbours
    uint32_t *sor_ibits = nullptr;     // interior unknowns, one bit per cell
    void *psi2 = nullptr;      // second psi buffer of the one-pass SOR iteration
    void *sor_save = nullptr;  // one-pass SOR: obstacle cells' values while they hold zeta
    uint32_t *sor_codes = nullptr;  // one-pass SOR: row codes of both colours per entry
    size_t psi2_bytes = 0;
    bool sor_fused = false;    // one-pass iteration (even nx, rows of up to 2048 cells)
    double *red = nullptr;
    int red_blocks = 0;
    int block_x = 128;
    int cpt = 1;  // cells per thread of the sweep (consecutive rows)
    int sor_zc = 8;   // planes per workgroup of the SOR's interior half-sweep (set per precision)
    int sor_wx = 4;   // waves along x of its workgroup tile (1, 2, 4)
    int sor_xcd = 1;  // XCD-contiguous tile order
    int sor_rows = 8; // rows per thread of the tile (4, 8; set per precision)
    int sor_near_blocks = 0;  // workgroups of the SOR's boundary list part (0: default)
    int sor_mzc = 16; // planes per workgroup of the one-pass SOR iteration
    int sor_mrw = 4;  // rows per thread of the one-pass SOR iteration (set per precision)
    int xcd_swizzle = 1;
    int sweep_wgcu = -1;  // sweep: workgroups per CU (0: no cap, -1: per precision and force)
    int sweep_nt = 2;  // streaming hints of the sweep: 0 none, 1 loads + stores, 2 stores
    // overlapped stepping (moving particles, prescribed kinematics): the
    // kinematics, mapping and classification of level n + 1 run on a second
    // stream during the exchange of level n
    bool overlap = false;
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_sweep = nullptr, ev_chain = nullptr;
    bool chain_pending = false;
    bool timing = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    // source of device memory (nullptr: hipMalloc / hipFree)
    lbmep::DevHeap *heap = nullptr;
};

namespace lbmep {
namespace rt {

// records the message of the last failure of the calling thread
int fail(int code, const std::string &msg);

#define LBMEP_HIP_TRY(expr)                                                                   \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::lbmep::rt::fail(LBMEP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t round_up(size_t n, size_t m);
size_t storage_bytes(int precision);
// stride (in elements) between the arrays of two populations: N rounded up
// to 128 plus a pad that staggers the 19 arrays against the HBM channel
// interleave
size_t population_stride(size_t N, int precision);
size_t compute_bytes(int precision);
bool finite_all(const double *p, size_t n);
int check_config(const lbmep_config *cfg);
// device bytes of a lattice (what lbmep_footprint reports)
size_t lattice_bytes(const lbmep_config *cfg, int32_t n_particles, double r_max,
                     int force_mode, bool overlap);

hipError_t dev_alloc(lbmep_lattice *L, void **p, size_t bytes);
void dev_free(lbmep_lattice *L, void *p);

// create / destroy with a given memory source; destroy without sync assumes
// the caller knows that no work of the lattice is pending
int create_lattice(const lbmep_config *cfg, DevHeap *heap, lbmep_lattice **out);
int destroy_lattice(lbmep_lattice *L, bool sync);

ParticleArgs particle_args(const lbmep_lattice *L);
// sweep arguments for a given (cur, cur_owner) state
SweepArgs sweep_args_state(const lbmep_lattice *L, int cur, int cur_owner);
SweepArgs sweep_args(const lbmep_lattice *L);
// gather the post-stream state into the spare grid (after a step)
int materialize(lbmep_lattice *L);
// host bookkeeping of one completed step (the grid / map buffers flip)
void advance_state(lbmep_lattice *L);

}  // namespace rt
}  // namespace lbmep
