// lbmep_api.hip -- host runtime behind the C ABI of include/lbmep.h: lattice
// object, argument checks, device memory, the per-step launch sequence and
// checkpointing.  Every step of the method runs in the device kernels of
// k_stream.hip, k_particles.hip and k_fields.hip.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lattice.h"

using namespace lbmep;
using namespace lbmep::rt;

namespace {
thread_local std::string g_err;
}  // namespace

namespace lbmep {
namespace rt {

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr) LBMEP_HIP_TRY(expr)

size_t round_up(size_t n, size_t m) { return (n + m - 1) / m * m; }

size_t storage_bytes(int precision) {
    return precision == LBMEP_FP64 ? 8 : (precision == LBMEP_FP32DEV ? 4 : 2);
}

// With a stride of exactly N = 2^k elements, the 19 source and 19
// destination streams of the sweep start at the same offset modulo every
// power of two, so the same cell of every population maps to the same HBM
// channel and bank; at 512^3 the pull pattern then moves ~7 % less data per
// second than with the arrays staggered.  The pad (in elements, a multiple
// of 128 so that the colour-split potential's halves stay aligned) is the
// best of a measured sweep per storage size (LBMEP_POP_PAD overrides it).
size_t population_stride(size_t N, int precision) {
    size_t pad = precision == LBMEP_FP64 ? 256 : 2048;
    if (const char *e = std::getenv("LBMEP_POP_PAD")) {
        const long v = std::atol(e);
        if (v >= 0) pad = round_up((size_t)v, 128);
    }
    return round_up(N, 128) + pad;
}

size_t compute_bytes(int precision) { return precision == LBMEP_FP64 ? 8 : 4; }

bool finite_all(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

hipError_t dev_alloc(lbmep_lattice *L, void **p, size_t bytes) {
    if (!L->heap) return hipMalloc(p, bytes);
    *p = L->heap->alloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_free(lbmep_lattice *L, void *p) {
    if (!p) return;
    if (!L->heap)
        hipFree(p);
    else
        L->heap->release(p);
}

}  // namespace rt
}  // namespace lbmep


namespace lbmep {
namespace rt {

int set_device(lbmep_lattice *L) {
    HIP_TRY(hipSetDevice(L->cfg.device));
    return LBMEP_OK;
}

ParticleArgs particle_args(const lbmep_lattice *L) {
    ParticleArgs pa;
    pa.g = L->g;
    pa.np = L->np;
    pa.moving = L->cfg.move_particles;
    pa.dynamic = L->dynamic ? 1 : 0;
    pa.X0 = L->X0;
    pa.R = L->R;
    pa.U = L->U;
    pa.W = L->W;
    pa.plist = L->plist_buf[L->lcur];
    pa.pcount = L->pcount_buf[L->lcur];
    pa.pcap = L->pcap;
    pa.halo_cap = L->halo_cap;
    return pa;
}

// map the particles at `level` into every owner buffer, classify the grid,
// list the cells with wall links, and write the particles' link lists
int remap_all(lbmep_lattice *L) {
    hipStream_t s = L->stream;
    L->lcur = 0;
    const ParticleArgs pa = particle_args(L);
    if (L->np > 0) {
        for (int b = 0; b < 2; ++b) {
            HIP_TRY(launch_fill_u32(L->owner[b], kNone, L->g.N, s));
            HIP_TRY(launch_positions(pa, L->level, L->Xheld[b], s));
            HIP_TRY(launch_map_set(pa, L->Xheld[b], L->flag, L->owner[b], s));
        }
        L->cur_owner = 0;
        L->ft_buf = 0;
        HIP_TRY(launch_fill_f64(L->FM, 0.0, 18 * (size_t)L->np, s));
    }
    HIP_TRY(launch_classify_all(L->g, L->flag, L->wallmask, L->np > 0 ? L->owner[0] : nullptr, s));
    HIP_TRY(launch_wall_list(L->g, L->wallmask, L->wall_list, L->wall_count, L->wall_scratch, s));
    if (L->np > 0)
        HIP_TRY(launch_classify_boxes(pa, L->Xheld[0], L->Xheld[0], L->flag, L->owner[0],
                                      L->owner[0], s));
    return LBMEP_OK;
}

// constants of the FP32-compute collision (see TrtF32), rounded once from
// FP64 products
TrtF32 trt_f32_constants(const lbmep_lattice *L) {
    const double kc = L->precision == LBMEP_FP16DEV ? (double)kHalfScale : 1.0;
    const double le = L->le, lo = L->lo, ae = L->ae, ao = L->ao;
    const double w0 = 1.0 / 3.0, wk[2] = {1.0 / 18.0, 1.0 / 36.0};
    TrtF32 t;
    t.hle = (float)(0.5 * le);
    t.le = (float)le;
    t.b15 = (float)(1.5 / kc);
    t.lw0 = (float)(le * w0);
    t.m0 = (float)(3.0 * ae * w0 / kc);
    for (int k = 0; k < 2; ++k) {
        t.lw[k] = (float)(le * wk[k]);
        t.m[k] = (float)(3.0 * ae * wk[k] / kc);
        t.k1[k] = (float)(4.5 * le * wk[k] / kc);
        t.k3[k] = (float)(9.0 * ae * wk[k] / kc);
        t.hlo[k] = (float)(lo * 3.0 * wk[k]);
        t.k4[k] = (float)(3.0 * ao * wk[k]);
    }
    t.fscale = (float)kc;
    for (int k = 0; k < 3; ++k) t.Ec[k] = (float)L->E[k] * (float)kc;
    return t;
}

SweepArgs sweep_args_state(const lbmep_lattice *L, int cur, int co) {
    SweepArgs a;
    a.g = L->g;
    a.src = L->f[cur];
    a.dst = L->f[1 - cur];
    a.flag = L->flag;
    a.nearmask = L->wallmask;
    const bool parts = L->np > 0;
    a.owner = parts ? L->owner[co] : nullptr;
    a.owner_old = parts ? L->owner[1 - co] : nullptr;
    a.Xc = parts ? L->Xheld[co] : nullptr;
    a.Xold = parts ? L->Xheld[1 - co] : nullptr;
    a.U = L->U;
    a.W = L->W;
    a.FM = parts ? L->FM : nullptr;
    a.force = L->force;
    for (int k = 0; k < 3; ++k) a.E[k] = L->E[k];
    a.le = L->le;
    a.lo = L->lo;
    a.ae = L->ae;
    a.ao = L->ao;
    a.tf = trt_f32_constants(L);
    a.nxb = 0;
    a.xcd_swizzle = L->xcd_swizzle;
    a.slip = L->slip;
    // measured at 512^3 (4096 moving spheres, two repeats): a cap of 4
    // workgroups per CU is fastest for FP32 (3.56-3.71 ms; 3: 4.1-4.5, none:
    // 3.56-3.84) and FP64 (7.03-7.21 ms; none: 7.19-8.06) with a charge or
    // dense force; FP16 and the force from the potential (its neighbour
    // reads of psi want every wave: 4.4-4.6 ms uncapped, 5.8-6.2 with 4) run
    // best uncapped
    int wgcu = L->sweep_wgcu;
    if (wgcu < 0)
        wgcu = L->force_mode == kForcePotential || L->precision == LBMEP_FP16DEV ? 0 : 4;
    a.lds = wgcu > 0 ? (uint32_t)((160 * 1024) / wgcu / 16 * 16) : 0u;
    a.keps = L->keps;
    a.zeta = L->force_mode == kForcePotential ? L->zeta : nullptr;
    a.np = L->np;
    a.pcap = L->pcap;
    a.plist = L->plist_buf[L->lcur];
    a.pcount = L->pcount_buf[L->lcur];
    a.wlist = L->wall_list;
    a.wcount = L->wall_count;
    return a;
}

SweepArgs sweep_args(const lbmep_lattice *L) { return sweep_args_state(L, L->cur, L->cur_owner); }

void advance_state(lbmep_lattice *L) {
    L->ft_buf = L->cur_owner;
    L->cur = 1 - L->cur;
    L->pmode = true;
    if (L->np > 0 && L->cfg.move_particles) {
        L->cur_owner = 1 - L->cur_owner;
        if (L->overlap) L->lcur ^= 1;
    }
    L->level += 1;
}

// bring the grid to the post-stream state of the current level (gather from
// the post-collision state), so that it can be read or modified in place
int materialize(lbmep_lattice *L) {
    if (!L->pmode) return LBMEP_OK;
    SweepArgs a = sweep_args(L);
    a.FM = nullptr;
    HIP_TRY(launch_sweep(L->precision, kSweepReadout, kForceNone, a, L->block_x, 1, L->stream));
    L->cur = 1 - L->cur;
    L->pmode = false;
    return LBMEP_OK;
}

void free_particles(lbmep_lattice *L) {
    dev_free(L, L->X0);
    dev_free(L, L->R);
    dev_free(L, L->U);
    dev_free(L, L->W);
    dev_free(L, L->FM);
    for (int b = 0; b < 2; ++b) {
        dev_free(L, L->Xheld[b]);
        L->Xheld[b] = nullptr;
    }
    for (int b = 0; b < 2; ++b) {
        dev_free(L, L->pcount_buf[b]);
        L->pcount_buf[b] = nullptr;
    }
    L->X0 = L->R = L->U = L->W = L->FM = nullptr;
    L->np_cap = 0;
}

size_t lattice_bytes(const lbmep_config *cfg, int32_t n_particles, double r_max,
                     int force_mode, bool overlap) {
    const size_t N = (size_t)cfg->nx * cfg->ny * cfg->nz;
    const size_t Ns = population_stride(N, cfg->precision);
    size_t b = 2 * (size_t)Q * Ns * storage_bytes(cfg->precision);  // two population grids
    b += round_up(N, 4096) + 4 * round_up(N, 4096) + 4 * N;      // flags, wall masks, wall list
    if (n_particles > 0) {
        b += 2 * 4 * N + (size_t)n_particles * (16 + 6 * 3) * 8;  // maps, particle table
        b += (size_t)n_particles * (8 * (size_t)link_capacity(r_max) + 4);  // link lists
        if (overlap)  // overlapped stepping: the next level's link lists
            b += (size_t)n_particles * (8 * (size_t)link_capacity(r_max) + 4);
    }
    if (force_mode == kForceDense) b += 3 * Ns * compute_bytes(cfg->precision);
    if (force_mode == kForceCharge || force_mode == kForcePotential)
        b += Ns * compute_bytes(cfg->precision);
    if (force_mode == kForcePotential) b += 8 * (size_t)n_particles;
    Grid g{};
    g.nx = cfg->nx;
    g.ny = cfg->ny;
    g.nz = cfg->nz;
    g.N = N;
    g.Ns = Ns;
    b += 4 * wall_list_scratch(g) + 256;                          // list scan, list length
    b += (5 * (size_t)invariants_blocks(g) + 4) * sizeof(double);  // reductions
    return b;
}

int check_config(const lbmep_config *cfg) {
    if (!cfg) return fail(LBMEP_EINVAL, "null config");
    if (cfg->nx <= 0 || cfg->ny <= 0 || cfg->nz <= 0)
        return fail(LBMEP_EINVAL, "grid sizes must be positive");
    if ((double)cfg->nx * cfg->ny * cfg->nz > 4.0e9)
        return fail(LBMEP_EINVAL, "grid larger than 4e9 cells");
    if (cfg->nx > (1 << 20) || cfg->ny > 65535 || cfg->nz > 65535)
        return fail(LBMEP_EINVAL, "ny and nz must be <= 65535");
    if (!(std::isfinite(cfg->nu) && cfg->nu > 0.0)) return fail(LBMEP_EINVAL, "nu must be > 0");
    if (!(std::isfinite(cfg->magic) && cfg->magic > 0.0))
        return fail(LBMEP_EINVAL, "magic parameter must be > 0");
    if (cfg->precision < LBMEP_FP64 || cfg->precision > LBMEP_FP16DEV)
        return fail(LBMEP_EINVAL, "unknown precision");
    if (cfg->reserved != 0) return fail(LBMEP_EINVAL, "reserved must be 0");
    return LBMEP_OK;
}

}  // namespace rt
}  // namespace lbmep

extern "C" {

const char *lbmep_last_error(void) { return g_err.c_str(); }

int lbmep_footprint(const lbmep_config *cfg, int32_t n_particles, double r_max, int with_charge,
                    size_t *bytes) {
    int rc = check_config(cfg);
    if (rc) return rc;
    if (!bytes || n_particles < 0 || !(r_max >= 0.0) || !std::isfinite(r_max))
        return fail(LBMEP_EINVAL, "bad footprint arguments");
    *bytes = lattice_bytes(cfg, n_particles, r_max, with_charge ? kForceCharge : kForceNone,
                           n_particles > 0 && cfg->move_particles);
    return LBMEP_OK;
}

int lbmep_copy_reference(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src) return fail(LBMEP_EINVAL, "null pointer");
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src) | bytes) & 15u)
        return fail(LBMEP_EINVAL, "pointers and size must be multiples of 16 bytes");
    HIP_TRY(launch_copy16(src, dst, bytes, (hipStream_t)stream));
    return LBMEP_OK;
}

int lbmep_destroy(lbmep_lattice *L) { return destroy_lattice(L, true); }

int lbmep_create(const lbmep_config *cfg, lbmep_lattice **out) {
    return create_lattice(cfg, nullptr, out);
}

}  // extern "C"

namespace lbmep {
namespace rt {

int destroy_lattice(lbmep_lattice *L, bool sync) {
    if (!L) return LBMEP_OK;
    hipSetDevice(L->cfg.device);
    if (sync) hipStreamSynchronize(L->stream);
    if (L->stream2) {
        hipStreamSynchronize(L->stream2);
        hipStreamDestroy(L->stream2);
        hipEventDestroy(L->ev_sweep);
        hipEventDestroy(L->ev_chain);
    }
    dev_free(L, L->f[0]);
    dev_free(L, L->f[1]);
    dev_free(L, L->flag);
    dev_free(L, L->wallmask);
    dev_free(L, L->wall_list);
    dev_free(L, L->wall_count);
    dev_free(L, L->wall_scratch);
    for (int b = 0; b < 2; ++b) dev_free(L, L->plist_buf[b]);
    for (int b = 0; b < 2; ++b) dev_free(L, L->owner[b]);
    dev_free(L, L->force);
    dev_free(L, L->red);
    dev_free(L, L->zeta);
    dev_free(L, L->q);
    dev_free(L, L->too_fast);
    dev_free(L, L->sor_ctl);
    dev_free(L, L->sor_partial);
    dev_free(L, L->sor_nlist);
    dev_free(L, L->sor_nscratch);
    dev_free(L, L->sor_nrow);
    dev_free(L, L->sor_nmask);
    dev_free(L, L->sor_ibits);
    dev_free(L, L->psi2);
    dev_free(L, L->sor_save);
    dev_free(L, L->sor_codes);
    free_particles(L);
    for (hipEvent_t e : L->ev) hipEventDestroy(e);
    delete L;
    return LBMEP_OK;
}

int create_lattice(const lbmep_config *cfg, DevHeap *heap, lbmep_lattice **out) {
    int rc = check_config(cfg);
    if (rc) return rc;
    if (!out) return fail(LBMEP_EINVAL, "null output pointer");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (cfg->device < 0 || cfg->device >= ndev) return fail(LBMEP_EINVAL, "no such device");
    HIP_TRY(hipSetDevice(cfg->device));
    lbmep_lattice *L = new lbmep_lattice();
    L->heap = heap;
    L->cfg = *cfg;
    L->stream = (hipStream_t)cfg->stream;
    // overlapped stepping for a lattice of its own with moving particles
    // (LBMEP_STEP_OVERLAP=0: every step in one stream, for comparisons)
    L->overlap = heap == nullptr && cfg->move_particles;
    if (const char *e = std::getenv("LBMEP_STEP_OVERLAP")) L->overlap = L->overlap && std::atoi(e) != 0;
    L->precision = cfg->precision;
    Grid &g = L->g;
    g.nx = cfg->nx;
    g.ny = cfg->ny;
    g.nz = cfg->nz;
    for (int k = 0; k < 3; ++k) g.per[k] = cfg->periodic[k] ? 1 : 0;
    g.N = (size_t)g.nx * g.ny * g.nz;
    g.Ns = population_stride(g.N, cfg->precision);
    // Eq. kinVisc: nu = (tau - 1/2) c_s^2; lambda_e = -1/tau (Sec. 3.1); the
    // odd rate from Lambda = (1/s_e - 1/2)(1/s_o - 1/2), s = -lambda
    L->tau = cfg->nu * 3.0 + 0.5;
    L->le = -1.0 / L->tau;
    L->lo = -1.0 / (0.5 + cfg->magic / (L->tau - 0.5));
    L->ae = 1.0 + 0.5 * L->le;
    L->ao = 1.0 + 0.5 * L->lo;
    if (!(L->lo > -2.0 && L->lo < 0.0)) {
        delete L;
        return fail(LBMEP_EINVAL, "odd relaxation rate outside ]-2,0[");
    }
    // launch shape of the sweep: x-segments of block_x threads (whole
    // wavefronts), cpt cells per thread on consecutive rows, dealt onto XCDs
    // in contiguous runs, streaming (non-temporal) hints on its loads and
    // stores (every value is read once and written once per step);
    // LBMEP_BLOCK_X, LBMEP_CPT, LBMEP_XCD_SWIZZLE and LBMEP_SWEEP_NT override
    // the defaults for launch-shape sweeps
    // measured at 512^3 (4096 spheres; segment width x block order x hints,
    // then repeated): FP32 is fastest with 256-cell segments in hardware
    // order (every XCD streams the same planes; 3.71 ms, XCD-contiguous 256:
    // 4.05-4.13), FP16 with 512-cell segments in hardware order (1.99 ms in
    // three repeats against 2.16-2.21 with 256 XCD-contiguous), FP64 with
    // 128-cell segments in XCD-contiguous order (7.75 ms; hardware 7.86)
    L->block_x = L->precision == LBMEP_FP64 ? 128 : L->precision == LBMEP_FP16DEV ? 512 : 256;
    L->xcd_swizzle = L->precision == LBMEP_FP64;
    L->cpt = 1;
    if (const char *e = std::getenv("LBMEP_CPT")) {
        const int c = std::atoi(e);
        if (c == 1 || c == 2) L->cpt = c;
    }
    // SOR tiles: 8 rows per thread and 8-plane chunks for FP32 psi; FP64 psi
    // needs twice the registers per row, so 4 and 4 (measured best of each)
    L->sor_rows = L->precision == LBMEP_FP64 ? 4 : 8;
    L->sor_zc = L->precision == LBMEP_FP64 ? 4 : 8;
    if (const char *e = std::getenv("LBMEP_SOR_ZC")) {
        const int c = std::atoi(e);
        if (c >= 1 && c <= 1024) L->sor_zc = c;
    }
    if (const char *e = std::getenv("LBMEP_SOR_WX")) {
        const int c = std::atoi(e);
        if (c == 1 || c == 2 || c == 4) L->sor_wx = c;
    }
    if (const char *e = std::getenv("LBMEP_SOR_XCD")) L->sor_xcd = std::atoi(e) != 0;
    if (const char *e = std::getenv("LBMEP_SOR_NEARBLK")) {
        const int c = std::atoi(e);
        if (c >= 8 && c <= 65536 && c % 8 == 0) L->sor_near_blocks = c;
    }
    // one-pass SOR iteration: rows per thread and planes per workgroup
    L->sor_mrw = 4;
    if (const char *e = std::getenv("LBMEP_SOR_MRW")) {
        const int c = std::atoi(e);
        if (c == 1 || c == 2 || c == 4 || c == 8) L->sor_mrw = c;
    }
    if (const char *e = std::getenv("LBMEP_SOR_MZC")) {
        const int c = std::atoi(e);
        if (c >= 1 && c <= 1024) L->sor_mzc = c;
    }
    if (const char *e = std::getenv("LBMEP_SOR_ROWS")) {
        const int c = std::atoi(e);
        if (c == 4 || c == 8) L->sor_rows = c;
    }
    if (const char *e = std::getenv("LBMEP_BLOCK_X")) {
        const int b = std::atoi(e);
        if (b >= 64 && b <= 512 && b % 64 == 0) L->block_x = b;
    }
    if (const char *e = std::getenv("LBMEP_XCD_SWIZZLE")) L->xcd_swizzle = std::atoi(e) != 0;
    // measured at 512^3: hints on the stores only are fastest for every
    // storage type (the loads' one-element overlaps along x then hit L2;
    // FP16 with 512-cell segments: 1.99 against 2.02-2.06 ms with hints on
    // the loads too)
    // workgroups per CU of the sweep capped by a dynamic LDS allocation per
    // workgroup (the kernel uses none of it; 160 KiB of LDS per CU), set per
    // force mode in sweep_args_state; LBMEP_SWEEP_WGCU (workgroups per CU, 0:
    // no cap) overrides it
    L->sweep_wgcu = -1;
    if (const char *e = std::getenv("LBMEP_SWEEP_WGCU")) {
        const int w = std::atoi(e);
        if (w >= 0 && w <= 32) L->sweep_wgcu = w;
    }
    L->sweep_nt = 2;
    if (const char *e = std::getenv("LBMEP_SWEEP_NT")) {
        const int v = std::atoi(e);
        if (v >= 0 && v <= 2) L->sweep_nt = v;
    }
    const size_t es = storage_bytes(L->precision);
    bool ok = true;
    ok = ok && dev_alloc(L, (void **)&L->f[0], Q * g.Ns * es) == hipSuccess;
    ok = ok && dev_alloc(L, (void **)&L->f[1], Q * g.Ns * es) == hipSuccess;
    // flags padded for the 16-byte reads of the NEAR-list compaction
    ok = ok && dev_alloc(L, (void **)&L->flag, round_up(g.N, 4096)) == hipSuccess;
    // wall masks padded for the 16-byte reads of the list compaction
    ok = ok && dev_alloc(L, (void **)&L->wallmask, 4 * round_up(g.N, 4096)) == hipSuccess;
    ok = ok && dev_alloc(L, (void **)&L->wall_list, 4 * g.N) == hipSuccess;
    ok = ok && dev_alloc(L, (void **)&L->wall_count, 256) == hipSuccess;
    ok = ok && dev_alloc(L, (void **)&L->wall_scratch, 4 * wall_list_scratch(g)) == hipSuccess;
    L->red_blocks = invariants_blocks(g);
    ok = ok && dev_alloc(L, (void **)&L->red, (5 * (size_t)L->red_blocks + 4) * sizeof(double)) == hipSuccess;
    if (!ok) {
        destroy_lattice(L, true);
        return fail(LBMEP_ENOMEM, "device allocation failed");
    }
    hipStream_t s = L->stream;
    hipError_t e = hipMemsetAsync(L->flag, 0, round_up(g.N, 4096), s);
    if (e == hipSuccess) e = hipMemsetAsync(L->wallmask, 0, 4 * round_up(g.N, 4096), s);
    if (e == hipSuccess) e = launch_classify_all(g, L->flag, L->wallmask, nullptr, s);
    if (e == hipSuccess)
        e = launch_wall_list(g, L->wallmask, L->wall_list, L->wall_count, L->wall_scratch, s);
    const double u0[3] = {0, 0, 0};
    if (e == hipSuccess) e = launch_init_equilibrium(L->precision, g, L->f[0], 1.0, u0, s);
    if (e == hipSuccess) e = launch_init_equilibrium(L->precision, g, L->f[1], 1.0, u0, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        destroy_lattice(L, true);
        return fail(LBMEP_EDEVICE, std::string("initialisation: ") + hipGetErrorString(e));
    }
    *out = L;
    return LBMEP_OK;
}

}  // namespace rt
}  // namespace lbmep

extern "C" {

int lbmep_set_flags(lbmep_lattice *L, const uint8_t *flags, int on_device) {
    if (!L || !flags) return fail(LBMEP_EINVAL, "null argument");
    int rc = set_device(L);
    if (rc) return rc;
    const size_t N = L->g.N;
    if (!on_device) {
        for (size_t i = 0; i < N; ++i)
            if (flags[i] != LBMEP_FLUID && flags[i] != LBMEP_WALL)
                return fail(LBMEP_EINVAL, "flag values must be LBMEP_FLUID or LBMEP_WALL");
    }
    rc = materialize(L);
    if (rc) return rc;
    uint8_t *tmp = nullptr;
    const uint8_t *src = flags;
    if (!on_device) {
        HIP_TRY(dev_alloc(L, (void **)&tmp, N));
        hipError_t e = hipMemcpyAsync(tmp, flags, N, hipMemcpyHostToDevice, L->stream);
        if (e != hipSuccess) {
            dev_free(L, tmp);
            return fail(LBMEP_EDEVICE, hipGetErrorString(e));
        }
        src = tmp;
    }
    hipError_t e = launch_import_flags(L->g, src, L->flag, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    dev_free(L, tmp);
    if (e != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(e));
    // the wall pass of the exchange kernel is launched only with wall cells
    // (device flags are not inspected on the host: assume some)
    L->has_walls = true;
    if (!on_device) {
        L->has_walls = false;
        for (size_t i = 0; i < N && !L->has_walls; ++i) L->has_walls = flags[i] == LBMEP_WALL;
    }
    return remap_all(L);
}

int lbmep_set_particles(lbmep_lattice *L, int32_t n, const double *X, const double *R,
                        const double *U, const double *W) {
    if (!L) return fail(LBMEP_EINVAL, "null lattice");
    if (n < 0) return fail(LBMEP_EINVAL, "negative particle count");
    if (n > 0 && (!X || !R || !U)) return fail(LBMEP_EINVAL, "null particle array");
    if (n > 0) {
        if (!finite_all(X, 3 * (size_t)n) || !finite_all(R, n) || !finite_all(U, 3 * (size_t)n) ||
            (W && !finite_all(W, 3 * (size_t)n)))
            return fail(LBMEP_EINVAL, "non-finite particle data");
        for (int i = 0; i < n; ++i)
            if (!(R[i] > 0.0)) return fail(LBMEP_EINVAL, "radii must be > 0");
        // the re-mapping of a step covers the boxes of two consecutive
        // positions grown by one cell: a body may move less than one cell
        if (L->cfg.move_particles)
            for (size_t i = 0; i < 3 * (size_t)n; ++i)
                if (!(std::fabs(U[i]) < 1.0))
                    return fail(LBMEP_EINVAL, "particles must move less than one cell per step");
    }
    int rc = set_device(L);
    if (rc) return rc;
    rc = materialize(L);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(L->stream));
    if (n > 0 && !L->owner[0]) {
        for (int b = 0; b < 2; ++b)
            if (dev_alloc(L, (void **)&L->owner[b], 4 * L->g.N) != hipSuccess)
                return fail(LBMEP_ENOMEM, "owner field allocation failed");
    }
    const int nlists = L->overlap ? 2 : 1;
    if ((size_t)n > L->np_cap) {
        free_particles(L);
        const size_t b = 3 * (size_t)n * sizeof(double);
        bool ok = dev_alloc(L, (void **)&L->X0, b) == hipSuccess && dev_alloc(L, (void **)&L->U, b) == hipSuccess &&
                  dev_alloc(L, (void **)&L->W, b) == hipSuccess && dev_alloc(L, (void **)&L->R, b / 3) == hipSuccess &&
                  dev_alloc(L, (void **)&L->FM, 6 * b) == hipSuccess;
        for (int r = 0; r < 2; ++r)
            ok = ok && dev_alloc(L, (void **)&L->Xheld[r], b) == hipSuccess;
        for (int r = 0; r < nlists; ++r)
            ok = ok && dev_alloc(L, (void **)&L->pcount_buf[r], 4 * (size_t)n) == hipSuccess;
        if (!ok) {
            free_particles(L);
            L->np = 0;
            return fail(LBMEP_ENOMEM, "particle table allocation failed");
        }
        L->np_cap = n;
    }
    // link lists: capacity per particle from the largest radius
    double rmax = 0.0;
    for (int i = 0; i < n; ++i) rmax = R[i] > rmax ? R[i] : rmax;
    const uint32_t pcap = n > 0 ? link_capacity(rmax) : 0;
    if ((size_t)n * pcap > L->plist_entries) {
        L->plist_entries = 0;
        for (int r = 0; r < 2; ++r) {
            dev_free(L, L->plist_buf[r]);
            L->plist_buf[r] = nullptr;
        }
        for (int r = 0; r < nlists; ++r)
            if (dev_alloc(L, (void **)&L->plist_buf[r], (size_t)n * pcap * sizeof(uint2)) != hipSuccess) {
                L->np = 0;
                return fail(LBMEP_ENOMEM, "link list allocation failed");
            }
        L->plist_entries = (size_t)n * pcap;
    }
    L->pcap = pcap;
    L->halo_cap = n > 0 ? halo_capacity(rmax) : 0;
    // boundary values of the potential and the dynamics belong to the
    // particle table they were given with
    dev_free(L, L->zeta);
    L->zeta = nullptr;
    L->hzeta.clear();
    dev_free(L, L->q);
    L->q = nullptr;
    L->hq.clear();
    L->dynamic = false;
    L->np = n;
    L->hX0.assign(X, X + 3 * (size_t)n);
    L->hR.assign(R, R + n);
    L->hU.assign(U, U + 3 * (size_t)n);
    if (W)
        L->hW.assign(W, W + 3 * (size_t)n);
    else
        L->hW.assign(3 * (size_t)n, 0.0);
    if (n > 0) {
        const size_t b = 3 * (size_t)n * sizeof(double);
        HIP_TRY(hipMemcpy(L->X0, L->hX0.data(), b, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(L->R, L->hR.data(), b / 3, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(L->U, L->hU.data(), b, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(L->W, L->hW.data(), b, hipMemcpyHostToDevice));
    }
    L->level = 0;
    rc = remap_all(L);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(L->stream));
    return LBMEP_OK;
}

static int set_force_common(lbmep_lattice *L, const void *in, int dtype, int on_device,
                            int ncomp, int mode) {
    if (!L || !in) return fail(LBMEP_EINVAL, "null argument");
    if (dtype != LBMEP_DTYPE_F64 && dtype != LBMEP_DTYPE_F32)
        return fail(LBMEP_EINVAL, "unknown dtype");
    int rc = set_device(L);
    if (rc) return rc;
    const size_t N = L->g.N, Ns = L->g.Ns;
    const size_t ib = dtype == LBMEP_DTYPE_F64 ? 8 : 4;
    if (!on_device) {
        for (size_t i = 0; i < (size_t)ncomp * N; ++i) {
            const double v = dtype == LBMEP_DTYPE_F64 ? ((const double *)in)[i]
                                                      : (double)((const float *)in)[i];
            if (!std::isfinite(v)) return fail(LBMEP_EINVAL, "non-finite force value");
        }
    }
    HIP_TRY(hipStreamSynchronize(L->stream));
    const size_t need = (size_t)ncomp * Ns * compute_bytes(L->precision);
    if (L->force_bytes < need) {
        dev_free(L, L->force);
        L->force = nullptr;
        L->force_bytes = 0;
        if (dev_alloc(L, (void **)&L->force, need) != hipSuccess) {
            L->force_mode = kForceNone;
            return fail(LBMEP_ENOMEM, "force field allocation failed");
        }
        L->force_bytes = need;
    }
    const void *src = in;
    void *tmp = nullptr;
    if (!on_device) {
        HIP_TRY(dev_alloc(L, (void **)&tmp, (size_t)ncomp * N * ib));
        hipError_t e = hipMemcpy(tmp, in, (size_t)ncomp * N * ib, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            dev_free(L, tmp);
            return fail(LBMEP_EDEVICE, hipGetErrorString(e));
        }
        src = tmp;
    }
    // psi goes into its storage order (colour-split for even nx)
    hipError_t e = mode == kForcePotential
                       ? launch_potential_pack(L->precision, L->g, src, dtype, L->force, L->stream)
                       : launch_convert_force(L->precision, src, dtype, L->force, N, N, Ns, ncomp,
                                              L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    dev_free(L, tmp);
    if (e != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(e));
    L->force_mode = mode;
    return LBMEP_OK;
}

int lbmep_set_force(lbmep_lattice *L, const void *fb, int dtype, int on_device) {
    int rc = set_force_common(L, fb, dtype, on_device, 3, kForceDense);
    if (rc == LBMEP_OK) L->E[0] = L->E[1] = L->E[2] = 0.0;
    return rc;
}

int lbmep_set_charge_force(lbmep_lattice *L, const void *rho_e, int dtype, const double E[3],
                           int on_device) {
    if (!E || !finite_all(E, 3)) return fail(LBMEP_EINVAL, "bad field E");
    int rc = set_force_common(L, rho_e, dtype, on_device, 1, kForceCharge);
    if (rc == LBMEP_OK) {
        L->E[0] = E[0];
        L->E[1] = E[1];
        L->E[2] = E[2];
    }
    return rc;
}

int lbmep_set_potential_force(lbmep_lattice *L, const void *psi, int dtype, double kappa2_eps,
                              const double E[3], const double *zeta, int on_device) {
    if (!L) return fail(LBMEP_EINVAL, "null lattice");
    if (!E || !finite_all(E, 3)) return fail(LBMEP_EINVAL, "bad field E");
    if (!std::isfinite(kappa2_eps)) return fail(LBMEP_EINVAL, "non-finite kappa^2 eps");
    if (zeta && !finite_all(zeta, (size_t)L->np)) return fail(LBMEP_EINVAL, "non-finite zeta");
    int rc = set_device(L);
    if (rc) return rc;
    double *dz = nullptr;
    if (zeta && L->np > 0) {
        if (dev_alloc(L, (void **)&dz, 8 * (size_t)L->np) != hipSuccess)
            return fail(LBMEP_ENOMEM, "zeta allocation failed");
    }
    rc = set_force_common(L, psi, dtype, on_device, 1, kForcePotential);
    if (rc) {
        dev_free(L, dz);
        return rc;
    }
    dev_free(L, L->zeta);
    L->zeta = dz;
    L->hzeta.clear();
    if (dz) {
        L->hzeta.assign(zeta, zeta + L->np);
        HIP_TRY(hipMemcpy(dz, zeta, 8 * (size_t)L->np, hipMemcpyHostToDevice));
    }
    L->keps = kappa2_eps;
    for (int k = 0; k < 3; ++k) L->E[k] = E[k];
    return LBMEP_OK;
}

static SorArgs sor_args(const lbmep_lattice *L) {
    SorArgs a;
    a.g = L->g;
    a.psi = L->force;
    a.psi2 = L->psi2;
    a.flag = L->flag;
    a.owner = L->np > 0 ? L->owner[L->cur_owner] : nullptr;
    a.zeta = L->zeta;
    a.kappa2 = L->sor_kappa2;
    a.omega = L->sor_omega;
    a.rf = L->sor_rf;
    a.ctl = L->sor_ctl;
    a.partial = L->sor_partial;
    a.nlist = L->sor_nlist;
    a.nscratch = L->sor_nscratch;
    a.nrow = L->sor_nrow;
    a.nmask = L->sor_nmask;
    a.ibits = L->sor_ibits;
    a.xcd_swizzle = (uint32_t)L->sor_xcd;
    a.zc = (uint32_t)L->sor_zc;
    a.wx = (uint32_t)L->sor_wx;
    a.rows = (uint32_t)L->sor_rows;
    a.near_blocks = (uint32_t)L->sor_near_blocks;
    a.codes = L->sor_codes;
    a.save = L->sor_save;
    a.mzc = (uint32_t)L->sor_mzc;
    a.mrw = (uint32_t)L->sor_mrw;
    return a;
}

// one solve as configured; the fused iteration may leave the result in the
// second buffer, which then becomes psi
static int run_solve(lbmep_lattice *L, hipStream_t s) {
    int swapped = 0;
    HIP_TRY(launch_sor_solve(L->precision, sor_args(L), L->sor_iters, L->sor_check,
                             L->sor_fused, s, &swapped));
    if (swapped) {
        std::swap(L->force, L->psi2);
        std::swap(L->force_bytes, L->psi2_bytes);
    }
    return LBMEP_OK;
}

int lbmep_set_potential_solver(lbmep_lattice *L, double kappa2, double omega, int32_t max_iter,
                               double rf, int32_t check_every) {
    if (!L) return fail(LBMEP_EINVAL, "null lattice");
    if (L->force_mode != kForcePotential) return fail(LBMEP_EINVAL, "no potential set");
    if (!(std::isfinite(kappa2) && kappa2 > 0.0)) return fail(LBMEP_EINVAL, "kappa^2 must be > 0");
    if (!(omega > 0.0 && omega < 2.0)) return fail(LBMEP_EINVAL, "omega outside (0, 2)");
    if (max_iter < 0 || check_every < 1 || !std::isfinite(rf))
        return fail(LBMEP_EINVAL, "bad iteration parameters");
    const int len[3] = {L->g.nx, L->g.ny, L->g.nz};
    for (int k = 0; k < 3; ++k)
        if (L->g.per[k] && (len[k] & 1))
            return fail(LBMEP_EINVAL, "red-black ordering needs even periodic extents");
    if (L->g.N + 2 >= ((size_t)1 << 32))
        return fail(LBMEP_EINVAL, "the solver lists cells with 32-bit indices (N < 2^32 - 2)");
    int rc = set_device(L);
    if (rc) return rc;
    if (!L->sor_ctl) {
        if (dev_alloc(L, (void **)&L->sor_ctl, sizeof(SorCtl)) != hipSuccess)
            return fail(LBMEP_ENOMEM, "solver control block");
        if (dev_alloc(L, (void **)&L->sor_partial, sizeof(double) * kSorPartials) != hipSuccess)
            return fail(LBMEP_ENOMEM, "solver partial sums");
        if (dev_alloc(L, (void **)&L->sor_nlist, 4 * sor_nlist_entries(L->g.N)) != hipSuccess)
            return fail(LBMEP_ENOMEM, "solver boundary list");
        if (dev_alloc(L, (void **)&L->sor_nscratch, 4 * sor_nscratch_entries(L->g.N)) != hipSuccess)
            return fail(LBMEP_ENOMEM, "solver list scratch");
        if (dev_alloc(L, &L->sor_nrow, 2 * compute_bytes(L->precision) *
                                           sor_nlist_entries(L->g.N)) != hipSuccess ||
            dev_alloc(L, (void **)&L->sor_nmask, sor_nlist_entries(L->g.N)) != hipSuccess ||
            dev_alloc(L, (void **)&L->sor_ibits, 6 * 4 * sor_ibits_words_per_colour(L->g.N)) !=
                hipSuccess)
            return fail(LBMEP_ENOMEM, "solver boundary rows");
        SorCtl c{};
        c.res0 = c.res = -1.0;
        HIP_TRY(hipMemcpy(L->sor_ctl, &c, sizeof c, hipMemcpyHostToDevice));
    }
    // one pass per iteration where it applies (even nx, rows of up to 2048
    // cells), else one launch per colour; LBMEP_SOR_FUSED=0 forces the latter
    L->sor_fused = L->g.nx % 2 == 0 && L->g.nx <= 2048;
    if (const char *e = std::getenv("LBMEP_SOR_FUSED")) L->sor_fused = L->sor_fused && std::atoi(e) != 0;
    const size_t need = L->g.Ns * compute_bytes(L->precision);
    if (L->sor_fused && L->psi2_bytes < need) {
        dev_free(L, L->psi2);
        dev_free(L, L->sor_save);
        L->psi2 = L->sor_save = nullptr;
        L->psi2_bytes = 0;
        if (dev_alloc(L, &L->psi2, need) != hipSuccess || dev_alloc(L, &L->sor_save, need) != hipSuccess)
            return fail(LBMEP_ENOMEM, "second potential buffer");
        L->psi2_bytes = need;
    }
    if (L->sor_fused && !L->sor_codes &&
        dev_alloc(L, (void **)&L->sor_codes, 4 * (L->g.N / 2 + 1)) != hipSuccess)
        return fail(LBMEP_ENOMEM, "solver row codes");
    L->sor_kappa2 = kappa2;
    L->sor_omega = omega;
    L->sor_iters = max_iter;
    L->sor_rf = rf;
    L->sor_check = check_every;
    L->sor_set = true;
    return LBMEP_OK;
}

int lbmep_solve_potential(lbmep_lattice *L, int32_t *iters, double res[2]) {
    if (!L) return fail(LBMEP_EINVAL, "null lattice");
    if (L->force_mode != kForcePotential || !L->sor_set)
        return fail(LBMEP_EINVAL, "no potential solver configured");
    int rc = set_device(L);
    if (rc) return rc;
    rc = run_solve(L, L->stream);
    if (rc) return rc;
    if (iters || res) {
        SorCtl c;
        HIP_TRY(hipMemcpyAsync(&c, L->sor_ctl, sizeof c, hipMemcpyDeviceToHost, L->stream));
        HIP_TRY(hipStreamSynchronize(L->stream));
        if (iters) *iters = c.iters;
        if (res) {
            res[0] = c.res0;
            res[1] = c.res;
        }
    }
    return LBMEP_OK;
}

int lbmep_get_solver_stats(lbmep_lattice *L, int32_t *iters, double res[2]) {
    if (!L || !iters || !res) return fail(LBMEP_EINVAL, "null argument");
    if (!L->sor_ctl) return fail(LBMEP_EINVAL, "no potential solver configured");
    int rc = set_device(L);
    if (rc) return rc;
    SorCtl c;
    HIP_TRY(hipMemcpyAsync(&c, L->sor_ctl, sizeof c, hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    *iters = c.iters;
    res[0] = c.res0;
    res[1] = c.res;
    return LBMEP_OK;
}

int lbmep_get_solver_shape(const lbmep_lattice *L, int32_t shape[4]) {
    if (!L || !shape) return fail(LBMEP_EINVAL, "null argument");
    if (!L->sor_set) return fail(LBMEP_EINVAL, "no potential solver configured");
    const bool one = L->sor_fused && L->g.nx % 2 == 0 && L->g.nx <= 2048;
    if (one) {
        int rw = L->sor_mrw >= 4 ? 4 : (L->sor_mrw >= 2 ? 2 : 1);  // as the solve picks it
        while (L->g.ny % rw) rw >>= 1;
        shape[0] = 1;
        shape[1] = rw;
        shape[2] = L->sor_mzc;
        shape[3] = (L->g.nx / 2 + 63) / 64;
    } else {
        shape[0] = 0;
        shape[1] = L->g.nx % 2 == 0 ? L->sor_rows : 4;
        shape[2] = L->g.nx % 2 == 0 ? L->sor_zc : 1;
        shape[3] = L->g.nx % 2 == 0 ? L->sor_wx : 1;
    }
    return LBMEP_OK;
}

int lbmep_get_potential(lbmep_lattice *L, double *psi, int on_device) {
    if (!L || !psi) return fail(LBMEP_EINVAL, "null argument");
    if (L->force_mode != kForcePotential) return fail(LBMEP_EINVAL, "no potential set");
    int rc = set_device(L);
    if (rc) return rc;
    const size_t N = L->g.N;
    double *d = psi;
    if (!on_device && dev_alloc(L, (void **)&d, N * sizeof(double)) != hipSuccess)
        return fail(LBMEP_ENOMEM, "temp");
    hipError_t e = launch_potential_to_f64(L->precision, L->g, L->force, d, L->stream);
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(psi, d, N * sizeof(double), hipMemcpyDeviceToHost, L->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (!on_device) dev_free(L, d);
    if (e != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(e));
    return LBMEP_OK;
}

int lbmep_set_dynamics(lbmep_lattice *L, double rho_p, const double *q, const double E[3]) {
    if (!L || !E) return fail(LBMEP_EINVAL, "null argument");
    if (!L->cfg.move_particles) return fail(LBMEP_EINVAL, "dynamics need move_particles = 1");
    if (!(std::isfinite(rho_p) && rho_p > 0.0)) return fail(LBMEP_EINVAL, "rho_p must be > 0");
    if (!finite_all(E, 3) || (q && !finite_all(q, (size_t)L->np)))
        return fail(LBMEP_EINVAL, "non-finite E or charge");
    int rc = set_device(L);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(L->stream));
    if (!L->too_fast) {
        if (dev_alloc(L, (void **)&L->too_fast, 64) != hipSuccess) return fail(LBMEP_ENOMEM, "flag");
        HIP_TRY(hipMemset(L->too_fast, 0, 64));
    }
    dev_free(L, L->q);
    L->q = nullptr;
    L->hq.clear();
    if (q && L->np > 0) {
        if (dev_alloc(L, (void **)&L->q, 8 * (size_t)L->np) != hipSuccess)
            return fail(LBMEP_ENOMEM, "charges");
        L->hq.assign(q, q + L->np);
        HIP_TRY(hipMemcpy(L->q, q, 8 * (size_t)L->np, hipMemcpyHostToDevice));
    }
    if (L->np > 0 && !L->dynamic) {
        // from now on X0 holds the current level's positions
        const ParticleArgs pa = particle_args(L);
        HIP_TRY(launch_positions(pa, L->level, L->X0, L->stream));
        HIP_TRY(hipStreamSynchronize(L->stream));
    }
    L->rho_p = rho_p;
    for (int k = 0; k < 3; ++k) L->Edyn[k] = E[k];
    L->dynamic = true;
    return LBMEP_OK;
}

int lbmep_get_particles(lbmep_lattice *L, double *X, double *U, double *W) {
    if (!L || (L->np > 0 && (!X || !U || !W))) return fail(LBMEP_EINVAL, "null argument");
    int rc = set_device(L);
    if (rc) return rc;
    if (L->np == 0) return LBMEP_OK;
    const size_t b = 3 * (size_t)L->np * sizeof(double);
    HIP_TRY(hipMemcpyAsync(X, L->Xheld[L->cur_owner], b, hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(hipMemcpyAsync(U, L->U, b, hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(hipMemcpyAsync(W, L->W, b, hipMemcpyDeviceToHost, L->stream));
    int32_t fast = 0;
    if (L->too_fast)
        HIP_TRY(hipMemcpyAsync(&fast, L->too_fast, 4, hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    if (fast) return fail(LBMEP_EINVAL, "a particle reached one cell per step: the mapping is not valid");
    return LBMEP_OK;
}

int lbmep_set_free_slip(lbmep_lattice *L, const int32_t faces[6]) {
    if (!L || !faces) return fail(LBMEP_EINVAL, "null argument");
    int bits = 0;
    for (int k = 0; k < 6; ++k) {
        if (faces[k] != 0 && faces[k] != 1) return fail(LBMEP_EINVAL, "face value not 0 / 1");
        if (faces[k] && L->g.per[k / 2]) return fail(LBMEP_EINVAL, "free-slip face on a periodic axis");
        if (faces[k]) bits |= 1 << k;
    }
    int rc = set_device(L);
    if (rc) return rc;
    // the stored state is the post-stream state of its level under the old
    // faces; bring it there before the faces change
    rc = materialize(L);
    if (rc) return rc;
    L->slip = bits;
    return LBMEP_OK;
}

int lbmep_get_particle_count(const lbmep_lattice *L, int32_t *n) {
    if (!L || !n) return fail(LBMEP_EINVAL, "null argument");
    *n = L->np;
    return LBMEP_OK;
}

int lbmep_init_equilibrium(lbmep_lattice *L, double rho, const double u[3]) {
    if (!L || !u) return fail(LBMEP_EINVAL, "null argument");
    if (!std::isfinite(rho) || !finite_all(u, 3)) return fail(LBMEP_EINVAL, "non-finite state");
    int rc = set_device(L);
    if (rc) return rc;
    HIP_TRY(launch_init_equilibrium(L->precision, L->g, L->f[L->cur], rho, u, L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    L->pmode = false;
    return LBMEP_OK;
}

int lbmep_set_pdfs(lbmep_lattice *L, const double *f, int on_device) {
    if (!L || !f) return fail(LBMEP_EINVAL, "null argument");
    int rc = set_device(L);
    if (rc) return rc;
    const size_t N = L->g.N;
    if (!on_device && !finite_all(f, Q * N)) return fail(LBMEP_EINVAL, "non-finite populations");
    double *tmp = nullptr;
    if (!on_device) HIP_TRY(dev_alloc(L, (void **)&tmp, N * sizeof(double)));
    hipError_t e = hipSuccess;
    for (int q = 0; q < Q && e == hipSuccess; ++q) {
        const double *src = f + (size_t)q * N;
        if (!on_device) {
            e = hipMemcpyAsync(tmp, src, N * sizeof(double), hipMemcpyHostToDevice, L->stream);
            src = tmp;
        }
        if (e == hipSuccess) e = launch_pdfs_from_f64(L->precision, L->g, q, src, L->f[L->cur], L->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    }
    dev_free(L, tmp);
    if (e != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(e));
    L->pmode = false;
    return LBMEP_OK;
}

int lbmep_get_pdfs(lbmep_lattice *L, double *f, int on_device) {
    if (!L || !f) return fail(LBMEP_EINVAL, "null argument");
    int rc = set_device(L);
    if (rc) return rc;
    rc = materialize(L);
    if (rc) return rc;
    const size_t N = L->g.N;
    double *tmp = nullptr;
    if (!on_device) HIP_TRY(dev_alloc(L, (void **)&tmp, N * sizeof(double)));
    hipError_t e = hipSuccess;
    for (int q = 0; q < Q && e == hipSuccess; ++q) {
        double *dst = on_device ? f + (size_t)q * N : tmp;
        e = launch_pdfs_to_f64(L->precision, L->g, q, L->f[L->cur], dst, L->stream);
        if (e == hipSuccess && !on_device)
            e = hipMemcpyAsync(f + (size_t)q * N, tmp, N * sizeof(double), hipMemcpyDeviceToHost,
                               L->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    }
    dev_free(L, tmp);
    if (e != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(e));
    return LBMEP_OK;
}

int lbmep_step(lbmep_lattice *L, int32_t nsteps) {
    if (!L) return fail(LBMEP_EINVAL, "null lattice");
    if (nsteps < 0) return fail(LBMEP_EINVAL, "negative step count");
    int rc = set_device(L);
    if (rc) return rc;
    hipStream_t s = L->stream;
    const ParticleArgs pa = particle_args(L);
    const bool solve = L->force_mode == kForcePotential && L->sor_set && L->sor_iters > 0;
    // overlapped stepping: prescribed kinematics (the next level's positions
    // do not depend on this step's forces)
    const bool ov = L->overlap && L->np > 0 && L->cfg.move_particles && !L->dynamic;
    if (ov && !L->stream2) {
        HIP_TRY(hipStreamCreateWithFlags(&L->stream2, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&L->ev_sweep, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&L->ev_chain, hipEventDisableTiming));
    }
    for (int32_t it = 0; it < nsteps; ++it) {
        // the sweep needs the flags, map and lists of its level
        if (ov && L->chain_pending) HIP_TRY(hipStreamWaitEvent(s, L->ev_chain, 0));
        // the EDL potential of this level's map, before the collision that
        // uses its force
        if (solve) {
            rc = run_solve(L, s);
            if (rc) return rc;
        }
        const SweepArgs a = sweep_args(L);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (L->timing) {
            while (L->ev.size() < L->ev_used + 2) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                L->ev.push_back(e);
            }
            e0 = L->ev[L->ev_used];
            e1 = L->ev[L->ev_used + 1];
            L->ev_used += 2;
            HIP_TRY(hipEventRecord(e0, s));
        }
        // gather + refill + collide + bounce-back slots (or, right after the
        // state was set, collide the stored post-stream state in place)
        const int mode = !L->pmode ? kSweepLocal
                         : L->sweep_nt == 1 ? kSweepPullNT
                         : L->sweep_nt == 2 ? kSweepPullNTS
                                            : kSweepPull;
        HIP_TRY(launch_sweep(L->precision, mode, L->force_mode, a, L->block_x, L->cpt, s));
        if (L->timing) HIP_TRY(hipEventRecord(e1, s));
        if (ov) HIP_TRY(hipEventRecord(L->ev_sweep, s));
        // bounce-back slots and momentum exchange next to solid cells
        HIP_TRY(launch_near(L->precision, a, near_wall_blocks(L->g, L->has_walls), s));
        if (L->dynamic && L->np > 0) {
            // the particles move under this step's force and torque
            DynArgs d;
            d.g = L->g;
            d.np = L->np;
            d.acc = L->FM;
            d.X = L->Xheld[L->cur_owner];
            d.R = L->R;
            d.q = L->q;
            d.U = L->U;
            d.W = L->W;
            d.X0 = L->X0;
            d.rho_p = L->rho_p;
            for (int k = 0; k < 3; ++k) d.E[k] = L->Edyn[k];
            d.too_fast = L->too_fast;
            HIP_TRY(launch_dynamics(d, s));
        }
        if (L->np > 0 && L->cfg.move_particles) {
            // kinematics, re-mapping and classification of the next level
            const int b = 1 - L->cur_owner;
            // the next level's link lists: the other buffer when overlapped
            ParticleArgs pn = pa;
            pn.plist = L->plist_buf[L->overlap ? L->lcur ^ 1 : L->lcur];
            pn.pcount = L->pcount_buf[L->overlap ? L->lcur ^ 1 : L->lcur];
            if (ov) {
                // on the second stream once the sweep has read the previous
                // map, the positions and the flags, while the exchange runs
                // (it reads the current link lists, positions and
                // post-collision state only): clear the map held two levels
                // back, map and classify the next level
                hipStream_t s2 = L->stream2;
                HIP_TRY(hipStreamWaitEvent(s2, L->ev_sweep, 0));
                HIP_TRY(launch_advance(pn, L->level + 1, L->Xheld[b], L->owner[b], s2));
                HIP_TRY(launch_map_set(pn, L->Xheld[b], L->flag, L->owner[b], s2));
                HIP_TRY(launch_classify_boxes(pn, L->Xheld[L->cur_owner], L->Xheld[b], L->flag,
                                              L->owner[b], L->owner[L->cur_owner], s2));
                HIP_TRY(hipEventRecord(L->ev_chain, s2));
                L->chain_pending = true;
            } else {
                // clear the map buffer b held two levels back, move to
                // level + 1
                HIP_TRY(launch_advance(pn, L->level + 1, L->Xheld[b], L->owner[b], s));
                HIP_TRY(launch_map_set(pn, L->Xheld[b], L->flag, L->owner[b], s));
                HIP_TRY(launch_classify_boxes(pn, L->Xheld[L->cur_owner], L->Xheld[b], L->flag,
                                              L->owner[b], L->owner[L->cur_owner], s));
            }
        }
        advance_state(L);
    }
    // later work on the lattice's stream follows the last classification
    if (L->chain_pending) {
        HIP_TRY(hipStreamWaitEvent(s, L->ev_chain, 0));
        L->chain_pending = false;
    }
    return LBMEP_OK;
}

int lbmep_sync(lbmep_lattice *L) {
    if (!L) return fail(LBMEP_EINVAL, "null lattice");
    int rc = set_device(L);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(L->stream));
    return LBMEP_OK;
}

int lbmep_get_macro(lbmep_lattice *L, double *rho, double *u, int on_device) {
    if (!L || !rho || !u) return fail(LBMEP_EINVAL, "null argument");
    int rc = set_device(L);
    if (rc) return rc;
    rc = materialize(L);
    if (rc) return rc;
    const size_t N = L->g.N;
    double *drho = rho, *du = u;
    if (!on_device) {
        if (dev_alloc(L, (void **)&drho, N * sizeof(double)) != hipSuccess) return fail(LBMEP_ENOMEM, "temp");
        if (dev_alloc(L, (void **)&du, 3 * N * sizeof(double)) != hipSuccess) {
            dev_free(L, drho);
            return fail(LBMEP_ENOMEM, "temp");
        }
    }
    hipError_t e = launch_macro(L->precision, L->force_mode, L->g, L->f[L->cur], L->flag,
                                L->np > 0 ? L->owner[L->cur_owner] : nullptr,
                                L->np > 0 ? L->Xheld[L->cur_owner] : nullptr, L->U, L->W, L->force,
                                L->E, L->keps, L->force_mode == kForcePotential ? L->zeta : nullptr,
                                drho, du, L->stream);
    if (e == hipSuccess && !on_device) {
        e = hipMemcpyAsync(rho, drho, N * sizeof(double), hipMemcpyDeviceToHost, L->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(u, du, 3 * N * sizeof(double), hipMemcpyDeviceToHost, L->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (!on_device) {
        dev_free(L, drho);
        dev_free(L, du);
    }
    if (e != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(e));
    return LBMEP_OK;
}

int lbmep_get_particle_ft(lbmep_lattice *L, double *F, double *M) {
    if (!L) return fail(LBMEP_EINVAL, "null lattice");
    if (L->np == 0) return LBMEP_OK;
    if (!F || !M) return fail(LBMEP_EINVAL, "null output");
    int rc = set_device(L);
    if (rc) return rc;
    std::vector<double> h(6 * (size_t)L->np);
    double *out = L->FM + 12 * (size_t)L->np;
    HIP_TRY(launch_finalize_ft(L->np, L->FM, L->Xheld[L->ft_buf], out, L->stream));
    HIP_TRY(hipMemcpyAsync(h.data(), out, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                           L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    for (int p = 0; p < L->np; ++p)
        for (int k = 0; k < 3; ++k) {
            F[3 * p + k] = h[6 * (size_t)p + k];
            M[3 * p + k] = h[6 * (size_t)p + 3 + k];
        }
    return LBMEP_OK;
}

int lbmep_get_map(lbmep_lattice *L, uint8_t *flags, int32_t *owner) {
    if (!L) return fail(LBMEP_EINVAL, "null lattice");
    int rc = set_device(L);
    if (rc) return rc;
    const size_t N = L->g.N;
    if (flags) {
        uint8_t *tmp = nullptr;
        HIP_TRY(dev_alloc(L, (void **)&tmp, N));
        hipError_t e = launch_export_flags(L->g, L->flag, tmp, L->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(flags, tmp, N, hipMemcpyDeviceToHost, L->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
        dev_free(L, tmp);
        if (e != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(e));
    }
    if (owner) {
        if (L->np > 0) {
            HIP_TRY(hipMemcpyAsync(owner, L->owner[L->cur_owner], 4 * N, hipMemcpyDeviceToHost,
                                   L->stream));
            HIP_TRY(hipStreamSynchronize(L->stream));
        } else {
            for (size_t i = 0; i < N; ++i) owner[i] = -1;
        }
    }
    return LBMEP_OK;
}

int lbmep_get_invariants(lbmep_lattice *L, double out[4]) {
    if (!L || !out) return fail(LBMEP_EINVAL, "null argument");
    int rc = set_device(L);
    if (rc) return rc;
    rc = materialize(L);
    if (rc) return rc;
    double *dout = L->red + 5 * (size_t)L->red_blocks;
    HIP_TRY(launch_invariants(L->precision, L->g, L->f[L->cur], L->flag, L->red, L->red_blocks,
                              dout, L->stream));
    HIP_TRY(hipMemcpyAsync(out, dout, 4 * sizeof(double), hipMemcpyDeviceToHost, L->stream));
    HIP_TRY(hipStreamSynchronize(L->stream));
    if (!finite_all(out, 4)) return fail(LBMEP_ENONFINITE, "non-finite mass or momentum");
    return LBMEP_OK;
}

int lbmep_get_time(lbmep_lattice *L, int64_t *step) {
    if (!L || !step) return fail(LBMEP_EINVAL, "null argument");
    *step = L->level;
    return LBMEP_OK;
}

int lbmep_set_timing(lbmep_lattice *L, int enable) {
    if (!L) return fail(LBMEP_EINVAL, "null lattice");
    L->timing = enable != 0;
    return LBMEP_OK;
}

int lbmep_get_timing(lbmep_lattice *L, double *total_ms, int64_t *launches) {
    if (!L || !total_ms || !launches) return fail(LBMEP_EINVAL, "null argument");
    int rc = set_device(L);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(L->stream));
    double tot = 0.0;
    for (size_t i = 0; i + 1 < L->ev_used; i += 2) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, L->ev[i], L->ev[i + 1]));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)(L->ev_used / 2);
    L->ev_used = 0;
    return LBMEP_OK;
}

// ---------------------------------------------------------------------------
// checkpoint
// ---------------------------------------------------------------------------

namespace {
const char kMagic[8] = {'L', 'B', 'M', 'E', 'P', 'c', 'k', '4'};  // 4: psi in cell order, FP64

struct Header {
    char magic[8];
    int32_t nx, ny, nz, per[3], precision, move;
    double nu, magic_param;
    int64_t level;
    int32_t np, force_mode;
    double E[3];
    double keps;       // potential force: kappa^2 eps_e
    int32_t nzeta, pad; // potential force: boundary values that follow the particles
    // red-black SOR of the potential (sor_set = 0: not configured)
    double sor_kappa2, sor_omega, sor_rf;
    int32_t sor_iters, sor_check, sor_set, pad2;
    // particle dynamics (dyn = 0: prescribed); with dynamics the particle
    // table holds the current positions and velocities
    double rho_p, Edyn[3];
    int32_t dyn, nq;
    int32_t slip, pad3;  // free-slip faces
};
}  // namespace

int lbmep_save_state(lbmep_lattice *L, const char *path) {
    if (!L || !path) return fail(LBMEP_EINVAL, "null argument");
    int rc = set_device(L);
    if (rc) return rc;
    rc = materialize(L);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(L->stream));
    FILE *fp = std::fopen(path, "wb");
    if (!fp) return fail(LBMEP_EINVAL, std::string("cannot open ") + path);
    Header h{};
    std::memcpy(h.magic, kMagic, 8);
    h.nx = L->g.nx;
    h.ny = L->g.ny;
    h.nz = L->g.nz;
    for (int k = 0; k < 3; ++k) h.per[k] = L->g.per[k];
    h.precision = L->precision;
    h.move = L->cfg.move_particles;
    h.nu = L->cfg.nu;
    h.magic_param = L->cfg.magic;
    h.level = L->level;
    h.np = L->np;
    h.force_mode = L->force_mode;
    for (int k = 0; k < 3; ++k) h.E[k] = L->E[k];
    h.keps = L->keps;
    h.nzeta = (int32_t)L->hzeta.size();
    h.sor_kappa2 = L->sor_kappa2;
    h.sor_omega = L->sor_omega;
    h.sor_rf = L->sor_rf;
    h.sor_iters = L->sor_iters;
    h.sor_check = L->sor_check;
    h.sor_set = L->sor_set ? 1 : 0;
    h.dyn = L->dynamic ? 1 : 0;
    h.rho_p = L->rho_p;
    for (int k = 0; k < 3; ++k) h.Edyn[k] = L->Edyn[k];
    h.nq = (int32_t)L->hq.size();
    h.slip = L->slip;
    // with dynamics the table's positions and velocities are the device state
    std::vector<double> pX = L->hX0, pU = L->hU, pW = L->hW;
    if (L->dynamic && L->np > 0) {
        const size_t b = 3 * (size_t)L->np * sizeof(double);
        if (hipMemcpy(pX.data(), L->X0, b, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(pU.data(), L->U, b, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(pW.data(), L->W, b, hipMemcpyDeviceToHost) != hipSuccess) {
            std::fclose(fp);
            return fail(LBMEP_EDEVICE, "particle state read-back failed");
        }
    }
    bool ok = std::fwrite(&h, sizeof h, 1, fp) == 1;
    const size_t N = L->g.N, Ns = L->g.Ns;
    if (ok && L->np > 0) {
        ok = std::fwrite(pX.data(), 8, pX.size(), fp) == pX.size() &&
             std::fwrite(L->hR.data(), 8, L->hR.size(), fp) == L->hR.size() &&
             std::fwrite(pU.data(), 8, pU.size(), fp) == pU.size() &&
             std::fwrite(pW.data(), 8, pW.size(), fp) == pW.size();
    }
    if (ok && h.nzeta > 0) ok = std::fwrite(L->hzeta.data(), 8, L->hzeta.size(), fp) == L->hzeta.size();
    if (ok && h.nq > 0) ok = std::fwrite(L->hq.data(), 8, L->hq.size(), fp) == L->hq.size();
    // user wall flags
    std::vector<uint8_t> fl(N);
    if (ok) {
        if (hipMemcpy(fl.data(), L->flag, N, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
        for (size_t i = 0; i < N; ++i) fl[i] = (fl[i] & kWall) ? LBMEP_WALL : LBMEP_FLUID;
        ok = ok && std::fwrite(fl.data(), 1, N, fp) == N;
    }
    // force (compute precision); the potential psi in cell order as FP64
    // (its storage order, colour-split for even nx, spans Ns/2 + N/2 slots
    // of a colour, not the first N)
    if (ok && L->force_mode == kForcePotential) {
        double *d = nullptr;
        std::vector<double> buf(N);
        ok = dev_alloc(L, (void **)&d, N * sizeof(double)) == hipSuccess;
        ok = ok && launch_potential_to_f64(L->precision, L->g, L->force, d, L->stream) == hipSuccess &&
             hipMemcpyAsync(buf.data(), d, N * sizeof(double), hipMemcpyDeviceToHost, L->stream) ==
                 hipSuccess &&
             hipStreamSynchronize(L->stream) == hipSuccess;
        if (d) dev_free(L, d);
        ok = ok && std::fwrite(buf.data(), 8, N, fp) == N;
    } else if (ok && L->force_mode != kForceNone) {
        const int nc = L->force_mode == kForceDense ? 3 : 1;
        std::vector<char> buf(N * compute_bytes(L->precision));
        for (int k = 0; k < nc && ok; ++k) {
            ok = hipMemcpy(buf.data(), (char *)L->force + k * Ns * compute_bytes(L->precision),
                           buf.size(), hipMemcpyDeviceToHost) == hipSuccess &&
                 std::fwrite(buf.data(), 1, buf.size(), fp) == buf.size();
        }
    }
    // populations, raw storage format
    if (ok) {
        const size_t es = storage_bytes(L->precision);
        std::vector<char> buf(N * es);
        for (int q = 0; q < Q && ok; ++q) {
            ok = hipMemcpy(buf.data(), (char *)L->f[L->cur] + q * Ns * es, buf.size(),
                           hipMemcpyDeviceToHost) == hipSuccess &&
                 std::fwrite(buf.data(), 1, buf.size(), fp) == buf.size();
        }
    }
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return fail(LBMEP_EDEVICE, "checkpoint write failed");
    return LBMEP_OK;
}

int lbmep_load_state(lbmep_lattice *L, const char *path) {
    if (!L || !path) return fail(LBMEP_EINVAL, "null argument");
    int rc = set_device(L);
    if (rc) return rc;
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return fail(LBMEP_EINVAL, std::string("cannot open ") + path);
    Header h{};
    bool ok = std::fread(&h, sizeof h, 1, fp) == 1 && std::memcmp(h.magic, kMagic, 8) == 0 &&
              h.nx == L->g.nx && h.ny == L->g.ny && h.nz == L->g.nz && h.per[0] == L->g.per[0] &&
              h.per[1] == L->g.per[1] && h.per[2] == L->g.per[2] &&
              h.precision == L->precision && h.move == L->cfg.move_particles &&
              h.nu == L->cfg.nu && h.magic_param == L->cfg.magic && h.np >= 0 && h.level >= 0 &&
              (h.nzeta == 0 || h.nzeta == h.np) && (h.nq == 0 || h.nq == h.np) &&
              (h.dyn == 0 || (h.dyn == 1 && h.move)) && (h.slip & ~63) == 0 &&
              h.force_mode >= kForceNone &&
              h.force_mode <= kForcePotential;
    if (!ok) {
        std::fclose(fp);
        return fail(LBMEP_EINVAL, "checkpoint does not match this lattice");
    }
    const size_t N = L->g.N, Ns = L->g.Ns;
    std::vector<double> X(3 * (size_t)h.np), R(h.np), U(3 * (size_t)h.np), W(3 * (size_t)h.np);
    if (h.np > 0)
        ok = std::fread(X.data(), 8, X.size(), fp) == X.size() &&
             std::fread(R.data(), 8, R.size(), fp) == R.size() &&
             std::fread(U.data(), 8, U.size(), fp) == U.size() &&
             std::fread(W.data(), 8, W.size(), fp) == W.size();
    std::vector<double> zeta(h.nzeta);
    if (h.nzeta > 0) ok = ok && std::fread(zeta.data(), 8, zeta.size(), fp) == zeta.size();
    std::vector<double> qv(h.nq);
    if (h.nq > 0) ok = ok && std::fread(qv.data(), 8, qv.size(), fp) == qv.size();
    std::vector<uint8_t> fl(N);
    ok = ok && std::fread(fl.data(), 1, N, fp) == N;
    const int nc = h.force_mode == kForceDense ? 3 : (h.force_mode == kForceNone ? 0 : 1);
    const size_t fbytes = h.force_mode == kForcePotential ? 8 : compute_bytes(L->precision);
    std::vector<char> force(nc * N * fbytes);
    ok = ok && std::fread(force.data(), 1, force.size(), fp) == force.size();
    const size_t es = storage_bytes(L->precision);
    std::vector<char> pdf(Q * N * es);
    ok = ok && std::fread(pdf.data(), 1, pdf.size(), fp) == pdf.size();
    std::fclose(fp);
    if (!ok) return fail(LBMEP_EINVAL, "truncated checkpoint");
    // walls, particles (time level 0 map), then the saved time level
    rc = lbmep_set_flags(L, fl.data(), 0);
    if (rc) return rc;
    L->slip = h.slip;
    rc = lbmep_set_particles(L, h.np, X.data(), R.data(), U.data(), W.data());
    if (rc) return rc;
    if (h.dyn) {
        // the table holds the saved level's positions and velocities
        rc = lbmep_set_dynamics(L, h.rho_p, h.nq > 0 ? qv.data() : nullptr, h.Edyn);
        if (rc) return rc;
    }
    L->level = h.level;
    rc = remap_all(L);
    if (rc) return rc;
    if (nc > 0) {
        const size_t need = nc * Ns * compute_bytes(L->precision);
        if (L->force_bytes < need) {
            dev_free(L, L->force);
            L->force = nullptr;
            L->force_bytes = 0;
            if (dev_alloc(L, (void **)&L->force, need) != hipSuccess) return fail(LBMEP_ENOMEM, "force");
            L->force_bytes = need;
        }
        if (h.force_mode == kForcePotential) {
            // psi from cell order into its storage order
            double *d = nullptr;
            if (dev_alloc(L, (void **)&d, N * sizeof(double)) != hipSuccess)
                return fail(LBMEP_ENOMEM, "psi staging");
            hipError_t e = hipMemcpy(d, force.data(), N * sizeof(double), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = launch_potential_pack(L->precision, L->g, d, LBMEP_DTYPE_F64, L->force, L->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
            dev_free(L, d);
            if (e != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(e));
        } else {
            const size_t cb = N * compute_bytes(L->precision);
            for (int k = 0; k < nc; ++k)
                HIP_TRY(hipMemcpy((char *)L->force + k * Ns * compute_bytes(L->precision),
                                  force.data() + k * cb, cb, hipMemcpyHostToDevice));
        }
    }
    L->force_mode = h.force_mode;
    for (int k = 0; k < 3; ++k) L->E[k] = h.E[k];
    L->keps = h.keps;
    dev_free(L, L->zeta);
    L->zeta = nullptr;
    L->hzeta.clear();
    if (h.nzeta > 0) {
        if (dev_alloc(L, (void **)&L->zeta, 8 * (size_t)h.nzeta) != hipSuccess)
            return fail(LBMEP_ENOMEM, "zeta");
        L->hzeta = zeta;
        HIP_TRY(hipMemcpy(L->zeta, zeta.data(), 8 * (size_t)h.nzeta, hipMemcpyHostToDevice));
    }
    for (int q = 0; q < Q; ++q)
        HIP_TRY(hipMemcpy((char *)L->f[L->cur] + q * Ns * es, pdf.data() + q * N * es, N * es,
                          hipMemcpyHostToDevice));
    HIP_TRY(hipStreamSynchronize(L->stream));
    L->sor_set = false;
    if (h.sor_set) {
        rc = lbmep_set_potential_solver(L, h.sor_kappa2, h.sor_omega, h.sor_iters, h.sor_rf,
                                        h.sor_check);
        if (rc) return rc;
    }
    L->pmode = false;
    return LBMEP_OK;
}

}  // extern "C"
