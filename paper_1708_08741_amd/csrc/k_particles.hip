// k_particles.hip -- prescribed kinematics, obstacle mapping and NEAR /
// uncovered cell classification (arXiv:1708.08741, Sec. 3.2: a cell is an
// obstacle cell of a particle iff its centre lies inside it; uncovered cells
// are refilled with f^eq(rho0, u_s) by the sweep).
//
// Every per-particle kernel runs one block per particle over the particle's
// bounding box of cells.  The inside test uses the same FP64 operation
// sequence as a plain CPU evaluation (no contraction), so maps are
// bit-identical to it; shared cells go to the lowest particle index via an
// atomic minimum.
#include <cmath>

#include "lbmep_internal.h"

namespace lbmep {
namespace {

constexpr int kBoxThreads = 256;

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

// cell range [lo, lo+cnt) of a box on one axis, before wrapping
struct Box {
    int lo[3], cnt[3];
};

__device__ __forceinline__ void axis_range(double xmin, double xmax, int len, int periodic,
                                           int &lo, int &cnt) {
    // computed in FP64 so that huge radii cannot overflow the integer range
    double l = floor(xmin) - 1.0;
    double h = floor(xmax) + 1.0;
    if (periodic) {
        if (h - l + 1.0 >= (double)len) {
            l = 0.0;
            h = (double)len - 1.0;
        }
    } else {
        if (l < 0.0) l = 0.0;
        if (h > (double)len - 1.0) h = (double)len - 1.0;
    }
    lo = (int)l;
    cnt = h >= l ? (int)(h - l + 1.0) : 0;
}

__device__ __forceinline__ int box_size(const Box &b) {
    return (b.cnt[0] > 0 && b.cnt[1] > 0 && b.cnt[2] > 0) ? b.cnt[0] * b.cnt[1] * b.cnt[2] : 0;
}

// box around the ball of radius R at X (generous: every cell whose centre
// can be inside is in it)
__device__ __forceinline__ Box ball_box(const Grid &g, const double *X, double R) {
    Box b;
    const int len[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) axis_range(X[k] - R, X[k] + R, len[k], g.per[k], b.lo[k], b.cnt[k]);
    return b;
}

// floor(i / d) for i >= 0, d >= 1, with rd ~ 1 / d: the product in single
// precision is within a few units of the quotient, the integer corrections
// make it exact (an integer division is a long instruction sequence)
__device__ __forceinline__ int div_exact(int i, int d, float rd) {
    int q = (int)((float)i * rd);
    int r = i - q * d;
    while (r < 0) {
        --q;
        r += d;
    }
    while (r >= d) {
        ++q;
        r -= d;
    }
    return q;
}

// v wrapped into [0, len): box coordinates lie within one period of the
// grid, so one addition or subtraction does it (the remainder otherwise)
__device__ __forceinline__ int wrap_axis(int v, int len) {
    if (v < 0) v += len;
    else if (v >= len) v -= len;
    if (v < 0 || v >= len) v = ((v % len) + len) % len;
    return v;
}

// box-relative coordinates (ix, iy, iz) of the i-th cell of a box of
// cx x cy x ... cells (rcx, rcy: reciprocals of cx, cy)
__device__ __forceinline__ void box_split(int i, int cx, int cy, float rcx, float rcy, int &ix,
                                          int &iy, int &iz) {
    const int q = div_exact(i, cx, rcx);
    ix = i - q * cx;
    iz = div_exact(q, cy, rcy);
    iy = q - iz * cy;
}

// the i-th cell of a box (wrapped on periodic axes)
__device__ __forceinline__ void box_cell(const Grid &g, const Box &b, int i, int &x, int &y,
                                         int &z) {
    const int cx = b.cnt[0], cy = b.cnt[1];
    int ix, iy, iz;
    box_split(i, cx, cy, 1.0f / (float)cx, 1.0f / (float)cy, ix, iy, iz);
    x = b.lo[0] + ix;
    y = b.lo[1] + iy;
    z = b.lo[2] + iz;
    if (g.per[0]) x = wrap_axis(x, g.nx);
    if (g.per[1]) y = wrap_axis(y, g.ny);
    if (g.per[2]) z = wrap_axis(z, g.nz);
}

__device__ __forceinline__ size_t cell_of(const Grid &g, int x, int y, int z) {
    return (size_t)x + (size_t)g.nx * ((size_t)y + (size_t)g.ny * (size_t)z);
}

__device__ __forceinline__ double position(const ParticleArgs &pa, int p, int k, int64_t level);

__global__ void k_positions(ParticleArgs pa, int64_t level, double *X) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pa.np) return;
    for (int k = 0; k < 3; ++k) X[3 * p + k] = position(pa, p, k, level);
}

// inside test of Sec. 3.2 (closed ball, minimum image), FP64 without
// contraction, as a plain CPU evaluation orders it
__device__ __forceinline__ bool inside_ball(const Grid &g, int x, int y, int z, const double *Xp,
                                            double R) {
    const double r0 = min_image(((double)x + 0.5) - Xp[0], g.nx, g.per[0]);
    const double r1 = min_image(((double)y + 0.5) - Xp[1], g.ny, g.per[1]);
    const double r2 = min_image(((double)z + 0.5) - Xp[2], g.nz, g.per[2]);
    const double d2 = (r0 * r0 + r1 * r1) + r2 * r2;
    return d2 <= R * R;
}

// clear the cells particle p covered at position X (every cell of the map
// lies in the ball of some particle, so clearing each particle's ball
// empties the map; the following set re-claims shared cells)
__device__ __forceinline__ void map_clear_particle(const ParticleArgs &pa, int p,
                                                   const double *X, uint32_t *owner) {
    const double *Xp = X + 3 * p;
    const double R = pa.R[p];
    const Box b = ball_box(pa.g, Xp, R);
    const int n = box_size(b);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int x, y, z;
        box_cell(pa.g, b, i, x, y, z);
        if (inside_ball(pa.g, x, y, z, Xp, R)) owner[cell_of(pa.g, x, y, z)] = kNone;
    }
}

__global__ void __launch_bounds__(kBoxThreads)
    k_map_clear(ParticleArgs pa, const double *X, uint32_t *owner) {
    map_clear_particle(pa, blockIdx.x, X, owner);
}

// X_p(level) of the prescribed kinematics, component k, wrapped into [0, L)
// on periodic axes
__device__ __forceinline__ double position(const ParticleArgs &pa, int p, int k, int64_t level) {
    const int len[3] = {pa.g.nx, pa.g.ny, pa.g.nz};
    double x = pa.X0[3 * p + k];
    // prescribed kinematics X(n) = X(0) + n U, evaluated in this form; with
    // dynamics X0 already holds the level's position
    if (pa.moving && !pa.dynamic) x = pa.X0[3 * p + k] + (double)level * pa.U[3 * p + k];
    if (pa.g.per[k]) {
        x = x - (double)len[k] * floor(x / (double)len[k]);
        if (x >= (double)len[k]) x -= (double)len[k];
    }
    return x;
}

// one particle of the step's kinematics: clear its cells of the map that the
// buffer held (two levels back), then store its position at `level`
__device__ __forceinline__ void advance_particle(const ParticleArgs &pa, int p, int64_t level,
                                                 double *X, uint32_t *owner) {
    map_clear_particle(pa, p, X, owner);
    __syncthreads();  // every thread has read the old position
    if (threadIdx.x < 3) X[3 * p + threadIdx.x] = position(pa, p, threadIdx.x, level);
}

__global__ void __launch_bounds__(kBoxThreads)
    k_advance(ParticleArgs pa, int64_t level, double *X, uint32_t *owner) {
    advance_particle(pa, blockIdx.x, level, X, owner);
}

__device__ __forceinline__ void map_set_particle(const ParticleArgs &pa, int p, const double *X,
                                                 const uint8_t *flag, uint32_t *owner) {
    const double *Xp = X + 3 * p;
    const double R = pa.R[p];
    const Box b = ball_box(pa.g, Xp, R);
    const int n = box_size(b);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int x, y, z;
        box_cell(pa.g, b, i, x, y, z);
        if (!inside_ball(pa.g, x, y, z, Xp, R)) continue;
        const size_t c = cell_of(pa.g, x, y, z);
        if (!(flag[c] & kWall)) atomicMin(&owner[c], (uint32_t)p);
    }
}

__global__ void __launch_bounds__(kBoxThreads)
    k_map_set(ParticleArgs pa, const double *X, const uint8_t *flag, uint32_t *owner) {
    map_set_particle(pa, blockIdx.x, X, flag, owner);
}

// exclusive prefix of `mine` over the workgroup (256 threads); returns the
// workgroup total in *total
__device__ __forceinline__ uint32_t block_scan(uint32_t mine, uint32_t *wsum, uint32_t *total) {
    const int tid = threadIdx.x, lane = (int)__lane_id(), wave = tid / 64;
    uint32_t incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t pre = incl - mine;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    return pre;
}

// one cell's classification from the wall bits and the map (global reads):
// its flag; *wmask = directions whose neighbour is a wall cell; *pmask =
// directions whose neighbour is an obstacle cell of particle p (p != kNone);
// with owner_old, a fluid cell that was an obstacle cell is marked uncovered
__device__ __forceinline__ uint8_t classify_cell(const Grid &g, int x, int y, int z,
                                                 const uint8_t *flag, const uint32_t *owner,
                                                 const uint32_t *owner_old, uint32_t p,
                                                 uint32_t *wmask, uint32_t *pmask) {
    const size_t c = cell_of(g, x, y, z);
    const uint8_t wall = flag[c] & kWall;
    uint8_t f = wall;
    uint32_t mask = 0, wm = 0, pm = 0;
    if (!wall) {
        if (owner && owner[c] != kNone) {
            f = kObst;
        } else {
#pragma unroll
            for (int q = 1; q < Q; ++q) {
                int sx = x + kCx[q], sy = y + kCy[q], sz = z + kCz[q];
                bool solid = false;
                if (sx < 0 || sx >= g.nx) {
                    if (g.per[0]) sx = sx < 0 ? sx + g.nx : sx - g.nx; else solid = true;
                }
                if (sy < 0 || sy >= g.ny) {
                    if (g.per[1]) sy = sy < 0 ? sy + g.ny : sy - g.ny; else solid = true;
                }
                if (sz < 0 || sz >= g.nz) {
                    if (g.per[2]) sz = sz < 0 ? sz + g.nz : sz - g.nz; else solid = true;
                }
                if (!solid) {
                    const size_t s = cell_of(g, sx, sy, sz);
                    const bool w = flag[s] & kWall;
                    const uint32_t o = owner ? owner[s] : kNone;
                    solid = w || o != kNone;
                    if (w) wm |= 1u << (q - 1);
                    if (!w && o != kNone && o == p) pm |= 1u << (q - 1);
                }
                if (solid) mask |= 1u << (q - 1);
            }
            f = (mask ? kNear : 0) | ((mask & kFaceDirs) ? kNear7 : 0);
            if (owner_old && owner_old[c] != kNone) f |= kUncov;
        }
    }
    *wmask = wm;
    *pmask = pm;
    return f | wall;
}

// the whole grid (after the flags or the particle table changed): flags and
// the wall-link masks of every cell
__global__ void k_classify_all(Grid g, uint8_t *flag, uint32_t *wallmask, const uint32_t *owner) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= g.nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    uint32_t wm, pm;
    const uint8_t f = classify_cell(g, x, y, z, flag, owner, nullptr, kNone, &wm, &pm);
    const size_t c = cell_of(g, x, y, z);
    flag[c] = f;
    wallmask[c] = wm;
}

// state bits of a box plus a one-cell halo, staged in LDS for the
// classification (boxes up to the staging capacity, at most kHaloCells
// cells; larger ones use the global path): solid (wall, obstacle of the new
// map, or beyond a non-periodic edge), obstacle cell of this particle,
// obstacle cell, wall cell
constexpr int kHaloCells = 32768;
constexpr uint8_t kHSolid = 1, kHMine = 2, kHObst = 4, kHWall = 8;

// Classification around one particle p (union of its boxes at the old and
// new positions, grown by one cell): flags of the new level and the list of
// p's links, (cell, directions whose neighbour is an obstacle cell of p), for
// the bounce-back / exchange kernel.  The list is compacted in box order.
__device__ __forceinline__ void classify_particle(const ParticleArgs &pa, int p,
                                                  const double *Xold, const double *Xnew,
                                                  uint8_t *flag, const uint32_t *owner_new,
                                                  const uint32_t *owner_old, uint8_t *solid,
                                                  int cap) {
    __shared__ uint32_t wcnt[kBoxThreads / 64][8];
    const Grid &g = pa.g;
    const double R = pa.R[p];
    Box b;
    {
        const int len[3] = {g.nx, g.ny, g.nz};
        for (int k = 0; k < 3; ++k) {
            const double a0 = Xold[3 * p + k], a1 = Xnew[3 * p + k];
            double mn = a0 < a1 ? a0 : a1, mx = a0 < a1 ? a1 : a0;
            // a particle that wrapped around a periodic axis: cover both ends
            if (g.per[k] && mx - mn > 0.5 * (double)len[k]) {
                mn = 0.0;
                mx = (double)len[k];
            }
            // one more cell on each side for the NEAR ring and for the
            // uncovered marks of the previous level (motion < 1 cell/step)
            axis_range(mn - R - 1.0, mx + R + 1.0, len[k], g.per[k], b.lo[k], b.cnt[k]);
        }
    }
    const int n = box_size(b);
    uint2 *plist = pa.plist + (size_t)p * pa.pcap;
    uint32_t base = 0;
    const int hx = b.cnt[0] + 2, hy = b.cnt[1] + 2, hz = b.cnt[2] + 2;
    const int hn = hx * hy * hz;
    const bool staged = n > 0 && hn <= cap;
    const float rhx = 1.0f / (float)hx, rhy = 1.0f / (float)hy;
    const float rcx = 1.0f / (float)b.cnt[0], rcy = 1.0f / (float)b.cnt[1];
    if (staged) {
        const int len[3] = {g.nx, g.ny, g.nz};
        // four halo cells per thread and pass, their loads issued together
        constexpr int kU = 4;
        for (int i0 = 0; i0 < hn; i0 += kU * (int)blockDim.x) {
            uint8_t fw[kU];
            uint32_t ow[kU];
            bool in[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                int ix, iy, iz;
                box_split(i, hx, hy, rhx, rhy, ix, iy, iz);
                int v[3] = {b.lo[0] - 1 + ix, b.lo[1] - 1 + iy, b.lo[2] - 1 + iz};
                bool out = i >= hn;
                for (int k = 0; k < 3; ++k) {
                    if (v[k] < 0 || v[k] >= len[k]) {
                        if (g.per[k]) v[k] = wrap_axis(v[k], len[k]); else out = true;
                    }
                }
                in[u] = !out;
                fw[u] = 0;
                ow[u] = kNone;
                if (!out) {
                    const size_t c = cell_of(g, v[0], v[1], v[2]);
                    fw[u] = flag[c];
                    ow[u] = owner_new[c];
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = i0 + u * (int)blockDim.x + (int)threadIdx.x;
                if (i >= hn) continue;
                uint8_t sv = kHSolid;
                if (in[u]) {
                    sv = 0;
                    if (fw[u] & kWall) sv = kHSolid | kHWall;
                    else if (ow[u] != kNone)
                        sv = kHSolid | kHObst | (ow[u] == (uint32_t)p ? kHMine : 0);
                }
                solid[i] = sv;
            }
        }
        __syncthreads();
    }
    // box cells: kPer cells per thread and pass, consecutive lanes on
    // consecutive cells (conflict-free LDS reads), their loads issued
    // together, one barrier per pass for the link-list positions
    constexpr int kPer = 8;
    for (int base0 = 0; base0 < n; base0 += kPer * (int)blockDim.x) {
        uint32_t cells[kPer], pms[kPer];
        uint8_t fl[kPer];
        bool fluid[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = base0 + j * (int)blockDim.x + (int)threadIdx.x;
            cells[j] = 0;
            pms[j] = 0;
            fl[j] = 0;
            fluid[j] = false;
            if (i >= n) continue;
            int ix, iy, iz;
            box_split(i, b.cnt[0], b.cnt[1], rcx, rcy, ix, iy, iz);
            int x = b.lo[0] + ix, y = b.lo[1] + iy, z = b.lo[2] + iz;
            if (g.per[0]) x = wrap_axis(x, g.nx);
            if (g.per[1]) y = wrap_axis(y, g.ny);
            if (g.per[2]) z = wrap_axis(z, g.nz);
            const size_t c = cell_of(g, x, y, z);
            cells[j] = (uint32_t)c;
            if (staged) {
                // the cell itself is in the staged box: no global re-reads
                const int h = (ix + 1) + hx * ((iy + 1) + hy * (iz + 1));
                const uint8_t me = solid[h];
                if (me & kHWall) {
                    fl[j] = kWall;
                } else if (me & kHObst) {
                    fl[j] = kObst;
                } else {
                    uint32_t mask = 0, pm = 0;
#pragma unroll
                    for (int q = 1; q < Q; ++q) {
                        const uint8_t sv = solid[h + kCx[q] + hx * (kCy[q] + hy * kCz[q])];
                        if (sv & kHSolid) mask |= 1u << (q - 1);
                        if (sv & kHMine) pm |= 1u << (q - 1);
                    }
                    fl[j] = (mask ? kNear : 0) | ((mask & kFaceDirs) ? kNear7 : 0);
                    pms[j] = pm;
                    fluid[j] = true;
                }
            } else {
                uint32_t wm;
                fl[j] = classify_cell(g, x, y, z, flag, owner_new, nullptr, (uint32_t)p, &wm,
                                      &pms[j]);
                fluid[j] = !(fl[j] & (kWall | kObst));
            }
        }
        // uncovered marks: the previous map, loads issued together
        uint32_t old[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) old[j] = fluid[j] ? owner_old[cells[j]] : kNone;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int i = base0 + j * (int)blockDim.x + (int)threadIdx.x;
            if (i >= n) continue;
            flag[cells[j]] = fl[j] | (old[j] != kNone ? kUncov : 0);
        }
        // append (cell, mask) of this pass's cells with links into p, in box
        // order (j-major, then wavefront, then lane): per-row ballots give
        // each lane's rank in its wavefront, one LDS exchange of the
        // wavefronts' counts gives the offsets
        const int lane = (int)__lane_id(), wave = (int)threadIdx.x / 64;
        const unsigned long long below = (1ull << lane) - 1ull;
        uint32_t rank[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const unsigned long long bj = __ballot(pms[j] != 0);
            rank[j] = (uint32_t)__popcll(bj & below);
            if (lane == 0) wcnt[wave][j] = (uint32_t)__popcll(bj);
        }
        __syncthreads();
        uint32_t run = base;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            uint32_t pre = 0, row = 0;
            for (int w = 0; w < kBoxThreads / 64; ++w) {
                row += wcnt[w][j];
                if (w < wave) pre += wcnt[w][j];
            }
            if (pms[j]) {
                const uint32_t pos = run + pre + rank[j];
                if (pos < pa.pcap) plist[pos] = make_uint2(cells[j], pms[j]);
            }
            run += row;
        }
        base = run;
        __syncthreads();  // wcnt is reused by the next pass
    }
    if (threadIdx.x == 0) pa.pcount[p] = base < pa.pcap ? base : pa.pcap;
}

// the staging array is dynamic LDS of pa.halo_cap bytes, sized for the
// largest particle: a 32 KiB array for R = 4 boxes of < 5 KiB would hold the
// CU to 5 workgroups
__global__ void __launch_bounds__(kBoxThreads, 6)
    k_classify_boxes(ParticleArgs pa, const double *Xold, const double *Xnew, uint8_t *flag,
                     const uint32_t *owner_new, const uint32_t *owner_old) {
    extern __shared__ uint8_t solid[];
    classify_particle(pa, blockIdx.x, Xold, Xnew, flag, owner_new, owner_old, solid,
                      (int)pa.halo_cap);
}

// compact list, in cell order, of the cells with a wall link (wall-link mask
// != 0), by a three-kernel scan (no contended atomics): per-block counts, a
// scan of the counts in tiles of 1024, then each block writing its cells
// from its offset.  A thread reads the masks of 16 consecutive cells as four
// 16-byte loads (the mask array is padded to a multiple of kListChunk).
// Built when the walls or the particle table are set, not per step.
constexpr int kListCells = 16;
constexpr int kListChunk = 256 * kListCells;

__device__ __forceinline__ uint32_t wall_bits(const Grid &g, const uint32_t *wallmask, size_t c0) {
    const uint4 *v = reinterpret_cast<const uint4 *>(wallmask + c0);
    uint32_t take = 0;  // bit k: cell c0 + k has a wall link
#pragma unroll
    for (int j = 0; j < kListCells / 4; ++j) {
        const uint4 m = v[j];
        const uint32_t w[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (w[i] && c0 + 4 * j + i < g.N) take |= 1u << (4 * j + i);
    }
    return take;
}

__global__ void __launch_bounds__(256) k_wall_count(Grid g, const uint32_t *wallmask,
                                                    uint32_t *bcount) {
    __shared__ uint32_t wsum[4];
    const size_t c0 = (size_t)blockIdx.x * kListChunk + (size_t)threadIdx.x * kListCells;
    uint32_t total;
    block_scan((uint32_t)__popc(wall_bits(g, wallmask, c0)), wsum, &total);
    if (threadIdx.x == 0) bcount[blockIdx.x] = total;
}

// second level of the scan: workgroup t turns the counts of list blocks
// [1024 t, 1024 t + 1024) into exclusive prefixes within that tile (one
// coalesced load per thread) and stores the tile total after the counts
constexpr int kTile = 1024;

__global__ void __launch_bounds__(kTile) k_wall_tiles(uint32_t *bcount, int nb) {
    const uint32_t tile = blockIdx.x;
    __shared__ uint32_t wsum[kTile / 64];
    const int tid = threadIdx.x, lane = (int)__lane_id(), wave = tid / 64;
    const size_t i = (size_t)tile * kTile + tid;
    const uint32_t mine = i < (size_t)nb ? bcount[i] : 0u;
    uint32_t incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)incl, off);
        if (lane >= off) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t pre = incl - mine;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    if (i < (size_t)nb) bcount[i] = pre;
    if (tid == kTile - 1) {
        uint32_t tot = 0;
        for (int w = 0; w < kTile / 64; ++w) tot += wsum[w];
        bcount[nb + tile] = tot;
    }
}

// list block blk writes its cells from its offset: the exclusive prefix
// within its tile plus the totals of the earlier tiles; the last block also
// stores the list length
__global__ void __launch_bounds__(256) k_wall_write(Grid g, const uint32_t *wallmask,
                                                    const uint32_t *bcount, int nb,
                                                    uint32_t *list, uint32_t *count) {
    __shared__ uint32_t wsum[4];
    const uint32_t blk = blockIdx.x;
    const size_t c0 = (size_t)blk * kListChunk + (size_t)threadIdx.x * kListCells;
    const uint32_t take = wall_bits(g, wallmask, c0);
    uint32_t off = bcount[blk];
    const uint32_t *tsum = bcount + nb;
    for (uint32_t t = 0; t < blk / kTile; ++t) off += tsum[t];
    uint32_t total;
    uint32_t pos = off + block_scan((uint32_t)__popc(take), wsum, &total);
#pragma unroll
    for (int k = 0; k < kListCells; ++k)
        if (take & (1u << k)) list[pos++] = (uint32_t)(c0 + k);
    if (blk == (uint32_t)nb - 1 && threadIdx.x == 0) *count = off + total;
}

// ---------------------------------------------------------------------------
// packed forms: one dispatch for several lattices (entry by binary search);
// the particle kernels use the map / position buffer the step writes,
// b = 1 - cur_owner
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBoxThreads) k_advance_packed(PackTable t) {
    const int e = pack_find(t, blockIdx.x);
    const LatticeDev *d = t.d[e];
    const ParticleArgs pa = d->pa;
    const int b = 1 - (int)(t.state[e] >> 1);
    advance_particle(pa, (int)(blockIdx.x - t.start[e]), t.level[e], d->Xheld[b], d->owner[b]);
}

__global__ void __launch_bounds__(kBoxThreads) k_map_set_packed(PackTable t) {
    const int e = pack_find(t, blockIdx.x);
    const LatticeDev *d = t.d[e];
    const ParticleArgs pa = d->pa;
    const int b = 1 - (int)(t.state[e] >> 1);
    map_set_particle(pa, (int)(blockIdx.x - t.start[e]), d->Xheld[b], d->flag, d->owner[b]);
}

__global__ void __launch_bounds__(kBoxThreads) k_classify_packed(PackTable t) {
    __shared__ uint8_t solid[kHaloCells];
    const int e = pack_find(t, blockIdx.x);
    const LatticeDev *d = t.d[e];
    const ParticleArgs pa = d->pa;
    const int co = (int)(t.state[e] >> 1), b = 1 - co;
    classify_particle(pa, (int)(blockIdx.x - t.start[e]), d->Xheld[co], d->Xheld[b], d->flag,
                      d->owner[b], d->owner[co], solid, kHaloCells);
}

// F = F_dev + K/18 and M = M_dev + (T - X x K)/18 from the per-particle
// accumulators F_dev[3], M_dev[3], K[3], T[3] of the sweep
__global__ void k_finalize_ft(int np, const double *acc, const double *X, double *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const double *t = acc + 12 * (size_t)p;
    const double *Xp = X + 3 * (size_t)p;
    out[6 * (size_t)p + 0] = t[0] + t[6] / 18.0;
    out[6 * (size_t)p + 1] = t[1] + t[7] / 18.0;
    out[6 * (size_t)p + 2] = t[2] + t[8] / 18.0;
    out[6 * (size_t)p + 3] = t[3] + (t[9] - (Xp[1] * t[8] - Xp[2] * t[7])) / 18.0;
    out[6 * (size_t)p + 4] = t[4] + (t[10] - (Xp[2] * t[6] - Xp[0] * t[8])) / 18.0;
    out[6 * (size_t)p + 5] = t[5] + (t[11] - (Xp[0] * t[7] - Xp[1] * t[6])) / 18.0;
}

// Newton-Euler update of particle p (Alg. "Electrophoresis Algorithm": the
// hydrodynamic force and torque of the step and the force q E of the
// applied field move the particle), one explicit step, velocities first:
//     U += (F_h + q E) / m,  W += M_h / I,  X(n+1) = X(n) + U,
// m = rho_p 4/3 pi R^3, I = 2/5 m R^2; F_h, M_h assembled as k_finalize_ft
// does, in the same order
__global__ void k_dynamics(DynArgs d) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.np) return;
    const double *t = d.acc + 12 * (size_t)p;
    const double *Xp = d.X + 3 * (size_t)p;
    double F[3], M[3];
    F[0] = t[0] + t[6] / 18.0;
    F[1] = t[1] + t[7] / 18.0;
    F[2] = t[2] + t[8] / 18.0;
    M[0] = t[3] + (t[9] - (Xp[1] * t[8] - Xp[2] * t[7])) / 18.0;
    M[1] = t[4] + (t[10] - (Xp[2] * t[6] - Xp[0] * t[8])) / 18.0;
    M[2] = t[5] + (t[11] - (Xp[0] * t[7] - Xp[1] * t[6])) / 18.0;
    const double R = d.R[p];
    const double m = d.rho_p * (4.0 / 3.0) * 3.14159265358979323846 * R * R * R;
    const double I = 0.4 * m * R * R;
    const double qp = d.q ? d.q[p] : 0.0;
    const int len[3] = {d.g.nx, d.g.ny, d.g.nz};
    bool fast = false;
    for (int a = 0; a < 3; ++a) {
        const double u = d.U[3 * p + a] + (F[a] + qp * d.E[a]) / m;
        d.U[3 * p + a] = u;
        d.W[3 * p + a] = d.W[3 * p + a] + M[a] / I;
        fast = fast || !(fabs(u) < 1.0);
        double x = Xp[a] + u;
        if (d.g.per[a]) {
            x = x - (double)len[a] * floor(x / (double)len[a]);
            if (x >= (double)len[a]) x -= (double)len[a];
        }
        d.X0[3 * p + a] = x;
    }
    if (fast) *d.too_fast = 1;
}

}  // namespace

hipError_t launch_dynamics(const DynArgs &d, hipStream_t s) {
    if (d.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dynamics, dim3((d.np + 127) / 128), dim3(128), 0, s, d);
    return hipGetLastError();
}

int wall_list_blocks(const Grid &g) { return (int)((g.N + kListChunk - 1) / kListChunk); }
int wall_list_tiles(const Grid &g) { return (wall_list_blocks(g) + kTile - 1) / kTile; }
size_t wall_list_scratch(const Grid &g) {
    return (size_t)wall_list_blocks(g) + (size_t)wall_list_tiles(g) + 64;
}

uint32_t halo_capacity(double r_max) {
    const double e = 2.0 * std::ceil(r_max) + 9.0;
    const double c = e * e * e;
    return c > (double)kHaloCells ? (uint32_t)kHaloCells : (uint32_t)c;
}

uint32_t link_capacity(double r_max) {
    const double e = 2.0 * std::ceil(r_max) + 3.0;
    return (uint32_t)(e * e * e);
}

hipError_t launch_wall_list(const Grid &g, const uint32_t *wallmask, uint32_t *list,
                            uint32_t *count, uint32_t *scratch, hipStream_t s) {
    const int nb = wall_list_blocks(g);
    hipLaunchKernelGGL(k_wall_count, dim3(nb), dim3(256), 0, s, g, wallmask, scratch);
    hipLaunchKernelGGL(k_wall_tiles, dim3(wall_list_tiles(g)), dim3(kTile), 0, s, scratch, nb);
    hipLaunchKernelGGL(k_wall_write, dim3(nb), dim3(256), 0, s, g, wallmask, scratch, nb, list,
                       count);
    return hipGetLastError();
}

hipError_t launch_finalize_ft(int np, const double *acc, const double *X, double *out,
                              hipStream_t s) {
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_ft, dim3((np + 127) / 128), dim3(128), 0, s, np, acc, X, out);
    return hipGetLastError();
}

hipError_t launch_advance(const ParticleArgs &pa, int64_t level, double *X, uint32_t *owner,
                          hipStream_t s) {
    if (pa.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_advance, dim3(pa.np), dim3(kBoxThreads), 0, s, pa, level, X, owner);
    return hipGetLastError();
}

namespace {
template <typename K>
hipError_t launch_packed(K kernel, const PackTable &t, int threads, hipStream_t s) {
    const uint32_t total = t.start[t.n];
    if (t.n == 0 || total == 0) return hipSuccess;
    hipLaunchKernelGGL(kernel, dim3(total), dim3(threads), 0, s, t);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_advance_packed(const PackTable &t, hipStream_t s) {
    return launch_packed(k_advance_packed, t, kBoxThreads, s);
}

hipError_t launch_map_set_packed(const PackTable &t, hipStream_t s) {
    return launch_packed(k_map_set_packed, t, kBoxThreads, s);
}

hipError_t launch_classify_packed(const PackTable &t, hipStream_t s) {
    return launch_packed(k_classify_packed, t, kBoxThreads, s);
}

hipError_t launch_positions(const ParticleArgs &pa, int64_t level, double *X, hipStream_t s) {
    if (pa.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_positions, dim3((pa.np + 127) / 128), dim3(128), 0, s, pa, level, X);
    return hipGetLastError();
}

hipError_t launch_map_clear(const ParticleArgs &pa, const double *X, uint32_t *owner,
                            hipStream_t s) {
    if (pa.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_clear, dim3(pa.np), dim3(kBoxThreads), 0, s, pa, X, owner);
    return hipGetLastError();
}

hipError_t launch_map_set(const ParticleArgs &pa, const double *X, const uint8_t *flag,
                          uint32_t *owner, hipStream_t s) {
    if (pa.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_set, dim3(pa.np), dim3(kBoxThreads), 0, s, pa, X, flag, owner);
    return hipGetLastError();
}

hipError_t launch_classify_all(const Grid &g, uint8_t *flag, uint32_t *wallmask,
                               const uint32_t *owner, hipStream_t s) {
    const int bx = 64;
    hipLaunchKernelGGL(k_classify_all, dim3((g.nx + bx - 1) / bx, g.ny, g.nz), dim3(bx), 0, s, g,
                       flag, wallmask, owner);
    return hipGetLastError();
}

hipError_t launch_classify_boxes(const ParticleArgs &pa, const double *Xold, const double *Xnew,
                                 uint8_t *flag, const uint32_t *owner_new,
                                 const uint32_t *owner_old, hipStream_t s) {
    if (pa.np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_classify_boxes, dim3(pa.np), dim3(kBoxThreads), pa.halo_cap, s, pa,
                       Xold, Xnew, flag, owner_new, owner_old);
    return hipGetLastError();
}

}  // namespace lbmep
