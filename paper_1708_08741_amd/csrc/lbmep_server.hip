// lbmep_server.hip -- request server: continuous batching of independent
// lattice Boltzmann simulations on one GPU (the C ABI lbmep_server_* of
// include/lbmep.h).
//
// Requests are queued on submit (all inputs copied).  A request is admitted
// (FIFO) when a slot is free and its device footprint fits the budget; its
// lattice is then built inside one pre-allocated device arena, so admission
// and retirement never call hipMalloc / hipFree (whose implicit device
// synchronisation would drain the pipeline of the other simulations).  Set-up
// runs on its own stream while the resident simulations keep stepping.
//
// Resident simulations advance together in chunks of steps.  Every step of a
// chunk is a short series of packed launches: one dispatch of each kernel of
// the step (sweep, bounce-back / exchange, kinematics, mapping,
// classification, NEAR-list scan) covers every resident lattice, each
// workgroup finding its lattice through a block table in the kernel
// arguments.  A simulation whose last step is in a chunk has its results
// (force and torque of the last step, FP64 mass / momentum of the final
// state, optionally the fields) computed right after that chunk on the same
// stream; when the host sees the completion event it copies them out and
// releases the lattice's memory to the arena.
//
// The arithmetic is that of the single-lattice path (the same device code):
// a simulation's fields, forces and torques are bitwise the same alone and
// in any mix (the per-particle sums are fixed-order wavefront and workgroup
// sums, no atomics).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>

#include "lattice.h"

using namespace lbmep;
using namespace lbmep::rt;

namespace {

// first-fit allocator over one device allocation; frees coalesce
class Arena final : public DevHeap {
  public:
    static constexpr size_t kAlign = 4096;

    ~Arena() override {
        if (base_) hipFree(base_);
    }
    hipError_t init(size_t bytes) {
        size_ = bytes / kAlign * kAlign;
        hipError_t e = hipMalloc(&base_, size_);
        if (e != hipSuccess) {
            base_ = nullptr;
            return e;
        }
        free_[0] = size_;
        return hipSuccess;
    }
    void *alloc(size_t bytes) override {
        const size_t need = std::max<size_t>(kAlign, (bytes + kAlign - 1) / kAlign * kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, rest = it->second - need;
            free_.erase(it);
            if (rest) free_[off + need] = rest;
            live_[off] = need;
            used_ += need;
            return base_ + off;
        }
        return nullptr;
    }
    void release(void *p) override {
        if (!p) return;
        const size_t off = (size_t)(static_cast<char *>(p) - base_);
        auto lv = live_.find(off);
        if (lv == live_.end()) return;
        size_t start = off, len = lv->second;
        live_.erase(lv);
        used_ -= len;
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    char *base_ = nullptr;
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;             // offset -> length
    std::unordered_map<size_t, size_t> live_;  // offset -> length
};

struct Request {
    uint64_t id = 0;
    lbmep_config cfg{};
    std::vector<uint8_t> flags;
    int32_t n = 0, steps = 0;
    std::vector<double> X, R, U, W;
    std::vector<char> rho_e;
    int32_t rho_dtype = 0;
    bool charge = false, keep_fields = false;
    double E[3] = {0, 0, 0};
    size_t footprint = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    // results
    bool done = false;
    int status = LBMEP_OK;
    std::string error;
    std::vector<double> F, M, rho, u;
    double inv[4] = {0, 0, 0, 0};
};

struct Slot {
    Request *req = nullptr;
    lbmep_lattice *L = nullptr;
    LatticeDev *d = nullptr;   // device descriptor (in the arena)
    int32_t to_enqueue = 0;    // steps not yet enqueued
    bool retiring = false;     // result read-out enqueued, waiting for its event
    hipEvent_t ev = nullptr;
    double *fields = nullptr;  // rho, u of the final state (arena), keep_fields only
};

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

bool small_offsets(const lbmep_config &c) {
    const size_t N = (size_t)c.nx * c.ny * c.nz;
    const size_t Ns = population_stride(N, c.precision);
    return 2 * Ns * storage_bytes(c.precision) < (size_t(1) << 32) && 4 * Ns < (size_t(1) << 32);
}

}  // namespace

struct lbmep_server {
    lbmep_server_config cfg{};
    std::chrono::steady_clock::time_point t0;
    Arena arena;
    hipStream_t main = nullptr, setup = nullptr;
    std::deque<std::unique_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> finished;
    std::deque<uint64_t> unreported;  // finished ids not yet returned by poll
    std::vector<Slot> slots;
    std::deque<hipEvent_t> chunk_ev;  // completion events of enqueued chunks
    std::deque<double> chunk_work;    // their cell updates
    std::vector<hipEvent_t> ev_pool;
    uint64_t next_id = 1;
    size_t reserved = 0;  // footprints of the resident requests
    lbmep_server_stats st{};
};

namespace {

hipEvent_t get_event(lbmep_server *S) {
    if (!S->ev_pool.empty()) {
        hipEvent_t e = S->ev_pool.back();
        S->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

size_t request_footprint(const lbmep_config &c, int32_t n, double r_max, bool charge, bool flags,
                         bool keep_fields) {
    const size_t N = (size_t)c.nx * c.ny * c.nz;
    size_t b = lattice_bytes(&c, n, r_max, charge ? kForceCharge : kForceNone, false);
    b += 32 * Arena::kAlign;                 // alignment of the lattice's arrays
    b += round_up(sizeof(LatticeDev), Arena::kAlign);
    // staging of the inputs during set-up
    size_t stage = 0;
    if (flags) stage = std::max(stage, N);
    if (charge) stage = std::max(stage, N * sizeof(double));
    b += round_up(stage, Arena::kAlign);
    if (keep_fields) b += round_up(4 * N * sizeof(double), Arena::kAlign);
    return b;
}

void fail_request(Request *r, int code, const std::string &msg) {
    r->status = code;
    r->error = msg;
}

// build the lattice of a request on the set-up stream, take its first step
// there (it starts from a post-stream state), and write its descriptor
int admit(lbmep_server *S, Slot &slot, Request *r) {
    lbmep_config c = r->cfg;
    c.device = S->cfg.device;
    c.stream = S->setup;
    lbmep_lattice *L = nullptr;
    int rc = create_lattice(&c, &S->arena, &L);
    if (rc) return rc;
    auto undo = [&](int code) {
        destroy_lattice(L, true);
        return code;
    };
    if (!r->flags.empty()) {
        rc = lbmep_set_flags(L, r->flags.data(), 0);
        if (rc) return undo(rc);
    }
    if (r->charge) {
        rc = lbmep_set_charge_force(L, r->rho_e.data(), r->rho_dtype, r->E, 0);
        if (rc) return undo(rc);
    }
    const double u0[3] = {0, 0, 0};
    rc = lbmep_init_equilibrium(L, 1.0, u0);
    if (rc) return undo(rc);
    rc = lbmep_set_particles(L, r->n, r->X.data(), r->R.data(), r->U.data(), r->W.data());
    if (rc) return undo(rc);
    rc = lbmep_step(L, 1);
    if (rc) return undo(rc);
    // device descriptor for the packed launches
    LatticeDev h{};
    for (int cur = 0; cur < 2; ++cur)
        for (int co = 0; co < 2; ++co) {
            SweepArgs a = sweep_args_state(L, cur, co);
            a.nxb = (L->g.nx + kPackBlockX - 1) / kPackBlockX;
            h.sweep[cur | (co << 1)] = a;
        }
    h.pa = particle_args(L);
    h.flag = L->flag;
    for (int b = 0; b < 2; ++b) {
        h.owner[b] = L->owner[b];
        h.Xheld[b] = L->Xheld[b];
    }
    h.wall_blocks = near_wall_blocks(L->g, L->has_walls);
    LatticeDev *d = static_cast<LatticeDev *>(S->arena.alloc(sizeof(LatticeDev)));
    if (!d) return undo(fail(LBMEP_ENOMEM, "arena exhausted (descriptor)"));
    double *fields = nullptr;
    if (r->keep_fields) {
        fields = static_cast<double *>(S->arena.alloc(4 * L->g.N * sizeof(double)));
        if (!fields) {
            S->arena.release(d);
            return undo(fail(LBMEP_ENOMEM, "arena exhausted (fields)"));
        }
    }
    hipError_t e = hipMemcpyAsync(d, &h, sizeof h, hipMemcpyHostToDevice, S->setup);
    if (e == hipSuccess) e = hipStreamSynchronize(S->setup);
    if (e != hipSuccess) {
        S->arena.release(d);
        S->arena.release(fields);
        return undo(fail(LBMEP_EDEVICE, std::string("descriptor: ") + hipGetErrorString(e)));
    }
    // from now on the lattice's work is enqueued on the main stream
    L->stream = S->main;
    slot.req = r;
    slot.L = L;
    slot.d = d;
    slot.fields = fields;
    slot.to_enqueue = r->steps - 1;
    slot.retiring = false;
    r->t_admit = now_s(S->t0);
    return LBMEP_OK;
}

// enqueue the result read-out of a slot whose last step is enqueued
int enqueue_readout(lbmep_server *S, Slot &slot) {
    lbmep_lattice *L = slot.L;
    hipStream_t s = S->main;
    if (L->np > 0)
        LBMEP_HIP_TRY(launch_finalize_ft(L->np, L->FM, L->Xheld[L->ft_buf],
                                         L->FM + 12 * (size_t)L->np, s));
    int rc = materialize(L);
    if (rc) return rc;
    double *dout = L->red + 5 * (size_t)L->red_blocks;
    LBMEP_HIP_TRY(launch_invariants(L->precision, L->g, L->f[L->cur], L->flag, L->red,
                                    L->red_blocks, dout, s));
    if (slot.fields) {
        const size_t N = L->g.N;
        LBMEP_HIP_TRY(launch_macro(L->precision, L->force_mode, L->g, L->f[L->cur], L->flag,
                                   L->np > 0 ? L->owner[L->cur_owner] : nullptr,
                                   L->np > 0 ? L->Xheld[L->cur_owner] : nullptr, L->U, L->W,
                                   L->force, L->E, L->keps, nullptr, slot.fields,
                                   slot.fields + N, s));
    }
    slot.ev = get_event(S);
    if (!slot.ev) return fail(LBMEP_EDEVICE, "event creation failed");
    LBMEP_HIP_TRY(hipEventRecord(slot.ev, s));
    slot.retiring = true;
    return LBMEP_OK;
}

// copy the results of a completed slot to its request and free the slot
void retire(lbmep_server *S, Slot &slot) {
    lbmep_lattice *L = slot.L;
    Request *r = slot.req;
    const size_t N = L->g.N;
    bool ok = true;
    if (L->np > 0) {
        std::vector<double> h(6 * (size_t)L->np);
        ok = hipMemcpy(h.data(), L->FM + 12 * (size_t)L->np, h.size() * sizeof(double),
                       hipMemcpyDeviceToHost) == hipSuccess;
        r->F.resize(3 * (size_t)L->np);
        r->M.resize(3 * (size_t)L->np);
        for (int p = 0; p < L->np; ++p)
            for (int k = 0; k < 3; ++k) {
                r->F[3 * p + k] = h[6 * (size_t)p + k];
                r->M[3 * p + k] = h[6 * (size_t)p + 3 + k];
            }
    }
    ok = ok && hipMemcpy(r->inv, L->red + 5 * (size_t)L->red_blocks, 4 * sizeof(double),
                         hipMemcpyDeviceToHost) == hipSuccess;
    if (slot.fields) {
        r->rho.resize(N);
        r->u.resize(3 * N);
        ok = ok && hipMemcpy(r->rho.data(), slot.fields, N * sizeof(double),
                             hipMemcpyDeviceToHost) == hipSuccess;
        ok = ok && hipMemcpy(r->u.data(), slot.fields + N, 3 * N * sizeof(double),
                             hipMemcpyDeviceToHost) == hipSuccess;
    }
    if (!ok) fail_request(r, LBMEP_EDEVICE, "result copy failed");
    r->t_done = now_s(S->t0);
    r->done = true;
    S->arena.release(slot.fields);
    S->arena.release(slot.d);
    destroy_lattice(L, false);  // its work is complete (event)
    S->ev_pool.push_back(slot.ev);
    S->reserved -= r->footprint;
    S->st.completed += 1;
    S->finished[r->id].reset(r);
    S->unreported.push_back(r->id);
    slot = Slot{};
}

// enqueue `k` steps of every active slot as packed launches
int enqueue_steps(lbmep_server *S, const std::vector<Slot *> &act, int k) {
    hipStream_t s = S->main;
    for (int it = 0; it < k; ++it) {
        // sweep and exchange, one packed launch pair per (precision, force mode)
        for (int prec = LBMEP_FP64; prec <= LBMEP_FP16DEV; ++prec)
            for (int fm = kForceNone; fm <= kForceCharge; ++fm) {
                PackTable ts{}, tn{};
                ts.xcd_swizzle = 1;
                auto flush = [&]() -> int {
                    if (ts.n == 0) return LBMEP_OK;
                    LBMEP_HIP_TRY(launch_sweep_packed(prec, fm, ts, s));
                    LBMEP_HIP_TRY(launch_near_packed(prec, tn, s));
                    S->st.packed_launches += 2;
                    ts.n = tn.n = 0;
                    ts.start[0] = tn.start[0] = 0;
                    return LBMEP_OK;
                };
                for (Slot *sl : act) {
                    lbmep_lattice *L = sl->L;
                    if (L->precision != prec || L->force_mode != fm) continue;
                    const uint32_t state = (uint32_t)(L->cur | (L->cur_owner << 1));
                    const uint32_t nxb = (uint32_t)((L->g.nx + kPackBlockX - 1) / kPackBlockX);
                    const uint32_t sb = nxb * (uint32_t)L->g.ny * (uint32_t)L->g.nz;
                    ts.d[ts.n] = tn.d[tn.n] = sl->d;
                    ts.state[ts.n] = tn.state[tn.n] = state;
                    ts.level[ts.n] = tn.level[tn.n] = L->level;
                    ts.start[ts.n + 1] = ts.start[ts.n] + sb;
                    tn.start[tn.n + 1] =
                        tn.start[tn.n] + (uint32_t)near_blocks(L->np, L->g, L->has_walls);
                    ts.n++;
                    tn.n++;
                    if (ts.n == kMaxPack) {
                        int rc = flush();
                        if (rc) return rc;
                    }
                }
                int rc = flush();
                if (rc) return rc;
            }
        // kinematics, re-mapping and classification (with the link lists)
        // of every moving lattice
        PackTable tp{};
        auto flush_p = [&]() -> int {
            if (tp.n == 0) return LBMEP_OK;
            LBMEP_HIP_TRY(launch_advance_packed(tp, s));
            LBMEP_HIP_TRY(launch_map_set_packed(tp, s));
            LBMEP_HIP_TRY(launch_classify_packed(tp, s));
            S->st.packed_launches += 3;
            tp.n = 0;
            return LBMEP_OK;
        };
        for (Slot *sl : act) {
            lbmep_lattice *L = sl->L;
            if (!(L->np > 0 && L->cfg.move_particles)) continue;
            tp.d[tp.n] = sl->d;
            tp.state[tp.n] = (uint32_t)(L->cur | (L->cur_owner << 1));
            tp.level[tp.n] = L->level + 1;
            tp.start[tp.n + 1] = tp.start[tp.n] + (uint32_t)L->np;
            tp.n++;
            if (tp.n == kMaxPack) {
                int rc = flush_p();
                if (rc) return rc;
            }
        }
        int rc = flush_p();
        if (rc) return rc;
        for (Slot *sl : act) {
            advance_state(sl->L);
            sl->to_enqueue -= 1;
            S->st.cell_updates += (double)sl->L->g.N;
        }
        S->st.steps += 1;
    }
    return LBMEP_OK;
}

int progress(lbmep_server *S) {
    // 1. retire slots whose read-out has completed
    for (Slot &sl : S->slots) {
        if (!sl.req || !sl.retiring) continue;
        const hipError_t q = hipEventQuery(sl.ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return fail(LBMEP_EDEVICE, std::string("event: ") + hipGetErrorString(q));
        retire(S, sl);
    }
    // 2. drop completed chunk events
    while (!S->chunk_ev.empty()) {
        const hipError_t q = hipEventQuery(S->chunk_ev.front());
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return fail(LBMEP_EDEVICE, std::string("event: ") + hipGetErrorString(q));
        S->ev_pool.push_back(S->chunk_ev.front());
        S->chunk_ev.pop_front();
        S->st.cell_updates_done += S->chunk_work.front();
        S->chunk_work.pop_front();
    }
    // 3. admit queued requests (FIFO) while a slot is free and the budget holds
    while (!S->queue.empty()) {
        Request *r = S->queue.front().get();
        if (S->reserved + r->footprint > S->arena.size()) break;
        Slot *free_slot = nullptr;
        for (Slot &sl : S->slots)
            if (!sl.req) {
                free_slot = &sl;
                break;
            }
        if (!free_slot) break;
        std::unique_ptr<Request> owned = std::move(S->queue.front());
        S->queue.pop_front();
        const int rc = admit(S, *free_slot, r);
        if (rc) {
            if (rc == LBMEP_ENOMEM && S->reserved > 0) {
                // fragmentation: wait for a resident request to finish
                S->queue.push_front(std::move(owned));
                break;
            }
            fail_request(r, rc, lbmep_last_error());
            r->t_admit = r->t_done = now_s(S->t0);
            r->done = true;
            S->st.failed += 1;
            S->unreported.push_back(r->id);
            S->finished[r->id] = std::move(owned);
            continue;
        }
        owned.release();  // held by the slot until it retires
        S->reserved += r->footprint;
        S->st.admitted += 1;
        if (free_slot->to_enqueue == 0) {
            int rc2 = enqueue_readout(S, *free_slot);
            if (rc2) return rc2;
        }
    }
    // 4. keep two chunks in flight
    while (S->chunk_ev.size() < 2) {
        std::vector<Slot *> act;
        int k = S->cfg.chunk_steps;
        for (Slot &sl : S->slots)
            if (sl.req && !sl.retiring && sl.to_enqueue > 0) {
                act.push_back(&sl);
                k = std::min(k, sl.to_enqueue);
            }
        if (act.empty()) break;
        const double before = S->st.cell_updates;
        int rc = enqueue_steps(S, act, k);
        if (rc) return rc;
        for (Slot *sl : act)
            if (sl->to_enqueue == 0) {
                rc = enqueue_readout(S, *sl);
                if (rc) return rc;
            }
        hipEvent_t e = get_event(S);
        if (!e) return fail(LBMEP_EDEVICE, "event creation failed");
        LBMEP_HIP_TRY(hipEventRecord(e, S->main));
        S->chunk_ev.push_back(e);
        S->chunk_work.push_back(S->st.cell_updates - before);
        S->st.chunks += 1;
    }
    return LBMEP_OK;
}

}  // namespace

extern "C" {

int lbmep_server_create(const lbmep_server_config *cfg, lbmep_server **out) {
    if (!cfg || !out) return fail(LBMEP_EINVAL, "null argument");
    *out = nullptr;
    if (cfg->max_slots < 1 || cfg->max_slots > kMaxPack)
        return fail(LBMEP_EINVAL, "max_slots must be in [1, 64]");
    if (cfg->chunk_steps < 1) return fail(LBMEP_EINVAL, "chunk_steps must be >= 1");
    if (cfg->max_queue < 1) return fail(LBMEP_EINVAL, "max_queue must be >= 1");
    if (cfg->hbm_budget < (size_t(1) << 20)) return fail(LBMEP_EINVAL, "budget below 1 MiB");
    int ndev = 0;
    LBMEP_HIP_TRY(hipGetDeviceCount(&ndev));
    if (cfg->device < 0 || cfg->device >= ndev) return fail(LBMEP_EINVAL, "no such device");
    LBMEP_HIP_TRY(hipSetDevice(cfg->device));
    auto S = std::make_unique<lbmep_server>();
    S->cfg = *cfg;
    S->t0 = std::chrono::steady_clock::now();
    if (S->arena.init(cfg->hbm_budget) != hipSuccess)
        return fail(LBMEP_ENOMEM, "device arena allocation failed");
    LBMEP_HIP_TRY(hipStreamCreateWithFlags(&S->main, hipStreamNonBlocking));
    LBMEP_HIP_TRY(hipStreamCreateWithFlags(&S->setup, hipStreamNonBlocking));
    S->slots.resize(cfg->max_slots);
    S->st.budget = S->arena.size();
    *out = S.release();
    return LBMEP_OK;
}

int lbmep_server_destroy(lbmep_server *S) {
    if (!S) return LBMEP_OK;
    hipSetDevice(S->cfg.device);
    hipStreamSynchronize(S->main);
    hipStreamSynchronize(S->setup);
    for (Slot &sl : S->slots) {
        if (!sl.req) continue;
        S->arena.release(sl.fields);
        S->arena.release(sl.d);
        destroy_lattice(sl.L, false);
        if (sl.ev) hipEventDestroy(sl.ev);
        delete sl.req;
    }
    for (hipEvent_t e : S->chunk_ev) hipEventDestroy(e);
    for (hipEvent_t e : S->ev_pool) hipEventDestroy(e);
    hipStreamDestroy(S->main);
    hipStreamDestroy(S->setup);
    delete S;
    return LBMEP_OK;
}

int lbmep_server_request_footprint(const lbmep_request *q, size_t *bytes) {
    if (!q || !bytes) return fail(LBMEP_EINVAL, "null argument");
    int rc = check_config(&q->cfg);
    if (rc) return rc;
    double rmax = 0.0;
    for (int i = 0; q->R && i < q->n; ++i) rmax = std::max(rmax, q->R[i]);
    *bytes = request_footprint(q->cfg, q->n, rmax, q->rho_e != nullptr, q->flags != nullptr,
                               q->keep_fields != 0);
    return LBMEP_OK;
}

int lbmep_server_submit(lbmep_server *S, const lbmep_request *q, uint64_t *id) {
    if (!S || !q || !id) return fail(LBMEP_EINVAL, "null argument");
    lbmep_config c = q->cfg;
    c.device = S->cfg.device;
    c.stream = nullptr;
    int rc = check_config(&c);
    if (rc) return rc;
    if (q->steps < 1) return fail(LBMEP_EINVAL, "steps must be >= 1");
    if (q->n < 0) return fail(LBMEP_EINVAL, "negative particle count");
    if (q->n > 0 && (!q->X || !q->R || !q->U)) return fail(LBMEP_EINVAL, "null particle array");
    if (q->rho_e && q->rho_e_dtype != LBMEP_DTYPE_F64 && q->rho_e_dtype != LBMEP_DTYPE_F32)
        return fail(LBMEP_EINVAL, "unknown rho_e dtype");
    if (q->rho_e && !finite_all(q->E, 3)) return fail(LBMEP_EINVAL, "bad field E");
    if (!small_offsets(c))
        return fail(LBMEP_EINVAL, "grid too large for the packed sweep (two population grids "
                                  "must be below 4 GiB)");
    const size_t N = (size_t)c.nx * c.ny * c.nz;
    double rmax = 0.0;
    for (int i = 0; i < q->n; ++i)
        if (std::isfinite(q->R[i])) rmax = std::max(rmax, q->R[i]);
    const size_t fp = request_footprint(c, q->n, rmax, q->rho_e != nullptr, q->flags != nullptr,
                                        q->keep_fields != 0);
    if (fp > S->arena.size()) return fail(LBMEP_EINVAL, "request footprint exceeds the budget");
    if ((int32_t)S->queue.size() >= S->cfg.max_queue) return fail(LBMEP_EBUSY, "queue full");
    auto r = std::make_unique<Request>();
    r->cfg = c;
    r->n = q->n;
    r->steps = q->steps;
    if (q->flags) r->flags.assign(q->flags, q->flags + N);
    if (q->n > 0) {
        r->X.assign(q->X, q->X + 3 * (size_t)q->n);
        r->R.assign(q->R, q->R + q->n);
        r->U.assign(q->U, q->U + 3 * (size_t)q->n);
        if (q->W)
            r->W.assign(q->W, q->W + 3 * (size_t)q->n);
        else
            r->W.assign(3 * (size_t)q->n, 0.0);
    }
    if (q->rho_e) {
        const size_t b = N * (q->rho_e_dtype == LBMEP_DTYPE_F64 ? 8 : 4);
        r->rho_e.assign(static_cast<const char *>(q->rho_e), static_cast<const char *>(q->rho_e) + b);
        r->rho_dtype = q->rho_e_dtype;
        r->charge = true;
        for (int k = 0; k < 3; ++k) r->E[k] = q->E[k];
    }
    r->keep_fields = q->keep_fields != 0;
    r->footprint = fp;
    r->id = S->next_id++;
    r->t_submit = now_s(S->t0);
    *id = r->id;
    S->queue.push_back(std::move(r));
    S->st.submitted += 1;
    return LBMEP_OK;
}

int lbmep_server_poll(lbmep_server *S, uint64_t *done_ids, int32_t cap, int32_t *ndone) {
    if (!S || !ndone || cap < 0 || (cap > 0 && !done_ids)) return fail(LBMEP_EINVAL, "bad argument");
    LBMEP_HIP_TRY(hipSetDevice(S->cfg.device));
    *ndone = 0;
    int rc = progress(S);
    if (rc) return rc;
    while (*ndone < cap && !S->unreported.empty()) {
        done_ids[(*ndone)++] = S->unreported.front();
        S->unreported.pop_front();
    }
    return LBMEP_OK;
}

int lbmep_server_result(lbmep_server *S, uint64_t id, double *F, double *M, double inv[4],
                        double times[3]) {
    if (!S) return fail(LBMEP_EINVAL, "null server");
    auto it = S->finished.find(id);
    if (it == S->finished.end()) return fail(LBMEP_ESTATE, "request not finished (or unknown)");
    Request *r = it->second.get();
    if (r->status != LBMEP_OK) return fail(r->status, "request failed: " + r->error);
    if (F && !r->F.empty()) std::memcpy(F, r->F.data(), r->F.size() * sizeof(double));
    if (M && !r->M.empty()) std::memcpy(M, r->M.data(), r->M.size() * sizeof(double));
    if (inv) std::memcpy(inv, r->inv, sizeof r->inv);
    if (times) {
        times[0] = r->t_submit;
        times[1] = r->t_admit;
        times[2] = r->t_done;
    }
    return LBMEP_OK;
}

int lbmep_server_fields(lbmep_server *S, uint64_t id, double *rho, double *u) {
    if (!S || !rho || !u) return fail(LBMEP_EINVAL, "null argument");
    auto it = S->finished.find(id);
    if (it == S->finished.end()) return fail(LBMEP_ESTATE, "request not finished (or unknown)");
    Request *r = it->second.get();
    if (r->status != LBMEP_OK) return fail(r->status, "request failed: " + r->error);
    if (r->rho.empty()) return fail(LBMEP_ESTATE, "request was submitted without keep_fields");
    std::memcpy(rho, r->rho.data(), r->rho.size() * sizeof(double));
    std::memcpy(u, r->u.data(), r->u.size() * sizeof(double));
    return LBMEP_OK;
}

int lbmep_server_release(lbmep_server *S, uint64_t id) {
    if (!S) return fail(LBMEP_EINVAL, "null server");
    auto it = S->finished.find(id);
    if (it == S->finished.end()) return fail(LBMEP_ESTATE, "request not finished (or unknown)");
    S->finished.erase(it);
    return LBMEP_OK;
}

int lbmep_server_get_stats(lbmep_server *S, lbmep_server_stats *out) {
    if (!S || !out) return fail(LBMEP_EINVAL, "null argument");
    S->st.queued = (int32_t)S->queue.size();
    int32_t res = 0;
    for (const Slot &sl : S->slots) res += sl.req ? 1 : 0;
    S->st.resident = res;
    S->st.bytes_reserved = S->reserved;
    S->st.bytes_in_use = S->arena.used();
    *out = S->st;
    return LBMEP_OK;
}

int lbmep_server_now(lbmep_server *S, double *t) {
    if (!S || !t) return fail(LBMEP_EINVAL, "null argument");
    *t = now_s(S->t0);
    return LBMEP_OK;
}

}  // extern "C"
