// lbmep_noalloc.hip -- the FP64 global sums of a lattice without any device
// allocation, for callers that cannot allocate (code under stream capture,
// tight serving loops): lbmep_get_invariants_noalloc.
//
// The per-workgroup partial sums that lbmep_get_invariants keeps in a buffer
// allocated with the lattice live here in one file-scope device array per
// GPU, `scratch`, held until the process ends.  Its device address is taken
// once per device (with that device current) by hipGetSymbolAddress and kept;
// host code never uses the array's name as an address.  Every workgroup of a
// call overwrites its own partials before the final reduction reads them,
// so nothing needs clearing between calls; calls that overlap in time on one
// GPU (other streams, other host threads) share the array and race.
#include <mutex>

#include "lattice.h"

using namespace lbmep;
using namespace lbmep::rt;

namespace {

// partials of at most kNoAllocBlocks workgroups: 4 sums and a fluid-cell
// count per workgroup, then the 4 results (the same layout as the lattice's
// own reduction buffer)
constexpr int kNoAllocBlocks = 4096;
constexpr size_t kScratchDoubles = 5 * (size_t)kNoAllocBlocks + 4;

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

// the device address of this device's scratch array (device current)
int scratch_ptr(int device, double **out) {
    if (device < 0 || device >= kMaxDevices) return fail(LBMEP_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBMEP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[device] = static_cast<double *>(p);
    }
    *out = g_ptr[device];
    return LBMEP_OK;
}

}  // namespace

extern "C" {

int lbmep_get_invariants_noalloc(lbmep_lattice *L, double *out) {
    if (!L || !out) return fail(LBMEP_EINVAL, "null argument");
    const hipError_t ed = hipSetDevice(L->cfg.device);
    if (ed != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(ed));
    const int nb = invariants_blocks(L->g);
    if (nb < 1 || nb > kNoAllocBlocks)
        return fail(LBMEP_EINVAL, "grid needs more partial sums than the static scratch holds");
    double *ptr = nullptr;
    int rc = scratch_ptr(L->cfg.device, &ptr);
    if (rc) return rc;
    // the post-stream state, as lbmep_get_invariants reads it (a kernel into
    // the lattice's spare grid; nothing is allocated)
    rc = materialize(L);
    if (rc) return rc;
    // partials and counts in the scratch array, the 4 results into out
    const hipError_t e = launch_invariants(L->precision, L->g, L->f[L->cur], L->flag, ptr, nb, out,
                                           L->stream);
    if (e != hipSuccess) return fail(LBMEP_EDEVICE, hipGetErrorString(e));
    return LBMEP_OK;
}

}  // extern "C"
