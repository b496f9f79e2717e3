// Permutation for callers that cannot allocate: hp_permute_plan and
// hp_permute_exec in one call, with both workspaces carved from a fixed
// device array of this library instead of caller or library allocations.
//
// The array (`scratch`, HP_NOALLOC_SCRATCH_BYTES) lives in the library's
// code object: every device the library runs on holds its own copy until
// the process ends.  Host code never passes the array's name to a kernel
// (on the host it is only a stand-in symbol); hp_create calls
// noalloc_setup() once per device, with that device current, to look up
// the copy's device address, and the entry point uses that address.
#include "hp_internal.hpp"

#include <mutex>

using namespace hp;

static constexpr size_t SCRATCH_BYTES = size_t(HP_NOALLOC_SCRATCH_BYTES);

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

void *g_scratch[MAX_DEVICES];   // device address of `scratch` on each device, once set up
std::mutex g_mu;

void *scratch_of(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_scratch[device];
}

size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace hp {

// Looks up this device's copy of the scratch array (the caller has made
// `device` current).  Idempotent; the first successful lookup is kept.
hp_status_t noalloc_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return HP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return HP_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return HP_ERR_HIP;
    g_scratch[device] = ptr;
    return HP_OK;
}

}  // namespace hp

extern "C" hp_status_t hp_permute_noalloc(hp_handle_t h, const hp_csr_t *A, const int32_t *p, const int32_t *q,
                                          hp_csr_t *C) {
    if (!h) return HP_ERR_INVALID_ARG;
    if (!A || !C) return fail(h, HP_ERR_INVALID_ARG, "permute_noalloc: A or C is NULL");
    if (h->timing) return fail(h, HP_ERR_INVALID_ARG, "permute_noalloc: stage timing must be off (it creates events)");
    char *ws = (char *)scratch_of(h->device);
    if (!ws) return fail(h, HP_ERR_HIP, "permute_noalloc: the scratch array of this device is not set up");
    if (!h->rb_done) return fail(h, HP_ERR_HIP, "permute_noalloc: the handle has no readback event");
    size_t plan_bytes = 0;
    hp_status_t st = hp_permute_workspace(h, A, &plan_bytes);
    if (st) return st;
    plan_bytes = round256(plan_bytes);
    if (plan_bytes > SCRATCH_BYTES)
        return fail(h, HP_ERR_WORKSPACE, "permute_noalloc: the matrix needs " + std::to_string(plan_bytes) +
                                             " bytes of scratch, above the fixed " +
                                             std::to_string(SCRATCH_BYTES));
    if (A->nnz > 0 && (!C->col || !C->val))
        return fail(h, HP_ERR_INVALID_ARG, "permute_noalloc: C->col and C->val must hold nnz(A) entries");
    const size_t ps = idx_size(A->ptr_type), vs = val_size(A->val_type);
    const void *outs[] = {C->rowptr, C->col, C->val};
    const size_t outsz[] = {(size_t)(A->nrows + 1) * ps, (size_t)A->nnz * 4, (size_t)A->nnz * vs};
    for (int k = 0; k < 3; k++)
        if (overlaps(outs[k], outsz[k], ws, SCRATCH_BYTES))
            return fail(h, HP_ERR_ALIAS, "permute_noalloc: an output overlaps the scratch array");
    hp_plan_info_t info{};
    st = hp_permute_plan(h, A, p, q, C, ws, plan_bytes, &info);
    if (st) return st;
    // the exec workspace with the row slots when the array holds it, else
    // the smallest one exec accepts (info.aux[0], without them)
    const size_t xbytes = plan_bytes + info.exec_ws_bytes <= SCRATCH_BYTES ? info.exec_ws_bytes : (size_t)info.aux[0];
    if (plan_bytes + xbytes > SCRATCH_BYTES)
        return fail(h, HP_ERR_WORKSPACE, "permute_noalloc: rows longer than the block sort need " +
                                             std::to_string(xbytes) + " more bytes of scratch than the fixed " +
                                             std::to_string(SCRATCH_BYTES) + " hold (C->rowptr is written)");
    return hp_permute_exec(h, A, p, q, C, ws, plan_bytes, &info, xbytes ? ws + plan_bytes : nullptr, xbytes);
}
