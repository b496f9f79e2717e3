// Handle, status, timing, and the shared kernels: status-block init, the
// exclusive scan with row classification, and the segmented sort used by
// every operation's Build step.
#include "hp_internal.hpp"
#include "hp_poll.hpp"
#include "hp_scan.hpp"

#include <algorithm>
#include <cstring>

using namespace hp;

// ===========================================================================
// Status / handle
// ===========================================================================
extern "C" const char *hp_status_string(hp_status_t s) {
    switch (s) {
        case HP_OK: return "HP_OK";
        case HP_ERR_INVALID_ARG: return "HP_ERR_INVALID_ARG";
        case HP_ERR_INDEX_RANGE: return "HP_ERR_INDEX_RANGE";
        case HP_ERR_NOT_PERMUTATION: return "HP_ERR_NOT_PERMUTATION";
        case HP_ERR_DUPLICATE_INDEX: return "HP_ERR_DUPLICATE_INDEX";
        case HP_ERR_NOT_CANONICAL: return "HP_ERR_NOT_CANONICAL";
        case HP_ERR_SHAPE: return "HP_ERR_SHAPE";
        case HP_ERR_OVERFLOW: return "HP_ERR_OVERFLOW";
        case HP_ERR_WORKSPACE: return "HP_ERR_WORKSPACE";
        case HP_ERR_CAPACITY: return "HP_ERR_CAPACITY";
        case HP_ERR_HIP: return "HP_ERR_HIP";
        case HP_ERR_ALIAS: return "HP_ERR_ALIAS";
        case HP_ERR_TIMEOUT: return "HP_ERR_TIMEOUT";
        case HP_ERR_REJECTED: return "HP_ERR_REJECTED";
    }
    return "HP_ERR_UNKNOWN";
}

namespace hp {

hp_status_t fail(hp_handle_t h, hp_status_t s, const std::string &msg) {
    if (h) h->last_error = std::string(hp_status_string(s)) + ": " + msg;
    return s;
}

hp_status_t hip_check(hp_handle_t h, hipError_t e, const char *what) {
    if (e == hipSuccess) return HP_OK;
    return fail(h, HP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

hp_status_t status_from_err(hp_handle_t h, uint32_t err, const char *op) {
    if (!err) return HP_OK;
    std::string o(op);
    if (err & E_TIMEOUT) return fail(h, HP_ERR_TIMEOUT, o + ": device wait limit reached");
    if (err & E_RANGE) return fail(h, HP_ERR_INDEX_RANGE, o + ": index out of range");
    if (err & E_NOTPERM) return fail(h, HP_ERR_NOT_PERMUTATION, o + ": index vector is not a permutation");
    if (err & E_DUP) return fail(h, HP_ERR_DUPLICATE_INDEX, o + ": repeated index in an assignment vector");
    if (err & E_NONCANON) return fail(h, HP_ERR_NOT_CANONICAL, o + ": CSR not canonical");
    if (err & E_OVERFLOW) return fail(h, HP_ERR_OVERFLOW, o + ": output nnz exceeds int32 rowptr");
    if (err & E_CAPACITY) return fail(h, HP_ERR_CAPACITY, o + ": output exceeds capacity");
    return fail(h, HP_ERR_INVALID_ARG, o + ": device error");
}

bool overlaps(const void *a, size_t an, const void *b, size_t bn) {
    if (!a || !b || an == 0 || bn == 0) return false;
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

size_t idx_size(int32_t t) { return t == HP_IDX_I64 ? 8 : 4; }
size_t val_size(int32_t t) { return t == HP_VAL_F64 ? 8 : 4; }

hp_status_t check_csr_args(hp_handle_t h, const hp_csr_t *A, const char *name) {
    std::string n(name);
    if (!A) return fail(h, HP_ERR_INVALID_ARG, n + " is NULL");
    if (A->nrows < 0 || A->ncols < 0 || A->nnz < 0)
        return fail(h, HP_ERR_INVALID_ARG, n + ": negative size");
    if (A->ncols > INT32_MAX || A->nrows > INT32_MAX)
        return fail(h, HP_ERR_INVALID_ARG, n + ": dimension exceeds int32 column/row index range");
    if (A->ptr_type != HP_IDX_I32 && A->ptr_type != HP_IDX_I64)
        return fail(h, HP_ERR_INVALID_ARG, n + ": bad ptr_type");
    if (A->val_type != HP_VAL_F32 && A->val_type != HP_VAL_F64)
        return fail(h, HP_ERR_INVALID_ARG, n + ": bad val_type");
    if (A->ptr_type == HP_IDX_I32 && A->nnz > INT32_MAX)
        return fail(h, HP_ERR_OVERFLOW, n + ": nnz exceeds int32 rowptr");
    if (!A->rowptr) return fail(h, HP_ERR_INVALID_ARG, n + ": rowptr is NULL");
    if (A->nnz > 0 && (!A->col || !A->val)) return fail(h, HP_ERR_INVALID_ARG, n + ": col/val NULL");
    return HP_OK;
}

// ---- stage timing ---------------------------------------------------------
// Events are recorded on the handle's stream between kernel stages and are
// only resolved by hp_stage_times(), so timing adds no synchronisation.
static hipEvent_t next_event(hp_handle_t h) {
    if (h->ev_used == h->ev.size()) {
        hipEvent_t e;
        hipEventCreate(&e);
        h->ev.push_back(e);
    }
    return h->ev[h->ev_used++];
}
void stage_begin(hp_handle_t h) {
    if (!h->timing) return;
    h->ev_cur = next_event(h);
    hipEventRecord(h->ev_cur, h->stream);
}
void stage_mark(hp_handle_t h, const char *name) {
    if (!h->timing) return;
    hipEvent_t e = next_event(h);
    hipEventRecord(e, h->stream);
    h->recs.push_back({name, h->ev_cur, e});
    h->ev_cur = e;
}
void stage_end(hp_handle_t h) { (void)h; }

}  // namespace hp

extern "C" hp_status_t hp_create(hp_handle_t *out, int device) {
    if (!out) return HP_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HP_ERR_INVALID_ARG;
    hp_handle_t h = new hp_handle_s();
    h->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipHostMalloc((void **)&h->host_hdr, sizeof(DevHdr), hipHostMallocDefault) != hipSuccess) {
        delete h;
        return HP_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        h->num_cus = prop.multiProcessorCount;
    h->validate = hp::validate_from_env();
    // the readback event, made here so that later calls create nothing
    if (hipEventCreateWithFlags(&h->rb_done, hipEventDisableTiming) != hipSuccess) h->rb_done = nullptr;
    // this device's copy of the fixed scratch array (hp_permute_noalloc);
    // a failure only leaves that entry point unavailable
    hp::noalloc_setup(device);
    *out = h;
    return HP_OK;
}

extern "C" hp_status_t hp_destroy(hp_handle_t h) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp::batch_release_handle(h);
    for (auto &e : h->ev) hipEventDestroy(e);
    if (h->rb_done) hipEventDestroy(h->rb_done);
    if (h->host_hdr) hipHostFree(h->host_hdr);
    delete h;
    return HP_OK;
}

extern "C" hp_status_t hp_set_stream(hp_handle_t h, void *stream) {
    if (!h) return HP_ERR_INVALID_ARG;
    h->stream = (hipStream_t)stream;
    return HP_OK;
}

extern "C" const char *hp_last_error(hp_handle_t h) { return h ? h->last_error.c_str() : "null handle"; }

extern "C" hp_status_t hp_enable_timing(hp_handle_t h, int enable) {
    if (!h) return HP_ERR_INVALID_ARG;
    h->timing = enable != 0;
    h->recs.clear();
    h->ev_used = 0;
    return HP_OK;
}

extern "C" int hp_stage_times(hp_handle_t h, float *ms, int *count, const char **names, int cap) {
    if (!h) return 0;
    std::vector<const char *> nm;
    std::vector<float> tot;
    std::vector<int> cnt;
    if (!h->recs.empty()) hipEventSynchronize(h->recs.back().e1);
    for (auto &r : h->recs) {
        float t = 0;
        hipEventElapsedTime(&t, r.e0, r.e1);
        size_t k = 0;
        while (k < nm.size() && std::strcmp(nm[k], r.name) != 0) k++;
        if (k == nm.size()) {
            nm.push_back(r.name);
            tot.push_back(0);
            cnt.push_back(0);
        }
        tot[k] += t;
        cnt[k] += 1;
    }
    h->recs.clear();
    h->ev_used = 0;
    int n = std::min<int>(cap, (int)nm.size());
    for (int k = 0; k < n; k++) {
        if (ms) ms[k] = tot[k];
        if (count) count[k] = cnt[k];
        if (names) names[k] = nm[k];
    }
    return n;
}

// ===========================================================================
// Small kernels
// ===========================================================================
__global__ void k_clear_words(uint32_t *p, size_t n) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    uint4 z = make_uint4(0, 0, 0, 0);
    size_t n4 = n / 4;
    for (size_t k = i; k < n4; k += stride) reinterpret_cast<uint4 *>(p)[k] = z;
    for (size_t k = n4 * 4 + i; k < n; k += stride) p[k] = 0;
}

__global__ void k_fill_words(uint32_t *p, size_t n, uint32_t v) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    uint4 z = make_uint4(v, v, v, v);
    size_t n4 = n / 4;
    for (size_t k = i; k < n4; k += stride) reinterpret_cast<uint4 *>(p)[k] = z;
    for (size_t k = n4 * 4 + i; k < n; k += stride) p[k] = v;
}

__global__ void k_init_hdr(DevHdr *h, uint64_t *tile_state, size_t ntiles) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    if (i < sizeof(DevHdr) / 4) reinterpret_cast<uint32_t *>(h)[i] = 0;
    for (size_t k = i; k < ntiles; k += stride) tile_state[k] = 0;
}

namespace hp {

static int grid_for(size_t n, int block, int cap = 1 << 16) {
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (size_t)cap) g = cap;
    return (int)g;
}

hipError_t launch_clear_words(hipStream_t s, void *p, size_t nwords32) {
    if (nwords32 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_words, dim3(grid_for(nwords32 / 4 + 1, 256, 8192)), dim3(256), 0, s,
                       (uint32_t *)p, nwords32);
    return hipGetLastError();
}

hipError_t launch_fill_words(hipStream_t s, void *p, size_t nwords32, uint32_t v) {
    if (nwords32 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_words, dim3(grid_for(nwords32 / 4 + 1, 256, 8192)), dim3(256), 0, s,
                       (uint32_t *)p, nwords32, v);
    return hipGetLastError();
}

hipError_t launch_init_hdr(hipStream_t s, DevHdr *h, uint64_t *tile_state, size_t ntiles) {
    size_t n = std::max(ntiles, sizeof(DevHdr) / 4);
    hipLaunchKernelGGL(k_init_hdr, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, h, tile_state, ntiles);
    return hipGetLastError();
}

// Bounded wait for an event recorded on a stream: polls it (spin, then
// yield, then sleep between polls) up to the host wait limit.  A failed or
// faulted stream ends the wait with its error; reaching the limit gives
// HP_ERR_TIMEOUT (the queued work may still run: the caller must
// synchronise the stream before it frees buffers that work uses).
hp_status_t wait_event(hp_handle_t h, hipEvent_t ev, const char *what) {
    hipError_t err = hipSuccess;
    const WaitResult r = wait_until(
        [&] {
            const hipError_t q = hipEventQuery(ev);
            if (q == hipSuccess) return Poll::READY;
            if (q == hipErrorNotReady) return Poll::PENDING;
            err = q;
            return Poll::FAILED;
        },
        default_wait_policy());
    if (r == WaitResult::DONE) return HP_OK;
    if (r == WaitResult::FAILED) return hip_check(h, err, what);
    return fail(h, HP_ERR_TIMEOUT, std::string(what) + ": host wait limit reached (HP_HOST_WAIT_MS)");
}

// The plan's one blocking step: the device header is copied to pinned host
// memory and an event behind the copy is polled, so the plan returns as soon
// as the few bytes have landed.
hp_status_t readback_hdr(hp_handle_t h, DevHdr *dev, const char *what) {
    const hipError_t e = hipMemcpyAsync(h->host_hdr, dev, sizeof(DevHdr), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_check(h, e, what);
    return wait_stream(h, what);
}

// Bounded wait for everything enqueued so far on the handle's stream.
hp_status_t wait_stream(hp_handle_t h, const char *what) {
    hipError_t e = hipSuccess;
    if (!h->rb_done) e = hipEventCreateWithFlags(&h->rb_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(h->rb_done, h->stream);
    if (e != hipSuccess) return hip_check(h, e, what);
    return wait_event(h, h->rb_done, what);
}

// ===========================================================================
// Exclusive scan with row classification: single pass (decoupled look-back)
// up to SCAN_ONEPASS_TILES tiles, three passes above.
//
// In the single pass, tiles are taken in launch order from an atomic ticket,
// so a tile only ever waits on tiles that are already running: every wait
// ends.  The wait is still bounded (SCAN_WAIT_TICKS); reaching it raises
// E_TIMEOUT and the kernel finishes normally.  The three passes never wait.
// ===========================================================================
size_t scan_tiles(int64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

// Up to this many tiles the single pass is used (its look-back chains are
// short); longer scans take three passes.
constexpr int64_t SCAN_ONEPASS_TILES = 256;

// Four wavefronts per SIMD (at most 128 VGPRs): left alone the compiler
// keeps all 16 staged values of a lane in flight and drops to two.  CLS
// false: the plain scan (no class lists), a smaller kernel.
template <typename PT, bool CLS>
__global__ __launch_bounds__(SCAN_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_scan_counts(
    const int32_t *__restrict__ cnt, PT *__restrict__ out, int64_t n, DevHdr *hdr, int slot,
    uint64_t *tile_state, int classify, uint32_t *lists, int64_t cap, uint64_t *goff,
    const uint8_t *__restrict__ force, const uint32_t *__restrict__ nmslots) {
    __shared__ ScanSmem sm;
    __shared__ uint32_t s_tile;
    if (threadIdx.x == 0) s_tile = atomicAdd(&hdr->ticket[slot], 1u);
    __syncthreads();
    scan_counts_tile<PT, CLS>(s_tile, sm, cnt, out, n, hdr, slot, tile_state, classify, lists, cap, goff, force,
                              nmslots);
}

// Three-pass form for long scans: tile sums, one workgroup scanning them,
// then every tile scans its counts from its prefix.  The single pass spends
// its time in look-back chains once there are thousands of tiles (16.8M
// counts: 145 us single pass).
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const int32_t *__restrict__ cnt, int64_t n,
                                                           uint64_t *partial) {
    __shared__ uint64_t s_wave[SCAN_BLOCK / WAVE];
    scan_reduce_tile(blockIdx.x, s_wave, cnt, n, partial);
}

__global__ __launch_bounds__(PSCAN_BLOCK) void k_scan_partials(uint64_t *partial, int64_t ntiles) {
    __shared__ uint64_t s_wave[PSCAN_BLOCK / WAVE];
    scan_partials_block(s_wave, partial, ntiles);
}

template <typename PT, bool CLS>
__global__ __launch_bounds__(SCAN_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_scan_down(
    const int32_t *__restrict__ cnt, PT *__restrict__ out, int64_t n, DevHdr *hdr, int slot,
    const uint64_t *__restrict__ prefix, int classify, uint32_t *lists, int64_t cap, uint64_t *goff,
    const uint8_t *__restrict__ force, const uint32_t *__restrict__ nmslots) {
    __shared__ ScanSmem sm;
    scan_counts_tile<PT, CLS>(blockIdx.x, sm, cnt, out, n, hdr, slot, nullptr, classify, lists, cap, goff, force,
                              nmslots, prefix);
}

template <typename PT>
__global__ void k_scan_empty(PT *out, DevHdr *hdr, int slot) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = 0;
        hdr->total[slot] = 0;
    }
}

template <typename PT>
hipError_t launch_scan_counts(hipStream_t s, const int32_t *cnt, PT *out, int64_t n, DevHdr *hdr,
                              int slot, uint64_t *tile_state, int classify, uint32_t *bin_lists,
                              int64_t bin_cap, const uint8_t *force, const uint32_t *nmslots) {
    if (n == 0) {
        hipLaunchKernelGGL(k_scan_empty<PT>, dim3(1), dim3(64), 0, s, out, hdr, slot);
        return hipGetLastError();
    }
    int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    uint64_t *goff = bin_lists ? reinterpret_cast<uint64_t *>(bin_lists + NBINS * bin_cap) : nullptr;
    if (tiles > SCAN_ONEPASS_TILES) {
        // tile_state (scan_tiles(n) words) holds the tile sums, then prefixes
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, cnt, n, tile_state);
        hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(PSCAN_BLOCK), 0, s, tile_state, tiles);
        auto down = classify ? k_scan_down<PT, true> : k_scan_down<PT, false>;
        hipLaunchKernelGGL(down, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, cnt, out, n, hdr, slot, (const uint64_t *)tile_state, classify,
                           bin_lists, bin_cap, goff, force, nmslots);
        return hipGetLastError();
    }
    auto one = classify ? k_scan_counts<PT, true> : k_scan_counts<PT, false>;
    hipLaunchKernelGGL(one, dim3((unsigned)tiles), dim3(SCAN_BLOCK), 0, s, cnt, out, n, hdr, slot, tile_state, classify, bin_lists, bin_cap, goff,
                       force, nmslots);
    return hipGetLastError();
}

template hipError_t launch_scan_counts<int32_t>(hipStream_t, const int32_t *, int32_t *, int64_t,
                                                DevHdr *, int, uint64_t *, int, uint32_t *, int64_t,
                                                const uint8_t *, const uint32_t *);
template hipError_t launch_scan_counts<int64_t>(hipStream_t, const int32_t *, int64_t *, int64_t,
                                                DevHdr *, int, uint64_t *, int, uint32_t *, int64_t,
                                                const uint8_t *, const uint32_t *);

}  // namespace hp
