// Internal definitions shared by the library's translation units.
// gfx950 only: 64-lane wavefronts, agent-scope atomics, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>
#include <vector>

#include "../../include/hipperm.h"

namespace hp {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Device-side status block, at offset 0 of every plan workspace.  Kernels
// raise error bits with atomicOr; the plan's single readback copies it out.
// ---------------------------------------------------------------------------
enum : uint32_t {
    E_RANGE = 1u, E_NOTPERM = 2u, E_DUP = 4u, E_NONCANON = 8u, E_OVERFLOW = 16u,
    E_TIMEOUT = 32u, E_CAPACITY = 64u,
};
enum : uint32_t { F_NOT_MONOTONE = 1u, F_NOT_RANGE = 2u };   // F_NOT_RANGE: J is not J[0] + (0, 1, 2, ...)

enum { BIN_THREAD = 0, BIN_WAVE = 1, BIN_BLOCK = 2, BIN_GLOBAL = 3, NBINS = 4 };
constexpr int64_t THREAD_MAX = 16;     // rows sorted in registers by one lane
constexpr int64_t SMALL_MAX = 64;      // rows k_sort_small sorts with one wavefront
constexpr int64_t WAVE_MAX = 256;      // rows sorted by one wavefront (4 keys per lane)
constexpr int64_t BLOCK_MAX = 2048;    // rows sorted in LDS by one workgroup

struct DevHdr {
    uint32_t err;
    uint32_t flags;
    uint32_t ticket[8];          // look-back scan tile tickets
    uint32_t bin_cnt[NBINS];     // rows per sort class
    uint32_t ndup;               // repeated-column records (spref)
    uint32_t pad0;
    uint64_t total[4];           // scan totals
    uint64_t bin_elems[NBINS];   // entries per sort class
    uint64_t aux[4];
};

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Column read from a caller's matrix, clamped into [0, n) so that a
// malformed input can never index past a table (results are then undefined).
__device__ __forceinline__ int64_t clampc(int32_t c, int64_t n) {
    return (uint32_t)c < (uint64_t)n ? (int64_t)c : 0;
}

__device__ __forceinline__ void raise_err(DevHdr *h, uint32_t bits) { atomicOr(&h->err, bits); }

// Fill n 32-bit words with v (sequential stores).
hipError_t launch_fill_words(hipStream_t s, void *p, size_t nwords32, uint32_t v);

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        T t = __shfl_up(v, o, WAVE);
        if (l >= o) v += t;
    }
    return v;
}
// 32-bit counts: data-parallel-primitive moves instead of LDS permutes:
// row shifts 1, 2, 4, 8 scan each row of 16 lanes, then row broadcasts of
// lanes 15 and 31 carry the row totals (lanes shifted in from outside a
// row read 0).  Every lane of the wavefront must be active.
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 -> rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 -> rows 2, 3
    return v;
}

// Exclusive scan over a workgroup of BLOCK threads; returns the exclusive
// prefix of `v` and writes the block total.  Uses BLOCK/64 words of LDS.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *s_wave, T &total) {
    const int w = threadIdx.x / WAVE, l = lane_id();
    T inc = wave_incl_scan(v);
    if (l == WAVE - 1) s_wave[w] = inc;
    __syncthreads();
    T wbase = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < BLOCK / WAVE; k++) {
        T x = s_wave[k];
        if (k < w) wbase += x;
        tot += x;
    }
    __syncthreads();
    total = tot;
    return wbase + inc - v;
}

// Bits needed to represent values in [0, n).
__host__ __device__ __forceinline__ int key_bits(int64_t n) {
    int b = 0;
    while (b < 63 && (int64_t(1) << b) < n) b++;
    return b < 1 ? 1 : b;
}

template <typename PT> struct PtrTag {};

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------
struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b) : base((char *)b) {}
    template <typename T> T *take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? (T *)(base + off) : nullptr;
        off += n * sizeof(T) + 16;
        return p;
    }
    size_t size() const { return (off + 255) & ~size_t(255); }
};


}  // namespace hp

// The handle (opaque to callers).
struct hp_stage_rec {
    const char *name;
    hipEvent_t e0, e1;
};
struct hp_handle_s {
    int device = 0;
    int num_cus = 256;                     // compute units of the device
    hipStream_t stream = nullptr;
    hp::DevHdr *host_hdr = nullptr;        // pinned readback block
    std::string last_error;
    bool timing = false;
    std::vector<hipEvent_t> ev;            // event pool for stage timing
    size_t ev_used = 0;
    hipEvent_t ev_cur = nullptr;
    std::vector<hp_stage_rec> recs;        // recorded (stage, start, end) triples
    hipEvent_t rb_done = nullptr;          // marks the end of a plan's readback copy
    bool validate = false;                 // plans check their CSR inputs first (HP_VALIDATE)
};

namespace hp {

// Status helpers -------------------------------------------------------------
hp_status_t fail(hp_handle_t h, hp_status_t s, const std::string &msg);
hp_status_t hip_check(hp_handle_t h, hipError_t e, const char *what);
hp_status_t status_from_err(hp_handle_t h, uint32_t err, const char *op);
bool overlaps(const void *a, size_t an, const void *b, size_t bn);
size_t idx_size(int32_t t);
size_t val_size(int32_t t);
hp_status_t check_csr_args(hp_handle_t h, const hp_csr_t *A, const char *name);

void batch_release_handle(hp_handle_t h);   // forget batch plans and graphs of h
// Input validation of the plans (hp_validate.hip): whether HP_VALIDATE asks
// for it, and the check itself (a no-op unless h->validate).
bool validate_from_env();
hp_status_t validate_input(hp_handle_t h, const hp_csr_t *M, DevHdr *hdr, const char *what);
// Looks up the device address of the fixed scratch array of hp_permute_noalloc
// on `device` (which the caller has made current); once per device.
hp_status_t noalloc_setup(int device);

// Stage timing (no-ops unless enabled).
void stage_begin(hp_handle_t h);
void stage_mark(hp_handle_t h, const char *name);   // closes the previous stage
void stage_end(hp_handle_t h);

// Common kernels, launched from host wrappers in hp_core.hip --------------
hipError_t launch_clear_words(hipStream_t s, void *p, size_t nwords32);
hipError_t launch_init_hdr(hipStream_t s, DevHdr *h, uint64_t *tile_state, size_t ntiles);
// Copies the device header into h->host_hdr and waits for it (bounded:
// HP_ERR_TIMEOUT past the host wait limit); `what` names the call in errors.
hp_status_t readback_hdr(hp_handle_t h, DevHdr *dev, const char *what);
// Bounded wait for an event already recorded on a stream (h may be NULL).
hp_status_t wait_event(hp_handle_t h, hipEvent_t ev, const char *what);
// Bounded wait for all work enqueued so far on the handle's stream.
hp_status_t wait_stream(hp_handle_t h, const char *what);

// Exclusive scan of n counts (int32 in) into out (PT, n+1 entries); out[n]
// = total; hdr->total[slot] = total.  classify: 0 none, 1 rows longer than
// THREAD_MAX, 2 all rows of >= 2 entries, 3 rows longer than WAVE_MAX when
// any of the 64 spread flag slots nmslots[32*k] is set (the column map is
// not monotone; F_NOT_MONOTONE is then raised), else only rows with
// force[i] != 0; 4 only rows with force[i] != 0 (class lists, see
// hp_segsort.hpp).  tile_state must hold scan_tiles(n)
// zeroed words and hdr->ticket[slot] must be zero (launch_init_hdr does both).
size_t scan_tiles(int64_t n);
template <typename PT>
hipError_t launch_scan_counts(hipStream_t s, const int32_t *cnt, PT *out, int64_t n, DevHdr *hdr,
                              int slot, uint64_t *tile_state, int classify, uint32_t *bin_lists,
                              int64_t bin_cap, const uint8_t *force = nullptr,
                              const uint32_t *nmslots = nullptr);

}  // namespace hp
