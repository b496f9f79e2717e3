// Exclusive scan with row classification, as tile functions shared by the
// plain per-call kernels and the batched persistent kernel: the single-pass
// tile (decoupled look-back), and the pieces of the three-pass form for long
// scans (tile sums, their scan, the tile pass from a given prefix).
//
// Single-pass tiles are started in launch order (an atomic ticket in the
// plain kernel, the batch queue order otherwise), so a tile only ever waits
// on tiles that are already running: every wait ends.  The wait is still
// bounded (SCAN_WAIT_TICKS); reaching it raises E_TIMEOUT and the kernel
// finishes.
#pragma once
#include "hp_internal.hpp"

namespace hp {

constexpr int SCAN_BLOCK = 256;   // threads of a scan tile
constexpr int SCAN_ITEMS = 16;   // 4096 counts per tile: fewer tiles, tickets and look-back rounds
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;
constexpr uint64_t ST_AGG = 1ull << 62, ST_PRE = 2ull << 62, ST_VAL = (1ull << 62) - 1;
constexpr uint64_t SCAN_WAIT_TICKS = 10000000ull;   // 0.1 s of the 100 MHz wall clock


// Sort class of a row of `len` entries under classification `mode`:
//   1  rows longer than 4 (shorter rows are sorted by the producer itself)
//   2  every row of >= 2 entries
//   3  when `all`: flagged rows and rows longer than SMALL_MAX (shorter
//      unflagged rows are sorted by the extraction gather or by
//      k_sort_small); else only flagged rows
//   4  only flagged rows
__device__ __forceinline__ int class_of(int64_t len, int mode, bool all, bool flagged) {
    if (len < 2) return -1;
    if (mode == 1 && len <= 4) return -1;
    if (mode == 4 && !flagged) return -1;
    if (mode == 3) {
        if (all) {
            if (len <= SMALL_MAX && !flagged) return -1;
        } else if (!flagged) {
            return -1;
        }
    }
    if (len <= THREAD_MAX) return BIN_THREAD;
    if (len <= WAVE_MAX) return BIN_WAVE;
    if (len <= BLOCK_MAX) return BIN_BLOCK;
    return BIN_GLOBAL;
}

// Per-wavefront staging of its WAVE*SCAN_ITEMS counts (and later its
// outputs): read and written 64-wide in index order, used 16 consecutive
// per lane.  One pad word per 16 keeps both patterns free of bank
// conflicts.
constexpr int SCAN_SEG = WAVE * SCAN_ITEMS;
constexpr int SCAN_STAGE = SCAN_SEG + SCAN_SEG / 16;
static_assert(SCAN_ITEMS == 16, "the staging offsets below assume 16 counts a lane");
// word of count j (j + j/16): lane l's item k sits at 17*l + k; the k-th
// 64-wide row at 68*k + l + l/16 (constant offsets from one base each)

struct ScanSmem {
    uint64_t wave[SCAN_BLOCK / WAVE];
    uint64_t excl;
    uint32_t bc[NBINS], bbase[NBINS];
    unsigned long long ge, gbase;
    int all;
    // 32-bit words: the counts on the way in, the outputs on the way out
    // (a 64-bit output in two rounds, low then high words), so a block
    // holds 17 KB of LDS
    uint32_t stage[SCAN_BLOCK / WAVE][SCAN_STAGE];
};

// One tile of the exclusive scan of n int32 counts into out (PT, n+1
// entries).  Single pass (tile_prefix == nullptr): tiles must be started in
// increasing order (the caller's ticket) so that a tile only waits on
// running tiles.  Second pass of the three-pass form: tile_prefix[tile] is
// the tile's exclusive prefix, and no tile waits.  CLS false: classify is
// 0 and the class-list code is left out of the kernel.
template <typename PT, bool CLS = true>
__device__ __forceinline__ void scan_counts_tile(int64_t tile, ScanSmem &sm, const int32_t *__restrict__ cnt,
                                 PT *__restrict__ out, int64_t n, DevHdr *hdr, int slot,
                                 uint64_t *tile_state, int classify, uint32_t *lists, int64_t cap,
                                 uint64_t *goff, const uint8_t *__restrict__ force,
                                 const uint32_t *__restrict__ nmslots,
                                 const uint64_t *__restrict__ tile_prefix = nullptr) {
    uint64_t *s_wave = sm.wave;
    uint64_t &s_excl = sm.excl;
    uint32_t *s_bc = sm.bc, *s_bbase = sm.bbase;
    unsigned long long &s_ge = sm.ge, &s_gbase = sm.gbase;
    int &s_all = sm.all;
    if (threadIdx.x == 0) {
        s_ge = 0;
        s_all = 1;
    }
    if (threadIdx.x < NBINS) s_bc[threadIdx.x] = 0;
    if (classify == 3 && threadIdx.x < WAVE) {
        // any block of the J-table build that saw J out of order
        uint64_t any = ballot(ld_agent(&nmslots[threadIdx.x * 32]) != 0);
        if (threadIdx.x == 0) s_all = any != 0;
    }
    __syncthreads();
    // Wavefront w owns the SCAN_SEG consecutive counts from seg; lane l
    // works on 16 consecutive ones (seg + l*16 + k), and the loads and
    // stores go 64-wide in index order through the wavefront's staging area.
    const int w = threadIdx.x / WAVE, l = lane_id();
    const int64_t seg = tile * SCAN_TILE + (int64_t)w * SCAN_SEG;
    uint32_t *st32 = sm.stage[w];
    const int rowb = l + (l >> 4), lanb = 17 * l;
    if (seg + SCAN_SEG <= n) {
        const int32_t *src = cnt + seg + l;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; k++) st32[rowb + 68 * k] = (uint32_t)src[k * WAVE];
    } else {
        for (int k = 0; k < SCAN_ITEMS; k++) {
            const int64_t idx = seg + k * WAVE + l;
            st32[rowb + 68 * k] = idx < n ? (uint32_t)cnt[idx] : 0u;
        }
    }
    __builtin_amdgcn_wave_barrier();
    int32_t v[SCAN_ITEMS];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) v[k] = (int32_t)st32[lanb + k];
    __builtin_amdgcn_wave_barrier();
    const int64_t base = seg + (int64_t)l * SCAN_ITEMS;   // this lane's first count
    uint64_t tsum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) tsum += (uint64_t)(uint32_t)v[k];
    uint64_t tile_total;
    uint64_t texcl = block_excl_scan<SCAN_BLOCK, uint64_t>(tsum, s_wave, tile_total);

    if (tile_prefix) {
        if (threadIdx.x == 0) s_excl = tile_prefix[tile];
    } else if (threadIdx.x < WAVE) {
        // publish this tile's aggregate, then look back for its prefix
        if (lane_id() == 0)
            st_agent(&tile_state[tile], (tile == 0 ? ST_PRE : ST_AGG) | (tile_total & ST_VAL));
        uint64_t excl = 0;
        if (tile > 0) {
            int64_t j = tile - 1;
            const uint64_t t0 = wall_clock64();
            uint32_t spins = 0;
            while (true) {
                int64_t idx = j - lane_id();
                uint64_t s = idx >= 0 ? ld_agent(&tile_state[idx]) : ST_PRE;
                uint64_t flag = s & ~ST_VAL;
                uint64_t pre = ballot(flag == ST_PRE);
                uint64_t inval = ballot(flag == 0);
                int fp = pre ? __ffsll((long long)pre) - 1 : 64;
                uint64_t need = fp >= 63 ? ~0ull : ((2ull << fp) - 1);
                if (inval & need) {
                    // bounded wait: 0.1 s of the 100 MHz wall clock, or stop at
                    // once when another wait of this request already gave up
                    ++spins;
                    const bool give_up = (wall_clock64() - t0 > SCAN_WAIT_TICKS) ||
                                         ((spins & 63) == 0 && (ld_agent(&hdr->err) & E_TIMEOUT));
                    if (__shfl(give_up ? 1 : 0, 0, WAVE)) {
                        if (lane_id() == 0) raise_err(hdr, E_TIMEOUT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                uint64_t part = (lane_id() <= fp) ? (s & ST_VAL) : 0;
                excl += wave_sum(part);
                if (pre) break;
                j -= WAVE;
            }
            if (lane_id() == 0) st_agent(&tile_state[tile], ST_PRE | ((excl + tile_total) & ST_VAL));
        }
        if (lane_id() == 0) s_excl = excl;
    }
    __syncthreads();
    {
        // the outputs' 32-bit words, transposed through LDS and stored
        // 64-wide in index order: all of an int32 output, or the low then
        // the high words of an int64 one
        const uint64_t run0 = s_excl + texcl;
        uint32_t *dst32 = reinterpret_cast<uint32_t *>(out);
        constexpr int NW = sizeof(PT) / 4;
#pragma unroll
        for (int hw = 0; hw < NW; hw++) {
            uint64_t run = run0;
#pragma unroll
            for (int k = 0; k < SCAN_ITEMS; k++) {
                st32[lanb + k] = (uint32_t)(run >> (32 * hw));
                run += (uint32_t)v[k];
            }
            __builtin_amdgcn_wave_barrier();
            if (seg + SCAN_SEG <= n) {
                uint32_t *dst = dst32 + (seg + l) * NW + hw;
#pragma unroll
                for (int k = 0; k < SCAN_ITEMS; k++) dst[k * WAVE * NW] = st32[rowb + 68 * k];
            } else {
                for (int k = 0; k < SCAN_ITEMS; k++) {
                    const int64_t idx = seg + k * WAVE + l;
                    if (idx < n) dst32[idx * NW + hw] = st32[rowb + 68 * k];
                }
            }
            __builtin_amdgcn_wave_barrier();   // the reads above before the next round's writes
        }
    }
    const int64_t last_base = (n - 1) / SCAN_TILE;
    if (tile == last_base && threadIdx.x == SCAN_BLOCK - 1) {
        uint64_t total = s_excl + tile_total;
        out[n] = (PT)total;
        hdr->total[slot] = total;
        if (sizeof(PT) == 4 && total > (uint64_t)INT32_MAX) raise_err(hdr, E_OVERFLOW);
        if (classify == 3 && s_all) atomicOr(&hdr->flags, F_NOT_MONOTONE);
    }
    if (CLS && classify) {
        // block-aggregated append to the class lists: each lane counts its
        // 16 rows per class, takes one LDS offset per class (and one for
        // the GLOBAL entries), the block one global offset per class; then
        // the lane recomputes its rows' classes and appends them in order
        // (no per-row offsets kept in registers)
        const bool all = s_all != 0;
        // bit k: row base + k flagged, force[base + k] != 0 in mode 3, 1 or 2
        // in mode 4 (3 marks a merged row its merge already sorted)
        uint32_t flags = 0;
        if (classify == 3 || classify == 4) {
#pragma unroll
            for (int k = 0; k < SCAN_ITEMS; k++) {
                const uint32_t f = base + k < n ? force[base + k] : 0u;
                if (classify == 3 ? f != 0 : (f == 1 || f == 2)) flags |= 1u << k;
            }
        }
        // modes that classify flagged rows only: a tile without one skips the
        // appends (its barriers included: the test is block-wide)
        const bool only_flagged = classify == 4 || (classify == 3 && !all);
        if (!(only_flagged && !__syncthreads_or(flags != 0))) {
            uint32_t lc[NBINS] = {0, 0, 0, 0};
            unsigned long long lge = 0;
#pragma unroll
            for (int k = 0; k < SCAN_ITEMS; k++) {
                const int b = base + k < n ? class_of(v[k], classify, all, (flags >> k) & 1u) : -1;
#pragma unroll
                for (int q = 0; q < NBINS; q++) lc[q] += b == q ? 1u : 0u;
                if (b == BIN_GLOBAL) lge += (uint32_t)v[k];
            }
            uint32_t lb[NBINS];
#pragma unroll
            for (int q = 0; q < NBINS; q++) lb[q] = lc[q] ? atomicAdd(&s_bc[q], lc[q]) : 0u;
            unsigned long long ge = lge ? atomicAdd(&s_ge, lge) : 0ull;
            __syncthreads();
            if (threadIdx.x < NBINS && s_bc[threadIdx.x])
                s_bbase[threadIdx.x] = atomicAdd(&hdr->bin_cnt[threadIdx.x], s_bc[threadIdx.x]);
            if (threadIdx.x == NBINS && s_ge)
                s_gbase = atomicAdd((unsigned long long *)&hdr->bin_elems[BIN_GLOBAL], s_ge);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < SCAN_ITEMS; k++) {
                const int b = base + k < n ? class_of(v[k], classify, all, (flags >> k) & 1u) : -1;
                if (b < 0) continue;
                uint32_t slot = 0;
#pragma unroll
                for (int q = 0; q < NBINS; q++)
                    if (b == q) slot = lb[q]++;
                const uint32_t pos = s_bbase[b] + slot;
                if (pos < cap) {
                    lists[(int64_t)b * cap + pos] = (uint32_t)(base + k);
                    if (b == BIN_GLOBAL) goff[pos] = s_gbase + ge;
                }
                if (b == BIN_GLOBAL) ge += (uint32_t)v[k];
            }
        }
    }
    __syncthreads();
}

// First pass of the three-pass form: the sum of the tile's counts (the
// same SCAN_TILE counts as scan_counts_tile, read in 64-wide rows) into
// partial[tile].
__device__ inline void scan_reduce_tile(int64_t tile, uint64_t *s_wave, const int32_t *__restrict__ cnt, int64_t n,
                                        uint64_t *partial) {
    const int64_t base = tile * SCAN_TILE + threadIdx.x;
    uint64_t tsum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; k++) {
        const int64_t idx = base + (int64_t)k * SCAN_BLOCK;
        tsum += idx < n ? (uint64_t)(uint32_t)cnt[idx] : 0;
    }
    uint64_t total;
    (void)block_excl_scan<SCAN_BLOCK, uint64_t>(tsum, s_wave, total);
    if (threadIdx.x == 0) partial[tile] = total;
}

// Middle pass: exclusive scan of the ntiles partial sums in place, by one
// workgroup of PSCAN_BLOCK threads, PSCAN_ITEMS consecutive sums a thread per
// round.
constexpr int PSCAN_BLOCK = 1024;
constexpr int PSCAN_ITEMS = 8;
__device__ inline void scan_partials_block(uint64_t *s_wave, uint64_t *partial, int64_t ntiles) {
    uint64_t run = 0;
    for (int64_t c0 = 0; c0 < ntiles; c0 += (int64_t)PSCAN_BLOCK * PSCAN_ITEMS) {
        const int64_t b = c0 + (int64_t)threadIdx.x * PSCAN_ITEMS;
        uint64_t v[PSCAN_ITEMS], t = 0;
#pragma unroll
        for (int k = 0; k < PSCAN_ITEMS; k++) {
            v[k] = b + k < ntiles ? partial[b + k] : 0;
            t += v[k];
        }
        uint64_t tot;
        uint64_t x = run + block_excl_scan<PSCAN_BLOCK, uint64_t>(t, s_wave, tot);
#pragma unroll
        for (int k = 0; k < PSCAN_ITEMS; k++) {
            if (b + k < ntiles) partial[b + k] = x;
            x += v[k];
        }
        run += tot;
    }
}

}  // namespace hp
