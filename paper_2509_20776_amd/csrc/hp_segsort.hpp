// Segmented sort used by the Build step of every operation (the paper sorts
// received tuples before forming the local matrix, Sec. 4.2 "Build").
//
// Every segment is one output row [rowptr[r], rowptr[r+1]); keys are the new
// column indices, distinct inside a row; values travel with their keys.  A
// Loader supplies element k of row r: either the row already written in
// place (LoadInPlace) or an operation-specific gather (permute reads row
// p[r] of A and maps its columns), so a gather and the sort are one pass.
//
// Length classes:
//   THREAD  2..16     one lane per row, bitonic network in registers
//   WAVE    17..256   one wavefront, rank = number of smaller keys (LDS)
//   BLOCK   257..2048 one workgroup: 64-element runs ranked per wavefront,
//                     then merged pairwise in LDS (merge-path ranks)
//   GLOBAL  > 2048    ranked through an LDS bitmap of the key range (one
//                     1024-thread workgroup per 2^20 columns of the row;
//                     wider rows are split by key range first).
// Rows of <= 64 entries can also be sorted without lists by k_sort_small,
// which walks all rows in groups of 64.
#pragma once
#include "hp_internal.hpp"

namespace hp {

template <typename PT, typename VT>
struct LoadInPlace {
    const PT *rowptr;
    const int32_t *key;
    const VT *val;
    __device__ __forceinline__ int64_t base(int64_t row) const { return rowptr[row]; }
    __device__ __forceinline__ void get(int64_t b, int64_t k, int32_t &kk, VT &vv) const {
        kk = key[b + k];
        vv = val[b + k];
    }
};

template <typename VT>
__device__ __forceinline__ void cswap(int32_t &ka, VT &va, int32_t &kb, VT &vb, bool up) {
    bool sw = (ka > kb) == up;
    int32_t tk = sw ? kb : ka;
    kb = sw ? ka : kb;
    ka = tk;
    VT tv = sw ? vb : va;
    vb = sw ? va : vb;
    va = tv;
}

template <int N, typename VT>
__device__ __forceinline__ void bitonic_regs(int32_t (&k)[N], VT (&v)[N]) {
#pragma unroll
    for (int size = 2; size <= N; size <<= 1)
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < N; i++) {
                int l = i ^ j;
                if (l > i) cswap(k[i], v[i], k[l], v[l], (i & size) == 0);
            }
}

// Sort up to N (4, 8 or 16) elements held by one lane and store the first len.
template <int N, typename VT>
__device__ __forceinline__ void sort_store_regs(int32_t (&k)[N], VT (&v)[N], int len, bool sorted,
                                                int32_t *okey, VT *oval) {
    if (!sorted) bitonic_regs<N, VT>(k, v);
#pragma unroll
    for (int i = 0; i < N; i++)
        if (i < len) {
            okey[i] = k[i];
            oval[i] = v[i];
        }
}

// One lane sorts one row of <= N entries read through the loader.  The
// entry indexes are clamped to the row (len >= 1), so every load, and every
// lookup a renaming loader makes, is issued without waiting on the one
// before (loads under a per-entry branch went out one at a time).
template <int N, typename VT, typename LD>
__device__ __forceinline__ void lane_sort_n(const LD &ld, int64_t sb, int len, bool sorted, int32_t *okey,
                                            VT *oval) {
    int32_t k[N];
    VT v[N];
#pragma unroll
    for (int i = 0; i < N; i++) ld.get(sb, i < len ? i : len - 1, k[i], v[i]);
#pragma unroll
    for (int i = 0; i < N; i++)
        if (i >= len) {
            k[i] = INT32_MAX;
            v[i] = VT(0);
        }
    sort_store_regs<N, VT>(k, v, len, sorted, okey, oval);
}

template <typename VT, typename LD>
__device__ __forceinline__ void lane_sort_row(const LD &ld, int64_t sb, int len, bool sorted,
                                              int32_t *okey, VT *oval) {
    if (len <= 0) return;
    if (len <= 4) lane_sort_n<4, VT>(ld, sb, len, sorted, okey, oval);
    else if (len <= 8) lane_sort_n<8, VT>(ld, sb, len, sorted, okey, oval);
    else lane_sort_n<16, VT>(ld, sb, len, sorted, okey, oval);
}

// Value held by lane l ^ d (d a power of two below 64; every lane of the
// wavefront active).  Distances 1 and 2 are DPP quad permutes, 4 and 8 DPP
// row shifts with a select (the partner is in the same row of 16 lanes);
// larger distances go through LDS permutes.
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v, int d) {
    const int iv = (int)v;
    const int l = lane_id();
    if (d == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, iv, 0xB1, 0xf, 0xf, false);   // quad [1,0,3,2]
    if (d == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, iv, 0x4E, 0xf, 0xf, false);   // quad [2,3,0,1]
    if (d == 4) {
        const int up = __builtin_amdgcn_update_dpp(0, iv, 0x104, 0xf, 0xf, false);   // row_shl:4
        const int dn = __builtin_amdgcn_update_dpp(0, iv, 0x114, 0xf, 0xf, false);   // row_shr:4
        return (uint32_t)((l & 4) ? dn : up);
    }
    if (d == 8) {
        const int up = __builtin_amdgcn_update_dpp(0, iv, 0x108, 0xf, 0xf, false);   // row_shl:8
        const int dn = __builtin_amdgcn_update_dpp(0, iv, 0x118, 0xf, 0xf, false);   // row_shr:8
        return (uint32_t)((l & 8) ? dn : up);
    }
    return (uint32_t)__shfl_xor(iv, d, WAVE);
}
template <typename W>
__device__ __forceinline__ W lane_xor(W v, int d) {
    if constexpr (sizeof(W) == 8) {
        const uint64_t u = (uint64_t)v;
        const uint64_t lo = lane_xor32((uint32_t)u, d), hi = lane_xor32((uint32_t)(u >> 32), d);
        return (W)(lo | (hi << 32));
    } else {
        return (W)lane_xor32((uint32_t)v, d);
    }
}

// Bitonic sorting network over 64*E 32-bit words held E per lane (element
// e = l*E + q), ascending.  Partners e ^ j with j < E sit in the same lane;
// larger j are lane distance j/E apart, swapped through cross-lane shuffles.
template <int E>
__device__ __forceinline__ void bitonic_wave(uint32_t (&x)[E]) {
    const int l = lane_id();
#pragma unroll
    for (int k = 2; k <= WAVE * E; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
            if (j < E) {
#pragma unroll
                for (int q = 0; q < E; q++) {
                    if (q & j) continue;
                    const bool asc = ((l * E + q) & k) == 0;
                    const uint32_t a = x[q], b = x[q | j];
                    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
                    x[q] = asc ? lo : hi;
                    x[q | j] = asc ? hi : lo;
                }
            } else {
                // k > j >= E: the direction and the pair side are lane bits
                const bool keep_min = (((l * E) & k) == 0) == (((l * E) & j) == 0);
#pragma unroll
                for (int q = 0; q < E; q++) {
                    const uint32_t o = lane_xor32(x[q], j / E);
                    x[q] = keep_min ? (o < x[q] ? o : x[q]) : (o < x[q] ? x[q] : o);
                }
            }
        }
    }
}

// Row of len <= 64*E entries whose keys are below 2^24: each key is packed
// with its position (key << 8 | position), the packed words are sorted by
// the network (distinct, so the order is total), and every output slot
// takes its value back from LDS by the position.  Padding words are all
// ones and sort last (a real word equals it only when len == 256).
template <int E, typename VT>
__device__ __forceinline__ void wave_sort_packed(const int32_t (&mk)[4], const VT (&mv)[4], int len,
                                                 int32_t *okey, VT *oval, uint32_t *s_k, VT *s_v) {
    const int l = lane_id();
    uint32_t x[E];
#pragma unroll
    for (int q = 0; q < E; q++) {
        const int e = q * WAVE + l;
        x[q] = 0xFFFFFFFFu;
        if (e < len) {
            x[q] = ((uint32_t)mk[q] << 8) | (uint32_t)e;
            s_v[e] = mv[q];
        }
    }
    bitonic_wave<E>(x);
#pragma unroll
    for (int q = 0; q < E; q++) s_k[l * E + q] = x[q];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < E; q++) {
        const int e = q * WAVE + l;
        if (e < len) {
            const uint32_t w = s_k[e];
            okey[e] = (int32_t)(w >> 8);
            oval[e] = s_v[w & 255u];
        }
    }
    __builtin_amdgcn_wave_barrier();
}

template <typename VT>
__device__ __forceinline__ void wave_sort_regs(const int32_t (&mk)[4], const VT (&mv)[4], int len, int32_t *okey,
                                               VT *oval, int32_t *s_k, VT *s_v);

// One wavefront sorts one row of <= 256 entries (up to 4 per lane).  Keys
// below 2^24 go through the packed bitonic network; otherwise every key's
// rank is the number of smaller keys, read 16 at a time from LDS.
template <typename VT, typename LD>
__device__ __forceinline__ void wave_sort_row(const LD &ld, int64_t sb, int len, bool sorted,
                                              int32_t *okey, VT *oval, int32_t *s_k, VT *s_v) {
    const int l = lane_id();
    int32_t mk[4];
    VT mv[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        mk[q] = INT32_MAX;
        mv[q] = VT(0);
        const int x = q * WAVE + l;
        if (x < len) ld.get(sb, x, mk[q], mv[q]);
    }
    if (sorted) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int x = q * WAVE + l;
            if (x < len) {
                okey[x] = mk[q];
                oval[x] = mv[q];
            }
        }
        return;
    }
    wave_sort_regs<VT>(mk, mv, len, okey, oval, s_k, s_v);
}

// The sorting part of wave_sort_row, on a row already in registers (entry
// e = q * WAVE + lane in mk[q], mv[q], padding INT32_MAX); s_k and s_v are
// the wavefront's staging area (free on entry).
template <typename VT>
__device__ __forceinline__ void wave_sort_regs(const int32_t (&mk)[4], const VT (&mv)[4], int len, int32_t *okey,
                                               VT *oval, int32_t *s_k, VT *s_v) {
    const int l = lane_id();
    bool wide = false;
#pragma unroll
    for (int q = 0; q < 4; q++) wide |= q * WAVE + l < len && (uint32_t)mk[q] >= (1u << 24);
    if (ballot(wide) == 0) {
        uint32_t *sk = reinterpret_cast<uint32_t *>(s_k);
        if (len <= WAVE) wave_sort_packed<1, VT>(mk, mv, len, okey, oval, sk, s_v);
        else if (len <= 2 * WAVE) wave_sort_packed<2, VT>(mk, mv, len, okey, oval, sk, s_v);
        else wave_sort_packed<4, VT>(mk, mv, len, okey, oval, sk, s_v);
        return;
    }
    const int len16 = (len + 15) & ~15;
#pragma unroll
    for (int q = 0; q < 4; q++)
        if (q * WAVE < len16) s_k[q * WAVE + l] = mk[q];   // padding keys are INT32_MAX
    __builtin_amdgcn_wave_barrier();
    int rank[4] = {0, 0, 0, 0};
    // 16 keys per round: four 16-byte LDS reads issued before any is used
    for (int i = 0; i < len16; i += 16) {
        int4 o[4];
#pragma unroll
        for (int r = 0; r < 4; r++) o[r] = *reinterpret_cast<const int4 *>(s_k + i + 4 * r);
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int q = 0; q < 4; q++)
                rank[q] += (o[r].x < mk[q]) + (o[r].y < mk[q]) + (o[r].z < mk[q]) + (o[r].w < mk[q]);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int x = q * WAVE + l;
        if (x < len) {
            okey[rank[q]] = mk[q];
            oval[rank[q]] = mv[q];
        }
    }
}

// Shared-memory blocks of the tile functions (the batched kernel overlays
// them in one buffer).
struct alignas(16) SegSmemWave {
    int32_t k[4][WAVE_MAX];
    uint64_t v[4][WAVE_MAX];   // values by source position (packed-key sort)
};

template <typename PT, typename VT, typename LD>
__device__ void seg_thread_tile(int64_t bid, const PT *__restrict__ rowptr, int32_t *okey, VT *oval,
                                const uint32_t *__restrict__ list, uint32_t count, const LD &ld, int sorted,
                                const DevHdr *hdr) {
    const int64_t t = bid * 256 + threadIdx.x;
    if (t >= count || hdr->err) return;
    int64_t row = list[t];
    int64_t b = rowptr[row];
    int len = (int)(rowptr[row + 1] - b);
    lane_sort_row<VT, LD>(ld, ld.base(row), len, sorted != 0, okey + b, oval + b);
}

template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(256) void k_seg_thread(const PT *__restrict__ rowptr, int32_t *okey,
                                                   VT *oval, const uint32_t *__restrict__ list,
                                                   uint32_t count, LD ld, int sorted,
                                                   const DevHdr *hdr) {
    seg_thread_tile<PT, VT, LD>(blockIdx.x, rowptr, okey, oval, list, count, ld, sorted, hdr);
}

template <typename PT, typename VT, typename LD>
__device__ void seg_wave_tile(int64_t bid, SegSmemWave &sm, const PT *__restrict__ rowptr, int32_t *okey,
                              VT *oval, const uint32_t *__restrict__ list, uint32_t count, const LD &ld,
                              int sorted, const DevHdr *hdr) {
    const int w = threadIdx.x / WAVE;
    const int64_t t = bid * 4 + w;
    if (t >= count || hdr->err) return;
    int64_t row = list[t];
    int64_t b = rowptr[row];
    int len = (int)(rowptr[row + 1] - b);
    wave_sort_row<VT, LD>(ld, ld.base(row), len, sorted != 0, okey + b, oval + b, sm.k[w],
                          reinterpret_cast<VT *>(sm.v[w]));
}

template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(256) void k_seg_wave(const PT *__restrict__ rowptr, int32_t *okey,
                                                 VT *oval, const uint32_t *__restrict__ list,
                                                 uint32_t count, LD ld, int sorted,
                                                 const DevHdr *hdr) {
    __shared__ __align__(16) SegSmemWave sm;
    seg_wave_tile<PT, VT, LD>(blockIdx.x, sm, rowptr, okey, oval, list, count, ld, sorted, hdr);
}

// All rows of <= SMALL_MAX entries, without lists: each wavefront takes 64
// consecutive rows; rows of <= 16 are sorted by their own lane, rows of
// 17..64 by the whole wavefront one after another.  Longer rows are left to
// the class kernels.  With gflag, only the 64-row groups flagged there are
// visited, and rows with skip[row] set (sorted through the class lists) are
// left alone.
template <typename PT, typename VT, typename LD>
__device__ void sort_small_tile(int64_t bid, SegSmemWave &sm, const PT *__restrict__ rowptr, int32_t *okey,
                                VT *oval, int64_t nrows, const LD &ld, const DevHdr *hdr,
                                const uint8_t *__restrict__ gflag = nullptr,
                                const uint8_t *__restrict__ skip = nullptr,
                                const int32_t *__restrict__ srows = nullptr, const uint64_t *nshort = nullptr) {
    if (hdr->err) return;
    const int w = threadIdx.x / WAVE, l = lane_id();
    const int64_t grp = bid * 4 + w;
    // srows: the groups are 64 consecutive entries of this row list
    // (*nshort of them) instead of 64 consecutive rows
    const uint64_t nsv = srows ? *nshort : (uint64_t)nrows;
    const int64_t ngrp = nsv < (uint64_t)nrows ? (int64_t)nsv : nrows;
    if (gflag && (grp * WAVE >= ngrp || !gflag[grp])) return;
    int64_t row = grp * WAVE + l;
    if (srows) {
        const int32_t r = row < ngrp ? srows[row] : -1;
        row = (uint32_t)r < (uint64_t)nrows ? (int64_t)r : nrows;
    }
    int len = 0;
    int64_t b = 0;
    if (row < nrows && !(skip && skip[row])) {
        b = rowptr[row];
        len = (int)(rowptr[row + 1] - b);
    }
    if (len >= 2 && len <= (int)THREAD_MAX) lane_sort_row<VT, LD>(ld, ld.base(row), len, false, okey + b, oval + b);
    uint64_t mid = ballot(len > (int)THREAD_MAX && len <= (int)SMALL_MAX);
    while (mid) {
        const int src = __ffsll((long long)mid) - 1;
        mid &= mid - 1;
        const int64_t r = __shfl(row, src, WAVE);
        const int64_t rb = __shfl(b, src, WAVE);
        const int rl = __shfl(len, src, WAVE);
        wave_sort_row<VT, LD>(ld, ld.base(r), rl, false, okey + rb, oval + rb, sm.k[w],
                              reinterpret_cast<VT *>(sm.v[w]));
    }
}

template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(256) void k_sort_small(const PT *__restrict__ rowptr, int32_t *okey,
                                                   VT *oval, int64_t nrows, LD ld,
                                                   const DevHdr *hdr, const uint8_t *gflag = nullptr,
                                                   const uint8_t *skip = nullptr, const int32_t *srows = nullptr,
                                                   const uint64_t *nshort = nullptr) {
    __shared__ __align__(16) SegSmemWave sm;
    sort_small_tile<PT, VT, LD>(blockIdx.x, sm, rowptr, okey, oval, nrows, ld, hdr, gflag, skip, srows, nshort);
}

// ---- workgroup bitonic sort of one row of up to 8*T entries -----------------
// Every key is packed with its position in the row (key << 32 | position, a
// 64-bit word; real words are distinct and below the all-ones padding), the
// words are sorted by a bitonic network held E per thread (element
// e = t*E + q), and each output slot takes its value back from LDS by the
// position.  Partners closer than E sit in the same thread, closer than 64*E
// in the same wavefront (shuffles); farther ones are exchanged through LDS,
// stored q-major so that consecutive threads hit consecutive words.

template <int T, int E, typename W>
__device__ __forceinline__ void bitonic_block(W (&x)[E], W *s_x) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 2; k <= T * E; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
            if (j < E) {
#pragma unroll
                for (int q = 0; q < E; q++) {
                    if (q & j) continue;
                    const bool asc = ((t * E + q) & k) == 0;
                    const W a = x[q], b = x[q | j];
                    const W lo = a < b ? a : b, hi = a < b ? b : a;
                    x[q] = asc ? lo : hi;
                    x[q | j] = asc ? hi : lo;
                }
            } else {
                // k > j >= E: direction and pair side are bits of t*E
                const bool keep_min = (((t * E) & k) == 0) == (((t * E) & j) == 0);
                const int d = j / E;   // partner thread t ^ d
                if (j < WAVE * E) {
#pragma unroll
                    for (int q = 0; q < E; q++) {
                        const W o = lane_xor<W>(x[q], d);
                        x[q] = keep_min ? (o < x[q] ? o : x[q]) : (o < x[q] ? x[q] : o);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < E; q++) s_x[q * T + t] = x[q];
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < E; q++) {
                        const W o = s_x[q * T + (t ^ d)];
                        x[q] = keep_min ? (o < x[q] ? o : x[q]) : (o < x[q] ? x[q] : o);
                    }
                    __syncthreads();
                }
            }
        }
    }
}

template <int N>
struct alignas(16) SegSmemBitonic {
    uint64_t x[N];   // exchange buffer of the network
    uint64_t v[N];   // values by source position
};

// W = uint64_t: word = key << 32 | position.  W = uint32_t: word = key <<
// PB | position, for keys below 2^(32 - PB) and rows of at most 2^PB
// entries (half the compare and shuffle work).
template <typename VT, typename LD, int T, int E, int N, typename W, int PB>
__device__ __forceinline__ void bitonic_row(const LD &ld, int64_t sb, int len, int32_t *okey, VT *oval,
                                            SegSmemBitonic<N> &sm) {
    const int t = threadIdx.x;
    VT *sv = reinterpret_cast<VT *>(sm.v);
    constexpr W PMASK = (W(1) << PB) - 1;
    W x[E];
    {
        // clamped entry indexes (len >= 1): the E loads, and a renaming
        // loader's lookups, go out together instead of one branch at a time
        int32_t kk[E];
        VT vv[E];
#pragma unroll
        for (int q = 0; q < E; q++) {
            const int i = q * T + t;
            ld.get(sb, i < len ? i : len - 1, kk[q], vv[q]);
        }
#pragma unroll
        for (int q = 0; q < E; q++) {
            const int i = q * T + t;
            x[q] = ~W(0);
            if (i < len) {
                x[q] = ((W)(uint32_t)kk[q] << PB) | (W)i;
                sv[i] = vv[q];
            }
        }
    }
    bitonic_block<T, E, W>(x, reinterpret_cast<W *>(sm.x));
    __syncthreads();   // every value staged (and, in place, every entry read) before any store
#pragma unroll
    for (int q = 0; q < E; q++) {
        const int e = t * E + q;
        if (e < len) {
            okey[e] = (int32_t)(x[q] >> PB);
            oval[e] = sv[(uint32_t)(x[q] & PMASK)];
        }
    }
}

template <typename VT, typename LD, int T, int EMAX, typename W, int PB>
__device__ __forceinline__ void bitonic_any(const LD &ld, int64_t sb, int len, int32_t *okey, VT *oval,
                                            SegSmemBitonic<EMAX * T> &sm) {
    constexpr int N = EMAX * T;
    if (len <= 2 * T) bitonic_row<VT, LD, T, 2, N, W, PB>(ld, sb, len, okey, oval, sm);
    else if (EMAX >= 4 && len <= 4 * T) bitonic_row<VT, LD, T, (EMAX >= 4 ? 4 : 2), N, W, PB>(ld, sb, len, okey, oval, sm);
    else if (EMAX >= 8 && len <= 8 * T) bitonic_row<VT, LD, T, (EMAX >= 8 ? 8 : 2), N, W, PB>(ld, sb, len, okey, oval, sm);
    else if (EMAX >= 16) bitonic_row<VT, LD, T, (EMAX >= 16 ? 16 : 2), N, W, PB>(ld, sb, len, okey, oval, sm);
}

// One workgroup of T threads per listed row of at most EMAX*T entries;
// E = 2, 4, 8 or 16 words a thread by length, LDS sized for EMAX.  narrow
// (every key below 2^(32 - log2(EMAX*T))): 32-bit words.  The row sort
// class BLOCK (257..2048 entries) uses T = 256, EMAX = 8.
template <typename PT, typename VT, typename LD, int T, int EMAX>
__device__ void seg_bitonic_tile(int64_t bid, SegSmemBitonic<EMAX * T> &sm, const PT *__restrict__ rowptr,
                                 int32_t *okey, VT *oval, const uint32_t *__restrict__ list, uint32_t count,
                                 const LD &ld, int narrow, const DevHdr *hdr) {
    constexpr int N = EMAX * T;
    constexpr int PB = N <= 2048 ? 11 : (N <= 4096 ? 12 : 13);
    static_assert(N <= 8192, "position field");
    if (bid >= count || hdr->err) return;
    const int64_t row = list[bid];
    const int64_t b = rowptr[row];
    const int64_t len = rowptr[row + 1] - b;
    if (len > N) return;
    const int64_t sb = ld.base(row);
    if (narrow) bitonic_any<VT, LD, T, EMAX, uint32_t, PB>(ld, sb, (int)len, okey + b, oval + b, sm);
    else bitonic_any<VT, LD, T, EMAX, uint64_t, 32>(ld, sb, (int)len, okey + b, oval + b, sm);
}

template <typename PT, typename VT, typename LD, int T, int EMAX>
__global__ __launch_bounds__(T) void k_seg_bitonic(const PT *__restrict__ rowptr, int32_t *okey, VT *oval,
                                                  const uint32_t *__restrict__ list, uint32_t count, LD ld,
                                                  int narrow, const DevHdr *hdr) {
    __shared__ SegSmemBitonic<EMAX * T> sm;
    seg_bitonic_tile<PT, VT, LD, T, EMAX>(blockIdx.x, sm, rowptr, okey, oval, list, count, ld, narrow, hdr);
}

// Block-class rows (257..BLOCK_MAX entries) in a 256-thread workgroup.
constexpr int BITONIC_EMAX = (int)(BLOCK_MAX / 256);
using SegSmemBlockBitonic = SegSmemBitonic<BLOCK_MAX>;
__host__ __device__ inline int bitonic_narrow(int64_t ncols_out) { return ncols_out <= (int64_t(1) << 21) ? 1 : 0; }

// ---- workgroup LDS sort of <= BLOCK_MAX keys with their 16-bit source index ----
// In: s_k0/s_i0 hold N (a multiple of 64) keys, real keys distinct, padded
// with INT_MAX.  Out: sorted (key, index) pairs in buffer 0 or 1 (returned).
__device__ int block_sort_lds(int32_t *s_k0, uint16_t *s_i0, int32_t *s_k1, uint16_t *s_i1, int N) {
    const int w = threadIdx.x / WAVE, l = lane_id();
    // 1. every 64-element run sorted by one wavefront (rank by counting)
    for (int c = w; c * WAVE < N; c += 4) {
        const int x = c * WAVE + l;
        const int32_t mk = s_k0[x];
        const uint16_t mi = s_i0[x];
        int rank = 0;
        const int32_t *run = s_k0 + c * WAVE;
        for (int i = 0; i < WAVE; i++) {
            const int32_t o = run[i];
            rank += (o < mk) || (o == mk && i < l);   // pads (equal keys) keep lane order
        }
        s_k1[c * WAVE + rank] = mk;
        s_i1[c * WAVE + rank] = mi;
    }
    __syncthreads();
    int cur = 1;
    int32_t *ka[2] = {s_k0, s_k1};
    uint16_t *ia[2] = {s_i0, s_i1};
    // 2. merge runs pairwise: an element's output rank is its rank in its own
    //    run plus the number of elements of the other run before it (ties:
    //    the left run first, which also keeps the padding in place)
    for (int width = WAVE; width < N; width <<= 1) {
        const int32_t *ik = ka[cur];
        const uint16_t *ii = ia[cur];
        int32_t *ok = ka[cur ^ 1];
        uint16_t *oi = ia[cur ^ 1];
        for (int x = threadIdx.x; x < N; x += 256) {
            const int a0 = (x / (2 * width)) * 2 * width;
            const bool in_a = (x - a0) < width;
            const int own = in_a ? (x - a0) : (x - a0 - width);
            const int o0 = in_a ? a0 + width : a0;
            const int olen = in_a ? min(width, N - (a0 + width)) : width;
            const int32_t key = ik[x];
            int lo = 0, hi = olen > 0 ? olen : 0;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const int32_t o = ik[o0 + mid];
                if (in_a ? (o < key) : (o <= key)) lo = mid + 1;
                else hi = mid;
            }
            ok[a0 + own + lo] = key;
            oi[a0 + own + lo] = ii[x];
        }
        __syncthreads();
        cur ^= 1;
    }
    return cur;
}

struct SegSmemBlock {
    int32_t k[2][BLOCK_MAX];
    uint16_t i[2][BLOCK_MAX];
};

template <typename PT, typename VT, typename LD>
__device__ void seg_block_tile(int64_t bid, SegSmemBlock &sm, const PT *__restrict__ rowptr, int32_t *okey,
                               VT *oval, const uint32_t *__restrict__ list, uint32_t count, const LD &ld,
                               int sorted, const DevHdr *hdr) {
    const int64_t t = bid;
    if (t >= count || hdr->err) return;
    int64_t row = list[t];
    int64_t b = rowptr[row];
    int64_t len64 = rowptr[row + 1] - b;
    int64_t sb = ld.base(row);
    if (sorted || len64 > BLOCK_MAX) {
        // already in order: copy through the loader
        for (int64_t i = threadIdx.x; i < len64; i += 256) {
            int32_t kk;
            VT vv;
            ld.get(sb, i, kk, vv);
            okey[b + i] = kk;
            oval[b + i] = vv;
        }
        return;
    }
    const int len = (int)len64;
    const int N = (len + WAVE - 1) / WAVE * WAVE;
    for (int i = threadIdx.x; i < N; i += 256) {
        int32_t kk = INT32_MAX;
        if (i < len) {
            VT vv;
            ld.get(sb, i, kk, vv);
        }
        sm.k[0][i] = kk;
        sm.i[0][i] = (uint16_t)i;
    }
    __syncthreads();
    const int cur = block_sort_lds(sm.k[0], sm.i[0], sm.k[1], sm.i[1], N);
    // gather every value first: with an in-place loader the row is both the
    // source and the destination
    constexpr int PER = BLOCK_MAX / 256;
    VT vr[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = q * 256 + threadIdx.x;
        vr[q] = VT(0);
        if (i < len) {
            int32_t kk;
            ld.get(sb, sm.i[cur][i], kk, vr[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = q * 256 + threadIdx.x;
        if (i < len) {
            okey[b + i] = sm.k[cur][i];
            oval[b + i] = vr[q];
        }
    }
}

template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(256) void k_seg_block(const PT *__restrict__ rowptr, int32_t *okey,
                                                  VT *oval, const uint32_t *__restrict__ list,
                                                  uint32_t count, LD ld, int sorted,
                                                  const DevHdr *hdr) {
    __shared__ SegSmemBlock sm;
    seg_block_tile<PT, VT, LD>(blockIdx.x, sm, rowptr, okey, oval, list, count, ld, sorted, hdr);
}

// ---- GLOBAL class ------------------------------------------------------------
// Keys of one row are distinct, so sorting a long row is ranking: mark every
// key in an LDS bitmap of its key range, prefix-count the bitmap, and the
// rank of a key is the number of marked bits below it.  A bitmap covers
// 2^RB_SHIFT keys (128 KB of LDS); rows whose output has more columns are
// first split by key range into buckets of that width (one workgroup per row,
// LDS histogram), and every non-empty bucket is ranked by its own workgroup.
// When one bucket covers all columns the split is skipped: the rank
// workgroup reads the row through the loader and stashes it in the row's
// temporary region, so in-place rows can be rewritten.
constexpr int BKT_SHIFT = 20;                        // keys per bucket = bitmap bits
constexpr int BKT_MAXNB = 4096;                      // buckets per row (2^31 columns need 2048)
constexpr int RANK_THREADS = 1024;
constexpr int RANK_U = 16;                           // elements per thread and pass
constexpr int RB_WORDS = 1 << (BKT_SHIFT - 5);       // 32768 bitmap words
constexpr int RB_GRP = 8;                            // words per prefix group
constexpr int RB_NGRP = RB_WORDS / RB_GRP;           // 4096 prefix entries

struct SegSmemBucket {
    uint32_t h[BKT_MAXNB + 1];
    uint32_t sw[4];
};

struct SegSmemRank {
    uint32_t bm[RB_WORDS];
    uint32_t pre[RB_NGRP];
    uint32_t sw[RANK_THREADS / WAVE];
};

// Split one long row into key buckets of width 2^BKT_SHIFT (256 threads).
// Elements are placed into the row's temporary region in bucket order
// (arbitrary order inside a bucket); the bucket start offsets go to
// bstart[t * (nb + 1) + ...].
template <typename PT, typename VT, typename LD>
__device__ void seg_bucket_tile(int64_t bid, SegSmemBucket &sm, const PT *__restrict__ rowptr,
                                const uint32_t *__restrict__ list, const uint64_t *__restrict__ goff,
                                uint32_t count, const LD &ld, int nb, int32_t *tkey, VT *tval, uint32_t *bstart,
                                const DevHdr *hdr) {
    uint32_t *s_h = sm.h;
    uint32_t *s_sw = sm.sw;
    const int64_t t = bid;
    if (t >= count || hdr->err) return;
    const int64_t row = list[t];
    const int64_t b = rowptr[row];
    const int64_t len = rowptr[row + 1] - b;
    const int64_t sb = ld.base(row);
    int32_t *yk = tkey + goff[t];
    VT *yv = tval + goff[t];
    for (int i = threadIdx.x; i <= nb; i += 256) s_h[i] = 0;
    __syncthreads();
    // BKT_U entries per thread and round, their loads (and a renaming
    // loader's lookups) issued together: indexes are clamped to the row
    // (len >= 1) and the extra lanes masked afterwards.  One entry per round
    // left a hub row of 67K entries at two dependent loads per 256 entries.
    constexpr int BKT_U = 8;
    for (int64_t i0 = 0; i0 < len; i0 += 256 * BKT_U) {
        int32_t kk[BKT_U];
        VT vv[BKT_U];
#pragma unroll
        for (int u = 0; u < BKT_U; u++) {
            const int64_t i = i0 + u * 256 + threadIdx.x;
            ld.get(sb, i < len ? i : len - 1, kk[u], vv[u]);
        }
#pragma unroll
        for (int u = 0; u < BKT_U; u++)
            if (i0 + u * 256 + threadIdx.x < len) atomicAdd(&s_h[(uint32_t)kk[u] >> BKT_SHIFT], 1u);
    }
    __syncthreads();
    // exclusive scan of the histogram, 256 threads over nb+1 counters
    const int per = (nb + 1 + 255) / 256;
    uint32_t loc = 0;
    for (int q = 0; q < per; q++) {
        int i = threadIdx.x * per + q;
        if (i <= nb) loc += s_h[i];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<256, uint32_t>(loc, s_sw, tot);
    for (int q = 0; q < per; q++) {
        int i = threadIdx.x * per + q;
        if (i <= nb) {
            uint32_t c = s_h[i];
            s_h[i] = run;
            bstart[(int64_t)t * (nb + 1) + i] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int64_t i0 = 0; i0 < len; i0 += 256 * BKT_U) {
        int32_t kk[BKT_U];
        VT vv[BKT_U];
#pragma unroll
        for (int u = 0; u < BKT_U; u++) {
            const int64_t i = i0 + u * 256 + threadIdx.x;
            ld.get(sb, i < len ? i : len - 1, kk[u], vv[u]);
        }
#pragma unroll
        for (int u = 0; u < BKT_U; u++) {
            if (i0 + u * 256 + threadIdx.x >= len) continue;
            const uint32_t pos = atomicAdd(&s_h[(uint32_t)kk[u] >> BKT_SHIFT], 1u);
            yk[pos] = kk[u];
            yv[pos] = vv[u];
        }
    }
    __syncthreads();
}

template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(256) void k_seg_bucket(const PT *__restrict__ rowptr,
                                                   const uint32_t *__restrict__ list,
                                                   const uint64_t *__restrict__ goff, uint32_t count,
                                                   LD ld, int nb, int32_t *tkey, VT *tval,
                                                   uint32_t *bstart, const DevHdr *hdr) {
    __shared__ SegSmemBucket sm;
    seg_bucket_tile<PT, VT, LD>(blockIdx.x, sm, rowptr, list, goff, count, ld, nb, tkey, tval, bstart, hdr);
}

// Rank one bucket (item = t * nb + bucket) of GLOBAL row list[t] with
// RANK_THREADS threads.  nb == 1: the row comes through the loader and is
// stashed in its temporary region first; nb > 1: the bucket is read from the
// temporary region the split wrote.  Every thread reads back only the
// elements it stashed itself.
template <typename PT, typename VT, typename LD>
__device__ void seg_rank_tile(int64_t item, SegSmemRank &sm, const PT *__restrict__ rowptr, int32_t *okey,
                              VT *oval, const uint32_t *__restrict__ list, const uint64_t *__restrict__ goff,
                              uint32_t count, const LD &ld, int nb, int32_t *tkey, VT *tval,
                              const uint32_t *__restrict__ bstart, const DevHdr *hdr) {
    const int64_t t = item / nb;
    const int bk = (int)(item % nb);
    if (t >= count || hdr->err) return;
    const int64_t row = list[t];
    const int64_t b = rowptr[row];
    int64_t s0 = 0, len = rowptr[row + 1] - b;
    if (nb > 1) {
        const uint32_t *bs = bstart + t * (nb + 1);
        s0 = bs[bk];
        len = (int64_t)bs[bk + 1] - s0;
    }
    if (len == 0) return;
    int32_t *yk = tkey + goff[t] + s0;
    VT *yv = tval + goff[t] + s0;
    const uint32_t kbase = (uint32_t)bk << BKT_SHIFT;
    const int tid = threadIdx.x;
    uint4 *bm4 = reinterpret_cast<uint4 *>(sm.bm);
    for (int i = tid; i < RB_WORDS / 4; i += RANK_THREADS) bm4[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    // Each pass handles RANK_U elements per thread with all loads issued
    // before any is used: a row of 17K entries is then 2 rounds of memory
    // latency per loop instead of 17.
    constexpr int64_t STEP = (int64_t)RANK_THREADS * RANK_U;
    if (nb == 1) {
        const int64_t sb = ld.base(row);
        for (int64_t i0 = 0; i0 < len; i0 += STEP) {
            int32_t kk[RANK_U];
            VT vv[RANK_U];
#pragma unroll
            for (int u = 0; u < RANK_U; u++) {
                const int64_t i = i0 + u * RANK_THREADS + tid;
                if (i < len) ld.get(sb, i, kk[u], vv[u]);
            }
#pragma unroll
            for (int u = 0; u < RANK_U; u++) {
                const int64_t i = i0 + u * RANK_THREADS + tid;
                if (i < len) {
                    yk[i] = kk[u];
                    yv[i] = vv[u];
                    const uint32_t d = (uint32_t)kk[u];
                    atomicOr(&sm.bm[d >> 5], 1u << (d & 31));
                }
            }
        }
    } else {
        for (int64_t i0 = 0; i0 < len; i0 += STEP) {
            uint32_t dd[RANK_U];
#pragma unroll
            for (int u = 0; u < RANK_U; u++) {
                const int64_t i = i0 + u * RANK_THREADS + tid;
                dd[u] = i < len ? (uint32_t)yk[i] - kbase : 0xFFFFFFFFu;
            }
#pragma unroll
            for (int u = 0; u < RANK_U; u++)
                if (dd[u] != 0xFFFFFFFFu) atomicOr(&sm.bm[dd[u] >> 5], 1u << (dd[u] & 31));
        }
    }
    __syncthreads();
    // prefix counts of the bitmap in groups of RB_GRP words
    constexpr int GPT = RB_NGRP / RANK_THREADS;   // groups per thread
    uint32_t c[GPT];
    uint32_t loc = 0;
#pragma unroll
    for (int g = 0; g < GPT; g++) {
        const uint4 *w4 = bm4 + (size_t)(tid * GPT + g) * (RB_GRP / 4);
        uint32_t n = 0;
#pragma unroll
        for (int q = 0; q < RB_GRP / 4; q++) {
            const uint4 w = w4[q];
            n += __popc(w.x) + __popc(w.y) + __popc(w.z) + __popc(w.w);
        }
        c[g] = n;
        loc += n;
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<RANK_THREADS, uint32_t>(loc, sm.sw, tot);
#pragma unroll
    for (int g = 0; g < GPT; g++) {
        sm.pre[tid * GPT + g] = run;
        run += c[g];
    }
    __syncthreads();
    const int64_t ob = b + s0;
    for (int64_t i0 = 0; i0 < len; i0 += STEP) {
        int32_t kk[RANK_U];
        VT vv[RANK_U];
#pragma unroll
        for (int u = 0; u < RANK_U; u++) {
            const int64_t i = i0 + u * RANK_THREADS + tid;
            if (i < len) {
                kk[u] = yk[i];
                vv[u] = yv[i];
            }
        }
#pragma unroll
        for (int u = 0; u < RANK_U; u++) {
            const int64_t i = i0 + u * RANK_THREADS + tid;
            if (i >= len) continue;
            const uint32_t d = (uint32_t)kk[u] - kbase;
            const uint32_t w = d >> 5;
            const uint32_t g0 = w & ~uint32_t(RB_GRP - 1);
            uint32_t r = sm.pre[w / RB_GRP] + __popc(sm.bm[w] & ((1u << (d & 31)) - 1u));
            for (uint32_t x = g0; x < w; x++) r += __popc(sm.bm[x]);
            okey[ob + r] = kk[u];
            oval[ob + r] = vv[u];
        }
    }
    __syncthreads();
}

template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(RANK_THREADS) void k_seg_rank(const PT *__restrict__ rowptr, int32_t *okey, VT *oval,
                                                          const uint32_t *__restrict__ list,
                                                          const uint64_t *__restrict__ goff, uint32_t count, LD ld,
                                                          int nb, int32_t *tkey, VT *tval,
                                                          const uint32_t *__restrict__ bstart,
                                                          const DevHdr *hdr) {
    __shared__ __align__(16) SegSmemRank sm;
    seg_rank_tile<PT, VT, LD>(blockIdx.x, sm, rowptr, okey, oval, list, goff, count, ld, nb, tkey, tval, bstart,
                              hdr);
}

// Class lists: NBINS lists of capacity cap, then cap uint64 temporary
// offsets for the GLOBAL class.  The exec workspace holds the GLOBAL rows'
// temporary keys (round256(elems*4) bytes), then their values, then the
// bucket tables (rows * (nb + 1) uint32).
inline int seg_nbuckets(int64_t ncols_out) {
    int64_t nb = (ncols_out + (1 << BKT_SHIFT) - 1) >> BKT_SHIFT;
    return nb < 1 ? 1 : (int)nb;
}

inline size_t seg_tmp_bytes(uint64_t glob_elems, uint64_t glob_rows, size_t vsize, int64_t ncols_out) {
    if (!glob_elems) return 0;
    size_t kb = (glob_elems * 4 + 255) & ~uint64_t(255);
    size_t vb = (glob_elems * vsize + 255) & ~uint64_t(255);
    int nb = seg_nbuckets(ncols_out);
    size_t bb = nb <= BKT_MAXNB ? glob_rows * (size_t)(nb + 1) * 4 : 0;
    return kb + vb + bb + 256;
}

inline size_t seg_list_words(int64_t cap) { return (size_t)cap * NBINS + (size_t)cap * 2 + 4; }

template <typename PT, typename VT, typename LD>
hipError_t launch_seg_classes(hipStream_t s, const PT *rowptr, int32_t *okey, VT *oval,
                              const uint32_t *lists, int64_t cap, const uint32_t *cnt, LD ld,
                              bool sorted, int64_t ncols_out, bool inplace, void *tmp,
                              uint64_t glob_elems, const DevHdr *hdr, bool do_thread,
                              bool do_wave = true) {
    const uint64_t *goff = reinterpret_cast<const uint64_t *>(lists + NBINS * cap);
    if (do_thread && cnt[BIN_THREAD])
        hipLaunchKernelGGL((k_seg_thread<PT, VT, LD>), dim3((cnt[BIN_THREAD] + 255) / 256), dim3(256),
                           0, s, rowptr, okey, oval, lists + BIN_THREAD * cap, cnt[BIN_THREAD], ld,
                           (int)sorted, hdr);
    if (do_wave && cnt[BIN_WAVE])
        hipLaunchKernelGGL((k_seg_wave<PT, VT, LD>), dim3((cnt[BIN_WAVE] + 3) / 4), dim3(256), 0, s,
                           rowptr, okey, oval, lists + BIN_WAVE * cap, cnt[BIN_WAVE], ld, (int)sorted,
                           hdr);
    if (cnt[BIN_BLOCK]) {
        if (sorted)
            hipLaunchKernelGGL((k_seg_block<PT, VT, LD>), dim3(cnt[BIN_BLOCK]), dim3(256), 0, s, rowptr,
                               okey, oval, lists + BIN_BLOCK * cap, cnt[BIN_BLOCK], ld, 1, hdr);
        else
            hipLaunchKernelGGL((k_seg_bitonic<PT, VT, LD, 256, BITONIC_EMAX>), dim3(cnt[BIN_BLOCK]), dim3(256), 0, s,
                               rowptr, okey, oval, lists + BIN_BLOCK * cap, cnt[BIN_BLOCK], ld,
                               bitonic_narrow(ncols_out), hdr);
    }
    if (cnt[BIN_GLOBAL]) {
        int32_t *tk = (int32_t *)tmp;
        char *p = (char *)tmp + ((glob_elems * sizeof(int32_t) + 255) & ~uint64_t(255));
        VT *tv = (VT *)p;
        uint32_t *bst = (uint32_t *)(p + ((glob_elems * sizeof(VT) + 255) & ~uint64_t(255)));
        const int nb = seg_nbuckets(ncols_out);
        if (sorted) {
            hipLaunchKernelGGL((k_seg_block<PT, VT, LD>), dim3(cnt[BIN_GLOBAL]), dim3(256), 0, s, rowptr,
                               okey, oval, lists + BIN_GLOBAL * cap, cnt[BIN_GLOBAL], ld, 1, hdr);
        } else {
            // LDS bitmap rank, one 1024-thread workgroup per row (after a
            // key-range split when the output is wider than 2^20 columns).
            // Its time is set by the longest rows, and the shorter rows of
            // the class finish under it: a bitonic workgroup per row of up
            // to 4096 entries ran 50 us beside a 60 us rank of the rest.
            if (nb > 1)
                hipLaunchKernelGGL((k_seg_bucket<PT, VT, LD>), dim3(cnt[BIN_GLOBAL]), dim3(256), 0, s, rowptr,
                                   lists + BIN_GLOBAL * cap, goff, cnt[BIN_GLOBAL], ld, nb, tk, tv, bst, hdr);
            hipLaunchKernelGGL((k_seg_rank<PT, VT, LD>), dim3((unsigned)((int64_t)cnt[BIN_GLOBAL] * nb)),
                               dim3(RANK_THREADS), 0, s, rowptr, okey, oval, lists + BIN_GLOBAL * cap, goff,
                               cnt[BIN_GLOBAL], ld, nb, tk, tv, bst, hdr);
        }
    }
    return hipGetLastError();
}

}  // namespace hp
