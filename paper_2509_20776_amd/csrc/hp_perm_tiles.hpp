// Tile functions of the permutation path (paper Sec. 2.1; Identify of
// Sec. 4.2 on one GPU), shared by the plain kernels in hp_permute.hip and
// the batched persistent kernel.  See hp_permute.hip for the algorithm.
#pragma once
#include "hp_internal.hpp"
#include "hp_segsort.hpp"

namespace hp {
namespace perm {

// pmark (optional): when the inverse of p itself is not needed (the pull
// fill of a general permutation only reads p and qinv), every value r of p
// just sets byte pmark[r] instead of pinv[r] = t: a quarter of the bytes.
template <typename PT>
__device__ inline void perm_prepare_tile(int64_t bid, const PT *__restrict__ arow, const int32_t *__restrict__ p,
                                         const int32_t *__restrict__ q, int64_t m, int64_t n, int32_t *pinv,
                                         int32_t *qinv, int32_t *cnt, DevHdr *hdr, uint8_t *pmark = nullptr) {
    const int64_t t = bid * 256 + threadIdx.x;
    if (t < m) {
        const int32_t r = p[t];
        if (r < 0 || r >= m) {
            atomicOr(&hdr->err, E_RANGE);     // error path only
            cnt[t] = 0;
        } else {
            if (pmark) pmark[r] = 1;
            else pinv[r] = (int32_t)t;
            cnt[t] = (int32_t)(arow[r + 1] - arow[r]);
        }
    }
    if (q && t < n) {
        const int32_t c = q[t];
        if (c < 0 || c >= n) atomicOr(&hdr->err, E_RANGE);
        else qinv[c] = (int32_t)t;
    }
}

// The q half of perm_prepare_tile on its own.  The plain permutation runs
// the two halves as two launches: one kernel that mixes the scatter of
// qinv with the gather of row lengths ran 957 us on a 16.7M-row grid,
// the two apart 508 + 199 us.
__device__ inline void perm_qinv_tile(int64_t bid, const int32_t *__restrict__ q, int64_t n, int32_t *qinv,
                                      DevHdr *hdr) {
    const int64_t t = bid * 256 + threadIdx.x;
    if (t < n) {
        const int32_t c = q[t];
        if (c < 0 || c >= n) atomicOr(&hdr->err, E_RANGE);   // error path only
        else qinv[c] = (int32_t)t;
    }
}

// pinv and qinv start filled with -1 (pmark with 0) and every in-range
// value of p (q) has been scattered: a slot left at -1 (0) means some value
// is missing, hence (m values in m slots) another is repeated.  Sequential
// reads only.
__device__ inline void perm_check_tile(int64_t bid, int64_t m, int64_t n, const int32_t *__restrict__ pinv,
                                       const int32_t *__restrict__ qinv, bool general, DevHdr *hdr,
                                       const uint8_t *__restrict__ pmark = nullptr) {
    const int64_t t = bid * 256 + threadIdx.x;
    bool bad = false;
    if (t < m) bad |= pmark ? pmark[t] == 0 : pinv[t] < 0;
    if (general && t < n) bad |= qinv[t] < 0;
    if (bad) atomicOr(&hdr->err, E_NOTPERM);   // error path only
}

// perm_check_tile with four slots a thread and vector loads (the plain
// kernels: ceil(max(m, n) / 1024) workgroups of 256); the tables start on
// 256-byte boundaries (pmark is allocated in 32-bit words).
__device__ __forceinline__ bool any_neg4(const int32_t *__restrict__ a, int64_t t, int64_t len) {
    if (t + 4 <= len) {
        const int4 v = *reinterpret_cast<const int4 *>(a + t);
        return (v.x | v.y | v.z | v.w) < 0;
    }
    bool bad = false;
    for (int k = 0; k < 4; k++)
        if (t + k < len) bad |= a[t + k] < 0;
    return bad;
}

__device__ inline void perm_check4_tile(int64_t bid, int64_t m, int64_t n, const int32_t *__restrict__ pinv,
                                        const int32_t *__restrict__ qinv, bool general, DevHdr *hdr,
                                        const uint8_t *__restrict__ pmark = nullptr) {
    const int64_t t = (bid * 256 + threadIdx.x) * 4;
    bool bad = false;
    if (t < m) {
        if (pmark) {
            if (t + 4 <= m) {
                const uint32_t w = *reinterpret_cast<const uint32_t *>(pmark + t);
                bad |= ((w - 0x01010101u) & ~w & 0x80808080u) != 0;   // a zero byte
            } else {
                for (int k = 0; k < 4; k++)
                    if (t + k < m) bad |= pmark[t + k] == 0;
            }
        } else {
            bad |= any_neg4(pinv, t, m);
        }
    }
    if (general && t < n) bad |= any_neg4(qinv, t, n);
    if (bad) atomicOr(&hdr->err, E_NOTPERM);   // error path only
}

// Longer rows: output row i is row p[i] of A with columns mapped (pull).
template <typename PT, typename VT>
struct LoadPerm {
    const PT *arow;
    const int32_t *acol;
    const VT *aval;
    const int32_t *p;
    const int32_t *cmap;
    int64_t n;
    __device__ __forceinline__ int64_t base(int64_t row) const { return arow[p[row]]; }
    __device__ __forceinline__ void get(int64_t b, int64_t k, int32_t &kk, VT &vv) const {
        kk = cmap[clampc(acol[b + k], n)];
        vv = aval[b + k];
    }
};

// ---- pull fill --------------------------------------------------------------
// Output row i is row p[i] of A with every column c renamed qinv[c]: the
// fill reads each source row at a random place and writes the output rows
// in order (random reads and coalesced writes, instead of the random
// partial-line writes of a push to row pinv[r]).

// Output rows of at most 4 entries, one lane per output row i (in order),
// columns renamed on the way.
template <typename PT, typename VT>
__device__ inline void perm_pull_short_tile(int64_t bid, const PT *__restrict__ arow, const int32_t *__restrict__ acol,
                                            const VT *__restrict__ aval, const int32_t *__restrict__ p,
                                            const int32_t *__restrict__ cmap, int64_t n, const PT *__restrict__ crow,
                                            int32_t *__restrict__ ccol, VT *__restrict__ cval, int64_t m,
                                            const DevHdr *hdr) {
    if (hdr->err) return;
    const int64_t i = bid * 256 + threadIdx.x;
    if (i >= m) return;
    const int32_t pr = p[i];
    const int64_t src = (uint32_t)pr < (uint64_t)m ? (int64_t)pr : 0;   // p was checked by the plan
    const int64_t s = arow[src];
    const int len = (int)(arow[src + 1] - s);
    if (len == 0 || len > 4) return;
    const int64_t d = crow[i];
    // clamped indexes (len >= 1): the four loads, then the four lookups, go
    // out together
    int32_t c[4], k[4];
    VT v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int64_t e = s + (u < len ? u : len - 1);
        c[u] = acol[e];
        v[u] = aval[e];
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int32_t mk = cmap[clampc(c[u], n)];
        k[u] = u < len ? mk : INT32_MAX;
        if (u >= len) v[u] = VT(0);
    }
    sort_store_regs<4, VT>(k, v, len, false, ccol + d, cval + d);
}

// Row slots: when rows of at most 4 entries hold most of the entries, a
// streaming pass first packs each such source row r, renamed and sorted,
// into a fixed slot of its own (4 column ids, then 4 values: 32 bytes for
// 4-byte values, 64 for 8-byte ones, aligned to the slot size).  The fill
// of output row i then reads one aligned slot, slot p[i], instead of the
// row bounds, columns and values of row p[i] in three places: one random
// line per row instead of about three, for a sequential pass over A.
template <typename VT>
constexpr int perm_slot_bytes() { return sizeof(VT) == 8 ? 64 : 32; }

__host__ __device__ inline bool perm_use_slots(int64_t nnz, int64_t long_entries) {
    return nnz > 0 && 2 * (nnz - long_entries) >= nnz;
}

// Entries of one wavefront's 64 rows staged through LDS by the pack when
// they are at most this many (rows of about 4 entries): the wavefront then
// reads them 64-wide in storage order, and each lane takes its row from LDS.
constexpr int PACK_STAGE = 256;

// Pack source rows bid*256 .. +255 (one lane each) into their slots; lk/lv
// hold PACK_STAGE entries per wavefront of the block.  The slot is written
// whole (unused entries as INT32_MAX / 0) so that its lines are full writes.
template <typename PT, typename VT>
__device__ inline void perm_pack_tile(int64_t bid, const PT *__restrict__ arow, const int32_t *__restrict__ acol,
                                      const VT *__restrict__ aval, const int32_t *__restrict__ cmap, int64_t n,
                                      int64_t m, char *__restrict__ slots, int32_t *lk, VT *lv) {
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    const int64_t r0 = bid * 256 + (int64_t)w * WAVE;
    if (r0 >= m) return;   // the whole wavefront
    const int64_t r = r0 + l;
    const int64_t rend = r0 + WAVE < m ? r0 + WAVE : m;
    const int64_t s0 = arow[r0], s1 = arow[rend];
    const int64_t s = r < m ? (int64_t)arow[r] : s1;
    const int len = r < m ? (int)(arow[r + 1] - s) : 0;
    const bool staged = s1 - s0 <= PACK_STAGE;
    int32_t *wk = lk + w * PACK_STAGE;
    VT *wv = lv + w * PACK_STAGE;
    if (staged) {
        // all column and value loads of the wavefront in one round, then all
        // renaming lookups in a second (a loop over the entries would make
        // each lookup wait on its own column load)
        static_assert(PACK_STAGE % WAVE == 0, "whole 64-wide rows of staged entries");
        int32_t ck[PACK_STAGE / WAVE];
        VT cv[PACK_STAGE / WAVE];
#pragma unroll
        for (int u = 0; u < PACK_STAGE / WAVE; u++) {
            const int64_t k = s0 + u * WAVE + l;
            ck[u] = k < s1 ? acol[k] : 0;
            cv[u] = k < s1 ? aval[k] : VT(0);
        }
        // every lane looks up (idle lanes column 0, one shared line), so
        // the lookups are issued together rather than one branch at a time
        int32_t mk[PACK_STAGE / WAVE];
#pragma unroll
        for (int u = 0; u < PACK_STAGE / WAVE; u++) mk[u] = cmap[clampc(ck[u], n)];
#pragma unroll
        for (int u = 0; u < PACK_STAGE / WAVE; u++) {
            const int64_t k = s0 + u * WAVE + l;
            if (k < s1) {
                wk[k - s0] = mk[u];
                wv[k - s0] = cv[u];
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (len == 0 || len > 4) return;
    int32_t k[4];
    VT v[4];
    if (staged) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            k[u] = u < len ? wk[s - s0 + u] : INT32_MAX;
            v[u] = u < len ? wv[s - s0 + u] : VT(0);
        }
    } else {
        // clamped indexes (len >= 1): the loads and lookups of the four
        // entries go out together
        int32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t e = s + (u < len ? u : len - 1);
            c[u] = acol[e];
            v[u] = aval[e];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int32_t mk = cmap[clampc(c[u], n)];
            k[u] = u < len ? mk : INT32_MAX;
            if (u >= len) v[u] = VT(0);
        }
    }
    bitonic_regs<4, VT>(k, v);
    char *slot = slots + r * perm_slot_bytes<VT>();
    *reinterpret_cast<uint4 *>(slot) = make_uint4((uint32_t)k[0], (uint32_t)k[1], (uint32_t)k[2], (uint32_t)k[3]);
    if constexpr (sizeof(VT) == 8) {
        reinterpret_cast<ulonglong2 *>(slot)[1] = make_ulonglong2(v[0], v[1]);
        reinterpret_cast<ulonglong2 *>(slot)[2] = make_ulonglong2(v[2], v[3]);
        reinterpret_cast<ulonglong2 *>(slot)[3] = make_ulonglong2(0, 0);
    } else {
        reinterpret_cast<uint4 *>(slot)[1] = make_uint4(v[0], v[1], v[2], v[3]);
    }
}

// Copy the first len (1..4) entries of the row slot of source row src to
// output position d.
template <typename VT>
__device__ __forceinline__ void perm_slot_copy(const char *__restrict__ slots, int64_t src, int len, int64_t d,
                                               int32_t *__restrict__ ccol, VT *__restrict__ cval) {
    const char *slot = slots + src * perm_slot_bytes<VT>();
    const uint4 kk = *reinterpret_cast<const uint4 *>(slot);
    VT v[4];
    if constexpr (sizeof(VT) == 8) {
        const ulonglong2 a = reinterpret_cast<const ulonglong2 *>(slot)[1];
        const ulonglong2 b = reinterpret_cast<const ulonglong2 *>(slot)[2];
        v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y;
    } else {
        const uint4 a = reinterpret_cast<const uint4 *>(slot)[1];
        v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
    }
    const int32_t k[4] = {(int32_t)kk.x, (int32_t)kk.y, (int32_t)kk.z, (int32_t)kk.w};
#pragma unroll
    for (int u = 0; u < 4; u++)
        if (u < len) {
            ccol[d + u] = k[u];
            cval[d + u] = v[u];
        }
}

// Output rows bid*256 .. +255 of at most 4 entries (one lane each), copied
// from slot p[i]; the row's length is that of output row i.
template <typename PT, typename VT>
__device__ inline void perm_slot_fill_tile(int64_t bid, const int32_t *__restrict__ p, const char *__restrict__ slots,
                                           const PT *__restrict__ crow, int32_t *__restrict__ ccol,
                                           VT *__restrict__ cval, int64_t m, const DevHdr *hdr) {
    if (hdr->err) return;
    const int64_t i = bid * 256 + threadIdx.x;
    if (i >= m) return;
    const int64_t d = crow[i];
    const int len = (int)(crow[i + 1] - d);
    if (len == 0 || len > 4) return;
    // (loading p[i] together with the row bounds, ahead of this branch, did
    // not speed the fill up: it is bound by the random slot reads)
    const int32_t pr = p[i];
    const int64_t src = (uint32_t)pr < (uint64_t)m ? (int64_t)pr : 0;   // p was checked by the plan
    perm_slot_copy<VT>(slots, src, len, d, ccol, cval);
}

}  // namespace perm
}  // namespace hp
