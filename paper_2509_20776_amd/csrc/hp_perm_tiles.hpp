// Tile functions of the permutation path (paper Sec. 2.1; Identify of
// Sec. 4.2 on one GPU), shared by the plain kernels in hp_permute.hip and
// the batched persistent kernel.  See hp_permute.hip for the algorithm.
#pragma once
#include "hp_internal.hpp"
#include "hp_segsort.hpp"

namespace hp {
namespace perm {

template <typename PT>
__device__ inline void perm_prepare_tile(int64_t bid, const PT *__restrict__ arow, const int32_t *__restrict__ p,
                                         const int32_t *__restrict__ q, int64_t m, int64_t n, int32_t *pinv,
                                         int32_t *qinv, int32_t *cnt, DevHdr *hdr) {
    const int64_t t = bid * 256 + threadIdx.x;
    if (t < m) {
        const int32_t r = p[t];
        if (r < 0 || r >= m) {
            atomicOr(&hdr->err, E_RANGE);     // error path only
            cnt[t] = 0;
        } else {
            pinv[r] = (int32_t)t;
            cnt[t] = (int32_t)(arow[r + 1] - arow[r]);
        }
    }
    if (q && t < n) {
        const int32_t c = q[t];
        if (c < 0 || c >= n) atomicOr(&hdr->err, E_RANGE);
        else qinv[c] = (int32_t)t;
    }
}

// pinv and qinv start filled with -1 and every in-range value of p (q) has
// been scattered: a slot left at -1 means some value is missing, hence
// (m values in m slots) another is repeated.  Sequential reads only.
__device__ inline void perm_check_tile(int64_t bid, int64_t m, int64_t n, const int32_t *__restrict__ pinv,
                                       const int32_t *__restrict__ qinv, bool general, DevHdr *hdr) {
    const int64_t t = bid * 256 + threadIdx.x;
    bool bad = false;
    if (t < m) bad |= pinv[t] < 0;
    if (general && t < n) bad |= qinv[t] < 0;
    if (bad) atomicOr(&hdr->err, E_NOTPERM);   // error path only
}

// Rows of at most 4 entries: one lane per SOURCE row r, streamed in order
// (coalesced reads of A, local reads of qinv for banded matrices), written
// to output row pinv[r] after an in-register sort of the mapped columns.
// Longer rows go through the class kernels (pull from A).
template <typename PT, typename VT>
__device__ inline void perm_fill_short_tile(
    int64_t bid, const PT *__restrict__ arow, const int32_t *__restrict__ acol, const VT *__restrict__ aval,
    const int32_t *__restrict__ pinv, const int32_t *__restrict__ cmap, const PT *__restrict__ crow,
    int32_t *__restrict__ ccol, VT *__restrict__ cval, int64_t m, int64_t n, const DevHdr *hdr) {
    if (hdr->err) return;
    const int64_t r = bid * 256 + threadIdx.x;
    if (r >= m) return;
    const int64_t s = arow[r];
    const int len = (int)(arow[r + 1] - s);
    if (len == 0 || len > 4) return;
    const int64_t d = crow[pinv[r]];
    int32_t k[4];
    VT v[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        k[i] = INT32_MAX;
        v[i] = VT(0);
        if (i < len) {
            k[i] = cmap[clampc(acol[s + i], n)];
            v[i] = aval[s + i];
        }
    }
    sort_store_regs<4, VT>(k, v, len, false, ccol + d, cval + d);
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

// ---- pull fill of the plain permutation ---------------------------------------
// Output row i is row p[i] of A with every column c renamed qinv[c].  The
// renaming is done once for all stored entries by a streaming pass (colq,
// in A's storage order: coalesced reads of the columns, and for banded
// matrices local reads of qinv), so the fill itself reads each source row
// once, at a random place, and writes the output rows in order: random
// reads and coalesced writes, instead of the random partial-line writes of
// a push to row pinv[r].

// colq[k] = cmap[col[k]] for the 1024 entries k of tile bid.
__device__ inline void perm_colmap_tile(int64_t bid, const int32_t *__restrict__ acol, int64_t nnz, int64_t n,
                                        const int32_t *__restrict__ cmap, int32_t *__restrict__ colq) {
    const int64_t b = bid * 1024 + threadIdx.x;
    int32_t c[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int64_t k = b + u * 256;
        c[u] = k < nnz ? acol[k] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int64_t k = b + u * 256;
        if (k < nnz) colq[k] = cmap[clampc(c[u], n)];
    }
}

// Output rows of at most 4 entries, one lane per output row i (in order).
// colq == nullptr: the columns are renamed here, cmap[col[k]] (used when
// short rows hold few of the entries, so the renaming pass is not run).
template <typename PT, typename VT>
__device__ inline void perm_pull_short_tile(int64_t bid, const PT *__restrict__ arow, const int32_t *__restrict__ colq,
                                            const VT *__restrict__ aval, const int32_t *__restrict__ p,
                                            const PT *__restrict__ crow, int32_t *__restrict__ ccol,
                                            VT *__restrict__ cval, int64_t m, const DevHdr *hdr,
                                            const int32_t *__restrict__ acol = nullptr,
                                            const int32_t *__restrict__ cmap = nullptr, int64_t n = 0) {
    if (hdr->err) return;
    const int64_t i = bid * 256 + threadIdx.x;
    if (i >= m) return;
    const int32_t pr = p[i];
    const int64_t src = (uint32_t)pr < (uint64_t)m ? (int64_t)pr : 0;   // p was checked by the plan
    const int64_t s = arow[src];
    const int len = (int)(arow[src + 1] - s);
    if (len == 0 || len > 4) return;
    const int64_t d = crow[i];
    int32_t k[4];
    VT v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        k[u] = INT32_MAX;
        v[u] = VT(0);
        if (u < len) {
            k[u] = colq ? colq[s + u] : cmap[clampc(acol[s + u], n)];
            v[u] = aval[s + u];
        }
    }
    sort_store_regs<4, VT>(k, v, len, false, ccol + d, cval + d);
}

// Rename the columns in a pass of their own when output rows of at most 4
// entries hold at least half of them (the pull fill of those rows then
// reads each row's renamed columns in one place); otherwise the fill and
// the class sorts look each column up in qinv as they go (LoadPerm), and
// the pass would only add its traffic.
__host__ __device__ inline bool perm_use_colq(int64_t nnz, int64_t long_entries) {
    return nnz > 0 && 2 * (nnz - long_entries) >= nnz;
}

// Longer output rows: the class sorts pull row p[i] with its columns
// already renamed in colq.
template <typename PT, typename VT>
struct LoadPermMapped {
    const PT *arow;
    const int32_t *colq;
    const VT *aval;
    const int32_t *p;
    int64_t m;
    __device__ __forceinline__ int64_t base(int64_t row) const {
        const int32_t pr = p[row];
        return arow[(uint32_t)pr < (uint64_t)m ? (int64_t)pr : 0];
    }
    __device__ __forceinline__ void get(int64_t b, int64_t k, int32_t &kk, VT &vv) const {
        kk = colq[b + k];
        vv = aval[b + k];
    }
};

}  // namespace perm
}  // namespace hp
