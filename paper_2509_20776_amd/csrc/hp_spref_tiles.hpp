// Tile functions of the extraction path (paper Sec. 2.2; Identify of
// Sec. 4.5 on one GPU), shared by the plain kernels in hp_spref.hip and the
// batched persistent kernel.  See hp_spref.hip for the algorithm.
#pragma once
#include "hp_internal.hpp"

namespace hp {
namespace spref {


constexpr int SR_BLOCK = 256;
constexpr int SR_U = 8;                       // entries per lane per step
constexpr int64_t SR_LB = 256;                // rows above this many entries are big
constexpr int64_t SR_BW = WAVE * SR_U;        // entries per big-row chunk
constexpr int SR_BIGBLOCKS = 2048;            // persistent workgroups for big chunks (launched first)
constexpr int NMSLOTS = 64;                   // spread "J not increasing" flag slots

// ---- J tables ---------------------------------------------------------------
__device__ inline void spref_jscatter_tile(int64_t bid, const int32_t *__restrict__ J, int64_t nJ,
                                           int64_t n, uint8_t *mark, int32_t *jpos, uint32_t *nm,
                                           DevHdr *hdr) {
    const int64_t j = bid * 256 + threadIdx.x;
    bool notmono = false;
    if (j < nJ) {
        const int32_t c = J[j];
        if (j + 1 < nJ && c >= J[j + 1]) notmono = true;
        if (c < 0 || c >= n) {
            atomicOr(&hdr->err, E_RANGE);   // error path only
        } else {
            mark[c] = 1;
            jpos[c] = (int32_t)j;
        }
    }
    if (__syncthreads_or(notmono) && threadIdx.x == 0) nm[(bid & (NMSLOTS - 1)) * 32] = 1u;
}

__device__ inline void spref_jpack_tile(int64_t bid, const int32_t *__restrict__ J, int64_t nJ, int64_t n,
                                        const uint8_t *__restrict__ mark, uint32_t *bm, int64_t nw,
                                        const int32_t *__restrict__ jpos, int32_t *Dn, uint32_t *dm) {
    const int64_t t = bid * 256 + threadIdx.x;
    if (t < nw) {
        const uint4 *p = reinterpret_cast<const uint4 *>(mark + t * 32);
        const uint4 a = p[0], b = p[1];
        const uint32_t w8[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        uint32_t m = 0;
#pragma unroll
        for (int q = 0; q < 8; q++)
#pragma unroll
            for (int y = 0; y < 4; y++) m |= ((w8[q] >> (8 * y)) & 0xffu ? 1u : 0u) << (4 * q + y);
        bm[t] = m;
    }
    if (t < nJ) {
        const int32_t c = J[t];
        int32_t loser = 0;
        if (c >= 0 && c < n && jpos[c] != (int32_t)t) {
            loser = 1;
            atomicOr(&dm[c >> 5], 1u << (c & 31));
        }
        Dn[t] = loser;
    }
}

// Link every non-winning position of a repeated column into the chain
// headed by jpos[c]: jpos[c] = ~t_last, Dn[t] = previous head, ..., ending
// in the winner (>= 0).  Chain order is arbitrary; rows are sorted later.
__device__ inline void spref_jlink_tile(int64_t bid, const int32_t *__restrict__ J, int64_t nJ, int32_t *jpos,
                                        int32_t *Dn) {
    const int64_t t = bid * 256 + threadIdx.x;
    if (t < nJ && Dn[t] == 1) Dn[t] = atomicExch(&jpos[J[t]], ~(int32_t)t);
}

// ---- selected rows ----------------------------------------------------------
template <typename PT>
__device__ inline void spref_rows_tile(int64_t bid, const PT *__restrict__ arow, const int32_t *__restrict__ I,
                                       int64_t nI, int64_t m, int64_t *rs, int32_t *rl, int32_t *ch, uint8_t *big,
                                       DevHdr *hdr) {
    const int64_t i = bid * 256 + threadIdx.x;
    if (i >= nI) return;
    const int32_t r = I[i];
    int64_t s = 0, len = 0;
    if (r < 0 || r >= m) atomicOr(&hdr->err, E_RANGE);   // error path only
    else {
        s = arow[r];
        len = arow[r + 1] - s;
    }
    rs[i] = s;
    rl[i] = (int32_t)len;
    ch[i] = len > SR_LB ? (int32_t)((len + SR_BW - 1) / SR_BW) : 0;
    big[i] = len > SR_LB ? 1 : 0;
}

// ---- shared pieces of count and gather -------------------------------------
__device__ __forceinline__ bool test_bit(const uint32_t *b, int64_t c) {
    return (b[c >> 5] >> (c & 31)) & 1u;
}

// Output entries produced by a hit on column c (its multiplicity in J).
__device__ __forceinline__ int mult_of(int64_t c, const uint32_t *dm, const int32_t *jpos,
                                       const int32_t *Dn) {
    if (!test_bit(dm, c)) return 1;
    int k = 1;
    int32_t v = jpos[c];
    while (v < 0) {
        k++;
        v = Dn[~v];
    }
    return k;
}

template <typename VT>
__device__ __forceinline__ void emit_hits(int64_t c, VT v, int64_t pos, const uint32_t *dm,
                                          const int32_t *jpos, const int32_t *Dn, int32_t *ccol,
                                          VT *cval) {
    int32_t x = jpos[c];
    if (test_bit(dm, c)) {
        while (x < 0) {
            ccol[pos] = ~x;
            cval[pos] = v;
            pos++;
            x = Dn[~x];
        }
    }
    ccol[pos] = x;
    cval[pos] = v;
}

// Largest i in [0, n) with a[i] <= x, a nondecreasing and a[0] <= x; the
// wavefront probes 64 positions per round (4 rounds for 2^24 entries).
__device__ __forceinline__ int64_t wave_search_le(const int64_t *a, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    const int l = lane_id();
    while (hi - lo > 1) {
        const int64_t step = (hi - lo + WAVE - 1) / WAVE;
        const int64_t idx = lo + (int64_t)l * step;
        const bool le = idx < hi && a[idx] <= x;
        const uint64_t msk = ballot(le);
        const int last = 63 - __clzll((long long)msk);
        lo = lo + (int64_t)last * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// Row (0..63) of the wave-local concatenation holding entry e.
__device__ __forceinline__ int row_of(const int32_t *start, int32_t e) {
    int lo = 0, hi = WAVE;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct GroupSmem {
    int32_t start[WAVE + 1];
    int32_t cnt[WAVE];
    int64_t rs[WAVE];
    int64_t crow[WAVE];
};

// ---- count (plan) -------------------------------------------------------------
// Tile bid of the count pass: bid < nbw are the long-row workers (persistent
// over the chunks), then one tile per 256 selected rows.
__device__ inline void spref_count_tile(
    int64_t bid, int64_t nbw, GroupSmem *gs, const int32_t *__restrict__ acol, int64_t n,
    const int64_t *__restrict__ rs, const int32_t *__restrict__ rl, const int64_t *__restrict__ cp, int64_t nI,
    const uint32_t *__restrict__ bm, const uint32_t *__restrict__ dm, const int32_t *__restrict__ jpos,
    const int32_t *__restrict__ Dn, int32_t *cnt, const DevHdr *hdr) {
    if (hdr->err) return;
    const int w = threadIdx.x / WAVE, l = lane_id();
    if (bid >= nbw) {
        GroupSmem &g = gs[w];
        const int64_t i = ((bid - nbw) * 4 + w) * WAVE + l;
        int len = 0;
        bool small = false;
        if (i < nI) {
            const int L = rl[i];
            small = L <= SR_LB;
            if (small) {
                len = L;
                g.rs[l] = rs[i];
            }
        }
        const int incl = wave_incl_scan(len);
        const int E = __shfl(incl, WAVE - 1, WAVE);
        g.start[l] = incl - len;
        g.cnt[l] = 0;
        __builtin_amdgcn_wave_barrier();
        for (int e0 = 0; e0 < E; e0 += SR_BW) {
            int64_t c[SR_U];
            int rr[SR_U];
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                const int e = e0 + u * WAVE + l;
                c[u] = -1;
                rr[u] = 0;
                if (e < E) {
                    const int r = row_of(g.start, e);
                    rr[u] = r;
                    c[u] = clampc(acol[g.rs[r] + (e - g.start[r])], n);
                }
            }
#pragma unroll
            for (int u = 0; u < SR_U; u++)
                if (c[u] >= 0 && test_bit(bm, c[u])) atomicAdd(&g.cnt[rr[u]], mult_of(c[u], dm, jpos, Dn));
        }
        __builtin_amdgcn_wave_barrier();
        if (small) cnt[i] = g.cnt[l];
        return;
    }
    // big-row chunks, one wavefront each (these workgroups come first)
    const int64_t nbig = cp[nI];
    const int64_t nwaves = nbw * 4;
    for (int64_t q = bid * 4 + w; q < nbig; q += nwaves) {
        const int64_t row = wave_search_le(cp, nI + 1, q);
        const int64_t b = (q - cp[row]) * SR_BW;
        const int64_t e = min(b + SR_BW, (int64_t)rl[row]);
        const int64_t base = rs[row];
        int sum = 0;
#pragma unroll
        for (int u = 0; u < SR_U; u++) {
            const int64_t k = b + u * WAVE + l;
            if (k < e) {
                const int64_t c = clampc(acol[base + k], n);
                if (test_bit(bm, c)) sum += mult_of(c, dm, jpos, Dn);
            }
        }
        sum = wave_sum(sum);
        if (l == 0 && sum) atomicAdd(&cnt[row], sum);
    }
}

// ---- gather (exec) ------------------------------------------------------------
// Within one step of SR_U slices, lane l of slice u holds entry e0+64u+l, so
// slices in order are entries in scan order.  For each slice the wavefront
// computes an exclusive scan of the hit multiplicities; a hit's position in
// its row is the row's running count plus the scan minus the scan at the
// row's first lane in the slice.
template <typename PT, typename VT>
__device__ inline void spref_gather_tile(
    int64_t bid, int64_t nbw, GroupSmem *gs, const int32_t *__restrict__ acol, const VT *__restrict__ aval,
    int64_t n, const int64_t *__restrict__ rs, const int32_t *__restrict__ rl, const int64_t *__restrict__ cp,
    int64_t nI, const uint32_t *__restrict__ bm, const uint32_t *__restrict__ dm,
    const int32_t *__restrict__ jpos, const int32_t *__restrict__ Dn, const PT *__restrict__ crow,
    int32_t *ccol, VT *cval, int32_t *cursor, const DevHdr *hdr) {
    if (hdr->err) return;
    const int w = threadIdx.x / WAVE, l = lane_id();
    const uint64_t le_mask = (l == 63) ? ~0ull : ((2ull << l) - 1);
    if (bid >= nbw) {
        GroupSmem &g = gs[w];
        const int64_t i = ((bid - nbw) * 4 + w) * WAVE + l;
        int len = 0;
        if (i < nI) {
            const int L = rl[i];
            if (L <= SR_LB) {
                len = L;
                g.rs[l] = rs[i];
                g.crow[l] = (int64_t)crow[i];
            }
        }
        const int incl = wave_incl_scan(len);
        const int E = __shfl(incl, WAVE - 1, WAVE);
        g.start[l] = incl - len;
        g.cnt[l] = 0;            // running output count per row
        __builtin_amdgcn_wave_barrier();
        for (int e0 = 0; e0 < E; e0 += SR_BW) {
            int64_t c[SR_U], k[SR_U];
            int rr[SR_U], mm[SR_U];
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                const int e = e0 + u * WAVE + l;
                c[u] = -1;
                rr[u] = -1 - l;  // distinct per idle lane: never joins a segment
                k[u] = 0;
                if (e < E) {
                    const int r = row_of(g.start, e);
                    rr[u] = r;
                    k[u] = g.rs[r] + (e - g.start[r]);
                    c[u] = clampc(acol[k[u]], n);
                }
            }
#pragma unroll
            for (int u = 0; u < SR_U; u++)
                mm[u] = (c[u] >= 0 && test_bit(bm, c[u])) ? mult_of(c[u], dm, jpos, Dn) : 0;
            VT v[SR_U];
#pragma unroll
            for (int u = 0; u < SR_U; u++) v[u] = mm[u] ? aval[k[u]] : VT(0);
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                const int ex = wave_incl_scan(mm[u]) - mm[u];
                const int prev_r = __shfl_up(rr[u], 1, WAVE);
                const int next_r = __shfl_down(rr[u], 1, WAVE);
                const bool is_start = l == 0 || prev_r != rr[u];
                const bool is_last = l == WAVE - 1 || next_r != rr[u];
                const uint64_t starts = ballot(is_start);
                const int first = 63 - __clzll((long long)(starts & le_mask));
                const int base_ex = __shfl(ex, first, WAVE);
                if (mm[u]) {
                    const int r = rr[u];
                    const int64_t pos = g.crow[r] + g.cnt[r] + (ex - base_ex);
                    emit_hits<VT>(c[u], v[u], pos, dm, jpos, Dn, ccol, cval);
                }
                __builtin_amdgcn_wave_barrier();
                if (rr[u] >= 0 && is_last) g.cnt[rr[u]] += ex + mm[u] - base_ex;
                __builtin_amdgcn_wave_barrier();
            }
        }
        return;
    }
    // big-row chunks: positions inside the chunk in scan order, the chunk's
    // block of the row reserved with the row's cursor (workgroups come first)
    const int64_t nbig = cp[nI];
    const int64_t nwaves = nbw * 4;
    for (int64_t q = bid * 4 + w; q < nbig; q += nwaves) {
        const int64_t row = wave_search_le(cp, nI + 1, q);
        const int64_t b = (q - cp[row]) * SR_BW;
        const int64_t e = min(b + SR_BW, (int64_t)rl[row]);
        const int64_t base = rs[row];
        int64_t c[SR_U];
        int mm[SR_U];
#pragma unroll
        for (int u = 0; u < SR_U; u++) {
            const int64_t kk = b + u * WAVE + l;
            c[u] = -1;
            if (kk < e) c[u] = clampc(acol[base + kk], n);
        }
        int run = 0;
        int ex[SR_U];
#pragma unroll
        for (int u = 0; u < SR_U; u++) {
            mm[u] = (c[u] >= 0 && test_bit(bm, c[u])) ? mult_of(c[u], dm, jpos, Dn) : 0;
            const int inc = wave_incl_scan(mm[u]);
            ex[u] = run + inc - mm[u];
            run += __shfl(inc, WAVE - 1, WAVE);
        }
        int32_t cb = 0;
        if (l == 0 && run) cb = atomicAdd(&cursor[row], run);
        cb = __shfl(cb, 0, WAVE);
        const int64_t ob = (int64_t)crow[row] + cb;
#pragma unroll
        for (int u = 0; u < SR_U; u++)
            if (mm[u]) emit_hits<VT>(c[u], aval[base + b + u * WAVE + l], ob + ex[u], dm, jpos, Dn, ccol, cval);
    }
}


}  // namespace spref
}  // namespace hp
