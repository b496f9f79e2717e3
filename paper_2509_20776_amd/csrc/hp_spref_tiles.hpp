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
constexpr int SR_STEPS = (int)(WAVE * SR_LB / SR_BW);   // most steps of a 64-row group (32)

// The count pass leaves, for every step of SR_U slots, one 64-bit word per
// slot with the lanes that hit (a ballot), so the gather pass reads one
// uniform word per slot instead of looking every entry up again:
//   small rows: hmS[(group * SR_STEPS + step) * SR_U + slot], group = 64 rows;
//   big rows:   hmB[chunk * SR_U + slot] while the chunk count fits capb
//               (both passes test nbig <= capb the same way).
inline int64_t hit_mask_small_words(int64_t nI) { return ((nI + WAVE - 1) / WAVE) * SR_STEPS * SR_U; }
inline int64_t hit_mask_big_cap(int64_t nnzA) { return nnzA / 256 + 64; }
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

// Spread the 16 low bits of x to the even bit positions.
__device__ __forceinline__ uint32_t spread16(uint32_t x) {
    x &= 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// Two independent pieces in one tile range:
//  * link every non-winning position of a repeated column into the chain
//    headed by jpos[c]: jpos[c] = ~t_last, Dn[t] = previous head, ...,
//    ending in the winner (>= 0); chain order is arbitrary (rows are sorted
//    later);
//  * interleave the column bitmap and the repeated-column bitmap into the
//    2-bit map b2 (bit 2k: column selected, bit 2k+1: selected more than
//    once, for column 16 w + k of word w), so a lookup is one load.
__device__ inline void spref_jlink_tile(int64_t bid, const int32_t *__restrict__ J, int64_t nJ, int32_t *jpos,
                                        int32_t *Dn, const uint32_t *__restrict__ bm,
                                        const uint32_t *__restrict__ dm, uint32_t *b2, int64_t nw) {
    const int64_t t = bid * 256 + threadIdx.x;
    if (t < nJ && Dn[t] == 1) Dn[t] = atomicExch(&jpos[J[t]], ~(int32_t)t);
    if (t < 2 * nw) {
        const int sh = (int)(t & 1) * 16;
        const uint32_t m16 = bm[t >> 1] >> sh, d16 = dm[t >> 1] >> sh;
        b2[t] = spread16(m16) | (spread16(d16) << 1);
    }
}

// ---- selected rows ----------------------------------------------------------
// Doubly compressed rows: only rows jc[0..nzc) (ascending) are stored, row
// jc[k] at arow[k].  bstart indexes them by bucket: the stored rows with
// id >> shift == b are jc[bstart[b] .. bstart[b+1]).  bstart == nullptr:
// plain row pointers.
constexpr int DX_PROBE = 8;   // bucket sizes looked up without a search

// rec (optional): one 64-byte record per bucket, so that the lookup of a
// bucket of at most DX_REC stored rows is one aligned line: the bucket's
// first row pointer, the row pointers of its rows (and the end) as 32-bit
// offsets from it, their ids' low bits and their count (DX_REC_OVER: look
// the bucket up through bstart instead).
constexpr int DX_REC = 8;
constexpr uint32_t DX_REC_OVER = 0xFFu;
struct alignas(64) DcscRec {
    int64_t base;                  // row pointer of the bucket's first stored row
    uint32_t off[DX_REC + 1];      // row pointers of its stored rows and the end, minus base
    uint8_t lid[DX_REC];           // their ids minus the bucket's first id
    uint32_t cnt;                  // stored rows, or DX_REC_OVER
};
static_assert(sizeof(DcscRec) == 64, "a bucket record is one aligned 64-byte line");

struct DcscIndex {
    const int32_t *jc;
    int64_t nzc;
    const int32_t *bstart;
    int shift;
    const DcscRec *rec;
};

// sflag (optional): 1 for a selected row with 1..SR_LB entries, else 0.
// Scanned and compacted into a row list, it lets the count and gather
// passes walk only those rows in their 64-row groups, so the empty selected
// rows (most of them, for a hypersparse matrix) cost nothing after this
// pass.
template <typename PT>
__device__ inline void spref_rows_tile(int64_t bid, const PT *__restrict__ arow, const int32_t *__restrict__ I,
                                       int64_t nI, int64_t m, int64_t *rs, int32_t *rl, int32_t *ch, uint8_t *big,
                                       DevHdr *hdr, DcscIndex dx = DcscIndex{nullptr, 0, nullptr, 0, nullptr},
                                       int32_t *sflag = nullptr) {
    const int64_t i = bid * 256 + threadIdx.x;
    if (i >= nI) return;
    const int32_t r = I[i];
    int64_t s = 0, len = 0;
    if (r < 0 || r >= m) {
        atomicOr(&hdr->err, E_RANGE);   // error path only
    } else if (dx.bstart) {
        const int32_t *jc = dx.jc;
        const int64_t nzc = dx.nzc;
        const int64_t b = r >> dx.shift;
        bool done = false;
        if (dx.rec) {
            // the bucket's record: one line, no dependent load
            const uint4 *q = reinterpret_cast<const uint4 *>(dx.rec + b);
            const uint4 w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3];
            const uint32_t wd[16] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w,
                                     w2.x, w2.y, w2.z, w2.w, w3.x, w3.y, w3.z, w3.w};
            DcscRec rc;
            __builtin_memcpy(&rc, wd, sizeof(DcscRec));
            if (rc.cnt != DX_REC_OVER) {
                const uint32_t want = (uint32_t)(r - (b << dx.shift));
#pragma unroll
                for (int t = 0; t < DX_REC; t++)
                    if ((uint32_t)t < rc.cnt && rc.lid[t] == want) {
                        s = rc.base + rc.off[t];
                        len = (int64_t)rc.off[t + 1] - (int64_t)rc.off[t];
                    }
                done = true;
            }
        }
        int64_t lo = done ? 0 : dx.bstart[b], hi = done ? 0 : dx.bstart[b + 1];
        if (done) {
        } else if (hi - lo <= DX_PROBE) {
            // a bucket of at most DX_PROBE stored rows: their ids and row
            // pointers are loaded together (both follow from the bucket
            // bounds), so the lookup is two rounds of memory latency
            int32_t cj[DX_PROBE];
            PT cpv[DX_PROBE + 1];
#pragma unroll
            for (int t = 0; t < DX_PROBE; t++) cj[t] = lo + t < hi ? jc[lo + t] : -1;
#pragma unroll
            for (int t = 0; t <= DX_PROBE; t++) cpv[t] = lo + t <= hi ? arow[lo + t] : PT(0);
#pragma unroll
            for (int t = 0; t < DX_PROBE; t++)
                if (cj[t] == r) {
                    s = cpv[t];
                    len = (int64_t)cpv[t + 1] - s;
                }
        } else {
            while (lo < hi) {   // first stored row >= r in the bucket
                const int64_t mid = (lo + hi) >> 1;
                if (jc[mid] < r) lo = mid + 1;
                else hi = mid;
            }
            if (lo < nzc && jc[lo] == r) {
                s = arow[lo];
                len = arow[lo + 1] - s;
            }
        }
    } else {
        s = arow[r];
        len = arow[r + 1] - s;
    }
    rs[i] = s;
    rl[i] = (int32_t)len;
    ch[i] = len > SR_LB ? (int32_t)((len + SR_BW - 1) / SR_BW) : 0;
    big[i] = len > SR_LB ? 1 : 0;
    if (sflag) sflag[i] = (len > 0 && len <= SR_LB) ? 1 : 0;
}

// Compaction of the flagged rows: row i goes to srows[spos[i]] (spos the
// exclusive scan of sflag), so the list is in row order.
__device__ inline void spref_compact_tile(int64_t bid, const int32_t *__restrict__ sflag,
                                          const int32_t *__restrict__ spos, int64_t nI, int32_t *srows) {
    const int64_t i = bid * 256 + threadIdx.x;
    if (i < nI && sflag[i]) srows[spos[i]] = (int32_t)i;
}

// Selected row of lane l in 64-row group gw: from the short list when there
// is one (nI past its end or for an entry out of range), else gw*64 + l.
__device__ __forceinline__ int64_t group_row(int64_t gw, int l, int64_t nI, const int32_t *__restrict__ srows,
                                             int64_t nshort) {
    const int64_t k = gw * WAVE + l;
    if (!srows) return k;
    if (k >= nshort) return nI;
    const int32_t r = srows[k];
    return (uint32_t)r < (uint64_t)nI ? (int64_t)r : nI;
}

// Length of the short-row list, never above nI.
__device__ __forceinline__ int64_t list_len(const uint64_t *nshort, int64_t nI) {
    const uint64_t v = *nshort;
    return v < (uint64_t)nI ? (int64_t)v : nI;
}

// ---- shared pieces of count and gather -------------------------------------
// Length of the chain of J positions of a repeated column: jpos[c] = ~t
// links to Dn[t], ..., ending in the winning position (>= 0).
__device__ __forceinline__ int chain_len(int32_t v, const int32_t *Dn) {
    int k = 1;
    while (v < 0) {
        k++;
        v = Dn[~v];
    }
    return k;
}

// Hit multiplicities of one step of SR_U slots (columns c, valid flags ok)
// from their words bw of the 2-bit map; the chain walk only runs for
// repeated columns.
__device__ __forceinline__ void step_mult_words(const int32_t (&c)[SR_U], const bool (&ok)[SR_U],
                                                const uint32_t (&bw)[SR_U], const int32_t *__restrict__ jpos,
                                                const int32_t *__restrict__ Dn, int (&mm)[SR_U]) {
    bool dup[SR_U], any = false;
#pragma unroll
    for (int u = 0; u < SR_U; u++) {
        const uint32_t f = bw[u] >> ((c[u] & 15) << 1);
        const bool hit = ok[u] && (f & 1u);
        mm[u] = hit ? 1 : 0;
        dup[u] = hit && (f & 2u);
        any |= dup[u];
    }
    if (ballot(any)) {
#pragma unroll
        for (int u = 0; u < SR_U; u++)
            if (dup[u]) mm[u] = chain_len(jpos[c[u]], Dn);
    }
}

// The same with the words loaded here: every slot's word is loaded (one
// divergent access per slot, all issued before any is used, so the loads
// of a step overlap).
__device__ __forceinline__ void step_mult(const int32_t (&c)[SR_U], const bool (&ok)[SR_U],
                                          const uint32_t *__restrict__ b2, const int32_t *__restrict__ jpos,
                                          const int32_t *__restrict__ Dn, int (&mm)[SR_U]) {
    uint32_t bw[SR_U];
#pragma unroll
    for (int u = 0; u < SR_U; u++) bw[u] = b2[c[u] >> 4];
    step_mult_words(c, ok, bw, jpos, Dn, mm);
}

// Gather side of the hit masks: the slots' hit bits come from the count
// pass's words w[0..SR_U), so only the hits look anything up (their J
// position; a negative one heads the chain of a repeated column).
__device__ __forceinline__ void hits_lookup(const uint64_t *__restrict__ w, const int32_t (&raw)[SR_U], int64_t n,
                                            const int32_t *__restrict__ jpos, int32_t (&c)[SR_U],
                                            int32_t (&jv)[SR_U], bool (&hit)[SR_U]) {
    const int l = lane_id();
#pragma unroll
    for (int u = 0; u < SR_U; u++) {
        hit[u] = (w[u] >> l) & 1ull;
        c[u] = (int32_t)clampc(raw[u], n);
    }
#pragma unroll
    for (int u = 0; u < SR_U; u++) jv[u] = hit[u] ? jpos[c[u]] : 0;
}

// Multiplicities of the hits once their J positions jv have arrived.
__device__ __forceinline__ void hits_mult(const bool (&hit)[SR_U], const int32_t (&jv)[SR_U],
                                          const int32_t *__restrict__ Dn, int (&mm)[SR_U]) {
    bool any = false;
#pragma unroll
    for (int u = 0; u < SR_U; u++) {
        mm[u] = hit[u] ? 1 : 0;
        any |= hit[u] && jv[u] < 0;
    }
    if (ballot(any)) {
#pragma unroll
        for (int u = 0; u < SR_U; u++)
            if (hit[u] && jv[u] < 0) mm[u] = chain_len(jv[u], Dn);
    }
}

__device__ __forceinline__ void hits_from_mask(const uint64_t *__restrict__ w, const int32_t (&raw)[SR_U],
                                               int64_t n, const int32_t *__restrict__ jpos,
                                               const int32_t *__restrict__ Dn, int32_t (&c)[SR_U],
                                               int32_t (&jv)[SR_U], int (&mm)[SR_U]) {
    bool hit[SR_U];
    hits_lookup(w, raw, n, jpos, c, jv, hit);
    hits_mult(hit, jv, Dn, mm);
}

// Write the output entries of one hit whose jpos entry is x: one entry for a
// column that occurs once in J (x >= 0), the whole chain otherwise.
template <typename VT>
__device__ __forceinline__ void emit_chain(int32_t x, VT v, int64_t pos, const int32_t *__restrict__ Dn,
                                           int32_t *ccol, VT *cval) {
    while (x < 0) {
        ccol[pos] = ~x;
        cval[pos] = v;
        pos++;
        x = Dn[~x];
    }
    ccol[pos] = x;
    cval[pos] = v;
}

template <typename VT>
__device__ __forceinline__ VT stage_val(uint64_t b) {
    if constexpr (sizeof(VT) == 8) return (VT)b;
    else return (VT)(uint32_t)b;
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

// Row of chunk q (largest r with cp[r] <= q), given the row of an earlier
// chunk: the next rows are probed 64 at a time (big rows are a few percent
// of the rows, so the answer is nearly always in the first probe), with a
// full search as the fallback.
__device__ __forceinline__ int64_t next_chunk_row(const int64_t *cp, int64_t nI, int64_t row, int64_t q) {
    const int l = lane_id();
    const int64_t idx = row + 1 + l;
    const bool le = idx <= nI && cp[idx] <= q;
    const uint64_t msk = ballot(le);
    if (!(msk >> 63)) return row + 1 + (63 - __clzll((long long)msk));   // lane 0 is always set
    const int64_t lo = row + 64;
    return lo + wave_search_le(cp + lo, nI + 1 - lo, q);
}

// Contiguous chunk range of big-row wavefront gw of nwaves.
__device__ __forceinline__ void chunk_range(int64_t nbig, int64_t gw, int64_t nwaves, int64_t &q0, int64_t &q1) {
    q0 = nbig * gw / nwaves;
    q1 = nbig * (gw + 1) / nwaves;
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

// Gather staging: when the output rows must be sorted, the short rows
// (<= SMALL_MAX output entries) of a 64-row group are assembled in LDS, then
// each entry is written at its rank within its row, so no separate sort pass
// touches them.  A group whose short rows hold more than SR_STAGE entries
// writes straight to the output and is flagged for the small-row sort.
constexpr int SR_STAGE = 512;

struct GroupCore {               // per-wavefront state of a 64-row group
    int32_t start[WAVE + 1];
    int32_t cnt[WAVE];
    int64_t rs[WAVE];
    int64_t crow[WAVE];
};

// SV holds the value bits: the value type itself in the plain kernel (an
// fp32 matrix stages 4-byte values, so more wavefronts fit in LDS), 64 bits
// in the batched kernel, which serves both widths from one layout.
template <typename SV>
struct GroupSmemT : GroupCore {  // the gather adds its staging area
    int32_t soff[WAVE];                 // staging offset of a staged row, else -1
    int32_t scnt[WAVE];                 // output entries of the row
    int32_t skey[SR_STAGE];
    SV sval[SR_STAGE];
    uint8_t srow[SR_STAGE];
};
using GroupSmem = GroupSmemT<uint64_t>;

// Like emit_chain, into the group's LDS staging area (with the row index).
template <typename VT, typename G>
__device__ __forceinline__ void stage_chain(int32_t x, VT v, int idx, int row, const int32_t *__restrict__ Dn,
                                            G &g) {
    using SV = decltype(+g.sval[0]);
    while (x < 0) {
        g.skey[idx] = ~x;
        g.sval[idx] = (SV)v;
        g.srow[idx] = (uint8_t)row;
        idx++;
        x = Dn[~x];
    }
    g.skey[idx] = x;
    g.sval[idx] = (SV)v;
    g.srow[idx] = (uint8_t)row;
}

// The columns and values of A are streamed with nontemporal loads in both
// passes: they are read once per pass, and keeping them out of the caches'
// way leaves the bitmap, the J positions and the output for the passes
// that follow (the R-MAT extraction step: 0.593 -> 0.574 ms, most of it in
// the sorts that read the freshly written output).

// ---- count (plan) -------------------------------------------------------------
// Tile bid of the count pass: bid < nbw are the long-row workers (a
// contiguous range of chunks per wavefront), then one tile per 256 selected
// rows (64 rows per wavefront, walked as one concatenation).  Every step
// issues its column loads together, then its bitmap loads together.  PIPE
// (the plain kernel): each step's column loads are issued one step ahead, a
// software pipeline (R-MAT scale-22 extraction: 146 -> 142 us); the batched
// kernel, which holds the other stages' code too, keeps the plain loop (the
// pipeline took its count stage from 89 to 180 VGPRs).
template <bool PIPE = false>
__device__ inline void spref_count_tile(
    int64_t bid, int64_t nbw, GroupCore *gs, const int32_t *__restrict__ acol, int64_t n,
    const int64_t *__restrict__ rs, const int32_t *__restrict__ rl, const int64_t *__restrict__ cp, int64_t nI,
    const uint32_t *__restrict__ b2, const int32_t *__restrict__ jpos, const int32_t *__restrict__ Dn,
    int32_t *cnt, uint64_t *hmS, uint64_t *hmB, int64_t capb, const DevHdr *hdr,
    const int32_t *__restrict__ srows = nullptr, const uint64_t *nshort = nullptr) {
    if (hdr->err) return;
    const int w = threadIdx.x / WAVE, l = lane_id();
    if (bid >= nbw) {
        GroupCore &g = gs[w];
        const int64_t gw = (bid - nbw) * 4 + w;
        const int64_t ns = srows ? list_len(nshort, nI) : 0;
        if (srows && gw * WAVE >= ns) return;
        const int64_t i = group_row(gw, l, nI, srows, ns);
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
        // Software pipeline: the column loads of the next step go out after
        // this step's bitmap loads and before their words are used, so a
        // step waits on one round of loads instead of two.
        // Carried between steps: the raw columns and the slots' rows, four
        // 6-bit rows to a word.
        static_assert(SR_U % 4 == 0, "rows packed four to a word");
        uint32_t rrp[SR_U / 4];
        int32_t raw[SR_U];
        auto issue = [&](int e0) {
            int64_t k[SR_U];
#pragma unroll
            for (int u = 0; u < SR_U / 4; u++) rrp[u] = 0;
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                const int e = e0 + u * WAVE + l;
                const int ec = e < E ? e : E - 1;
                const int r = row_of(g.start, ec);
                rrp[u / 4] |= (uint32_t)r << (8 * (u % 4));
                k[u] = g.rs[r] + (ec - g.start[r]);
            }
#pragma unroll
            for (int u = 0; u < SR_U; u++) raw[u] = __builtin_nontemporal_load(&acol[k[u]]);
        };
        if (PIPE && E > 0) issue(0);
        for (int e0 = 0; e0 < E; e0 += SR_BW) {
            if (!PIPE) issue(e0);
            int32_t c[SR_U];
            int rc[SR_U], mm[SR_U];
            bool okc[SR_U];
            uint32_t bw[SR_U];
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                c[u] = (int32_t)clampc(raw[u], n);
                rc[u] = (int)((rrp[u / 4] >> (8 * (u % 4))) & 0xFFu);
                okc[u] = e0 + u * WAVE + l < E;
            }
#pragma unroll
            for (int u = 0; u < SR_U; u++) bw[u] = b2[c[u] >> 4];
            if (PIPE && e0 + SR_BW < E) issue(e0 + SR_BW);
            step_mult_words(c, okc, bw, jpos, Dn, mm);
            uint64_t hm = 0;
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                const uint64_t b = ballot(mm[u] != 0);
                if (l == u) hm = b;
            }
            if (l < SR_U) hmS[(gw * SR_STEPS + e0 / SR_BW) * SR_U + l] = hm;
#pragma unroll
            for (int u = 0; u < SR_U; u++)
                if (mm[u]) atomicAdd(&g.cnt[rc[u]], mm[u]);
        }
        __builtin_amdgcn_wave_barrier();
        if (small) cnt[i] = g.cnt[l];
        return;
    }
    // big-row chunks: every wavefront takes a contiguous range of chunks
    // (these workgroups come first); pipelined like the short rows
    const int64_t nbig = cp[nI];
    int64_t q0, q1;
    chunk_range(nbig, bid * 4 + w, nbw * 4, q0, q1);
    if (q0 >= q1) return;
    int64_t row = wave_search_le(cp, nI + 1, q0);
    int64_t rbeg = cp[row], rend = cp[row + 1], base = rs[row];
    int64_t rlen = rl[row];
    int32_t raw[SR_U];
    int nq = 0;   // entries of the chunk whose columns are in raw
    auto issue = [&](int64_t q) {
        if (q >= rend) {
            row = next_chunk_row(cp, nI, row, q);
            rbeg = cp[row];
            rend = cp[row + 1];
            base = rs[row];
            rlen = rl[row];
        }
        const int64_t b = (q - rbeg) * SR_BW;
        nq = (int)(min(b + SR_BW, rlen) - b);
        const int64_t kb = base + b;
#pragma unroll
        for (int u = 0; u < SR_U; u++) {
            const int kk = u * WAVE + l;
            raw[u] = __builtin_nontemporal_load(&acol[kb + (kk < nq ? kk : nq - 1)]);
        }
    };
    if (PIPE) issue(q0);
    for (int64_t q = q0; q < q1; q++) {
        if (!PIPE) issue(q);
        const int64_t crow_q = row;   // the row of chunk q
        const int nc = nq;
        int32_t c[SR_U];
        int mm[SR_U];
        bool okc[SR_U];
        uint32_t bw[SR_U];
#pragma unroll
        for (int u = 0; u < SR_U; u++) {
            c[u] = (int32_t)clampc(raw[u], n);
            okc[u] = u * WAVE + l < nc;
        }
#pragma unroll
        for (int u = 0; u < SR_U; u++) bw[u] = b2[c[u] >> 4];
        if (PIPE && q + 1 < q1) issue(q + 1);
        step_mult_words(c, okc, bw, jpos, Dn, mm);
        if (nbig <= capb) {
            uint64_t hm = 0;
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                const uint64_t bb = ballot(mm[u] != 0);
                if (l == u) hm = bb;
            }
            if (l < SR_U) hmB[q * SR_U + l] = hm;
        }
        int sum = 0;
#pragma unroll
        for (int u = 0; u < SR_U; u++) sum += mm[u];
        sum = wave_sum(sum);
        if (l == 0 && sum) atomicAdd(&cnt[crow_q], sum);
    }
}

// ---- gather (exec) ------------------------------------------------------------
// Within one step of SR_U slices, lane l of slice u holds entry e0+64u+l, so
// slices in order are entries in scan order.  For each slice the wavefront
// computes an exclusive scan of the hit multiplicities; a hit's position in
// its row is the row's running count plus the scan minus the scan at the
// row's first lane in the slice.  Loads go in three rounds per step: columns
// and values, bitmap words, then the J positions of the hits.
template <typename PT, typename VT, typename G>
__device__ inline void spref_gather_tile(
    int64_t bid, int64_t nbw, G *gs, const int32_t *__restrict__ acol, const VT *__restrict__ aval,
    int64_t n, const int64_t *__restrict__ rs, const int32_t *__restrict__ rl, const int64_t *__restrict__ cp,
    int64_t nI, const uint32_t *__restrict__ b2, const int32_t *__restrict__ jpos,
    const int32_t *__restrict__ Dn, const PT *__restrict__ crow,
    int32_t *ccol, VT *cval, int32_t *cursor, const uint64_t *__restrict__ hmS,
    const uint64_t *__restrict__ hmB, int64_t capb, bool sort_out, uint8_t *gflag, const DevHdr *hdr,
    const int32_t *__restrict__ srows = nullptr, const uint64_t *nshort = nullptr) {
    if (hdr->err) return;
    const int w = threadIdx.x / WAVE, l = lane_id();
    const uint64_t le_mask = (l == 63) ? ~0ull : ((2ull << l) - 1);
    if (bid >= nbw) {
        G &g = gs[w];
        const int64_t gw = (bid - nbw) * 4 + w;
        const int64_t ns = srows ? list_len(nshort, nI) : 0;
        if (srows && gw * WAVE >= ns) return;
        const int64_t i = group_row(gw, l, nI, srows, ns);
        int len = 0, nout = 0;
        if (i < nI) {
            const int L = rl[i];
            if (L <= SR_LB) {
                len = L;
                g.rs[l] = rs[i];
                const int64_t c0 = (int64_t)crow[i];
                g.crow[l] = c0;
                nout = (int)((int64_t)crow[i + 1] - c0);
            }
        }
        // rows staged in LDS (sorted output wanted, 1..SMALL_MAX entries)
        const bool st_row = sort_out && nout >= 1 && nout <= (int)SMALL_MAX;
        const int sc = st_row ? nout : 0;
        const int sincl = wave_incl_scan(sc);
        const int stot = __shfl(sincl, WAVE - 1, WAVE);
        const bool staging = stot <= SR_STAGE;
        g.soff[l] = (staging && st_row) ? sincl - sc : -1;
        g.scnt[l] = nout;
        if (sort_out && l == 0) gflag[gw] = staging ? 0 : 1;   // 1: left for the small-row sort
        const int incl = wave_incl_scan(len);
        const int E = __shfl(incl, WAVE - 1, WAVE);
        g.start[l] = incl - len;
        __builtin_amdgcn_wave_barrier();
        // Rows are contiguous in scan order, so only the row running across
        // a slice boundary needs its hit count carried: `cur` is the row of
        // the previous slice's last lane and `carry` its hits so far.
        int carry = 0, cur = INT32_MIN;
        // The slots' rows are kept four 6-bit rows to a word (82 VGPRs
        // instead of 90).  Issuing the next step's column and value loads
        // before this step's J positions are used (a software pipeline, as
        // in the count pass) needed 116 VGPRs and took the gather from 187
        // to 204 us at four wavefronts per SIMD.
        uint32_t rrp[SR_U / 4];
        int32_t raw[SR_U];
        VT v[SR_U];
        auto issue = [&](int e0) {
            int64_t k[SR_U];
#pragma unroll
            for (int u = 0; u < SR_U / 4; u++) rrp[u] = 0;
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                const int e = e0 + u * WAVE + l;
                const int ec = e < E ? e : E - 1;
                const int r = row_of(g.start, ec);
                rrp[u / 4] |= (uint32_t)r << (8 * (u % 4));
                k[u] = g.rs[r] + (ec - g.start[r]);
            }
#pragma unroll
            for (int u = 0; u < SR_U; u++) raw[u] = __builtin_nontemporal_load(&acol[k[u]]);
#pragma unroll
            for (int u = 0; u < SR_U; u++) v[u] = __builtin_nontemporal_load(&aval[k[u]]);
        };
        for (int e0 = 0; e0 < E; e0 += SR_BW) {
            issue(e0);
            int32_t c[SR_U], jv[SR_U];
            int rr[SR_U], mm[SR_U];
            bool hit[SR_U];
            VT vc[SR_U];
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                const bool ok = e0 + u * WAVE + l < E;
                const int r = (int)((rrp[u / 4] >> (8 * (u % 4))) & 0xFFu);
                rr[u] = ok ? r : -1 - l;   // distinct per idle lane: never joins a segment
                vc[u] = v[u];
            }
            const uint64_t *hw = hmS + (gw * SR_STEPS + e0 / SR_BW) * SR_U;
            hits_lookup(hw, raw, n, jpos, c, jv, hit);
            hits_mult(hit, jv, Dn, mm);
#pragma unroll
            for (int u = 0; u < SR_U; u++) {
                const int r = rr[u];
                const int ex = wave_incl_scan(mm[u]) - mm[u];
                const int prev_r = __shfl_up(r, 1, WAVE);
                const bool is_start = r != (l == 0 ? cur : prev_r);
                const uint64_t mine = ballot(is_start) & le_mask;
                const int first = mine ? 63 - __clzll((long long)mine) : 0;
                const int base_ex = __shfl(ex, first, WAVE);
                // position of the hit within its row: from the row's first
                // lane in this slice, or after the carried hits
                const int pos = mine ? ex - base_ex : carry + ex;
                if (mm[u] && pos + mm[u] <= g.scnt[r]) {   // within the planned count
                    const int so = g.soff[r];
                    if (so >= 0) stage_chain<VT>(jv[u], vc[u], so + pos, r, Dn, g);
                    else emit_chain<VT>(jv[u], vc[u], g.crow[r] + pos, Dn, ccol, cval);
                }
                carry = __builtin_amdgcn_readlane(pos + mm[u], WAVE - 1);
                cur = __builtin_amdgcn_readlane(r, WAVE - 1);
            }
        }
        if (staging && stot > 0) {
            // every staged entry goes to its rank within its row
            __builtin_amdgcn_wave_barrier();
            for (int e = l; e < stot; e += WAVE) {
                // (the masks and checks only matter if the inputs changed
                // after the plan: every write stays inside its row)
                const int r = g.srow[e] & (WAVE - 1);
                const int s0 = g.soff[r], nr = g.scnt[r];
                if (s0 < 0) continue;
                const int32_t key = g.skey[e];
                int rank = 0;
                for (int q = 0; q < nr; q++) rank += g.skey[s0 + q] < key;
                if (rank >= nr) continue;
                const int64_t o = g.crow[r] + rank;
                ccol[o] = key;
                cval[o] = stage_val<VT>(g.sval[e]);
            }
        }
        return;
    }
    // big-row chunks: positions inside the chunk in scan order, the chunk's
    // block of the row reserved with the row's cursor (workgroups come first)
    const int64_t nbig = cp[nI];
    const bool use_mask = nbig <= capb;
    int64_t q0, q1;
    chunk_range(nbig, bid * 4 + w, nbw * 4, q0, q1);
    if (q0 >= q1) return;
    int64_t row = wave_search_le(cp, nI + 1, q0);
    int64_t rbeg = cp[row], rend = cp[row + 1], base = rs[row];
    int64_t rlen = rl[row], orow = (int64_t)crow[row], oend = (int64_t)crow[row + 1];
    int32_t raw[SR_U];
    VT v[SR_U];
    int nq = 0;   // entries of the chunk whose columns and values are in raw, v
    auto issue = [&](int64_t q) {
        if (q >= rend) {
            row = next_chunk_row(cp, nI, row, q);
            rbeg = cp[row];
            rend = cp[row + 1];
            base = rs[row];
            rlen = rl[row];
            orow = (int64_t)crow[row];
            oend = (int64_t)crow[row + 1];
        }
        const int64_t b = (q - rbeg) * SR_BW;
        nq = (int)(min(b + SR_BW, rlen) - b);
        const int64_t kb = base + b;
#pragma unroll
        for (int u = 0; u < SR_U; u++) {
            const int kk = u * WAVE + l;
            const int64_t kc = kb + (kk < nq ? kk : nq - 1);
            raw[u] = __builtin_nontemporal_load(&acol[kc]);
            v[u] = __builtin_nontemporal_load(&aval[kc]);
        }
    };
    for (int64_t q = q0; q < q1; q++) {
        issue(q);
        const int64_t row_q = row, orow_q = orow, oend_q = oend;   // chunk q's row
        const int nc = nq;
        int32_t c[SR_U], jv[SR_U];
        int mm[SR_U];
        bool ok[SR_U];
        VT vc[SR_U];
#pragma unroll
        for (int u = 0; u < SR_U; u++) {
            ok[u] = u * WAVE + l < nc;
            vc[u] = v[u];
        }
        if (use_mask) {
            bool hit[SR_U];
            hits_lookup(hmB + q * SR_U, raw, n, jpos, c, jv, hit);
            hits_mult(hit, jv, Dn, mm);
        } else {
#pragma unroll
            for (int u = 0; u < SR_U; u++) c[u] = (int32_t)clampc(raw[u], n);
            step_mult(c, ok, b2, jpos, Dn, mm);
#pragma unroll
            for (int u = 0; u < SR_U; u++) jv[u] = mm[u] ? jpos[c[u]] : 0;
        }
        int run = 0;
        int ex[SR_U];
#pragma unroll
        for (int u = 0; u < SR_U; u++) {
            const int inc = wave_incl_scan(mm[u]);
            ex[u] = run + inc - mm[u];
            run += __shfl(inc, WAVE - 1, WAVE);
        }
        int32_t cb = 0;
        if (l == 0 && run) cb = atomicAdd(&cursor[row_q], run);
        cb = __shfl(cb, 0, WAVE);
        const int64_t ob = orow_q + cb;
#pragma unroll
        for (int u = 0; u < SR_U; u++)
            if (mm[u] && ob + ex[u] + mm[u] <= oend_q) emit_chain<VT>(jv[u], vc[u], ob + ex[u], Dn, ccol, cval);
    }
}


}  // namespace spref
}  // namespace hp
