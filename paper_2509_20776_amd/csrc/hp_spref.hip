// spref: C = A(I, J), C[i,j] = A[I[i], J[j]] over I x J (paper Sec. 2.2).
//
// Identify (Sec. 4.5 Step 1) on one GPU: instead of converting I and J to
// sparse vectors and binary-searching each selected column (the appendix
// algorithm for extraction), J becomes an O(1) lookup structure over A's
// columns, built without contended atomics:
//   mark  one byte per column, set for selected columns (plain stores),
//   bm    the same as a bitmap (L2 resident), packed from mark,
//   jpos  for a selected column c a position j with J[j] = c (the last
//         plain store wins), or, for a column selected several times, the
//         head ~t of a chain through Dn that visits every other position
//         and ends in the winner,
//   dm    bitmap of columns selected more than once,
//   b2    bm and dm interleaved (2 bits per column), the one table the
//         count and gather passes read per scanned entry.
// Every selected row I[i] is then streamed twice: once to count its hits
// (with multiplicity: a column selected k times yields k entries), once in
// exec to write them.  Work is split per wavefront:
//   row groups  64 consecutive selected rows of <= SR_LB entries (or 64
//               consecutive entries of the list of selected rows that have
//               entries, when most may have none); a wave-local merge path
//               assigns 8 entries per lane per step; hits are written in
//               scan order (so already sorted when J increases);
//   big rows    chunks of SR_BW entries, one wavefront each, located with a
//               cooperative 64-ary search over the chunk prefix; each chunk
//               reserves its block of the row with an atomic cursor, and big
//               rows are always sorted afterwards.
// Build (Sec. 4.2 Step 3) is the segmented sort of hp_segsort.hpp.
#include "hp_internal.hpp"
#include "hp_segsort.hpp"
#include "hp_spref_tiles.hpp"

using namespace hp;
using namespace hp::spref;

namespace {

struct SprefLayout {
    DevHdr *hdr;
    uint64_t *tiles;       // 2 scans
    uint32_t *zero;        // mark | dm | cnt | nmslots, cleared together
    uint8_t *mark;
    uint32_t *dm, *nm;
    int32_t *cnt;
    uint32_t *bm, *b2;     // column bitmap; 2-bit map (selected, repeated)
    int32_t *jpos, *Dn;
    int64_t *rs;           // start of row I[i] in A
    int32_t *rl, *ch;
    uint8_t *big;          // 1 for rows assembled by big-row chunks
    int64_t *cp;
    int32_t *cursor;       // big-row fill cursors (exec)
    uint32_t *lists;
    uint64_t *hmS, *hmB;   // hit masks of the count pass (small-row steps, big-row chunks)
    uint8_t *gflag;        // 64-row groups left unsorted by the gather
    int32_t *sflag, *spos; // DCSC: selected rows with 1..SR_LB entries (flags, scan) ...
    int32_t *srows;        // ... compacted in row order; hdr->total[3] of them
    int64_t capb;          // big-row chunks the masks can hold
    size_t nzero, nw;
};

SprefLayout spref_layout(Carve &c, int64_t n, int64_t nI, int64_t nJ, int64_t nnzA) {
    SprefLayout L;
    L.nw = (((size_t)((n + 31) / 32) + 1) + 3) & ~size_t(3);   // keeps cnt 16-byte aligned
    const size_t st = scan_tiles(nI);
    L.hdr = c.take<DevHdr>(1);
    L.tiles = c.take<uint64_t>(3 * st);
    const size_t markw = L.nw * 8;             // nw*32 bytes of marks
    L.nzero = markw + L.nw + (size_t)nI + NMSLOTS * 32 + 8;
    L.zero = c.take<uint32_t>(L.nzero);
    L.mark = (uint8_t *)L.zero;
    L.dm = L.zero ? L.zero + markw : nullptr;
    L.cnt = L.zero ? (int32_t *)(L.zero + markw + L.nw) : nullptr;
    L.nm = L.zero ? L.zero + markw + L.nw + nI + 8 : nullptr;
    L.bm = c.take<uint32_t>(L.nw);
    L.b2 = c.take<uint32_t>(2 * L.nw);
    L.jpos = c.take<int32_t>(n + 1);
    L.Dn = c.take<int32_t>(nJ + 1);
    L.rs = c.take<int64_t>(nI + 1);
    L.rl = c.take<int32_t>(nI + 1);
    L.ch = c.take<int32_t>(nI + 1);
    L.big = c.take<uint8_t>(nI + 1);
    L.cp = c.take<int64_t>(nI + 1);
    L.cursor = c.take<int32_t>(nI + 1);
    L.lists = c.take<uint32_t>(seg_list_words(nI));
    L.capb = hit_mask_big_cap(nnzA);
    L.hmS = c.take<uint64_t>((size_t)hit_mask_small_words(nI));
    L.hmB = c.take<uint64_t>((size_t)L.capb * SR_U);
    L.gflag = c.take<uint8_t>((size_t)((nI + WAVE - 1) / WAVE) + 1);
    L.sflag = c.take<int32_t>(nI + 1);
    L.spos = c.take<int32_t>(nI + 1);
    L.srows = c.take<int32_t>(nI + 1);
    return L;
}

// ---- kernels: one tile per workgroup ---------------------------------------
__global__ __launch_bounds__(256) void k_spref_jscatter(const int32_t *__restrict__ J, int64_t nJ, int64_t n,
                                                       uint8_t *mark, int32_t *jpos, uint32_t *nm, DevHdr *hdr) {
    spref_jscatter_tile(blockIdx.x, J, nJ, n, mark, jpos, nm, hdr);
}
__global__ __launch_bounds__(256) void k_spref_jpack(const int32_t *__restrict__ J, int64_t nJ, int64_t n,
                                                    const uint8_t *__restrict__ mark, uint32_t *bm, int64_t nw,
                                                    const int32_t *__restrict__ jpos, int32_t *Dn, uint32_t *dm) {
    spref_jpack_tile(blockIdx.x, J, nJ, n, mark, bm, nw, jpos, Dn, dm);
}
__global__ __launch_bounds__(256) void k_spref_jlink(const int32_t *__restrict__ J, int64_t nJ, int32_t *jpos,
                                                    int32_t *Dn, const uint32_t *__restrict__ bm,
                                                    const uint32_t *__restrict__ dm, uint32_t *b2, int64_t nw) {
    spref_jlink_tile(blockIdx.x, J, nJ, jpos, Dn, bm, dm, b2, nw);
}
template <typename PT>
__global__ __launch_bounds__(256) void k_spref_rows(const PT *__restrict__ arow, const int32_t *__restrict__ I,
                                                   int64_t nI, int64_t m, int64_t *rs, int32_t *rl, int32_t *ch,
                                                   uint8_t *big, DevHdr *hdr, DcscIndex dx, int32_t *sflag) {
    spref_rows_tile<PT>(blockIdx.x, arow, I, nI, m, rs, rl, ch, big, hdr, dx, sflag);
}
__global__ __launch_bounds__(256) void k_spref_compact(const int32_t *__restrict__ sflag,
                                                      const int32_t *__restrict__ spos, int64_t nI, int32_t *srows) {
    spref_compact_tile(blockIdx.x, sflag, spos, nI, srows);
}

// Stored rows per bucket of the doubly compressed index (ids outside
// [0, m) are skipped: the input is then malformed, never read out of bounds).
// jc is ascending, so equal buckets sit in runs of lanes: the first lane of
// each run adds the run's length (one atomic per run, not per row).
__global__ __launch_bounds__(256) void k_dcsc_buckets(const int32_t *__restrict__ jc, int64_t nzc, int64_t m,
                                                     int shift, int32_t *cnt) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int l = lane_id();
    const int32_t r = k < nzc ? jc[k] : -1;
    const bool ok = r >= 0 && r < m;
    const int64_t b = ok ? (int64_t)(r >> shift) : -1;
    const int64_t bp = __shfl_up(b, 1, WAVE);
    const bool head = ok && (l == 0 || bp != b);
    const uint64_t heads = ballot(head) | ballot(!ok);   // a run also ends before an invalid lane
    if (!head) return;
    const uint64_t after = l == WAVE - 1 ? 0ull : heads >> (l + 1);
    const int len = after ? __ffsll((long long)after) : WAVE - l;
    atomicAdd(&cnt[b], len);
}

// Bucket index of a doubly compressed matrix with m row ids and nzc stored
// rows: two to four stored rows per bucket on average, and per bucket a
// 64-byte record (DcscRec) when the bucket spans at most 256 ids, so a
// lookup is one line (buckets of more than DX_REC rows, about 1% of them at
// those averages, go through the bucket bounds and a short search); the
// index takes O(nzc) memory, never O(m).
struct DcscPlan {
    int shift = 0;
    int64_t nb = 1;
    bool rec = false;
    size_t bytes = 0;
};
DcscPlan dcsc_plan(int64_t m, int64_t nzc) {
    DcscPlan d;
    const int64_t target = std::max<int64_t>(1, nzc / 2);
    while (((m + (int64_t(1) << d.shift) - 1) >> d.shift) > target) d.shift++;
    d.nb = std::max<int64_t>(1, (m + (int64_t(1) << d.shift) - 1) >> d.shift);
    d.rec = d.shift <= 8;   // ids within a bucket fit the record's bytes
    Carve c(nullptr);
    c.take<int32_t>(d.nb + 1);
    c.take<int32_t>(d.nb + 1);
    c.take<uint64_t>(scan_tiles(d.nb));
    if (d.rec) c.take<DcscRec>(d.nb);
    d.bytes = c.size();
    return d;
}

// Record of bucket b (one thread each): its stored rows' row pointers as
// offsets from the first, their ids' low bits and their count; DX_REC_OVER
// for a bucket of more rows, offsets past 32 bits or ids outside the bucket.
template <typename PT>
__global__ __launch_bounds__(256) void k_dcsc_rec(const int32_t *__restrict__ jc, const PT *__restrict__ colptr,
                                                 const int32_t *__restrict__ bstart, int64_t nb, int shift,
                                                 DcscRec *rec) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int64_t lo = bstart[b], cnt = (int64_t)bstart[b + 1] - lo;
    const bool fits = cnt >= 0 && cnt <= DX_REC;
    // every slot loaded with a constant index (predicated), so nothing
    // lands in scratch memory
    const int64_t base = fits && cnt > 0 ? (int64_t)colptr[lo] : 0;
    uint32_t off[DX_REC + 1], lid[DX_REC];
    bool ok = fits;
#pragma unroll
    for (int t = 0; t <= DX_REC; t++) {
        const int64_t d = (fits && t <= cnt && cnt > 0) ? (int64_t)colptr[lo + t] - base : 0;
        ok &= d >= 0 && d <= (int64_t)UINT32_MAX;
        off[t] = (uint32_t)d;
    }
#pragma unroll
    for (int t = 0; t < DX_REC; t++) {
        const int64_t id = (fits && t < cnt) ? (int64_t)jc[lo + t] - (b << shift) : 0;
        ok &= id >= 0 && id < 256;
        lid[t] = (uint32_t)id & 0xffu;
    }
    // the record's 16 words: base (2), off[0..8] (9), lid packed four to a
    // word (2), cnt (1), two unused (the layout of DcscRec)
    static_assert(offsetof(DcscRec, off) == 8 && offsetof(DcscRec, lid) == 44 && offsetof(DcscRec, cnt) == 52,
                  "record layout");
    const uint32_t l0 = lid[0] | (lid[1] << 8) | (lid[2] << 16) | (lid[3] << 24);
    const uint32_t l1 = lid[4] | (lid[5] << 8) | (lid[6] << 16) | (lid[7] << 24);
    const uint32_t c = ok ? (uint32_t)cnt : DX_REC_OVER;
    uint4 *q = reinterpret_cast<uint4 *>(rec + b);
    q[0] = make_uint4((uint32_t)base, (uint32_t)((uint64_t)base >> 32), off[0], off[1]);
    q[1] = make_uint4(off[2], off[3], off[4], off[5]);
    q[2] = make_uint4(off[6], off[7], off[8], l0);
    q[3] = make_uint4(l1, c, 0u, 0u);
}__global__ __launch_bounds__(SR_BLOCK) void k_spref_count(
    const int32_t *__restrict__ acol, int64_t n, const int64_t *__restrict__ rs,
    const int32_t *__restrict__ rl, const int64_t *__restrict__ cp, int64_t nI, int64_t ngb,
    const uint32_t *__restrict__ b2, const int32_t *__restrict__ jpos, const int32_t *__restrict__ Dn,
    int32_t *cnt, uint64_t *hmS, uint64_t *hmB, int64_t capb, const DevHdr *hdr, const int32_t *srows,
    const uint64_t *nshort) {
    __shared__ GroupCore gs[SR_BLOCK / WAVE];
    (void)ngb;
    spref_count_tile<true>(blockIdx.x, SR_BIGBLOCKS, gs, acol, n, rs, rl, cp, nI, b2, jpos, Dn, cnt, hmS, hmB, capb,
                           hdr, srows, nshort);
}
// Five wavefronts per SIMD (at most 96 VGPRs; the fp32 staging area keeps
// five workgroups in LDS): the gather is bound by the latency of its
// dependent loads, and 4 -> 5 wavefronts took it from 218 to 195 us on the
// R-MAT scale-22 extraction.  The count pass gained nothing from 6 -> 8.
template <typename PT, typename VT>
__global__ __launch_bounds__(SR_BLOCK) __attribute__((amdgpu_waves_per_eu(5))) void k_spref_gather(
    const int32_t *__restrict__ acol, const VT *__restrict__ aval, int64_t n,
    const int64_t *__restrict__ rs, const int32_t *__restrict__ rl, const int64_t *__restrict__ cp,
    int64_t nI, int64_t ngb, const uint32_t *__restrict__ b2, const int32_t *__restrict__ jpos,
    const int32_t *__restrict__ Dn, const PT *__restrict__ crow, int32_t *ccol, VT *cval, int32_t *cursor,
    const uint64_t *__restrict__ hmS, const uint64_t *__restrict__ hmB, int64_t capb, int sort_out,
    uint8_t *gflag, const DevHdr *hdr, const int32_t *srows, const uint64_t *nshort) {
    __shared__ GroupSmemT<VT> gs[SR_BLOCK / WAVE];
    (void)ngb;
    spref_gather_tile<PT, VT>(blockIdx.x, SR_BIGBLOCKS, gs, acol, aval, n, rs, rl, cp, nI, b2, jpos, Dn, crow,
                              ccol, cval, cursor, hmS, hmB, capb, sort_out != 0, gflag, hdr, srows, nshort);
}

hp_status_t spref_check_args(hp_handle_t h, const hp_csr_t *A, const int32_t *I, int64_t nI,
                             const int32_t *J, int64_t nJ, const hp_csr_t *C) {
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    if (!C) return fail(h, HP_ERR_INVALID_ARG, "C is NULL");
    if (nI < 0 || nJ < 0) return fail(h, HP_ERR_INVALID_ARG, "negative index-vector length");
    if (nI > INT32_MAX || nJ > INT32_MAX) return fail(h, HP_ERR_INVALID_ARG, "index vector too long");
    if ((nI > 0 && !I) || (nJ > 0 && !J)) return fail(h, HP_ERR_INVALID_ARG, "I or J is NULL");
    if (C->nrows != nI || C->ncols != nJ) return fail(h, HP_ERR_SHAPE, "C must be |I| x |J|");
    if (C->ptr_type != A->ptr_type || C->val_type != A->val_type)
        return fail(h, HP_ERR_INVALID_ARG, "C must have A's ptr_type and val_type");
    if (!C->rowptr) return fail(h, HP_ERR_INVALID_ARG, "C->rowptr is NULL");
    return HP_OK;
}

inline int grid1(int64_t n) { return (int)std::max<int64_t>(1, (n + 255) / 256); }

// dcsc: A's rows are doubly compressed (only the nzc rows jc[k] stored, the
// row pointers then have nzc+1 entries; the bucket index follows the
// extraction's workspace).
template <typename PT>
hp_status_t spref_plan_t(hp_handle_t h, const hp_csr_t *A, const int32_t *I, int64_t nI,
                         const int32_t *J, int64_t nJ, hp_csr_t *C, void *ws, size_t ws_bytes,
                         hp_plan_info_t *info, bool dcsc = false, const int32_t *jc = nullptr, int64_t nzc = 0) {
    const int64_t m = A->nrows, n = A->ncols;
    const int64_t nptr = dcsc ? nzc + 1 : m + 1;
    // List the selected rows that have entries when most may have none (a
    // DCSC matrix, or fewer stored entries than rows), so that count and
    // gather skip the rest; elsewhere the scan and compaction would cost more
    // than the empty rows.
    const bool listed = dcsc || A->nnz < m;
    Carve need(nullptr);
    spref_layout(need, n, nI, nJ, A->nnz);
    const size_t base = need.size();
    const DcscPlan dp = dcsc ? dcsc_plan(m, nzc) : DcscPlan{};
    if (!ws || ws_bytes < base + dp.bytes) return fail(h, HP_ERR_WORKSPACE, "spref plan workspace too small");
    const size_t ps = sizeof(PT), vs = val_size(A->val_type);
    const void *ins[] = {A->rowptr, A->col, A->val, I, J, jc};
    const size_t insz[] = {(size_t)nptr * ps, (size_t)A->nnz * 4, (size_t)A->nnz * vs,
                           (size_t)nI * 4, (size_t)nJ * 4, jc ? (size_t)nzc * 4 : 0};
    for (int k = 0; k < 6; k++)
        if (overlaps(C->rowptr, (nI + 1) * ps, ins[k], insz[k]) || overlaps(ws, ws_bytes, ins[k], insz[k]))
            return fail(h, HP_ERR_ALIAS, "output or workspace overlaps an input");
    if (overlaps(C->rowptr, (nI + 1) * ps, ws, ws_bytes))
        return fail(h, HP_ERR_ALIAS, "C->rowptr overlaps the workspace");
    Carve c(ws);
    SprefLayout L = spref_layout(c, n, nI, nJ, A->nnz);
    const size_t st = scan_tiles(nI);
    hipStream_t s = h->stream;
    if (!dcsc)
        if (hp_status_t v = validate_input(h, A, L.hdr, "spref plan: A")) return v;
    stage_begin(h);
    hipError_t e = launch_init_hdr(s, L.hdr, L.tiles, 3 * st);
    if (e == hipSuccess) e = launch_clear_words(s, L.zero, L.nzero);
    DcscIndex dx{nullptr, 0, nullptr, 0, nullptr};
    if (dcsc && e == hipSuccess) {
        Carve cx((char *)ws + base);
        int32_t *bcnt = cx.take<int32_t>(dp.nb + 1);
        int32_t *bstart = cx.take<int32_t>(dp.nb + 1);
        uint64_t *btiles = cx.take<uint64_t>(scan_tiles(dp.nb));
        e = launch_clear_words(s, bcnt, (size_t)dp.nb + 1);
        if (e == hipSuccess) e = launch_clear_words(s, btiles, scan_tiles(dp.nb) * 2);
        if (e == hipSuccess && nzc > 0)
            hipLaunchKernelGGL(k_dcsc_buckets, dim3(grid1(nzc)), dim3(256), 0, s, jc, nzc, m, dp.shift, bcnt);
        if (e == hipSuccess)
            e = launch_scan_counts<int32_t>(s, bcnt, bstart, dp.nb, L.hdr, 2, btiles, 0, nullptr, 0);
        DcscRec *rec = nullptr;
        if (e == hipSuccess && dp.rec) {
            rec = cx.take<DcscRec>(dp.nb);
            hipLaunchKernelGGL(k_dcsc_rec<PT>, dim3(grid1(dp.nb)), dim3(256), 0, s, jc, (const PT *)A->rowptr, bstart,
                               dp.nb, dp.shift, rec);
            e = hipGetLastError();
        }
        dx = DcscIndex{jc, nzc, bstart, dp.shift, rec};
    }
    stage_mark(h, "spref.init");
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_spref_jscatter, dim3(grid1(nJ)), dim3(256), 0, s, J, nJ, n, L.mark, L.jpos,
                           L.nm, L.hdr);
        hipLaunchKernelGGL(k_spref_jpack, dim3(grid1(std::max<int64_t>(nJ, (int64_t)L.nw))), dim3(256), 0,
                           s, J, nJ, n, L.mark, L.bm, (int64_t)L.nw, L.jpos, L.Dn, L.dm);
        hipLaunchKernelGGL(k_spref_jlink, dim3(grid1(std::max<int64_t>(nJ, 2 * (int64_t)L.nw))), dim3(256), 0, s, J,
                           nJ, L.jpos, L.Dn, L.bm, L.dm, L.b2, (int64_t)L.nw);
        stage_mark(h, "spref.jtables");
        hipLaunchKernelGGL(k_spref_rows<PT>, dim3(grid1(nI)), dim3(256), 0, s, (const PT *)A->rowptr, I,
                           nI, m, L.rs, L.rl, L.ch, L.big, L.hdr, dx, listed ? L.sflag : nullptr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_scan_counts<int64_t>(s, L.ch, L.cp, nI, L.hdr, 0, L.tiles, 0, nullptr, 0);
    // the short-row list (scan slots: 0 chunks, 1 counts, 2 the DCSC bucket
    // index, 3 this list)
    const int32_t *srows = listed ? L.srows : nullptr;
    const uint64_t *d_nshort = &L.hdr->total[3];
    if (listed && e == hipSuccess) {
        e = launch_scan_counts<int32_t>(s, L.sflag, L.spos, nI, L.hdr, 3, L.tiles + 2 * st, 0, nullptr, 0);
        if (e == hipSuccess && nI > 0)
            hipLaunchKernelGGL(k_spref_compact, dim3(grid1(nI)), dim3(256), 0, s, (const int32_t *)L.sflag,
                               (const int32_t *)L.spos, nI, L.srows);
    }
    stage_mark(h, "spref.rows");
    const int64_t ngb = (nI + 4 * WAVE - 1) / (4 * WAVE);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_spref_count, dim3((unsigned)(ngb + SR_BIGBLOCKS)), dim3(SR_BLOCK), 0, s, A->col,
                           n, L.rs, L.rl, L.cp, nI, ngb, L.b2, L.jpos, L.Dn, L.cnt, L.hmS, L.hmB, L.capb,
                           L.hdr, srows, d_nshort);
        stage_mark(h, "spref.count");
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        e = launch_scan_counts<PT>(s, L.cnt, (PT *)C->rowptr, nI, L.hdr, 1, L.tiles + st, 3, L.lists, nI,
                                   L.big, L.nm);
        stage_mark(h, "spref.scan");
    }
    if (e != hipSuccess) return hip_check(h, e, "spref plan");
    if (hp_status_t rb = readback_hdr(h, L.hdr, "spref plan")) return rb;
    stage_end(h);
    const DevHdr &H = *h->host_hdr;
    hp_status_t stt = status_from_err(h, H.err, "spref");
    if (stt) return stt;
    C->nnz = (int64_t)H.total[1];
    if (info) {
        *info = hp_plan_info_t{};
        info->nnz_out = C->nnz;
        info->map_monotone = (H.flags & F_NOT_MONOTONE) ? 0 : 1;
        info->op = 2;
        for (int b = 0; b < NBINS; b++) {
            info->rows_sorted[b] = H.bin_cnt[b];
            info->class_elems[b] = (int64_t)H.bin_elems[b];
        }
        info->aux[1] = (int64_t)H.total[0];   // big-row chunks
        info->aux[2] = listed ? (int64_t)H.total[3] : -1;   // listed short rows, or no list
        info->exec_ws_bytes = seg_tmp_bytes(H.bin_elems[BIN_GLOBAL], H.bin_cnt[BIN_GLOBAL], vs, nJ);
    }
    return HP_OK;
}

template <typename PT, typename VT>
hp_status_t spref_exec_t(hp_handle_t h, const hp_csr_t *A, const int32_t *I, int64_t nI,
                         const int32_t *J, int64_t nJ, hp_csr_t *C, void *ws, size_t ws_bytes,
                         const hp_plan_info_t *info, void *xws, size_t xws_bytes, int64_t nptr = -1) {
    const int64_t m = A->nrows, n = A->ncols;
    if (nptr < 0) nptr = m + 1;
    Carve need(nullptr);
    spref_layout(need, n, nI, nJ, A->nnz);
    if (!ws || ws_bytes < need.size()) return fail(h, HP_ERR_WORKSPACE, "spref workspace too small");
    if (!info || info->op != 2) return fail(h, HP_ERR_INVALID_ARG, "info is not from hp_spref_plan");
    if (xws_bytes < info->exec_ws_bytes || (info->exec_ws_bytes && !xws))
        return fail(h, HP_ERR_WORKSPACE, "spref exec workspace too small");
    if (C->nnz != info->nnz_out) return fail(h, HP_ERR_INVALID_ARG, "C->nnz differs from the plan");
    if (C->nnz > 0 && (!C->col || !C->val)) return fail(h, HP_ERR_INVALID_ARG, "C->col/val is NULL");
    const size_t vs = sizeof(VT);
    const void *ins[] = {A->rowptr, A->col, A->val, I, J, ws, xws, C->rowptr};
    const size_t insz[] = {(size_t)nptr * sizeof(PT), (size_t)A->nnz * 4, (size_t)A->nnz * vs,
                           (size_t)nI * 4, (size_t)nJ * 4, ws_bytes, xws_bytes,
                           (size_t)(nI + 1) * sizeof(PT)};
    for (int k = 0; k < 8; k++)
        if (overlaps(C->col, (size_t)C->nnz * 4, ins[k], insz[k]) ||
            overlaps(C->val, (size_t)C->nnz * vs, ins[k], insz[k]))
            return fail(h, HP_ERR_ALIAS, "C->col/val overlaps an input or workspace");
    Carve c(ws);
    SprefLayout L = spref_layout(c, n, nI, nJ, A->nnz);
    hipStream_t s = h->stream;
    // workgroups of four 64-row groups: over the plan's short-row list when
    // it made one, else over all selected rows
    const bool listed = info->aux[2] >= 0;
    const int64_t nshort = listed ? std::min<int64_t>(info->aux[2], nI) : nI;
    const int64_t ngs = (nshort + 4 * WAVE - 1) / (4 * WAVE);
    const int32_t *srows = listed ? L.srows : nullptr;
    const uint64_t *d_nshort = &L.hdr->total[3];
    hipError_t e = hipSuccess;
    if (info->aux[1] > 0) e = launch_clear_words(s, L.cursor, (size_t)nI);
    stage_begin(h);   // the gather stage is the gather kernel alone
    if (e == hipSuccess && info->nnz_out > 0) {
        hipLaunchKernelGGL((k_spref_gather<PT, VT>), dim3((unsigned)(ngs + SR_BIGBLOCKS)), dim3(SR_BLOCK), 0,
                           s, A->col, (const VT *)A->val, n, L.rs, L.rl, L.cp, nI, ngs, L.b2, L.jpos,
                           L.Dn, (const PT *)C->rowptr, C->col, (VT *)C->val, L.cursor, L.hmS, L.hmB, L.capb,
                           info->map_monotone ? 0 : 1, L.gflag, L.hdr, srows, d_nshort);
        stage_mark(h, "spref.gather");
        e = hipGetLastError();
    }
    if (e == hipSuccess && info->nnz_out > 0) {
        uint32_t cnt[NBINS];
        for (int b = 0; b < NBINS; b++) cnt[b] = (uint32_t)info->rows_sorted[b];
        LoadInPlace<PT, VT> ld{(const PT *)C->rowptr, C->col, (const VT *)C->val};
        if (!info->map_monotone && ngs > 0)
            hipLaunchKernelGGL((k_sort_small<PT, VT, LoadInPlace<PT, VT>>), dim3((unsigned)ngs), dim3(256), 0,
                               s, (const PT *)C->rowptr, C->col, (VT *)C->val, nI, ld, L.hdr,
                               (const uint8_t *)L.gflag, (const uint8_t *)L.big, srows, d_nshort);
        e = launch_seg_classes<PT, VT, LoadInPlace<PT, VT>>(
            s, (const PT *)C->rowptr, C->col, (VT *)C->val, L.lists, nI, cnt, ld, false, nJ, true, xws,
            (uint64_t)info->class_elems[BIN_GLOBAL], L.hdr, true);
        stage_mark(h, "spref.sort");
    }
    stage_end(h);
    return hip_check(h, e == hipSuccess ? hipGetLastError() : e, "spref exec");
}

}  // namespace

extern "C" hp_status_t hp_spref_workspace(hp_handle_t h, const hp_csr_t *A, int64_t nI, int64_t nJ,
                                          size_t *bytes) {
    if (!h || !bytes) return HP_ERR_INVALID_ARG;
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    if (nI < 0 || nJ < 0) return fail(h, HP_ERR_INVALID_ARG, "negative index-vector length");
    Carve c(nullptr);
    spref_layout(c, A->ncols, nI, nJ, A->nnz);
    *bytes = c.size();
    return HP_OK;
}

extern "C" hp_status_t hp_spref_plan(hp_handle_t h, const hp_csr_t *A, const int32_t *I, int64_t nI,
                                     const int32_t *J, int64_t nJ, hp_csr_t *C, void *ws,
                                     size_t ws_bytes, hp_plan_info_t *info) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = spref_check_args(h, A, I, nI, J, nJ, C);
    if (st) return st;
    if (A->ptr_type == HP_IDX_I32) return spref_plan_t<int32_t>(h, A, I, nI, J, nJ, C, ws, ws_bytes, info);
    return spref_plan_t<int64_t>(h, A, I, nI, J, nJ, C, ws, ws_bytes, info);
}

extern "C" hp_status_t hp_spref_exec(hp_handle_t h, const hp_csr_t *A, const int32_t *I, int64_t nI,
                                     const int32_t *J, int64_t nJ, hp_csr_t *C, void *ws,
                                     size_t ws_bytes, const hp_plan_info_t *info, void *xws,
                                     size_t xws_bytes) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = spref_check_args(h, A, I, nI, J, nJ, C);
    if (st) return st;
    const bool p64 = A->ptr_type == HP_IDX_I64, v64 = A->val_type == HP_VAL_F64;
    if (!p64 && !v64)
        return spref_exec_t<int32_t, uint32_t>(h, A, I, nI, J, nJ, C, ws, ws_bytes, info, xws, xws_bytes);
    if (!p64 && v64)
        return spref_exec_t<int32_t, uint64_t>(h, A, I, nI, J, nJ, C, ws, ws_bytes, info, xws, xws_bytes);
    if (p64 && !v64)
        return spref_exec_t<int64_t, uint32_t>(h, A, I, nI, J, nJ, C, ws, ws_bytes, info, xws, xws_bytes);
    return spref_exec_t<int64_t, uint64_t>(h, A, I, nI, J, nJ, C, ws, ws_bytes, info, xws, xws_bytes);
}

// ---- column-compressed input ----------------------------------------------
// A(I, J) on CSC/DCSC is the row extraction of the transpose: the column
// pointers and row indices of A are the row pointers and columns of A^T,
// C^T = A^T(J, I), and the CSR of C^T is the CSC of C.
namespace {
hp_csr_t transpose_view(const hp_dcsc_t *A) {
    hp_csr_t T;
    T.nrows = A->ncols;
    T.ncols = A->nrows;
    T.nnz = A->nnz;
    T.ptr_type = A->ptr_type;
    T.val_type = A->val_type;
    T.rowptr = A->colptr;
    T.col = A->row;
    T.val = A->val;
    return T;
}

hp_status_t dcsc_check(hp_handle_t h, const hp_dcsc_t *A, const hp_dcsc_t *C) {
    if (!A) return fail(h, HP_ERR_INVALID_ARG, "A is NULL");
    if (A->dcsc != 0 && A->dcsc != 1) return fail(h, HP_ERR_INVALID_ARG, "A: dcsc must be 0 or 1");
    if (A->dcsc && (A->nzc < 0 || A->nzc > A->ncols)) return fail(h, HP_ERR_INVALID_ARG, "A: nzc outside [0, ncols]");
    if (A->dcsc && A->nzc > 0 && !A->jc) return fail(h, HP_ERR_INVALID_ARG, "A: jc is NULL");
    if (!A->colptr) return fail(h, HP_ERR_INVALID_ARG, "A: colptr is NULL");
    if (C && C->dcsc) return fail(h, HP_ERR_INVALID_ARG, "C is returned in CSC: C->dcsc must be 0");
    return HP_OK;
}
}  // namespace

extern "C" hp_status_t hp_spref_dcsc_workspace(hp_handle_t h, const hp_dcsc_t *A, int64_t nI, int64_t nJ,
                                               size_t *bytes) {
    if (!h || !bytes) return HP_ERR_INVALID_ARG;
    hp_status_t st = dcsc_check(h, A, nullptr);
    if (st) return st;
    const hp_csr_t T = transpose_view(A);
    st = hp_spref_workspace(h, &T, nJ, nI, bytes);
    if (st == HP_OK && A->dcsc) *bytes += dcsc_plan(T.nrows, A->nzc).bytes;
    return st;
}

extern "C" hp_status_t hp_spref_dcsc_plan(hp_handle_t h, const hp_dcsc_t *A, const int32_t *I, int64_t nI,
                                          const int32_t *J, int64_t nJ, hp_dcsc_t *C, void *ws, size_t ws_bytes,
                                          hp_plan_info_t *info) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = dcsc_check(h, A, C);
    if (st) return st;
    if (!C) return fail(h, HP_ERR_INVALID_ARG, "C is NULL");
    const hp_csr_t T = transpose_view(A);
    hp_csr_t CT = transpose_view(C);
    st = spref_check_args(h, &T, J, nJ, I, nI, &CT);
    if (st) return st;
    const bool dc = A->dcsc != 0;
    st = T.ptr_type == HP_IDX_I32
             ? spref_plan_t<int32_t>(h, &T, J, nJ, I, nI, &CT, ws, ws_bytes, info, dc, A->jc, A->nzc)
             : spref_plan_t<int64_t>(h, &T, J, nJ, I, nI, &CT, ws, ws_bytes, info, dc, A->jc, A->nzc);
    if (st == HP_OK) C->nnz = CT.nnz;
    return st;
}

extern "C" hp_status_t hp_spref_dcsc_exec(hp_handle_t h, const hp_dcsc_t *A, const int32_t *I, int64_t nI,
                                          const int32_t *J, int64_t nJ, hp_dcsc_t *C, void *ws, size_t ws_bytes,
                                          const hp_plan_info_t *info, void *xws, size_t xws_bytes) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = dcsc_check(h, A, C);
    if (st) return st;
    if (!C) return fail(h, HP_ERR_INVALID_ARG, "C is NULL");
    const hp_csr_t T = transpose_view(A);
    hp_csr_t CT = transpose_view(C);
    st = spref_check_args(h, &T, J, nJ, I, nI, &CT);
    if (st) return st;
    const int64_t nptr = A->dcsc ? A->nzc + 1 : A->ncols + 1;
    const bool p64 = T.ptr_type == HP_IDX_I64, v64 = T.val_type == HP_VAL_F64;
    if (!p64 && !v64)
        return spref_exec_t<int32_t, uint32_t>(h, &T, J, nJ, I, nI, &CT, ws, ws_bytes, info, xws, xws_bytes, nptr);
    if (!p64 && v64)
        return spref_exec_t<int32_t, uint64_t>(h, &T, J, nJ, I, nI, &CT, ws, ws_bytes, info, xws, xws_bytes, nptr);
    if (p64 && !v64)
        return spref_exec_t<int64_t, uint32_t>(h, &T, J, nJ, I, nI, &CT, ws, ws_bytes, info, xws, xws_bytes, nptr);
    return spref_exec_t<int64_t, uint64_t>(h, &T, J, nJ, I, nI, &CT, ws, ws_bytes, info, xws, xws_bytes, nptr);
}
