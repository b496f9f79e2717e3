// spref: C = A(I, J), C[i,j] = A[I[i], J[j]] over I x J (paper Sec. 2.2).
//
// Identify (Sec. 4.5 Step 1) on one GPU: instead of converting I and J to
// sparse vectors and binary-searching each selected column (the appendix
// algorithm for extraction), J becomes an O(1) lookup structure:
//   bm    membership bitmap over A's columns (L2 resident),
//   dm    "column selected more than once" bitmap,
//   jpos  for a selected column c: a position j with J[j] = c, or, for a
//         repeated column, the head (~t) of a chain through the repeat
//         records (Dj, Dn) ending in the first position.
// Every selected row I[i] is streamed once to count its hits (with
// multiplicity: a column selected k times yields k entries), and once more
// in exec to write them.  Rows are processed in two ways:
//   small rows (<= SR_LB entries) in row chunks: all rows whose merge-path
//     start i + sps[i] falls in [w*SR_D, (w+1)*SR_D); rows never split, so
//     entries land in scan order (already sorted when J is increasing);
//   big rows in fixed chunks of SR_BD entries spread over workgroups; each
//     chunk reserves its block of the row with an atomic cursor, and big
//     rows are always sorted afterwards (deterministic final order).
// Build (Sec. 4.2 Step 3) is the segmented sort of hp_segsort.hpp.
#include "hp_internal.hpp"
#include "hp_segsort.hpp"

using namespace hp;

namespace {

constexpr int SR_BLOCK = 256;
constexpr int64_t SR_D = 1024;    // merge-path items (rows + entries) per small chunk
constexpr int64_t SR_LB = 1024;   // rows above this many entries are big
constexpr int64_t SR_BD = 4096;   // entries per big-row chunk
constexpr int SR_GRID = 2048;     // persistent workgroups for count and gather

struct SprefLayout {
    DevHdr *hdr;
    uint64_t *tiles;       // 3 scans
    uint32_t *zero;        // bm | dm | cnt, cleared together
    uint32_t *bm, *dm;
    int32_t *cnt;
    int32_t *jpos;
    int32_t *Dc, *Dj, *Dn; // repeat records
    int64_t *rs;           // start of row I[i] in A
    int32_t *rl, *rls, *ch;
    int64_t *sps, *cp;
    int32_t *cursor;       // big-row fill cursors (exec)
    uint32_t *lists;
    size_t nzero;
};

SprefLayout spref_layout(Carve &c, int64_t n, int64_t nI, int64_t nJ) {
    SprefLayout L;
    const size_t nw = (size_t)((n + 31) / 32) + 1;
    const size_t st = scan_tiles(nI);
    L.hdr = c.take<DevHdr>(1);
    L.tiles = c.take<uint64_t>(3 * st);
    L.nzero = 2 * nw + (size_t)nI;
    L.zero = c.take<uint32_t>(L.nzero);
    L.bm = L.zero;
    L.dm = L.zero ? L.zero + nw : nullptr;
    L.cnt = L.zero ? (int32_t *)(L.zero + 2 * nw) : nullptr;
    L.jpos = c.take<int32_t>(n + 1);
    L.Dc = c.take<int32_t>(nJ + 1);
    L.Dj = c.take<int32_t>(nJ + 1);
    L.Dn = c.take<int32_t>(nJ + 1);
    L.rs = c.take<int64_t>(nI + 1);
    L.rl = c.take<int32_t>(nI + 1);
    L.rls = c.take<int32_t>(nI + 1);
    L.ch = c.take<int32_t>(nI + 1);
    L.sps = c.take<int64_t>(nI + 1);
    L.cp = c.take<int64_t>(nI + 1);
    L.cursor = c.take<int32_t>(nI + 1);
    L.lists = c.take<uint32_t>(seg_list_words(nI));
    return L;
}

// ---- J tables -------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spref_jbuild(const int32_t *__restrict__ J, int64_t nJ,
                                                     int64_t n, uint32_t *bm, uint32_t *dm,
                                                     int32_t *jpos, int32_t *Dc, int32_t *Dj,
                                                     DevHdr *hdr) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool notmono = false;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nJ; j += stride) {
        const int32_t c = J[j];
        if (j + 1 < nJ && c >= J[j + 1]) notmono = true;
        if (c < 0 || c >= n) {
            atomicOr(&hdr->err, E_RANGE);
            continue;
        }
        const uint32_t bit = 1u << (c & 31);
        const uint32_t old = atomicOr(&bm[c >> 5], bit);
        if (old & bit) {
            // a later occurrence of column c: record it for the chain
            atomicOr(&dm[c >> 5], bit);
            uint32_t t = atomicAdd(&hdr->ndup, 1u);
            Dc[t] = c;
            Dj[t] = (int32_t)j;
        } else {
            jpos[c] = (int32_t)j;     // the single first occurrence
        }
    }
    uint64_t b = ballot(notmono);
    if (b && lane_id() == __ffsll((long long)b) - 1) atomicOr(&hdr->flags, F_NOT_MONOTONE);
}

// Link the repeat records of each column into a chain headed by jpos[c]:
// jpos[c] = ~t_last, Dn[t] = previous head, ..., the last link holds the
// first occurrence (>= 0).  Chain order is arbitrary; rows are sorted later.
__global__ __launch_bounds__(256) void k_spref_jlink(int32_t *jpos, const int32_t *__restrict__ Dc,
                                                    int32_t *Dn, const DevHdr *hdr) {
    const uint32_t nd = hdr->ndup;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nd; t += gridDim.x * blockDim.x)
        Dn[t] = atomicExch(&jpos[Dc[t]], ~(int32_t)t);
}

// ---- selected rows --------------------------------------------------------
template <typename PT>
__global__ __launch_bounds__(256) void k_spref_rows(const PT *__restrict__ arow,
                                                   const int32_t *__restrict__ I, int64_t nI,
                                                   int64_t m, int64_t *rs, int32_t *rl, int32_t *rls,
                                                   int32_t *ch, DevHdr *hdr) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nI; i += stride) {
        const int32_t r = I[i];
        int64_t s = 0, len = 0;
        if (r < 0 || r >= m) atomicOr(&hdr->err, E_RANGE);
        else {
            s = arow[r];
            len = arow[r + 1] - s;
        }
        rs[i] = s;
        rl[i] = (int32_t)len;
        const bool big = len > SR_LB;
        rls[i] = big ? 0 : (int32_t)len;
        ch[i] = big ? (int32_t)((len + SR_BD - 1) / SR_BD) : 0;
    }
}

// ---- shared pieces of count and gather -------------------------------------
__device__ __forceinline__ bool test_bit(const uint32_t *bm, int64_t c) {
    return (bm[c >> 5] >> (c & 31)) & 1u;
}

// Number of output entries a hit on column c produces (its multiplicity in J).
__device__ __forceinline__ int mult_of(int64_t c, const uint32_t *dm, const int32_t *jpos,
                                       const int32_t *Dn) {
    if (!test_bit(dm, c)) return 1;
    int m = 1;
    int32_t v = jpos[c];
    while (v < 0) {
        m++;
        v = Dn[~v];
    }
    return m;
}

// Smallest i in [0, nI] with i + sps[i] >= d.
__device__ __forceinline__ int64_t diag_lb(const int64_t *sps, int64_t nI, int64_t d) {
    int64_t lo = 0, hi = nI;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (mid + sps[mid] < d) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Largest i in [0, n) with a[i] <= x (a nondecreasing, a[0] <= x).
template <typename T>
__device__ __forceinline__ int64_t last_le(const T *a, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct ChunkSmem {
    int64_t sps[SR_D + 2];
    int64_t rs[SR_D + 1];
    int32_t cnt[SR_D + 1];
    int32_t scan[2 * SR_LB + 8];
    int64_t misc[8];
    int32_t red[8];
};

// Load the rows of small chunk w into shared memory; returns the row count.
__device__ __forceinline__ int64_t load_small_chunk(ChunkSmem &sm, int64_t w, const int64_t *sps,
                                                    const int64_t *rs, int64_t nI, int64_t &i0) {
    if (threadIdx.x == 0) {
        sm.misc[0] = diag_lb(sps, nI, w * SR_D);
        sm.misc[1] = diag_lb(sps, nI, (w + 1) * SR_D);
    }
    __syncthreads();
    i0 = sm.misc[0];
    const int64_t nr = sm.misc[1] - i0;
    for (int64_t r = threadIdx.x; r <= nr; r += SR_BLOCK) {
        sm.sps[r] = sps[i0 + r];
        if (r < nr) {
            sm.rs[r] = rs[i0 + r];
            sm.cnt[r] = 0;
        }
    }
    __syncthreads();
    return nr;
}

// ---- count (plan) -----------------------------------------------------------
__global__ __launch_bounds__(SR_BLOCK) void k_spref_count(
    const int32_t *__restrict__ acol, int64_t n, const int64_t *__restrict__ rs,
    const int32_t *__restrict__ rl, const int64_t *__restrict__ sps, const int64_t *__restrict__ cp,
    int64_t nI, const uint32_t *__restrict__ bm, const uint32_t *__restrict__ dm,
    const int32_t *__restrict__ jpos, const int32_t *__restrict__ Dn, int32_t *cnt,
    const DevHdr *hdr) {
    __shared__ ChunkSmem sm;
    if (hdr->err) return;
    const int64_t S = sps[nI];
    const int64_t nsmall = (nI + S + SR_D - 1) / SR_D;
    const int64_t total = nsmall + cp[nI];
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        if (w < nsmall) {
            int64_t i0;
            const int64_t nr = load_small_chunk(sm, w, sps, rs, nI, i0);
            const int64_t E0 = sm.sps[0], E = sm.sps[nr] - E0;
            for (int64_t e = threadIdx.x; e < E; e += SR_BLOCK) {
                const int64_t r = last_le(sm.sps, nr + 1, E0 + e);
                const int64_t c = clampc(acol[sm.rs[r] + (E0 + e - sm.sps[r])], n);
                if (test_bit(bm, c)) atomicAdd(&sm.cnt[r], mult_of(c, dm, jpos, Dn));
            }
            __syncthreads();
            for (int64_t r = threadIdx.x; r < nr; r += SR_BLOCK)
                if (rl[i0 + r] <= SR_LB) cnt[i0 + r] = sm.cnt[r];
            __syncthreads();
        } else {
            const int64_t g = w - nsmall;
            if (threadIdx.x == 0) sm.misc[0] = last_le(cp, nI + 1, g);
            __syncthreads();
            const int64_t i = sm.misc[0];
            const int64_t b = (g - cp[i]) * SR_BD;
            const int64_t e = min(b + SR_BD, (int64_t)rl[i]);
            const int64_t base = rs[i];
            int32_t local = 0;
            for (int64_t k = b + threadIdx.x; k < e; k += SR_BLOCK) {
                const int64_t c = clampc(acol[base + k], n);
                if (test_bit(bm, c)) local += mult_of(c, dm, jpos, Dn);
            }
            int32_t tot;
            block_excl_scan<SR_BLOCK, int32_t>(local, sm.red, tot);
            if (threadIdx.x == 0 && tot) atomicAdd(&cnt[i], tot);
            __syncthreads();
        }
    }
}

// ---- gather (exec) ----------------------------------------------------------
template <typename PT, typename VT>
__device__ __forceinline__ void emit_hits(int64_t c, VT v, int64_t pos, const uint32_t *dm,
                                          const int32_t *jpos, const int32_t *Dj,
                                          const int32_t *Dn, int32_t *ccol, VT *cval) {
    int32_t x = jpos[c];
    if (!test_bit(dm, c)) {
        ccol[pos] = x;
        cval[pos] = v;
        return;
    }
    while (x < 0) {
        ccol[pos] = Dj[~x];
        cval[pos] = v;
        pos++;
        x = Dn[~x];
    }
    ccol[pos] = x;
    cval[pos] = v;
}

template <typename PT, typename VT>
__global__ __launch_bounds__(SR_BLOCK) void k_spref_gather(
    const int32_t *__restrict__ acol, const VT *__restrict__ aval, int64_t n,
    const int64_t *__restrict__ rs, const int32_t *__restrict__ rl, const int64_t *__restrict__ sps,
    const int64_t *__restrict__ cp, int64_t nI, const uint32_t *__restrict__ bm,
    const uint32_t *__restrict__ dm, const int32_t *__restrict__ jpos, const int32_t *__restrict__ Dj,
    const int32_t *__restrict__ Dn, const PT *__restrict__ crow, int32_t *ccol, VT *cval,
    int32_t *cursor, const DevHdr *hdr) {
    __shared__ ChunkSmem sm;
    if (hdr->err) return;
    const int64_t S = sps[nI];
    const int64_t nsmall = (nI + S + SR_D - 1) / SR_D;
    const int64_t total = nsmall + cp[nI];
    constexpr int EPT = (int)((2 * SR_LB + SR_BLOCK - 1) / SR_BLOCK);   // entries per thread
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        if (w < nsmall) {
            int64_t i0;
            const int64_t nr = load_small_chunk(sm, w, sps, rs, nI, i0);
            const int64_t E0 = sm.sps[0], E = sm.sps[nr] - E0;
            int64_t cc[EPT];
            int32_t mm[EPT], rr[EPT];
            int64_t kk[EPT];
            int32_t run = 0;
#pragma unroll
            for (int q = 0; q < EPT; q++) {
                const int64_t e = q * SR_BLOCK + threadIdx.x;
                int32_t mult = 0;
                cc[q] = 0;
                rr[q] = 0;
                kk[q] = 0;
                if (e < E) {
                    const int64_t r = last_le(sm.sps, nr + 1, E0 + e);
                    const int64_t k = sm.rs[r] + (E0 + e - sm.sps[r]);
                    const int64_t c = clampc(acol[k], n);
                    if (test_bit(bm, c)) mult = mult_of(c, dm, jpos, Dn);
                    cc[q] = c;
                    rr[q] = (int32_t)r;
                    kk[q] = k;
                }
                mm[q] = mult;
                int32_t tot;
                const int32_t ex = block_excl_scan<SR_BLOCK, int32_t>(mult, sm.red, tot);
                if (e < E) sm.scan[e] = run + ex;
                run += tot;
                if (E <= (q + 1) * SR_BLOCK) break;   // uniform across the block
            }
            if (threadIdx.x == 0) sm.scan[E] = run;
            __syncthreads();
#pragma unroll
            for (int q = 0; q < EPT; q++) {
                const int64_t e = q * SR_BLOCK + threadIdx.x;
                if (e < E && mm[q]) {
                    const int64_t r = rr[q];
                    const int64_t first = sm.sps[r] - E0;
                    const int64_t pos = (int64_t)crow[i0 + r] + sm.scan[e] - sm.scan[first];
                    emit_hits<PT, VT>(cc[q], aval[kk[q]], pos, dm, jpos, Dj, Dn, ccol, cval);
                }
            }
            __syncthreads();
        } else {
            const int64_t g = w - nsmall;
            if (threadIdx.x == 0) sm.misc[0] = last_le(cp, nI + 1, g);
            __syncthreads();
            const int64_t i = sm.misc[0];
            const int64_t b = (g - cp[i]) * SR_BD;
            const int64_t e = min(b + SR_BD, (int64_t)rl[i]);
            const int64_t base = rs[i];
            constexpr int BPT = (int)(SR_BD / SR_BLOCK);
            int64_t cc[BPT];
            int32_t mm[BPT];
            int32_t mine = 0;
#pragma unroll
            for (int q = 0; q < BPT; q++) {
                const int64_t k = b + (int64_t)threadIdx.x * BPT + q;    // blocked: keeps entry order
                int32_t mult = 0;
                cc[q] = 0;
                if (k < e) {
                    const int64_t c = clampc(acol[base + k], n);
                    if (test_bit(bm, c)) mult = mult_of(c, dm, jpos, Dn);
                    cc[q] = c;
                }
                mm[q] = mult;
                mine += mult;
            }
            int32_t tot;
            int32_t ex = block_excl_scan<SR_BLOCK, int32_t>(mine, sm.red, tot);
            if (threadIdx.x == 0) sm.misc[1] = tot ? atomicAdd(&cursor[i], tot) : 0;
            __syncthreads();
            int64_t pos = (int64_t)crow[i] + sm.misc[1] + ex;
#pragma unroll
            for (int q = 0; q < BPT; q++) {
                if (mm[q]) {
                    const int64_t k = b + (int64_t)threadIdx.x * BPT + q;
                    emit_hits<PT, VT>(cc[q], aval[base + k], pos, dm, jpos, Dj, Dn, ccol, cval);
                    pos += mm[q];
                }
            }
            __syncthreads();
        }
    }
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

template <typename PT>
hp_status_t spref_plan_t(hp_handle_t h, const hp_csr_t *A, const int32_t *I, int64_t nI,
                         const int32_t *J, int64_t nJ, hp_csr_t *C, void *ws, size_t ws_bytes,
                         hp_plan_info_t *info) {
    const int64_t m = A->nrows, n = A->ncols;
    Carve need(nullptr);
    spref_layout(need, n, nI, nJ);
    if (!ws || ws_bytes < need.size()) return fail(h, HP_ERR_WORKSPACE, "spref plan workspace too small");
    const size_t ps = sizeof(PT), vs = val_size(A->val_type);
    const void *ins[] = {A->rowptr, A->col, A->val, I, J};
    const size_t insz[] = {(size_t)(m + 1) * ps, (size_t)A->nnz * 4, (size_t)A->nnz * vs,
                           (size_t)nI * 4, (size_t)nJ * 4};
    for (int k = 0; k < 5; k++)
        if (overlaps(C->rowptr, (nI + 1) * ps, ins[k], insz[k]) || overlaps(ws, ws_bytes, ins[k], insz[k]))
            return fail(h, HP_ERR_ALIAS, "output or workspace overlaps an input");
    if (overlaps(C->rowptr, (nI + 1) * ps, ws, ws_bytes))
        return fail(h, HP_ERR_ALIAS, "C->rowptr overlaps the workspace");
    Carve c(ws);
    SprefLayout L = spref_layout(c, n, nI, nJ);
    const size_t st = scan_tiles(nI);
    hipStream_t s = h->stream;
    stage_begin(h);
    hipError_t e = launch_init_hdr(s, L.hdr, L.tiles, 3 * st);
    if (e == hipSuccess) e = launch_clear_words(s, L.zero, L.nzero);
    stage_mark(h, "spref.init");
    const int gj = (int)std::max<int64_t>(1, std::min<int64_t>((nJ + 255) / 256, 4096));
    const int gi = (int)std::max<int64_t>(1, std::min<int64_t>((nI + 255) / 256, 4096));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_spref_jbuild, dim3(gj), dim3(256), 0, s, J, nJ, n, L.bm, L.dm, L.jpos, L.Dc,
                           L.Dj, L.hdr);
        hipLaunchKernelGGL(k_spref_jlink, dim3(gj), dim3(256), 0, s, L.jpos, L.Dc, L.Dn, L.hdr);
        stage_mark(h, "spref.jtables");
        hipLaunchKernelGGL(k_spref_rows<PT>, dim3(gi), dim3(256), 0, s, (const PT *)A->rowptr, I, nI, m,
                           L.rs, L.rl, L.rls, L.ch, L.hdr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_scan_counts<int64_t>(s, L.rls, L.sps, nI, L.hdr, 0, L.tiles, 0, nullptr, 0);
    if (e == hipSuccess) e = launch_scan_counts<int64_t>(s, L.ch, L.cp, nI, L.hdr, 1, L.tiles + st, 0, nullptr, 0);
    stage_mark(h, "spref.rows");
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_spref_count, dim3(SR_GRID), dim3(SR_BLOCK), 0, s, A->col, n, L.rs, L.rl, L.sps,
                           L.cp, nI, L.bm, L.dm, L.jpos, L.Dn, L.cnt, L.hdr);
        stage_mark(h, "spref.count");
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        e = launch_scan_counts<PT>(s, L.cnt, (PT *)C->rowptr, nI, L.hdr, 2, L.tiles + 2 * st, 3, L.lists, nI,
                                   L.ch);
        stage_mark(h, "spref.scan");
    }
    if (e == hipSuccess) e = readback_hdr(h, L.hdr);
    stage_end(h);
    if (e != hipSuccess) return hip_check(h, e, "spref plan");
    const DevHdr &H = *h->host_hdr;
    hp_status_t stt = status_from_err(h, H.err, "spref");
    if (stt) return stt;
    C->nnz = (int64_t)H.total[2];
    if (info) {
        *info = hp_plan_info_t{};
        info->nnz_out = C->nnz;
        info->map_monotone = (H.flags & F_NOT_MONOTONE) ? 0 : 1;
        info->op = 2;
        for (int b = 0; b < NBINS; b++) {
            info->rows_sorted[b] = H.bin_cnt[b];
            info->class_elems[b] = (int64_t)H.bin_elems[b];
        }
        info->aux[0] = (int64_t)H.total[0];   // entries scanned in small rows
        info->aux[1] = (int64_t)H.total[1];   // big-row chunks
        info->aux[2] = (int64_t)H.ndup;       // repeated J positions
        info->exec_ws_bytes = seg_tmp_bytes(H.bin_elems[BIN_GLOBAL], vs);
    }
    return HP_OK;
}

template <typename PT, typename VT>
hp_status_t spref_exec_t(hp_handle_t h, const hp_csr_t *A, const int32_t *I, int64_t nI,
                         const int32_t *J, int64_t nJ, hp_csr_t *C, void *ws, size_t ws_bytes,
                         const hp_plan_info_t *info, void *xws, size_t xws_bytes) {
    const int64_t m = A->nrows, n = A->ncols;
    Carve need(nullptr);
    spref_layout(need, n, nI, nJ);
    if (!ws || ws_bytes < need.size()) return fail(h, HP_ERR_WORKSPACE, "spref workspace too small");
    if (!info || info->op != 2) return fail(h, HP_ERR_INVALID_ARG, "info is not from hp_spref_plan");
    if (xws_bytes < info->exec_ws_bytes || (info->exec_ws_bytes && !xws))
        return fail(h, HP_ERR_WORKSPACE, "spref exec workspace too small");
    if (C->nnz != info->nnz_out) return fail(h, HP_ERR_INVALID_ARG, "C->nnz differs from the plan");
    if (C->nnz > 0 && (!C->col || !C->val)) return fail(h, HP_ERR_INVALID_ARG, "C->col/val is NULL");
    const size_t vs = sizeof(VT);
    const void *ins[] = {A->rowptr, A->col, A->val, I, J, ws, xws, C->rowptr};
    const size_t insz[] = {(size_t)(m + 1) * sizeof(PT), (size_t)A->nnz * 4, (size_t)A->nnz * vs,
                           (size_t)nI * 4, (size_t)nJ * 4, ws_bytes, xws_bytes,
                           (size_t)(nI + 1) * sizeof(PT)};
    for (int k = 0; k < 8; k++)
        if (overlaps(C->col, (size_t)C->nnz * 4, ins[k], insz[k]) ||
            overlaps(C->val, (size_t)C->nnz * vs, ins[k], insz[k]))
            return fail(h, HP_ERR_ALIAS, "C->col/val overlaps an input or workspace");
    Carve c(ws);
    SprefLayout L = spref_layout(c, n, nI, nJ);
    hipStream_t s = h->stream;
    stage_begin(h);
    hipError_t e = hipSuccess;
    if (info->aux[1] > 0) e = launch_clear_words(s, L.cursor, (size_t)nI);
    if (e == hipSuccess && info->nnz_out > 0) {
        hipLaunchKernelGGL((k_spref_gather<PT, VT>), dim3(SR_GRID), dim3(SR_BLOCK), 0, s, A->col,
                           (const VT *)A->val, n, L.rs, L.rl, L.sps, L.cp, nI, L.bm, L.dm, L.jpos, L.Dj,
                           L.Dn, (const PT *)C->rowptr, C->col, (VT *)C->val, L.cursor, L.hdr);
        stage_mark(h, "spref.gather");
        e = hipGetLastError();
    }
    if (e == hipSuccess && info->nnz_out > 0) {
        uint32_t cnt[NBINS];
        for (int b = 0; b < NBINS; b++) cnt[b] = (uint32_t)info->rows_sorted[b];
        LoadInPlace<PT, VT> ld{(const PT *)C->rowptr, C->col, (const VT *)C->val};
        e = launch_seg_classes<PT, VT, LoadInPlace<PT, VT>>(
            s, (const PT *)C->rowptr, C->col, (VT *)C->val, L.lists, nI, cnt, ld, false, key_bits(nJ),
            true, xws, (uint64_t)info->class_elems[BIN_GLOBAL], L.hdr, true);
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
    spref_layout(c, A->ncols, nI, nJ);
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
