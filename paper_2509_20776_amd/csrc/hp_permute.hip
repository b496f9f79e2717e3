// permute: C = P A Q^T, C[i,j] = A[p[i], q[j]] (paper Sec. 2.1).
//
// Identify (Sec. 4.2 Step 1): the index/value swap of p and q gives pinv
// and qinv; the destination of source row r is output row pinv[r] and of
// column c is qinv[c].  On one GPU the Exchange step disappears, and the
// paper's two-pass count / prefix / scatter becomes count -> scan -> fill,
// with the Build-step sort folded into the fill:
//   plan : fill -1      pinv, qinv
//          k_perm_prepare  scatter pinv (marks of p); per-output-row counts;
//                          range of p
//          k_perm_qinv     scatter qinv; range of q
//          k_perm_check    no slot left at -1 (every value occurs once)
//          scan            rowptr of C + row classes by length
//   exec : k_perm_pack       rows of <= 4 entries renamed, sorted and packed
//                            into fixed slots (a sequential pass over A;
//                            only when such rows hold most entries)
//          k_perm_slot_fill  output rows of <= 4 entries copied from slot
//                            p[i] (or k_perm_pull_short: read from row p[i]
//                            of A, renamed and sorted in registers)
//          class kernels     longer rows gathered from A (pull) and sorted
#include "hp_internal.hpp"
#include "hp_segsort.hpp"
#include "hp_perm_tiles.hpp"

using namespace hp;
using namespace hp::perm;

namespace {

// The symmetric form renames columns with pinv itself; the general form
// needs only qinv, and marks the values of p in bytes (pmark) for the check.
struct PermLayout {
    DevHdr *hdr;
    uint64_t *tiles;
    int32_t *pinv, *qinv, *cnt;
    uint8_t *pmark;
    uint32_t *lists;
};

PermLayout perm_layout(Carve &c, int64_t m, int64_t n, bool sym) {
    PermLayout L;
    L.hdr = c.take<DevHdr>(1);
    L.tiles = c.take<uint64_t>(scan_tiles(m));
    L.pinv = sym ? c.take<int32_t>(m) : nullptr;
    L.pmark = sym ? nullptr : reinterpret_cast<uint8_t *>(c.take<uint32_t>((m + 3) / 4));
    L.qinv = sym ? L.pinv : c.take<int32_t>(n);
    L.cnt = c.take<int32_t>(m);
    L.lists = c.take<uint32_t>(seg_list_words(m));
    return L;
}

template <typename PT>
__global__ __launch_bounds__(256) void k_perm_prepare(const PT *__restrict__ arow, const int32_t *__restrict__ p,
                                                     const int32_t *__restrict__ q, int64_t m, int64_t n,
                                                     int32_t *pinv, int32_t *qinv, int32_t *cnt, DevHdr *hdr,
                                                     uint8_t *pmark) {
    perm_prepare_tile<PT>(blockIdx.x, arow, p, q, m, n, pinv, qinv, cnt, hdr, pmark);
}
__global__ __launch_bounds__(256) void k_perm_qinv(const int32_t *__restrict__ q, int64_t n, int32_t *qinv,
                                                  DevHdr *hdr) {
    perm_qinv_tile(blockIdx.x, q, n, qinv, hdr);
}
__global__ __launch_bounds__(256) void k_perm_check(int64_t m, int64_t n, const int32_t *__restrict__ pinv,
                                                   const int32_t *__restrict__ qinv, bool general, DevHdr *hdr,
                                                   const uint8_t *__restrict__ pmark) {
    perm_check4_tile(blockIdx.x, m, n, pinv, qinv, general, hdr, pmark);
}
template <typename PT, typename VT>
__global__ __launch_bounds__(256) void k_perm_pack(const PT *__restrict__ arow, const int32_t *__restrict__ acol,
                                                  const VT *__restrict__ aval, const int32_t *__restrict__ cmap,
                                                  int64_t n, int64_t m, char *__restrict__ slots) {
    __shared__ int32_t lk[4 * PACK_STAGE];
    __shared__ VT lv[4 * PACK_STAGE];
    perm_pack_tile<PT, VT>(blockIdx.x, arow, acol, aval, cmap, n, m, slots, lk, lv);
}
template <typename PT, typename VT>
__global__ __launch_bounds__(256) void k_perm_slot_fill(const int32_t *__restrict__ p, const char *__restrict__ slots,
                                                       const PT *__restrict__ crow, int32_t *__restrict__ ccol,
                                                       VT *__restrict__ cval, int64_t m, const DevHdr *hdr) {
    perm_slot_fill_tile<PT, VT>(blockIdx.x, p, slots, crow, ccol, cval, m, hdr);
}
template <typename PT, typename VT>
__global__ __launch_bounds__(256) void k_perm_pull_short(const PT *__restrict__ arow, const int32_t *__restrict__ acol,
                                                        const VT *__restrict__ aval, const int32_t *__restrict__ p,
                                                        const int32_t *__restrict__ cmap, int64_t n,
                                                        const PT *__restrict__ crow, int32_t *__restrict__ ccol,
                                                        VT *__restrict__ cval, int64_t m, const DevHdr *hdr) {
    perm_pull_short_tile<PT, VT>(blockIdx.x, arow, acol, aval, p, cmap, n, crow, ccol, cval, m, hdr);
}

// Entries in output rows of more than 4 entries (the class sorts' rows).
int64_t long_entries(const hp_plan_info_t *info) {
    int64_t e = 0;
    for (int b = 0; b < NBINS; b++) e += info->class_elems[b];
    return e;
}

// Exec workspace: the class sorts' temporaries, then the row slots when
// they are used (m slots of slot_bytes, from the first 256-byte boundary
// after the temporaries, wherever the caller's workspace starts).
size_t perm_xws_bytes(size_t seg_bytes, int64_t m, int slot_bytes) {
    const size_t seg = (seg_bytes + 255) & ~size_t(255);
    return slot_bytes ? seg + 256 + (((size_t)m * slot_bytes + 255) & ~size_t(255)) : seg;
}

hp_status_t perm_check_args(hp_handle_t h, const hp_csr_t *A, const int32_t *p, const int32_t *q,
                            const hp_csr_t *C) {
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    if (!C) return fail(h, HP_ERR_INVALID_ARG, "C is NULL");
    if (!q && A->nrows != A->ncols) return fail(h, HP_ERR_SHAPE, "symmetric permute needs a square A");
    if (C->nrows != A->nrows || C->ncols != A->ncols)
        return fail(h, HP_ERR_SHAPE, "C must have A's shape");
    if (C->ptr_type != A->ptr_type || C->val_type != A->val_type)
        return fail(h, HP_ERR_INVALID_ARG, "C must have A's ptr_type and val_type");
    if (!C->rowptr) return fail(h, HP_ERR_INVALID_ARG, "C->rowptr is NULL");
    if (A->nrows > 0 && !p) return fail(h, HP_ERR_INVALID_ARG, "p is NULL");
    return HP_OK;
}

template <typename PT>
hp_status_t perm_plan_t(hp_handle_t h, const hp_csr_t *A, const int32_t *p, const int32_t *q,
                        hp_csr_t *C, void *ws, size_t ws_bytes, hp_plan_info_t *info) {
    const int64_t m = A->nrows, n = A->ncols;
    const bool sym = q == nullptr;
    Carve need(nullptr);
    perm_layout(need, m, n, sym);
    if (!ws || ws_bytes < need.size()) return fail(h, HP_ERR_WORKSPACE, "permute plan workspace too small");
    const size_t ps = sizeof(PT), vs = val_size(A->val_type);
    const void *ins[] = {A->rowptr, A->col, A->val, p, q};
    const size_t insz[] = {(size_t)(m + 1) * ps, (size_t)A->nnz * 4, (size_t)A->nnz * vs,
                           (size_t)m * 4, q ? (size_t)n * 4 : 0};
    for (int k = 0; k < 5; k++)
        if (overlaps(C->rowptr, (m + 1) * ps, ins[k], insz[k]) || overlaps(ws, ws_bytes, ins[k], insz[k]))
            return fail(h, HP_ERR_ALIAS, "output or workspace overlaps an input");
    if (overlaps(C->rowptr, (m + 1) * ps, ws, ws_bytes))
        return fail(h, HP_ERR_ALIAS, "C->rowptr overlaps the workspace");
    Carve c(ws);
    PermLayout L = perm_layout(c, m, n, sym);
    hipStream_t s = h->stream;
    if (hp_status_t v = validate_input(h, A, L.hdr, "permute plan: A")) return v;
    stage_begin(h);
    hipError_t e = launch_init_hdr(s, L.hdr, L.tiles, scan_tiles(m));
    if (e == hipSuccess) e = sym ? launch_fill_words(s, L.pinv, (size_t)m, 0xFFFFFFFFu)
                                 : launch_fill_words(s, L.pmark, (size_t)(m + 3) / 4, 0u);
    if (e == hipSuccess && !sym) e = launch_fill_words(s, L.qinv, (size_t)n, 0xFFFFFFFFu);
    const int64_t hi = m > n ? m : n;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_perm_prepare<PT>, dim3((unsigned)std::max<int64_t>(1, (m + 255) / 256)), dim3(256), 0,
                           s, (const PT *)A->rowptr, p, nullptr, m, n, L.pinv, L.qinv, L.cnt, L.hdr, L.pmark);
        if (!sym)
            hipLaunchKernelGGL(k_perm_qinv, dim3((unsigned)std::max<int64_t>(1, (n + 255) / 256)), dim3(256), 0, s,
                               q, n, L.qinv, L.hdr);
        stage_mark(h, "perm.prepare");
        hipLaunchKernelGGL(k_perm_check, dim3((unsigned)std::max<int64_t>(1, (hi + 1023) / 1024)), dim3(256), 0, s, m,
                           n, L.pinv, L.qinv, !sym, L.hdr, L.pmark);
        stage_mark(h, "perm.check");
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        e = launch_scan_counts<PT>(s, L.cnt, (PT *)C->rowptr, m, L.hdr, 0, L.tiles, 1, L.lists, m);
        stage_mark(h, "perm.scan");
    }
    if (e != hipSuccess) return hip_check(h, e, "permute plan");
    if (hp_status_t rb = readback_hdr(h, L.hdr, "permute plan")) return rb;
    stage_end(h);
    const DevHdr &H = *h->host_hdr;
    hp_status_t st = status_from_err(h, H.err, "permute");
    if (st) return st;
    C->nnz = (int64_t)H.total[0];
    if (info) {
        *info = hp_plan_info_t{};
        info->nnz_out = C->nnz;
        info->map_monotone = 0;   // rows are always sorted
        info->op = 1;
        for (int b = 0; b < NBINS; b++) {
            info->rows_sorted[b] = H.bin_cnt[b];
            info->class_elems[b] = (int64_t)H.bin_elems[b];
        }
        // exec_ws_bytes: with the row slots when they pay; aux[0]: the
        // smallest exec workspace, without them
        const size_t seg = seg_tmp_bytes(H.bin_elems[BIN_GLOBAL], H.bin_cnt[BIN_GLOBAL], vs, n);
        const int sb = vs == 8 ? perm_slot_bytes<uint64_t>() : perm_slot_bytes<uint32_t>();
        info->aux[0] = (int64_t)perm_xws_bytes(seg, m, 0);
        info->exec_ws_bytes = perm_use_slots(A->nnz, long_entries(info)) ? perm_xws_bytes(seg, m, sb)
                                                                          : (size_t)info->aux[0];
    }
    return HP_OK;
}

template <typename PT, typename VT>
hp_status_t perm_exec_t(hp_handle_t h, const hp_csr_t *A, const int32_t *p, const int32_t *q,
                        hp_csr_t *C, void *ws, size_t ws_bytes, const hp_plan_info_t *info, void *xws,
                        size_t xws_bytes) {
    const int64_t m = A->nrows, n = A->ncols;
    const bool sym = q == nullptr;
    Carve need(nullptr);
    perm_layout(need, m, n, sym);
    if (!ws || ws_bytes < need.size()) return fail(h, HP_ERR_WORKSPACE, "permute workspace too small");
    if (!info || info->op != 1) return fail(h, HP_ERR_INVALID_ARG, "info is not from hp_permute_plan");
    if (info->aux[0] < 0 || xws_bytes < (size_t)info->aux[0] || (info->aux[0] && !xws))
        return fail(h, HP_ERR_WORKSPACE, "permute exec workspace too small");
    if (C->nnz != A->nnz) return fail(h, HP_ERR_INVALID_ARG, "C->nnz must equal nnz(A) (set by plan)");
    if (C->nnz > 0 && (!C->col || !C->val)) return fail(h, HP_ERR_INVALID_ARG, "C->col/val is NULL");
    const size_t vs = sizeof(VT);
    const void *ins[] = {A->rowptr, A->col, A->val, p, q, ws, xws, C->rowptr};
    const size_t insz[] = {(size_t)(m + 1) * sizeof(PT), (size_t)A->nnz * 4, (size_t)A->nnz * vs,
                           (size_t)m * 4, q ? (size_t)n * 4 : 0, ws_bytes, xws_bytes,
                           (size_t)(m + 1) * sizeof(PT)};
    for (int k = 0; k < 8; k++)
        if (overlaps(C->col, (size_t)C->nnz * 4, ins[k], insz[k]) ||
            overlaps(C->val, (size_t)C->nnz * vs, ins[k], insz[k]))
            return fail(h, HP_ERR_ALIAS, "C->col/val overlaps an input or workspace");
    Carve c(ws);
    PermLayout L = perm_layout(c, m, n, sym);
    hipStream_t s = h->stream;
    const int sorted = info->map_monotone;
    stage_begin(h);
    const size_t seg_bytes = seg_tmp_bytes((uint64_t)info->class_elems[BIN_GLOBAL], (uint64_t)info->rows_sorted[BIN_GLOBAL],
                                           vs, n);
    if ((size_t)info->aux[0] != perm_xws_bytes(seg_bytes, m, 0))
        return fail(h, HP_ERR_INVALID_ARG, "info is not from hp_permute_plan of this matrix");
    // the row slots when they pay and the workspace holds them
    const int sb = perm_slot_bytes<VT>();
    const bool slots = perm_use_slots(A->nnz, long_entries(info)) && xws_bytes >= perm_xws_bytes(seg_bytes, m, sb);
    const unsigned grid = (unsigned)((m + 255) / 256);
    if (m > 0 && slots) {
        const uintptr_t at = (uintptr_t)xws + ((seg_bytes + 255) & ~size_t(255));
        char *sl = (char *)((at + 255) & ~uintptr_t(255));
        hipLaunchKernelGGL((k_perm_pack<PT, VT>), dim3(grid), dim3(256), 0, s, (const PT *)A->rowptr, A->col,
                           (const VT *)A->val, L.qinv, n, m, sl);
        stage_mark(h, "perm.pack");
        hipLaunchKernelGGL((k_perm_slot_fill<PT, VT>), dim3(grid), dim3(256), 0, s, p, (const char *)sl,
                           (const PT *)C->rowptr, C->col, (VT *)C->val, m, L.hdr);
        stage_mark(h, "perm.fill_short");
    } else if (m > 0) {
        hipLaunchKernelGGL((k_perm_pull_short<PT, VT>), dim3(grid), dim3(256), 0, s, (const PT *)A->rowptr, A->col,
                           (const VT *)A->val, p, L.qinv, n, (const PT *)C->rowptr, C->col, (VT *)C->val, m, L.hdr);
        stage_mark(h, "perm.fill_short");
    }
    uint32_t cnt[NBINS];
    for (int b = 0; b < NBINS; b++) cnt[b] = (uint32_t)info->rows_sorted[b];
    LoadPerm<PT, VT> ld{(const PT *)A->rowptr, A->col, (const VT *)A->val, p, L.qinv, n};
    hipError_t e = launch_seg_classes<PT, VT, LoadPerm<PT, VT>>(
        s, (const PT *)C->rowptr, C->col, (VT *)C->val, L.lists, m, cnt, ld, sorted != 0, n, false, xws,
        (uint64_t)info->class_elems[BIN_GLOBAL], L.hdr, true);
    stage_mark(h, "perm.fill_long");
    stage_end(h);
    return hip_check(h, e == hipSuccess ? hipGetLastError() : e, "permute exec");
}

}  // namespace

extern "C" hp_status_t hp_permute_workspace(hp_handle_t h, const hp_csr_t *A, size_t *bytes) {
    if (!h || !bytes) return HP_ERR_INVALID_ARG;
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    Carve c(nullptr);
    perm_layout(c, A->nrows, A->ncols, false);
    *bytes = c.size();
    return HP_OK;
}

extern "C" hp_status_t hp_permute_plan(hp_handle_t h, const hp_csr_t *A, const int32_t *p,
                                       const int32_t *q, hp_csr_t *C, void *ws, size_t ws_bytes,
                                       hp_plan_info_t *info) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = perm_check_args(h, A, p, q, C);
    if (st) return st;
    if (A->ptr_type == HP_IDX_I32) return perm_plan_t<int32_t>(h, A, p, q, C, ws, ws_bytes, info);
    return perm_plan_t<int64_t>(h, A, p, q, C, ws, ws_bytes, info);
}

extern "C" hp_status_t hp_permute_exec(hp_handle_t h, const hp_csr_t *A, const int32_t *p,
                                       const int32_t *q, hp_csr_t *C, void *ws, size_t ws_bytes,
                                       const hp_plan_info_t *info, void *xws, size_t xws_bytes) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = perm_check_args(h, A, p, q, C);
    if (st) return st;
    const bool p64 = A->ptr_type == HP_IDX_I64, v64 = A->val_type == HP_VAL_F64;
    if (!p64 && !v64) return perm_exec_t<int32_t, uint32_t>(h, A, p, q, C, ws, ws_bytes, info, xws, xws_bytes);
    if (!p64 && v64) return perm_exec_t<int32_t, uint64_t>(h, A, p, q, C, ws, ws_bytes, info, xws, xws_bytes);
    if (p64 && !v64) return perm_exec_t<int64_t, uint32_t>(h, A, p, q, C, ws, ws_bytes, info, xws, xws_bytes);
    return perm_exec_t<int64_t, uint64_t>(h, A, p, q, C, ws, ws_bytes, info, xws, xws_bytes);
}
