// Canonical-CSR check: rowptr[0] = 0, rowptr non-decreasing, rowptr[m] =
// nnz, every column in [0, ncols) and columns strictly increasing inside a
// row.  Row starts are marked in a byte array so that the entry pass can
// tell "first entry of a row" from "follows an entry of the same row".
#include "hp_internal.hpp"

#include <algorithm>
#include <cstdlib>

using namespace hp;

namespace {

template <typename PT>
__global__ __launch_bounds__(256) void k_val_rows(const PT *__restrict__ rowptr, int64_t m, int64_t nnz,
                                                 uint8_t *start, DevHdr *hdr) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r > m) return;
    const int64_t s = rowptr[r];
    bool bad = false;
    if (r == 0) bad |= s != 0;
    if (r == m) bad |= s != nnz;
    if (r < m) {
        const int64_t e = rowptr[r + 1];
        bad |= e < s || s < 0 || e > nnz;
        if (!bad && e > s) start[s] = 1;
    }
    if (bad) atomicOr(&hdr->err, E_NONCANON);   // error path only
}

__global__ __launch_bounds__(256) void k_val_entries(const int32_t *__restrict__ col, int64_t nnz,
                                                    int64_t n, const uint8_t *__restrict__ start,
                                                    DevHdr *hdr) {
    if (hdr->err) return;
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nnz) return;
    const int32_t c = col[k];
    uint32_t e = 0;
    if (c < 0 || c >= n) e |= E_RANGE;
    if (k > 0 && !start[k] && col[k - 1] >= c) e |= E_NONCANON;
    if (e) atomicOr(&hdr->err, e);   // error path only
}

// Row-parallel form of the same check (one lane walks one row), which needs
// no workspace beyond a status block: the plans run it first when
// validation is switched on.
template <typename PT>
__global__ __launch_bounds__(256) void k_val_rowwise(const PT *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                    int64_t m, int64_t n, int64_t nnz, DevHdr *hdr) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r > m) return;
    const int64_t s = rowptr[r];
    uint32_t e = 0;
    if (r == 0 && s != 0) e |= E_NONCANON;
    if (r == m && s != nnz) e |= E_NONCANON;
    if (r < m) {
        const int64_t t = rowptr[r + 1];
        if (t < s || s < 0 || t > nnz) {
            e |= E_NONCANON;
        } else {
            int64_t prev = -1;
            for (int64_t k = s; k < t && !e; k++) {
                const int32_t c = col[k];
                if (c < 0 || c >= n) e |= E_RANGE;
                else if (c <= prev) e |= E_NONCANON;
                prev = c;
            }
        }
    }
    if (e) atomicOr(&hdr->err, e);   // error path only
}

size_t val_ws(const hp_csr_t *A) {
    Carve c(nullptr);
    c.take<DevHdr>(1);
    c.take<uint8_t>((size_t)A->nnz + 16);
    return c.size();
}

}  // namespace

extern "C" hp_status_t hp_validate_workspace(hp_handle_t h, const hp_csr_t *A, size_t *bytes) {
    if (!h || !bytes) return HP_ERR_INVALID_ARG;
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    *bytes = val_ws(A);
    return HP_OK;
}

extern "C" hp_status_t hp_validate_csr(hp_handle_t h, const hp_csr_t *A, void *ws, size_t ws_bytes) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    if (!ws || ws_bytes < val_ws(A)) return fail(h, HP_ERR_WORKSPACE, "validate workspace too small");
    Carve c(ws);
    DevHdr *hdr = c.take<DevHdr>(1);
    uint8_t *start = c.take<uint8_t>((size_t)A->nnz + 16);
    hipStream_t s = h->stream;
    const int64_t m = A->nrows, nnz = A->nnz;
    hipError_t e = launch_init_hdr(s, hdr, nullptr, 0);
    if (e == hipSuccess) e = launch_clear_words(s, start, ((size_t)nnz + 16) / 4);
    if (e == hipSuccess) {
        const unsigned gr = (unsigned)std::max<int64_t>(1, (m + 1 + 255) / 256);
        if (A->ptr_type == HP_IDX_I64)
            hipLaunchKernelGGL(k_val_rows<int64_t>, dim3(gr), dim3(256), 0, s, (const int64_t *)A->rowptr, m, nnz,
                               start, hdr);
        else
            hipLaunchKernelGGL(k_val_rows<int32_t>, dim3(gr), dim3(256), 0, s, (const int32_t *)A->rowptr, m, nnz,
                               start, hdr);
        if (nnz > 0)
            hipLaunchKernelGGL(k_val_entries, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s, A->col, nnz,
                               A->ncols, start, hdr);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_check(h, e, "validate");
    if (hp_status_t rb = readback_hdr(h, hdr, "validate")) return rb;
    return status_from_err(h, h->host_hdr->err, "validate");
}

namespace hp {

bool validate_from_env() {
    const char *v = std::getenv("HP_VALIDATE");
    return v && *v && !(v[0] == '0' && v[1] == 0);
}

// When validation is on for h: the canonical-CSR check of M (named `what`)
// into the status block `hdr` of the calling plan's workspace, read back
// before the plan launches anything else.
hp_status_t validate_input(hp_handle_t h, const hp_csr_t *M, DevHdr *hdr, const char *what) {
    if (!h->validate) return HP_OK;
    hipStream_t s = h->stream;
    hipError_t e = launch_init_hdr(s, hdr, nullptr, 0);
    if (e == hipSuccess) {
        const unsigned gr = (unsigned)std::max<int64_t>(1, (M->nrows + 1 + 255) / 256);
        if (M->ptr_type == HP_IDX_I64)
            hipLaunchKernelGGL(k_val_rowwise<int64_t>, dim3(gr), dim3(256), 0, s, (const int64_t *)M->rowptr, M->col,
                               M->nrows, M->ncols, M->nnz, hdr);
        else
            hipLaunchKernelGGL(k_val_rowwise<int32_t>, dim3(gr), dim3(256), 0, s, (const int32_t *)M->rowptr, M->col,
                               M->nrows, M->ncols, M->nnz, hdr);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_check(h, e, what);
    if (hp_status_t rb = readback_hdr(h, hdr, what)) return rb;
    return status_from_err(h, h->host_hdr->err, what);
}

}  // namespace hp

extern "C" hp_status_t hp_set_validate(hp_handle_t h, int enable) {
    if (!h) return HP_ERR_INVALID_ARG;
    h->validate = enable != 0;
    return HP_OK;
}
