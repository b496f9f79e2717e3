// Bookkeeping of the incremental-update workload (paper Sec. 5.9): a graph
// is rebuilt from a large part by assigning small parts back, with a fresh
// random permutation fused into every step.  Between steps the driver maps
// the parts' original row and column labels to the current ones, composes
// the permutations, and measures the load balance of the current matrix
// over a process grid (the paper's load-imbalance metric: the largest block
// nonzero count over the mean).  None of these calls blocks.
#include "hp_internal.hpp"

namespace hp {
namespace {

__global__ __launch_bounds__(256) void k_gather_index(const int32_t *__restrict__ map, int64_t nmap,
                                                     const int32_t *idx, int64_t n, int32_t *out) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t i = idx[t];
    out[t] = (i >= 0 && i < nmap) ? map[i] : -1;
}

__global__ __launch_bounds__(256) void k_invert_perm(const int32_t *__restrict__ p, int64_t n,
                                                    int32_t *__restrict__ pinv) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int32_t r = p[t];
    if (r >= 0 && r < n) pinv[r] = (int32_t)t;
}

constexpr int BLK_MAX = 4096;   // grid blocks a histogram holds in LDS
constexpr int BN_CHUNK = 1024;  // consecutive entries a wavefront takes at a time
// Row r lies in grid row r*gr/m, column c in grid column c*gc/n.  The rows
// of grid row b are R_b = ceil(b*m/gr) .. R_{b+1}-1, so its entries are the
// contiguous range rowptr[R_b] .. rowptr[R_{b+1}) of col: the pass streams
// col in chunks of BN_CHUNK entries per wavefront (lanes over consecutive
// entries), finds an entry's grid row among the gr+1 entry boundaries in LDS,
// and adds into a workgroup histogram in LDS, flushed once with 64-bit
// atomics.  The lanes of one step add per distinct block (one LDS atomic per
// block present, by ballot), not per entry: the columns of a power-law
// matrix crowd into few blocks, and 64 lanes adding to one LDS word
// serialise.  (Walking rows, a wavefront per row, took 9.2 ms for the 128M
// entries of an R-MAT scale-22 matrix: a chain of dependent loads per row.)
template <typename PT>
__global__ __launch_bounds__(256) void k_block_nnz(const PT *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                  int64_t m, int64_t n, int gr, int gc,
                                                  unsigned long long *counts) {
    __shared__ uint32_t hist[BLK_MAX];
    extern __shared__ int64_t eb[];   // gr + 1 entry boundaries of the grid rows (dynamic: small grids keep occupancy)
    const int nb = gr * gc;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) hist[k] = 0u;
    for (int b = threadIdx.x; b <= gr; b += blockDim.x) eb[b] = (int64_t)rowptr[((int64_t)b * m + gr - 1) / gr];
    __syncthreads();
    const int w = threadIdx.x / WAVE, l = lane_id();
    const int64_t e0 = eb[0], e1 = eb[gr];
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t c0 = e0 + ((int64_t)blockIdx.x * (blockDim.x / WAVE) + w) * BN_CHUNK; c0 < e1;
         c0 += nwaves * BN_CHUNK) {
        const int64_t c1 = c0 + BN_CHUNK < e1 ? c0 + BN_CHUNK : e1;
        for (int64_t k0 = c0; k0 < c1; k0 += WAVE) {
            const int64_t k = k0 + l;
            int bin = -1;
            if (k < c1) {
                // largest b with eb[b] <= k (eb[0] <= k < eb[gr])
                int lo = 0, hi = gr;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (eb[mid] <= k) lo = mid;
                    else hi = mid;
                }
                bin = (int)((int64_t)lo * gc + clampc(col[k], n) * gc / n);
            }
            uint64_t left = ballot(bin >= 0);
            while (left) {
                const int lead = __ffsll((long long)left) - 1;
                const int b = __shfl(bin, lead, WAVE);
                const uint64_t same = ballot(bin == b);
                if (l == lead) atomicAdd(&hist[b], (uint32_t)__popcll(same));
                left &= ~same;
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += blockDim.x)
        if (hist[k]) atomicAdd(&counts[k], (unsigned long long)hist[k]);
}
inline int grid_of(int64_t n) { return (int)std::max<int64_t>(1, (n + 255) / 256); }

}  // namespace
}  // namespace hp

using namespace hp;

extern "C" hp_status_t hp_gather_index(hp_handle_t h, const int32_t *map, int64_t nmap, const int32_t *idx,
                                       int64_t n, int32_t *out) {
    if (!h) return HP_ERR_INVALID_ARG;
    if (n < 0 || nmap < 0) return fail(h, HP_ERR_INVALID_ARG, "negative length");
    if (n == 0) return HP_OK;
    if (!idx || !out || (nmap > 0 && !map)) return fail(h, HP_ERR_INVALID_ARG, "NULL array");
    if (overlaps(out, (size_t)n * 4, map, (size_t)nmap * 4))
        return fail(h, HP_ERR_ALIAS, "out overlaps map");
    if (out != idx && overlaps(out, (size_t)n * 4, idx, (size_t)n * 4))
        return fail(h, HP_ERR_ALIAS, "out partly overlaps idx");
    hipLaunchKernelGGL(k_gather_index, dim3(grid_of(n)), dim3(256), 0, h->stream, map, nmap, idx, n, out);
    return hip_check(h, hipGetLastError(), "gather_index");
}

extern "C" hp_status_t hp_invert_perm(hp_handle_t h, const int32_t *p, int64_t n, int32_t *pinv) {
    if (!h) return HP_ERR_INVALID_ARG;
    if (n < 0) return fail(h, HP_ERR_INVALID_ARG, "negative length");
    if (n == 0) return HP_OK;
    if (!p || !pinv) return fail(h, HP_ERR_INVALID_ARG, "NULL array");
    if (overlaps(p, (size_t)n * 4, pinv, (size_t)n * 4)) return fail(h, HP_ERR_ALIAS, "pinv overlaps p");
    hipLaunchKernelGGL(k_invert_perm, dim3(grid_of(n)), dim3(256), 0, h->stream, p, n, pinv);
    return hip_check(h, hipGetLastError(), "invert_perm");
}

extern "C" hp_status_t hp_block_nnz(hp_handle_t h, const hp_csr_t *A, int32_t gr, int32_t gc, uint64_t *counts) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    if (gr < 1 || gc < 1 || (int64_t)gr * gc > BLK_MAX)
        return fail(h, HP_ERR_INVALID_ARG, "grid must have 1..4096 blocks");
    if (!counts) return fail(h, HP_ERR_INVALID_ARG, "counts is NULL");
    hipError_t e = launch_clear_words(h->stream, counts, (size_t)gr * gc * 2);
    const int64_t m = A->nrows;
    if (e == hipSuccess && m > 0 && A->ncols > 0 && A->nnz > 0) {
        // one workgroup per CU-slot's worth of chunks, at most 1024 (each
        // flushes its histogram once)
        const int64_t chunks = (A->nnz + BN_CHUNK - 1) / BN_CHUNK;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (chunks + 3) / 4));
        unsigned long long *cnt = reinterpret_cast<unsigned long long *>(counts);
        const size_t ebytes = (size_t)(gr + 1) * sizeof(int64_t);
        if (A->ptr_type == HP_IDX_I64)
            hipLaunchKernelGGL(k_block_nnz<int64_t>, dim3(grid), dim3(256), ebytes, h->stream,
                               (const int64_t *)A->rowptr, A->col, m, A->ncols, gr, gc, cnt);
        else
            hipLaunchKernelGGL(k_block_nnz<int32_t>, dim3(grid), dim3(256), ebytes, h->stream,
                               (const int32_t *)A->rowptr, A->col, m, A->ncols, gr, gc, cnt);
        e = hipGetLastError();
    }
    return hip_check(h, e, "block_nnz");
}
