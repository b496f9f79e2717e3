// Segmented sort used by the Build step of every operation (the paper sorts
// received tuples before forming the local matrix, Sec. 4.2 "Build").
//
// Every segment is one output row [rowptr[r], rowptr[r+1]); keys are the new
// column indices, distinct inside a row; values travel with their keys.  A
// Loader supplies element k of row r: either the row already written in
// place (LoadInPlace) or an operation-specific gather (for example permute
// reads row p[r] of A and maps its columns), so a gather and the sort are
// one pass.  Rows are grouped by length into classes decided during the
// count scan:
//   THREAD  2..16     one lane, bitonic network in registers
//   WAVE    17..64    one wavefront, rank = number of smaller keys (LDS)
//   BLOCK   65..4096  one workgroup, bitonic sort in LDS
//   GLOBAL  > 4096    one workgroup, LSD radix (8-bit digits) through a
//                     temporary region; stable ranks from wavefront match
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

// Sort up to N (4 or 16) elements held by one lane and store the first len.
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

template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(256) void k_seg_thread(const PT *__restrict__ rowptr, int32_t *okey,
                                                   VT *oval, const uint32_t *__restrict__ list,
                                                   uint32_t count, LD ld, int sorted,
                                                   const DevHdr *hdr) {
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count || hdr->err) return;
    int64_t row = list[t];
    int64_t b = rowptr[row];
    int len = (int)(rowptr[row + 1] - b);
    int64_t sb = ld.base(row);
    if (len <= 4) {
        int32_t k[4];
        VT v[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            k[i] = INT32_MAX;
            v[i] = VT(0);
            if (i < len) ld.get(sb, i, k[i], v[i]);
        }
        sort_store_regs<4, VT>(k, v, len, sorted, okey + b, oval + b);
        return;
    }
    int32_t k[16];
    VT v[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        k[i] = INT32_MAX;
        v[i] = VT(0);
        if (i < len) ld.get(sb, i, k[i], v[i]);
    }
    sort_store_regs<16, VT>(k, v, len, sorted, okey + b, oval + b);
}

template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(256) void k_seg_wave(const PT *__restrict__ rowptr, int32_t *okey,
                                                 VT *oval, const uint32_t *__restrict__ list,
                                                 uint32_t count, LD ld, int sorted,
                                                 const DevHdr *hdr) {
    __shared__ int32_t s_k[4][WAVE];
    const int w = threadIdx.x / WAVE, l = lane_id();
    uint32_t t = blockIdx.x * 4 + w;
    if (t >= count || hdr->err) return;
    int64_t row = list[t];
    int64_t b = rowptr[row];
    int len = (int)(rowptr[row + 1] - b);
    int64_t sb = ld.base(row);
    int32_t mk = INT32_MAX;
    VT mv = VT(0);
    if (l < len) ld.get(sb, l, mk, mv);
    int rank = l;
    if (!sorted) {
        s_k[w][l] = mk;
        __builtin_amdgcn_wave_barrier();
        rank = 0;
        for (int i = 0; i < len; i++) rank += s_k[w][i] < mk;
    }
    if (l < len) {
        okey[b + rank] = mk;
        oval[b + rank] = mv;
    }
}

template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(256) void k_seg_block(const PT *__restrict__ rowptr, int32_t *okey,
                                                  VT *oval, const uint32_t *__restrict__ list,
                                                  uint32_t count, LD ld, int sorted,
                                                  const DevHdr *hdr) {
    __shared__ int32_t s_k[BLOCK_MAX];
    __shared__ VT s_v[BLOCK_MAX];
    uint32_t t = blockIdx.x;
    if (t >= count || hdr->err) return;
    int64_t row = list[t];
    int64_t b = rowptr[row];
    int len = (int)(rowptr[row + 1] - b);
    int64_t sb = ld.base(row);
    if (sorted) {
        for (int i = threadIdx.x; i < len; i += 256) {
            int32_t kk;
            VT vv;
            ld.get(sb, i, kk, vv);
            okey[b + i] = kk;
            oval[b + i] = vv;
        }
        return;
    }
    int N = 128;
    while (N < len) N <<= 1;
    for (int i = threadIdx.x; i < N; i += 256) {
        int32_t kk = INT32_MAX;
        VT vv = VT(0);
        if (i < len) ld.get(sb, i, kk, vv);
        s_k[i] = kk;
        s_v[i] = vv;
    }
    __syncthreads();
    for (int size = 2; size <= N; size <<= 1) {
        for (int j = size >> 1; j > 0; j >>= 1) {
            for (int p = threadIdx.x; p < N / 2; p += 256) {
                int i = 2 * j * (p / j) + (p % j);
                int l = i + j;
                bool up = (i & size) == 0;
                int32_t a = s_k[i], c = s_k[l];
                if ((a > c) == up) {
                    s_k[i] = c;
                    s_k[l] = a;
                    VT tv = s_v[i];
                    s_v[i] = s_v[l];
                    s_v[l] = tv;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < len; i += 256) {
        okey[b + i] = s_k[i];
        oval[b + i] = s_v[i];
    }
}

// LSD radix over one long row.  X = the output row, Y = its temporary
// region.  Pass 0 reads through the loader; the last pass writes X.  When
// the loader reads X itself (in-place) and the pass count is odd, the data
// is first copied to Y so that no pass reads and writes the same array.
template <typename PT, typename VT, typename LD>
__global__ __launch_bounds__(256) void k_seg_global(const PT *__restrict__ rowptr, int32_t *okey,
                                                   VT *oval, const uint32_t *__restrict__ list,
                                                   const uint64_t *__restrict__ goff, uint32_t count,
                                                   LD ld, int sorted, int kbits, int inplace,
                                                   int32_t *tkey, VT *tval, const DevHdr *hdr) {
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_wc[4][256];
    __shared__ uint32_t s_sw[4];
    uint32_t t = blockIdx.x;
    if (t >= count || hdr->err) return;
    int64_t row = list[t];
    int64_t b = rowptr[row];
    int64_t len = rowptr[row + 1] - b;
    int64_t sb = ld.base(row);
    int32_t *xk = okey + b;
    VT *xv = oval + b;
    int32_t *yk = tkey + goff[t];
    VT *yv = tval + goff[t];
    if (sorted) {
        for (int64_t i = threadIdx.x; i < len; i += 256) {
            int32_t kk;
            VT vv;
            ld.get(sb, i, kk, vv);
            xk[i] = kk;
            xv[i] = vv;
        }
        return;
    }
    const int w = threadIdx.x / WAVE;
    const uint64_t lt = lanemask_lt();
    const int passes = (kbits + 7) / 8;
    bool from_loader = true;
    if (inplace && (passes & 1)) {
        for (int64_t i = threadIdx.x; i < len; i += 256) {
            yk[i] = xk[i];
            yv[i] = xv[i];
        }
        __syncthreads();
        from_loader = false;   // data now in Y
    }
    // destination of pass p: X when (passes-1-p) is even, else Y
    for (int i = threadIdx.x; i < 4 * 256; i += 256) (&s_wc[0][0])[i] = 0;
    for (int pass = 0; pass < passes; pass++) {
        const int shift = 8 * pass;
        const bool to_x = ((passes - 1 - pass) & 1) == 0;
        int32_t *dk = to_x ? xk : yk;
        VT *dv = to_x ? xv : yv;
        const int32_t *sk = to_x ? yk : xk;
        const VT *sv = to_x ? yv : xv;
        const bool use_ld = pass == 0 && from_loader;
        s_hist[threadIdx.x] = 0;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < len; i += 256) {
            int32_t kk;
            if (use_ld) {
                VT vv;
                ld.get(sb, i, kk, vv);
            } else {
                kk = sk[i];
            }
            atomicAdd(&s_hist[((uint32_t)kk >> shift) & 255u], 1u);
        }
        __syncthreads();
        {
            uint32_t tot;
            uint32_t ex = block_excl_scan<256, uint32_t>(s_hist[threadIdx.x], s_sw, tot);
            s_base[threadIdx.x] = ex;
        }
        __syncthreads();
        for (int64_t c0 = 0; c0 < len; c0 += 256) {
            int64_t i = c0 + threadIdx.x;
            bool valid = i < len;
            int32_t k = 0;
            VT v = VT(0);
            if (valid) {
                if (use_ld) ld.get(sb, i, k, v);
                else { k = sk[i]; v = sv[i]; }
            }
            uint32_t d = ((uint32_t)k >> shift) & 255u;
            uint64_t peers = ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; bit++) {
                uint64_t bb = ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? bb : ~bb;
            }
            uint32_t rank = (uint32_t)__popcll(peers & lt);
            if (valid && rank == 0) s_wc[w][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (valid) {
                uint32_t off = s_base[d] + rank;
                for (int ww = 0; ww < w; ww++) off += s_wc[ww][d];
                dk[off] = k;
                dv[off] = v;
            }
            __syncthreads();
            {
                const uint32_t dd = threadIdx.x;
                s_base[dd] += s_wc[0][dd] + s_wc[1][dd] + s_wc[2][dd] + s_wc[3][dd];
                s_wc[0][dd] = 0;
                s_wc[1][dd] = 0;
                s_wc[2][dd] = 0;
                s_wc[3][dd] = 0;
            }
            __syncthreads();
        }
    }
}

// Launch the classes present in the plan's bin counts.  lists holds NBINS
// lists of capacity cap, followed by cap uint64 temporary offsets for the
// GLOBAL class; tmp holds round256(glob_elems*4) key bytes then the values.
template <typename PT, typename VT, typename LD>
hipError_t launch_seg_classes(hipStream_t s, const PT *rowptr, int32_t *okey, VT *oval,
                              const uint32_t *lists, int64_t cap, const uint32_t *cnt, LD ld,
                              bool sorted, int kbits, bool inplace, void *tmp, uint64_t glob_elems,
                              const DevHdr *hdr, bool do_thread) {
    const uint64_t *goff = reinterpret_cast<const uint64_t *>(lists + NBINS * cap);
    if (do_thread && cnt[BIN_THREAD])
        hipLaunchKernelGGL((k_seg_thread<PT, VT, LD>), dim3((cnt[BIN_THREAD] + 255) / 256), dim3(256),
                           0, s, rowptr, okey, oval, lists + BIN_THREAD * cap, cnt[BIN_THREAD], ld,
                           (int)sorted, hdr);
    if (cnt[BIN_WAVE])
        hipLaunchKernelGGL((k_seg_wave<PT, VT, LD>), dim3((cnt[BIN_WAVE] + 3) / 4), dim3(256), 0, s,
                           rowptr, okey, oval, lists + BIN_WAVE * cap, cnt[BIN_WAVE], ld, (int)sorted,
                           hdr);
    if (cnt[BIN_BLOCK])
        hipLaunchKernelGGL((k_seg_block<PT, VT, LD>), dim3(cnt[BIN_BLOCK]), dim3(256), 0, s, rowptr,
                           okey, oval, lists + BIN_BLOCK * cap, cnt[BIN_BLOCK], ld, (int)sorted, hdr);
    if (cnt[BIN_GLOBAL]) {
        int32_t *tk = (int32_t *)tmp;
        VT *tv = (VT *)((char *)tmp + ((glob_elems * sizeof(int32_t) + 255) & ~uint64_t(255)));
        hipLaunchKernelGGL((k_seg_global<PT, VT, LD>), dim3(cnt[BIN_GLOBAL]), dim3(256), 0, s, rowptr,
                           okey, oval, lists + BIN_GLOBAL * cap, goff, cnt[BIN_GLOBAL], ld, (int)sorted,
                           kbits, (int)inplace, tk, tv, hdr);
    }
    return hipGetLastError();
}

inline size_t seg_tmp_bytes(uint64_t glob_elems, size_t vsize) {
    if (!glob_elems) return 0;
    return ((glob_elems * 4 + 255) & ~uint64_t(255)) + glob_elems * vsize + 256;
}

inline size_t seg_list_words(int64_t cap) { return (size_t)cap * NBINS + (size_t)cap * 2 + 4; }

}  // namespace hp
