// Batched form: many extraction / permutation requests planned and executed
// together.
//
// Every request is broken into phases of tiles (a tile = one workgroup of
// work, run by the same tile functions as the plain per-call kernels):
//   spref  plan  0 clear  1 J scatter  2 selected rows  3 J pack  4 J link
//                5 long-row chunk scan  6 count  7 rowptr scan (+ classes)
//          exec  0 clear cursors, copy rowptr  1 gather  2 short-row sort
//                3-7 class sorts (thread, wave, block, bucket split, bucket)
//   permute plan 0 clear, fill -1  1 scatter inverses + counts  2 check
//                3 rowptr scan (+ classes)
//          exec  0 copy rowptr  1 short rows (pull)
//                3-7 class sorts (pull from A)
//                (columns looked up in qinv as rows are read)
// Phases are grouped into stages (stage_of): a stage only holds phases
// whose inputs were written by earlier stages, so one launch per stage runs
// the tiles of every request of the batch, and stream order between the
// launches is the only dependency mechanism -- no workgroup ever waits for
// another one's tile, except inside a scan.  The workgroups of a launch are
// persistent and take tiles from an atomic ticket in queue order, so the
// tiles of one scan start in order and its look-back only waits on tiles
// that are already running (the same argument as the plain scan kernel).
// The exec half is captured once as a hipGraph and replayed.  Each stage
// runs a kernel compiled for that stage's phases alone (in_stage).
#include "hp_internal.hpp"
#include "hp_scan.hpp"
#include "hp_segsort.hpp"
#include "hp_spref_tiles.hpp"
#include "hp_perm_tiles.hpp"
#include "hp_tunecache.hpp"

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace hp;

namespace {

constexpr int NPH = 8;                 // phases per half
constexpr int NST = 6;                 // stages per half (at most)
constexpr int CLEAR_PER_TILE = 4096;   // words cleared / copied per tile

// Stage of each phase, per half and request kind (-1: phase not used).
//   spref plan: {0} {1,2} {3,5} {4} {6} {7}; exec: {0} {1} {2..6} {7}
//   permute plan: {0} {1} {2} {3};  exec: {0} {1} {3..6} {7}
// (the permutation's class sorts share exec stage 2 with the extraction's
// sorts rather than stage 1 with the gathers: 29.5 against 30.9 ms summed
// stage time on the 512-request batch, each stage with its own tuned shape)
// Phase 7 of exec (ranking long rows through a 128 KB LDS bitmap) is the
// only content of exec stage RANK_STAGE, which runs its own kernel.
constexpr int8_t STAGE_OF[2][2][NPH] = {
    {{0, 1, 1, 2, 3, 2, 4, 5}, {0, 1, 2, 3, -1, -1, -1, -1}},
    {{0, 1, 2, 2, 2, 2, 2, 3}, {0, 1, -1, 2, 2, 2, 2, 3}},
};
constexpr int RANK_STAGE = 3;

struct ReqDev {
    int32_t kind, sym, monotone, active;
    int64_t m, n, nnz, nI, nJ, nrows_out, ncols_out;
    const void *arow;
    const int32_t *acol;
    const void *aval;
    const int32_t *I, *J, *p, *q;
    DevHdr *hdr;
    uint32_t *zero;          // cleared in plan phase 0
    int64_t nzero;
    int32_t *fill;           // filled with -1 in plan phase 0 (permute)
    int64_t nfill;
    uint64_t *tiles0, *tiles1;
    uint8_t *mark;
    uint32_t *dm, *nm, *bm, *b2;
    int64_t nw;
    int32_t *cnt, *jpos, *Dn;
    int64_t *rs;
    int32_t *rl, *ch;
    uint8_t *big;
    int64_t *cp;
    int32_t *cursor;
    uint32_t *lists;
    int32_t *pinv, *qinv;
    void *crow_tmp;          // rowptr of the result, written by plan
    void *crow;              // exec: arena copies
    int32_t *ccol;
    void *cval;
    void *tmp;
    uint64_t *hmS, *hmB;     // spref hit masks
    uint8_t *gflag;          // spref 64-row groups left unsorted by the gather
    int64_t capb;
    uint64_t glob_elems;
    int32_t nb, nbw;
    uint32_t cls[NBINS];
    void *aws;               // assignment: its own plan workspace (host-side use only)
    size_t aws_bytes;
};

struct QEntry {
    int64_t first;       // first ticket of the entry within its stage
    int32_t req, phase;
};

union BatchSmem {
    ScanSmem scan;
    spref::GroupSmem gs[4];
    spref::GroupCore gc[4];
    SegSmemWave wave;
    SegSmemBlockBitonic block;
    SegSmemBucket bucket;
};

__device__ inline void clear_tile(int64_t tile, uint32_t *p, int64_t n) {
    const int64_t b = tile * CLEAR_PER_TILE;
    for (int64_t k = b + threadIdx.x; k < min(b + CLEAR_PER_TILE, n); k += 256) p[k] = 0u;
}
__device__ inline void fill_tile(int64_t tile, int32_t *p, int64_t n) {
    const int64_t b = tile * CLEAR_PER_TILE;
    for (int64_t k = b + threadIdx.x; k < min(b + CLEAR_PER_TILE, n); k += 256) p[k] = -1;
}
template <typename PT>
__device__ inline void copy_rowptr_tile(int64_t tile, const PT *src, PT *dst, int64_t n) {
    const int64_t b = tile * CLEAR_PER_TILE;
    for (int64_t k = b + threadIdx.x; k < min(b + CLEAR_PER_TILE, n); k += 256) dst[k] = src[k];
}
__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Whether phase ph of a request of kind k (0 extraction, 1 permutation) runs
// in stage st of half h: each stage kernel is compiled with only its own
// phases, so its register use (and hence occupancy) is that of its own
// tiles, not of the heaviest tile of the whole batch.
constexpr bool in_stage(int h, int st, int k, int ph) { return STAGE_OF[h][k][ph] == st; }
#define HP_PHASE(k, ph) case ph: if constexpr (in_stage(HALF, STAGE, k, ph))

template <typename PT, typename VT, int HALF, int STAGE>
__device__ void perm_exec_phase(int phase, int64_t tile, const ReqDev &r, BatchSmem &sm, const PT *crow, int64_t cap,
                                const uint64_t *goff, int32_t *tk, VT *tv, uint32_t *bst);

template <typename PT, typename VT, int HALF, int STAGE>
__device__ void run_tile(int phase, int64_t tile, const ReqDev &r, BatchSmem &sm) {
    uint64_t *goff = reinterpret_cast<uint64_t *>(r.lists + NBINS * (r.kind == HP_REQ_SPREF ? r.nI : r.m));
    const int64_t cap = r.kind == HP_REQ_SPREF ? r.nI : r.m;
    if constexpr (HALF == 0) {
        if (r.kind == HP_REQ_SPREF) {
            switch (phase) {
                HP_PHASE(0, 0) {
                    clear_tile(tile, r.zero, r.nzero);
                    if (tile == 0 && threadIdx.x == 0 && r.nrows_out == 0) ((PT *)r.crow_tmp)[0] = 0;
                }
                break;
                HP_PHASE(0, 1) { spref::spref_jscatter_tile(tile, r.J, r.nJ, r.n, r.mark, r.jpos, r.nm, r.hdr); }
                break;
                HP_PHASE(0, 2) {
                    spref::spref_rows_tile<PT>(tile, (const PT *)r.arow, r.I, r.nI, r.m, r.rs, r.rl, r.ch, r.big,
                                               r.hdr);
                }
                break;
                HP_PHASE(0, 3) { spref::spref_jpack_tile(tile, r.J, r.nJ, r.n, r.mark, r.bm, r.nw, r.jpos, r.Dn, r.dm); }
                break;
                HP_PHASE(0, 4) { spref::spref_jlink_tile(tile, r.J, r.nJ, r.jpos, r.Dn, r.bm, r.dm, r.b2, r.nw); }
                break;
                HP_PHASE(0, 5) {
                    scan_counts_tile<int64_t>(tile, sm.scan, r.ch, r.cp, r.nI, r.hdr, 0, r.tiles0, 0, nullptr, 0,
                                              nullptr, nullptr, nullptr);
                }
                break;
                HP_PHASE(0, 6) {
                    spref::spref_count_tile(tile, r.nbw, sm.gc, r.acol, r.n, r.rs, r.rl, r.cp, r.nI, r.b2, r.jpos,
                                            r.Dn, r.cnt, r.hmS, r.hmB, r.capb, r.hdr);
                }
                break;
                HP_PHASE(0, 7) {
                    scan_counts_tile<PT>(tile, sm.scan, r.cnt, (PT *)r.crow_tmp, r.nI, r.hdr, 1, r.tiles1, 3,
                                         r.lists, cap, goff, r.big, r.nm);
                }
                break;
            }
        } else {
            switch (phase) {
                HP_PHASE(1, 0) {
                    const int64_t nct = cdiv(r.nzero, CLEAR_PER_TILE);
                    if (tile < nct) {
                        clear_tile(tile, r.zero, r.nzero);
                        if (tile == 0 && threadIdx.x == 0 && r.nrows_out == 0) ((PT *)r.crow_tmp)[0] = 0;
                    } else {
                        fill_tile(tile - nct, r.fill, r.nfill);
                    }
                }
                break;
                HP_PHASE(1, 1) {
                    perm::perm_prepare_tile<PT>(tile, (const PT *)r.arow, r.p, r.sym ? nullptr : r.q, r.m, r.n,
                                                r.pinv, r.qinv, r.cnt, r.hdr);
                }
                break;
                HP_PHASE(1, 2) { perm::perm_check_tile(tile, r.m, r.n, r.pinv, r.qinv, !r.sym, r.hdr); }
                break;
                HP_PHASE(1, 3) {
                    scan_counts_tile<PT>(tile, sm.scan, r.cnt, (PT *)r.crow_tmp, r.m, r.hdr, 0, r.tiles0, 1, r.lists,
                                         cap, goff, nullptr, nullptr);
                }
                break;
            }
        }
        return;
    } else {
        // exec half
        const PT *crow = (const PT *)r.crow_tmp;
        int32_t *tk = (int32_t *)r.tmp;
        char *tp = (char *)r.tmp + ((r.glob_elems * sizeof(int32_t) + 255) & ~uint64_t(255));
        VT *tv = (VT *)tp;
        uint32_t *bst = (uint32_t *)(tp + ((r.glob_elems * sizeof(VT) + 255) & ~uint64_t(255)));
        if (r.kind == HP_REQ_SPREF) {
            LoadInPlace<PT, VT> ld{crow, r.ccol, (const VT *)r.cval};
            switch (phase) {
                HP_PHASE(0, 0) {
                    const int64_t nct = cdiv(r.nI, CLEAR_PER_TILE);
                    if (tile < nct) clear_tile(tile, (uint32_t *)r.cursor, r.nI);
                    else copy_rowptr_tile<PT>(tile - nct, crow, (PT *)r.crow, r.nrows_out + 1);
                }
                break;
                HP_PHASE(0, 1) {
                    spref::spref_gather_tile<PT, VT>(tile, r.nbw, sm.gs, r.acol, (const VT *)r.aval, r.n, r.rs, r.rl,
                                                     r.cp, r.nI, r.b2, r.jpos, r.Dn, crow, r.ccol, (VT *)r.cval,
                                                     r.cursor, r.hmS, r.hmB, r.capb, !r.monotone, r.gflag, r.hdr);
                }
                break;
                HP_PHASE(0, 2) {
                    sort_small_tile<PT, VT>(tile, sm.wave, crow, r.ccol, (VT *)r.cval, r.nI, ld, r.hdr, r.gflag,
                                            r.big);
                }
                break;
                HP_PHASE(0, 3) {
                    seg_thread_tile<PT, VT>(tile, crow, r.ccol, (VT *)r.cval, r.lists + BIN_THREAD * cap,
                                            r.cls[BIN_THREAD], ld, 0, r.hdr);
                }
                break;
                HP_PHASE(0, 4) {
                    seg_wave_tile<PT, VT>(tile, sm.wave, crow, r.ccol, (VT *)r.cval, r.lists + BIN_WAVE * cap,
                                          r.cls[BIN_WAVE], ld, 0, r.hdr);
                }
                break;
                HP_PHASE(0, 5) {
                    seg_bitonic_tile<PT, VT, decltype(ld), 256, BITONIC_EMAX>(
                        tile, sm.block, crow, r.ccol, (VT *)r.cval, r.lists + BIN_BLOCK * cap, r.cls[BIN_BLOCK], ld,
                        bitonic_narrow(r.ncols_out), r.hdr);
                }
                break;
                HP_PHASE(0, 6) {
                    seg_bucket_tile<PT, VT>(tile, sm.bucket, crow, r.lists + BIN_GLOBAL * cap, goff,
                                            r.cls[BIN_GLOBAL], ld, r.nb, tk, tv, bst, r.hdr);
                }
                break;
            }
        } else {
            perm_exec_phase<PT, VT, HALF, STAGE>(phase, tile, r, sm, crow, cap, goff, tk, tv, bst);
        }
    }
}

// Exec phases 0-6 of a permutation request: output row i is row p[i] of A
// with its columns looked up in qinv on the way (a pass that renames all
// columns first measured slower here: its tiles add to every batch's
// queue, while most batched matrices keep the bulk of their entries in the
// long rows that the class sorts pull).
template <typename PT, typename VT, int HALF, int STAGE>
__device__ void perm_exec_phase(int phase, int64_t tile, const ReqDev &r, BatchSmem &sm, const PT *crow, int64_t cap,
                                const uint64_t *goff, int32_t *tk, VT *tv, uint32_t *bst) {
    perm::LoadPerm<PT, VT> ld{(const PT *)r.arow, r.acol, (const VT *)r.aval, r.p, r.qinv, r.n};
    switch (phase) {
        HP_PHASE(1, 0) { copy_rowptr_tile<PT>(tile, crow, (PT *)r.crow, r.nrows_out + 1); }
        break;
        HP_PHASE(1, 1) {
            perm::perm_pull_short_tile<PT, VT>(tile, (const PT *)r.arow, r.acol, (const VT *)r.aval, r.p, r.qinv,
                                               r.n, crow, r.ccol, (VT *)r.cval, r.m, r.hdr);
        }
        break;
        HP_PHASE(1, 3) {
            seg_thread_tile<PT, VT>(tile, crow, r.ccol, (VT *)r.cval, r.lists + BIN_THREAD * cap, r.cls[BIN_THREAD],
                                    ld, 0, r.hdr);
        }
        break;
        HP_PHASE(1, 4) {
            seg_wave_tile<PT, VT>(tile, sm.wave, crow, r.ccol, (VT *)r.cval, r.lists + BIN_WAVE * cap,
                                  r.cls[BIN_WAVE], ld, 0, r.hdr);
        }
        break;
        HP_PHASE(1, 5) {
            seg_bitonic_tile<PT, VT, decltype(ld), 256, BITONIC_EMAX>(
                tile, sm.block, crow, r.ccol, (VT *)r.cval, r.lists + BIN_BLOCK * cap, r.cls[BIN_BLOCK], ld,
                bitonic_narrow(r.ncols_out), r.hdr);
        }
        break;
        HP_PHASE(1, 6) {
            seg_bucket_tile<PT, VT>(tile, sm.bucket, crow, r.lists + BIN_GLOBAL * cap, goff, r.cls[BIN_GLOBAL], ld,
                                    r.nb, tk, tv, bst, r.hdr);
        }
        break;
    }
}
#undef HP_PHASE

// Exec phase 7: rank one bucket of a long row (RANK_THREADS threads).
template <typename PT, typename VT>
__device__ void run_rank_tile(int64_t tile, const ReqDev &r, SegSmemRank &sm) {
    const PT *crow = (const PT *)r.crow_tmp;
    const int64_t cap = r.kind == HP_REQ_SPREF ? r.nI : r.m;
    const uint64_t *goff = reinterpret_cast<const uint64_t *>(r.lists + NBINS * cap);
    int32_t *tk = (int32_t *)r.tmp;
    char *tp = (char *)r.tmp + ((r.glob_elems * sizeof(int32_t) + 255) & ~uint64_t(255));
    VT *tv = (VT *)tp;
    const uint32_t *bst = (const uint32_t *)(tp + ((r.glob_elems * sizeof(VT) + 255) & ~uint64_t(255)));
    if (r.kind == HP_REQ_SPREF) {
        LoadInPlace<PT, VT> ld{crow, r.ccol, (const VT *)r.cval};
        seg_rank_tile<PT, VT>(tile, sm, crow, r.ccol, (VT *)r.cval, r.lists + BIN_GLOBAL * cap, goff,
                              r.cls[BIN_GLOBAL], ld, r.nb, tk, tv, bst, r.hdr);
    } else {
        perm::LoadPerm<PT, VT> ld{(const PT *)r.arow, r.acol, (const VT *)r.aval, r.p, r.qinv, r.n};
        seg_rank_tile<PT, VT>(tile, sm, crow, r.ccol, (VT *)r.cval, r.lists + BIN_GLOBAL * cap, goff,
                              r.cls[BIN_GLOBAL], ld, r.nb, tk, tv, bst, r.hdr);
    }
}

__global__ void k_batch_reset(uint32_t *ticket, int nticket, DevHdr *hdrs, int64_t nhdr_words) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (i < nticket) ticket[i] = 0;
    for (int64_t k = i; k < nhdr_words; k += stride) reinterpret_cast<uint32_t *>(hdrs)[k] = 0;
}

// One stage: persistent workgroups take tickets until the stage's tiles run
// out.  q holds the stage's (request, phase) entries in queue order.  A
// ticket is `per` consecutive tiles, run in order (so the tiles of a scan
// still start in increasing order), which divides the ticket atomics and
// the searches for the tile's queue entry by `per`.
template <typename PT, typename VT, int HALF, int STAGE>
__global__ __launch_bounds__(256) void k_batch_stage(const QEntry *__restrict__ q, int nq, int64_t total,
                                                    const ReqDev *__restrict__ reqs, uint32_t *ticket, int per) {
    __shared__ __align__(16) BatchSmem sm;
    __shared__ int64_t s_t;
    __shared__ int32_t s_e;
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t t = (int64_t)atomicAdd(ticket, (uint32_t)per);
            int lo = 0;
            if (t < total) {
                int hi = nq;   // last entry with first <= t
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (q[mid].first <= t) lo = mid;
                    else hi = mid;
                }
            }
            s_t = t;
            s_e = lo;
        }
        __syncthreads();
        const int64_t t0 = s_t;
        if (t0 >= total) break;
        int e = s_e;
        const int64_t t1 = t0 + per < total ? t0 + per : total;
        for (int64_t t = t0; t < t1; t++) {
            while (e + 1 < nq && q[e + 1].first <= t) e++;
            const QEntry qe = q[e];
            run_tile<PT, VT, HALF, STAGE>(qe.phase, t - qe.first, reqs[qe.req], sm);
            __syncthreads();   // LDS and s_t are reused by the next tile
        }
    }
}

// The rank stage of exec, same scheme with RANK_THREADS-wide workgroups.
template <typename PT, typename VT>
__global__ __launch_bounds__(RANK_THREADS) void k_batch_rank_stage(const QEntry *__restrict__ q, int nq,
                                                                  int64_t total, const ReqDev *__restrict__ reqs,
                                                                  uint32_t *ticket) {
    __shared__ __align__(16) SegSmemRank sm;
    __shared__ int64_t s_t;
    __shared__ int32_t s_e;
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t t = atomicAdd(ticket, 1u);
            int lo = 0;
            if (t < total) {
                int hi = nq;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (q[mid].first <= t) lo = mid;
                    else hi = mid;
                }
            }
            s_t = t;
            s_e = lo;
        }
        __syncthreads();
        const int64_t t = s_t;
        if (t >= total) break;
        const QEntry e = q[s_e];
        run_rank_tile<PT, VT>(t - e.first, reqs[e.req], sm);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct Global {
    uint32_t *ticket;    // [0, NST): plan stages, [NST, 2 NST): exec stages
    DevHdr *hdrs;
    ReqDev *reqs;
    QEntry *queue;
};

size_t req_scratch(hp_handle_t h, hp::Carve &c, const hp_request_t &rq, ReqDev &d) {
    const size_t before = c.off;
    const int64_t m = rq.A.nrows, n = rq.A.ncols;
    const size_t ps = rq.A.ptr_type == HP_IDX_I64 ? 8 : 4;
    if (rq.kind == HP_REQ_SPASGN) {
        // an assignment runs through the assignment's own kernels: its plan
        // workspace and its row pointers (written by plan, copied into the
        // arena by exec) live here
        size_t b = 0;
        hp_spasgn_workspace(h, &rq.A, &rq.B, &b);
        d.aws_bytes = b;
        d.aws = c.take<char>(b);
        d.crow_tmp = c.take<char>((size_t)(m + 1) * ps);
        return c.off - before;
    }
    if (rq.kind == HP_REQ_SPREF) {
        const int64_t nI = rq.nI, nJ = rq.nJ;
        const size_t st = scan_tiles(nI);
        d.nw = (int64_t)((((size_t)((n + 31) / 32) + 1) + 3) & ~size_t(3));
        const size_t markw = (size_t)d.nw * 8;
        // zero region: tile states (2 scans) | marks | dm | cnt | nm
        d.nzero = (int64_t)(4 * st + markw + d.nw + nI + 8 + 64 * 32);
        d.zero = c.take<uint32_t>((size_t)d.nzero);
        if (d.zero) {
            d.tiles0 = (uint64_t *)d.zero;
            d.tiles1 = (uint64_t *)d.zero + st;
            uint32_t *z = d.zero + 4 * st;
            d.mark = (uint8_t *)z;
            d.dm = z + markw;
            d.cnt = (int32_t *)(z + markw + d.nw);
            d.nm = z + markw + d.nw + nI + 8;
        }
        d.bm = c.take<uint32_t>((size_t)d.nw);
        d.b2 = c.take<uint32_t>(2 * (size_t)d.nw);
        d.jpos = c.take<int32_t>(n + 1);
        d.Dn = c.take<int32_t>(nJ + 1);
        d.rs = c.take<int64_t>(nI + 1);
        d.rl = c.take<int32_t>(nI + 1);
        d.ch = c.take<int32_t>(nI + 1);
        d.big = c.take<uint8_t>(nI + 16);
        d.cp = c.take<int64_t>(nI + 1);
        d.cursor = c.take<int32_t>(nI + 1);
        d.lists = c.take<uint32_t>(seg_list_words(nI));
        d.crow_tmp = c.take<char>((size_t)(nI + 1) * ps);
        d.capb = spref::hit_mask_big_cap(rq.A.nnz);
        d.hmS = c.take<uint64_t>((size_t)spref::hit_mask_small_words(nI));
        d.hmB = c.take<uint64_t>((size_t)d.capb * spref::SR_U);
        d.gflag = c.take<uint8_t>((size_t)((nI + WAVE - 1) / WAVE) + 1);
    } else {
        const size_t st = scan_tiles(m);
        const bool sym = rq.q == nullptr;
        d.nzero = (int64_t)(2 * st);
        d.zero = c.take<uint32_t>((size_t)d.nzero);
        if (d.zero) d.tiles0 = (uint64_t *)d.zero;
        d.nfill = m + (sym ? 0 : n);
        d.fill = c.take<int32_t>((size_t)d.nfill + 1);
        if (d.fill) {
            d.pinv = d.fill;
            d.qinv = sym ? d.fill : d.fill + m;
        }
        d.cnt = c.take<int32_t>(m + 1);
        d.lists = c.take<uint32_t>(seg_list_words(m));
        d.crow_tmp = c.take<char>((size_t)(m + 1) * ps);
    }
    return c.off - before;
}

Global global_layout(hp::Carve &c, int n) {
    Global g;
    g.ticket = c.take<uint32_t>(64);
    g.hdrs = c.take<DevHdr>((size_t)n);
    g.reqs = c.take<ReqDev>((size_t)n);
    g.queue = c.take<QEntry>((size_t)n * NPH + 8);
    return g;
}

hp_status_t check_req(hp_handle_t h, const hp_request_t &r, int k, int32_t pt, int32_t vt) {
    std::string w = "request " + std::to_string(k);
    hp_status_t st = check_csr_args(h, &r.A, w.c_str());
    if (st) return st;
    if (r.A.ptr_type != pt || r.A.val_type != vt)
        return fail(h, HP_ERR_INVALID_ARG, w + ": all requests of a batch share ptr_type and val_type");
    if (r.kind == HP_REQ_SPREF) {
        if (r.nI < 0 || r.nJ < 0 || r.nI > INT32_MAX || r.nJ > INT32_MAX)
            return fail(h, HP_ERR_INVALID_ARG, w + ": bad index-vector length");
        if ((r.nI > 0 && !r.I) || (r.nJ > 0 && !r.J)) return fail(h, HP_ERR_INVALID_ARG, w + ": I or J is NULL");
    } else if (r.kind == HP_REQ_PERMUTE) {
        if (!r.q && r.A.nrows != r.A.ncols) return fail(h, HP_ERR_SHAPE, w + ": symmetric permute needs square A");
        if (r.A.nrows > 0 && !r.p) return fail(h, HP_ERR_INVALID_ARG, w + ": p is NULL");
    } else if (r.kind == HP_REQ_SPASGN) {
        st = check_csr_args(h, &r.B, (w + " B").c_str());
        if (st) return st;
        if (r.B.ptr_type != pt || r.B.val_type != vt)
            return fail(h, HP_ERR_INVALID_ARG, w + ": B must have the batch's ptr_type and val_type");
        if (r.nI != r.B.nrows || r.nJ != r.B.ncols) return fail(h, HP_ERR_SHAPE, w + ": B must be |I| x |J|");
        if ((r.nI > 0 && !r.I) || (r.nJ > 0 && !r.J)) return fail(h, HP_ERR_INVALID_ARG, w + ": I or J is NULL");
        if (r.op < HP_OP_SECOND || r.op > HP_OP_REPLACE) return fail(h, HP_ERR_INVALID_ARG, w + ": bad op");
    } else {
        return fail(h, HP_ERR_INVALID_ARG, w + ": unknown request kind");
    }
    return HP_OK;
}

struct BatchState {
    const void *ws = nullptr;
    int n = -1;
    DevHdr *hdrs = nullptr;      // pinned readback of the request headers
    int hdr_cap = 0;
    std::vector<ReqDev> devs;
    std::vector<hp_plan_info_t> asg;   // plan infos of the assignment requests
};

std::map<hp_handle_t, BatchState> g_state;        // last plan per handle
struct GraphKey {
    const void *ws, *arena;
    std::array<int, NST> shape;   // launch shape code per stage
    int pv;
    std::array<int64_t, NST> total;
    std::array<int, NST + 1> off;
    std::vector<int64_t> asg;    // shapes of the assignment requests' launches
    bool operator<(const GraphKey &o) const {
        return std::tie(ws, arena, shape, pv, total, off, asg) <
               std::tie(o.ws, o.arena, o.shape, o.pv, o.total, o.off, o.asg);
    }
};
struct GraphEntry {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
};
std::map<hp_handle_t, std::map<GraphKey, GraphEntry>> g_graphs;
std::map<std::string, int> g_tuned;                // autotuned grid per size class
std::mutex g_mu;                                   // guards the three maps (handles may run concurrently)

int num_cus(hp_handle_t h) { return h->num_cus; }

// Phase tile counts of one request.
void plan_tiles(const hp_request_t &rq, const ReqDev &d, int64_t *nt) {
    for (int k = 0; k < NPH; k++) nt[k] = 0;
    if (rq.kind == HP_REQ_SPASGN) return;   // runs its own kernels
    if (rq.kind == HP_REQ_SPREF) {
        const int64_t ngb = cdiv(rq.nI, 4 * WAVE);
        nt[0] = cdiv(d.nzero, CLEAR_PER_TILE);
        nt[1] = cdiv(rq.nJ, 256);
        nt[2] = cdiv(rq.nI, 256);
        nt[3] = cdiv(std::max<int64_t>(rq.nJ, d.nw), 256);
        nt[4] = cdiv(std::max<int64_t>(rq.nJ, 2 * d.nw), 256);
        nt[5] = cdiv(rq.nI, SCAN_TILE);
        nt[6] = d.nbw + ngb;
        nt[7] = cdiv(rq.nI, SCAN_TILE);
    } else {
        const int64_t hi = std::max(rq.A.nrows, rq.A.ncols);
        nt[0] = cdiv(d.nzero, CLEAR_PER_TILE) + cdiv(d.nfill, CLEAR_PER_TILE);
        nt[1] = cdiv(hi, 256);
        nt[2] = cdiv(hi, 256);
        nt[3] = cdiv(rq.A.nrows, SCAN_TILE);
    }
}

void exec_tiles(const hp_request_t &rq, const ReqDev &d, int64_t *nt) {
    for (int k = 0; k < NPH; k++) nt[k] = 0;
    if (!d.active || rq.kind == HP_REQ_SPASGN) return;
    const uint32_t *c = d.cls;
    if (rq.kind == HP_REQ_SPREF) {
        const int64_t ngb = cdiv(rq.nI, 4 * WAVE);
        nt[0] = cdiv(rq.nI, CLEAR_PER_TILE) + cdiv(rq.nI + 1, CLEAR_PER_TILE);
        nt[1] = d.nbw + ngb;
        nt[2] = d.monotone ? 0 : ngb;
    } else {
        nt[0] = cdiv(rq.A.nrows + 1, CLEAR_PER_TILE);
        nt[1] = cdiv(rq.A.nrows, 256);
    }
    nt[3] = cdiv(c[BIN_THREAD], 256);
    nt[4] = cdiv(c[BIN_WAVE], 4);
    nt[5] = c[BIN_BLOCK];
    nt[6] = d.nb > 1 ? c[BIN_GLOBAL] : 0;
    nt[7] = (int64_t)c[BIN_GLOBAL] * d.nb;
}

// Stage queues of one half: the entries of every stage, phase by phase and
// request by request, with stage-relative first tickets.
struct Stages {
    std::vector<QEntry> q;        // all stages, concatenated
    int off[NST + 1] = {0};       // entries of stage s: q[off[s], off[s+1])
    int64_t total[NST] = {0};     // tiles of stage s
    int64_t tiles() const {
        int64_t t = 0;
        for (int k = 0; k < NST; k++) t += total[k];
        return t;
    }
};

void build_stages(int half, const hp_request_t *reqs, const std::vector<std::array<int64_t, NPH>> &nt, Stages &S) {
    S.q.clear();
    const int n = (int)nt.size();
    for (int st = 0; st < NST; st++) {
        S.off[st] = (int)S.q.size();
        int64_t t = 0;
        for (int ph = 0; ph < NPH; ph++)
            for (int r = 0; r < n; r++) {
                const int kind = reqs[r].kind == HP_REQ_SPREF ? 0 : 1;
                const int64_t k = nt[r][ph];
                if (k <= 0 || STAGE_OF[half][kind][ph] != st) continue;
                QEntry e;
                e.first = t;
                e.req = r;
                e.phase = ph;
                S.q.push_back(e);
                t += k;
            }
        S.total[st] = t;
    }
    S.off[NST] = (int)S.q.size();
}

// Stages that have a compiled stage kernel (launch_stage below): plan
// stages 0-5, exec stages 0-2 (exec stage RANK_STAGE has its own kernel).
constexpr bool stage_compiled(int h, int st) { return h == 0 ? st < NST : st < RANK_STAGE; }
constexpr bool stages_covered() {
    for (int h = 0; h < 2; h++)
        for (int k = 0; k < 2; k++)
            for (int ph = 0; ph < NPH; ph++) {
                const int st = STAGE_OF[h][k][ph];
                if (st >= 0 && !stage_compiled(h, st) && !(h == 1 && st == RANK_STAGE)) return false;
            }
    return true;
}
static_assert(stages_covered(), "every stage of the table needs a stage kernel");

// The stage kernel compiled for (half, stage); false if there is none.
template <typename PT, typename VT>
bool launch_stage(hipStream_t s, int half, int st, int grid, int per, const QEntry *q, int nq, int64_t tot,
                  const ReqDev *reqs, uint32_t *tk) {
#define HP_STAGE(H, ST)                                                                                      \
    case H * NST + ST:                                                                                       \
        static_assert(stage_compiled(H, ST), "stage list");                                                  \
        hipLaunchKernelGGL((k_batch_stage<PT, VT, H, ST>), dim3(grid), dim3(256), 0, s, q, nq, tot, reqs, tk, per); \
        return true;
    switch (half * NST + st) {
        HP_STAGE(0, 0) HP_STAGE(0, 1) HP_STAGE(0, 2) HP_STAGE(0, 3) HP_STAGE(0, 4) HP_STAGE(0, 5)
        HP_STAGE(1, 0) HP_STAGE(1, 1) HP_STAGE(1, 2)
        default: return false;
    }
#undef HP_STAGE
}

// Launch shape of a half: persistent workgroups per stage and tiles per
// ticket (the autotuner's two knobs).  Encoded in one int for the tuner
// cache and the graph key: grid in the low 20 bits, tiles per ticket above.
struct Shape {
    int grid, per;
    int code() const { return grid | (per << 20); }
    static Shape of(int code) { return Shape{code & 0xFFFFF, (code >> 20) > 0 ? code >> 20 : 1}; }
};

using Shapes = std::array<Shape, NST>;   // one launch shape per stage of a half

int max_grid(const Shapes &s) {
    int g = 0;
    for (const Shape &x : s) g = std::max(g, x.grid);
    return g;
}

// ev (tuning only): NST + 1 events, ev[st] recorded before stage st is
// launched (or skipped) and ev[NST] after the last.
template <typename PT, typename VT>
hipError_t launch_half(hp_handle_t h, int half, const Global &g, int n, const Stages &S, const Shapes &shape,
                       hipEvent_t *ev = nullptr) {
    hipStream_t s = h->stream;
    const int64_t hw = half == 0 ? (int64_t)n * (int64_t)(sizeof(DevHdr) / 4) : 0;
    uint32_t *tk = g.ticket + half * NST;
    hipLaunchKernelGGL(k_batch_reset, dim3(half == 0 ? 64 : 1), dim3(256), 0, s, tk, NST, g.hdrs, hw);
    for (int st = 0; st < NST; st++) {
        if (ev) hipEventRecord(ev[st], s);
        const int64_t tot = S.total[st];
        if (tot <= 0) continue;
        const Shape &sh = shape[st];
        const int gr = (int)std::min<int64_t>((tot + sh.per - 1) / sh.per, sh.grid);
        if (half == 1 && st == RANK_STAGE)   // one 1024-thread workgroup per CU at most
            hipLaunchKernelGGL((k_batch_rank_stage<PT, VT>), dim3((int)std::min<int64_t>(tot, num_cus(h))),
                               dim3(RANK_THREADS), 0, s, g.queue + S.off[st], S.off[st + 1] - S.off[st], tot,
                               g.reqs, tk + st);
        else if (!launch_stage<PT, VT>(s, half, st, gr, sh.per, g.queue + S.off[st], S.off[st + 1] - S.off[st],
                                       tot, g.reqs, tk + st))
            return hipErrorInvalidValue;
    }
    if (ev) hipEventRecord(ev[NST], s);
    return hipGetLastError();
}

// Time one half at a few launch shapes (persistent grid x tiles per ticket)
// and keep, for every stage, the shape under which that stage ran fastest
// (stages are separate launches, so each is timed between events and
// chosen on its own: a scan stage wants one tile per ticket, a streaming
// stage many).  Both halves are idempotent: every run starts from cleared
// state and rewrites the same outputs.  Each candidate runs TUNE_SAMPLES
// times and counts with its median.  Choices persist in the tuner cache
// file (hp_tunecache.hpp, one entry per stage), loaded on first use, so a
// size class is timed once per machine.
constexpr int TUNE_SAMPLES = 3;
// Tiles per ticket without tuning (4 workgroups per CU), per half and
// stage: what the tuner picked for the 512-request batch (one for the
// stages holding the rowptr and chunk scans).
constexpr int DEFAULT_PER[2][NST] = {{16, 4, 4, 1, 1, 1}, {4, 16, 16, 1, 1, 1}};
bool g_cache_loaded = false;

std::string stage_key(const std::string &key, int st) { return key + "/s" + std::to_string(st); }

template <typename PT, typename VT>
Shapes tune_shape(hp_handle_t h, int half, const Global &g, int n, const Stages &S, const std::string &key,
                  bool tune) {
    const int cus = num_cus(h);
    Shapes best;
    for (int st = 0; st < NST; st++) best[st] = Shape{4 * cus, DEFAULT_PER[half][st]};
    if (!tune || getenv("HP_NO_TUNE")) return best;
    const std::string path = tune_cache_path();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_cache_loaded) {
            for (auto &kv : tune_cache_load(path)) g_tuned.emplace(kv.first, kv.second);
            g_cache_loaded = true;
        }
        bool all = true;
        Shapes got = best;
        for (int st = 0; st < NST && all; st++) {
            auto it = g_tuned.find(stage_key(key, st));
            if (it == g_tuned.end()) all = false;
            else got[st] = Shape::of(it->second);
        }
        if (all) return got;
    }
    std::vector<Shape> cand;
    for (int gm : {1, 2, 4, 8, 16})
        for (int per : {1, 4, 16, 64}) cand.push_back(Shape{gm * cus, per});
    std::array<float, NST> best_ms;
    best_ms.fill(1e30f);
    bool ok = true;
    hipEvent_t ev[NST + 1];
    for (auto &e : ev) hipEventCreate(&e);
    for (const Shape &c : cand) {
        Shapes all;
        all.fill(c);
        float t[NST][TUNE_SAMPLES];
        for (int r = 0; r < TUNE_SAMPLES && ok; r++) {
            launch_half<PT, VT>(h, half, g, n, S, all, ev);
            if (wait_event(h, ev[NST], "batch tuner") != HP_OK) ok = false;
            for (int st = 0; st < NST; st++) {
                t[st][r] = 0;
                hipEventElapsedTime(&t[st][r], ev[st], ev[st + 1]);
            }
        }
        if (!ok) break;
        for (int st = 0; st < NST; st++) {
            std::sort(t[st], t[st] + TUNE_SAMPLES);
            const float med = t[st][TUNE_SAMPLES / 2];
            if (med < best_ms[st]) {
                best_ms[st] = med;
                best[st] = c;
            }
        }
    }
    for (auto &e : ev) hipEventDestroy(e);
    std::lock_guard<std::mutex> lk(g_mu);
    for (int st = 0; st < NST; st++) {
        g_tuned[stage_key(key, st)] = best[st].code();
        if (ok) tune_cache_store(path, stage_key(key, st), best[st].code());
    }
    return best;
}

// Size class of a half: device (compute units), index and value types, and
// log2 of its tile count.
std::string size_class(hp_handle_t h, const char *half, int32_t pt, int32_t vt, int64_t total) {
    int lg = 0;
    while ((int64_t(1) << lg) < total) lg++;
    char buf[96];
    snprintf(buf, sizeof buf, "batch2/cu%d/%s/p%d/v%d/t2^%d", num_cus(h), half, pt, vt, lg);
    return buf;
}

__global__ void k_copy_words(uint32_t *__restrict__ dst, const uint32_t *__restrict__ src, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

// The assignment requests of a batch: row pointers from the plan's copy in
// the workspace into the arena (a kernel, so that a captured graph holds no
// copy node), then the assignment's own exec kernels on the handle's stream.
hp_status_t run_assignments(hp_handle_t h, hp_request_t *reqs, int n, const std::vector<ReqDev> &devs,
                            const std::vector<hp_plan_info_t> &asg) {
    for (int k = 0; k < n; k++) {
        hp_request_t &r = reqs[k];
        const ReqDev &d = devs[k];
        if (r.kind != HP_REQ_SPASGN || !d.active) continue;
        const int64_t words = (r.A.nrows + 1) * (r.A.ptr_type == HP_IDX_I64 ? 2 : 1);
        const int grid = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (words + 255) / 256));
        hipLaunchKernelGGL(k_copy_words, dim3(grid), dim3(256), 0, h->stream, (uint32_t *)d.crow,
                           (const uint32_t *)d.crow_tmp, words);
        if (hipError_t e = hipGetLastError()) return hip_check(h, e, "batch assignment rowptr copy");
        const hp_status_t st = hp_spasgn_exec(h, &r.A, &r.B, r.I, r.J, (hp_asgn_op_t)r.op, &r.C, d.aws, d.aws_bytes,
                                              &asg[k], d.tmp, asg[k].exec_ws_bytes);
        if (st) return st;
    }
    return HP_OK;
}

template <typename PT, typename VT>
hp_status_t batch_plan_t(hp_handle_t h, hp_request_t *reqs, int n, void *ws, size_t ws_bytes,
                         hp_batch_info_t *info) {
    hp::Carve need(nullptr);
    global_layout(need, n);
    std::vector<ReqDev> devs(n);
    for (int k = 0; k < n; k++) req_scratch(h, need, reqs[k], devs[k]);
    if (!ws || ws_bytes < need.size()) return fail(h, HP_ERR_WORKSPACE, "batch workspace too small");
    hp::Carve c(ws);
    Global g = global_layout(c, n);
    const int cus = num_cus(h);
    for (int k = 0; k < n; k++) {
        ReqDev &d = devs[k];
        d = ReqDev{};
        req_scratch(h, c, reqs[k], d);
        const hp_request_t &r = reqs[k];
        d.kind = r.kind;
        d.sym = r.q == nullptr;
        d.active = 1;
        d.m = r.A.nrows;
        d.n = r.A.ncols;
        d.nnz = r.A.nnz;
        d.arow = r.A.rowptr;
        d.acol = r.A.col;
        d.aval = r.A.val;
        d.I = r.I;
        d.J = r.J;
        d.p = r.p;
        d.q = r.q;
        d.nI = r.kind == HP_REQ_SPREF ? r.nI : 0;
        d.nJ = r.kind == HP_REQ_SPREF ? r.nJ : 0;
        d.nrows_out = r.kind == HP_REQ_SPREF ? r.nI : r.A.nrows;
        d.ncols_out = r.kind == HP_REQ_SPREF ? r.nJ : r.A.ncols;
        d.hdr = g.hdrs + k;
        // long-row workers: about one per 2^20 nonzeros of A, at most one per CU
        d.nbw = (r.kind == HP_REQ_SPREF && r.nI > 0)
                    ? (int32_t)std::min<int64_t>(cus, std::max<int64_t>(1, r.A.nnz >> 20)) : 0;
    }
    std::vector<std::array<int64_t, NPH>> nt(n);
    for (int k = 0; k < n; k++) plan_tiles(reqs[k], devs[k], nt[k].data());
    Stages S;
    build_stages(0, reqs, nt, S);
    const int64_t total = S.tiles();
    hipStream_t s = h->stream;
    hipError_t e = hipMemcpyAsync(g.reqs, devs.data(), sizeof(ReqDev) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !S.q.empty())
        e = hipMemcpyAsync(g.queue, S.q.data(), sizeof(QEntry) * S.q.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_check(h, e, "batch plan upload");
    const std::string key = size_class(h, "plan", reqs[0].A.ptr_type, reqs[0].A.val_type, total);
    const Shapes shape = tune_shape<PT, VT>(h, 0, g, n, S, key, !(info && (info->flags & HP_BATCH_NO_TUNE)));
    stage_begin(h);
    e = launch_half<PT, VT>(h, 0, g, n, S, shape);
    stage_mark(h, "batch.plan");
    BatchState *bsp;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        bsp = &g_state[h];   // map nodes are stable; one handle is used by one thread at a time
    }
    BatchState &bs = *bsp;
    if (e == hipSuccess && bs.hdr_cap < n) {
        if (bs.hdrs) hipHostFree(bs.hdrs);
        bs.hdrs = nullptr;
        bs.hdr_cap = 0;
        e = hipHostMalloc((void **)&bs.hdrs, sizeof(DevHdr) * n, hipHostMallocDefault);
        if (e == hipSuccess) bs.hdr_cap = n;
        else bs.hdrs = nullptr;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(bs.hdrs, g.hdrs, sizeof(DevHdr) * n, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_check(h, e, "batch plan");
    if (hp_status_t ws = wait_stream(h, "batch plan")) return ws;
    // assignment requests: the assignment's own plan on the same stream,
    // row pointers into the batch workspace (exec copies them to the arena)
    std::vector<hp_plan_info_t> asg(n);
    std::vector<hp_status_t> asg_st(n, HP_OK);
    std::vector<int64_t> asg_nnz(n, 0);
    for (int k = 0; k < n; k++) {
        hp_request_t &r = reqs[k];
        if (r.kind != HP_REQ_SPASGN) continue;
        hp_csr_t Ct{};
        Ct.nrows = r.A.nrows;
        Ct.ncols = r.A.ncols;
        Ct.ptr_type = r.A.ptr_type;
        Ct.val_type = r.A.val_type;
        Ct.rowptr = devs[k].crow_tmp;
        asg_st[k] = hp_spasgn_plan(h, &r.A, &r.B, r.I, r.J, (hp_asgn_op_t)r.op, &Ct, devs[k].aws, devs[k].aws_bytes,
                                   &asg[k]);
        asg_nnz[k] = Ct.nnz;
    }
    // per-request results and the arena
    const size_t ps = sizeof(PT), vs = sizeof(VT);
    size_t arena = 0;
    int failed = 0;
    int64_t nnz_total = 0;
    for (int k = 0; k < n; k++) {
        hp_request_t &r = reqs[k];
        ReqDev &d = devs[k];
        if (r.kind == HP_REQ_SPASGN) {
            const hp_status_t st = asg_st[k];
            r.C = hp_csr_t{};
            r.C.nrows = r.A.nrows;
            r.C.ncols = r.A.ncols;
            r.C.ptr_type = r.A.ptr_type;
            r.C.val_type = r.A.val_type;
            r.C.nnz = st == HP_OK ? asg_nnz[k] : 0;
            r.status = st;
            d.active = st == HP_OK;
            if (st != HP_OK) {
                failed++;
                continue;
            }
            nnz_total += r.C.nnz;
            arena = (arena + 255) & ~size_t(255);
            arena += (size_t)(r.A.nrows + 1) * ps + 256;
            arena = (arena + 255) & ~size_t(255);
            arena += (size_t)r.C.nnz * 4 + 256;
            arena = (arena + 255) & ~size_t(255);
            arena += (size_t)r.C.nnz * vs + 256;
            arena = (arena + 255) & ~size_t(255);
            arena += asg[k].exec_ws_bytes + 256;
            continue;
        }
        const DevHdr &H = bs.hdrs[k];
        hp_status_t st = status_from_err(h, H.err, "batch request");
        r.C = hp_csr_t{};
        r.C.nrows = d.nrows_out;
        r.C.ncols = d.ncols_out;
        r.C.ptr_type = r.A.ptr_type;
        r.C.val_type = r.A.val_type;
        const int slot = r.kind == HP_REQ_SPREF ? 1 : 0;
        r.C.nnz = st == HP_OK ? (int64_t)H.total[slot] : 0;
        d.monotone = r.kind == HP_REQ_SPREF ? ((H.flags & F_NOT_MONOTONE) ? 0 : 1) : 0;
        d.glob_elems = H.bin_elems[BIN_GLOBAL];
        d.nb = seg_nbuckets(d.ncols_out);
        for (int b = 0; b < NBINS; b++) d.cls[b] = H.bin_cnt[b];
        r.status = st;
        d.active = st == HP_OK;
        if (st != HP_OK) {
            failed++;
            continue;
        }
        nnz_total += r.C.nnz;
        arena = (arena + 255) & ~size_t(255);
        arena += (size_t)(d.nrows_out + 1) * ps + 256;
        arena = (arena + 255) & ~size_t(255);
        arena += (size_t)r.C.nnz * 4 + 256;
        arena = (arena + 255) & ~size_t(255);
        arena += (size_t)r.C.nnz * vs + 256;
        arena = (arena + 255) & ~size_t(255);
        arena += seg_tmp_bytes(d.glob_elems, d.cls[BIN_GLOBAL], vs, d.ncols_out);
    }
    bs.ws = ws;
    bs.n = n;
    bs.devs = devs;
    bs.asg = asg;
    if (info) {
        const int32_t flags = info->flags;   // caller's option bits survive the plan
        *info = hp_batch_info_t{};
        info->flags = flags;
        info->arena_bytes = arena + 256;
        info->nnz_total = nnz_total;
        info->failed = failed;
        info->grid_plan = max_grid(shape);
        info->tiles_plan = total;
    }
    return HP_OK;
}

template <typename PT, typename VT>
hp_status_t batch_exec_t(hp_handle_t h, hp_request_t *reqs, int n, void *ws, size_t ws_bytes,
                         hp_batch_info_t *info, void *arena, size_t arena_bytes) {
    BatchState *bsp = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_state.find(h);
        if (it != g_state.end()) bsp = &it->second;
    }
    if (!bsp || bsp->ws != ws || bsp->n != n)
        return fail(h, HP_ERR_INVALID_ARG, "hp_batch_exec needs the preceding hp_batch_plan of this batch");
    BatchState &bs = *bsp;
    if (!info || arena_bytes < info->arena_bytes || (info->arena_bytes > 256 && !arena))
        return fail(h, HP_ERR_WORKSPACE, "batch arena too small");
    hp::Carve c(ws);
    Global g = global_layout(c, n);
    std::vector<ReqDev> devs = bs.devs;
    const size_t ps = sizeof(PT), vs = sizeof(VT);
    hp::Carve a(arena);
    for (int k = 0; k < n; k++) {
        ReqDev &d = devs[k];
        hp_request_t &r = reqs[k];
        if (!d.active) continue;
        d.crow = a.take<char>((size_t)(d.nrows_out + 1) * ps);
        d.ccol = a.take<int32_t>((size_t)r.C.nnz);
        d.cval = a.take<char>((size_t)r.C.nnz * vs);
        d.tmp = r.kind == HP_REQ_SPASGN ? a.take<char>(bs.asg[k].exec_ws_bytes)
                                        : a.take<char>(seg_tmp_bytes(d.glob_elems, d.cls[BIN_GLOBAL], vs, d.ncols_out));
        r.C.rowptr = d.crow;
        r.C.col = d.ccol;
        r.C.val = d.cval;
    }
    if (a.size() > arena_bytes) return fail(h, HP_ERR_WORKSPACE, "batch arena too small");
    std::vector<std::array<int64_t, NPH>> nt(n);
    for (int k = 0; k < n; k++) exec_tiles(reqs[k], devs[k], nt[k].data());
    Stages S;
    build_stages(1, reqs, nt, S);
    const int64_t total = S.tiles();
    hipStream_t s = h->stream;
    hipError_t e = hipMemcpyAsync(g.reqs, devs.data(), sizeof(ReqDev) * n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !S.q.empty())
        e = hipMemcpyAsync(g.queue, S.q.data(), sizeof(QEntry) * S.q.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_check(h, e, "batch exec upload");
    const std::string key = size_class(h, "exec", reqs[0].A.ptr_type, reqs[0].A.val_type, total);
    const Shapes shape = tune_shape<PT, VT>(h, 1, g, n, S, key, !(info->flags & HP_BATCH_NO_TUNE));
    // exec runs from a captured graph, replayed for any batch with the same
    // workspace, arena, grid and stage shapes (queue and request records are
    // uploaded before every launch)
    GraphKey gk{ws, arena, {}, (int)(ps * 16 + vs), {}, {}, {}};
    for (int st = 0; st < NST; st++) gk.shape[st] = shape[st].code();
    std::copy(S.total, S.total + NST, gk.total.begin());
    std::copy(S.off, S.off + NST + 1, gk.off.begin());
    for (int k = 0; k < n; k++) {
        if (reqs[k].kind != HP_REQ_SPASGN || !devs[k].active) continue;
        const hp_plan_info_t &pi = bs.asg[k];
        gk.asg.insert(gk.asg.end(), {k, pi.nnz_out, (int64_t)pi.exec_ws_bytes, pi.map_monotone, pi.op,
                                     (int64_t)reqs[k].op});
        for (int b = 0; b < 4; b++) gk.asg.insert(gk.asg.end(), {pi.rows_sorted[b], pi.class_elems[b], pi.aux[b]});
    }
    stage_begin(h);
    if (info->flags & HP_BATCH_NO_GRAPH) {
        e = launch_half<PT, VT>(h, 1, g, n, S, shape);
        if (e == hipSuccess) {
            if (hp_status_t as = run_assignments(h, reqs, n, devs, bs.asg)) return as;
        }
        stage_mark(h, "batch.exec");
        if (e != hipSuccess) return hip_check(h, e, "batch exec");
        info->tiles_exec = total;
        info->grid_exec = max_grid(shape);
        return HP_OK;
    }
    GraphEntry *gep;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto &graphs = g_graphs[h];
        if (graphs.size() >= 64 && !graphs.count(gk)) {
            // bound the cache: drop every graph of this handle (its stream is idle
            // only after the last launch, so synchronise before destroying)
            hipStreamSynchronize(s);
            for (auto &kv : graphs) {
                if (kv.second.ge) hipGraphExecDestroy(kv.second.ge);
                if (kv.second.g) hipGraphDestroy(kv.second.g);
            }
            graphs.clear();
        }
        gep = &graphs[gk];
    }
    GraphEntry &ge = *gep;
    if (!ge.ge) {
        hipStream_t cs;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) {
            hipStream_t keep = h->stream;
            h->stream = cs;
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t le = launch_half<PT, VT>(h, 1, g, n, S, shape);
                const hp_status_t as = le == hipSuccess ? run_assignments(h, reqs, n, devs, bs.asg) : HP_OK;
                e = hipStreamEndCapture(cs, &ge.g);
                if (e == hipSuccess) e = le;
                if (e == hipSuccess && as != HP_OK) e = hipErrorUnknown;
            }
            h->stream = keep;
            hipStreamDestroy(cs);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&ge.ge, ge.g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            ge.ge = nullptr;
            return hip_check(h, e, "batch exec graph capture");
        }
    }
    e = hipGraphLaunch(ge.ge, s);
    stage_mark(h, "batch.exec");
    if (e != hipSuccess) return hip_check(h, e, "batch exec");
    if (info) {
        info->tiles_exec = total;
        info->grid_exec = max_grid(shape);
    }
    return HP_OK;
}

}  // namespace

namespace hp {
// Drops the per-handle batch state and graphs (called by hp_destroy).
void batch_release_handle(hp_handle_t h) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto st = g_state.find(h);
    if (st != g_state.end()) {
        if (st->second.hdrs) hipHostFree(st->second.hdrs);
        g_state.erase(st);
    }
    auto it = g_graphs.find(h);
    if (it != g_graphs.end()) {
        for (auto &kv : it->second) {
            if (kv.second.ge) hipGraphExecDestroy(kv.second.ge);
            if (kv.second.g) hipGraphDestroy(kv.second.g);
        }
        g_graphs.erase(it);
    }
}
}  // namespace hp

extern "C" hp_status_t hp_batch_workspace(hp_handle_t h, const hp_request_t *reqs, int n, size_t *bytes) {
    if (!h || !bytes || n < 0 || (n > 0 && !reqs)) return HP_ERR_INVALID_ARG;
    hp::Carve c(nullptr);
    global_layout(c, n);
    for (int k = 0; k < n; k++) {
        hp_status_t st = check_req(h, reqs[k], k, reqs[0].A.ptr_type, reqs[0].A.val_type);
        if (st) return st;
        ReqDev d{};
        req_scratch(h, c, reqs[k], d);
    }
    *bytes = c.size();
    return HP_OK;
}

extern "C" hp_status_t hp_batch_plan(hp_handle_t h, hp_request_t *reqs, int n, void *ws, size_t ws_bytes,
                                     hp_batch_info_t *info) {
    if (!h || n < 0 || (n > 0 && !reqs)) return HP_ERR_INVALID_ARG;
    if (n == 0) {
        if (info) *info = hp_batch_info_t{};
        return HP_OK;
    }
    for (int k = 0; k < n; k++) {
        hp_status_t st = check_req(h, reqs[k], k, reqs[0].A.ptr_type, reqs[0].A.val_type);
        if (st) return st;
    }
    const bool p64 = reqs[0].A.ptr_type == HP_IDX_I64, v64 = reqs[0].A.val_type == HP_VAL_F64;
    if (!p64 && !v64) return batch_plan_t<int32_t, uint32_t>(h, reqs, n, ws, ws_bytes, info);
    if (!p64 && v64) return batch_plan_t<int32_t, uint64_t>(h, reqs, n, ws, ws_bytes, info);
    if (p64 && !v64) return batch_plan_t<int64_t, uint32_t>(h, reqs, n, ws, ws_bytes, info);
    return batch_plan_t<int64_t, uint64_t>(h, reqs, n, ws, ws_bytes, info);
}

extern "C" hp_status_t hp_batch_exec(hp_handle_t h, hp_request_t *reqs, int n, void *ws, size_t ws_bytes,
                                     hp_batch_info_t *info, void *arena, size_t arena_bytes) {
    if (!h || n < 0 || (n > 0 && !reqs)) return HP_ERR_INVALID_ARG;
    if (n == 0) return HP_OK;
    const bool p64 = reqs[0].A.ptr_type == HP_IDX_I64, v64 = reqs[0].A.val_type == HP_VAL_F64;
    if (!p64 && !v64) return batch_exec_t<int32_t, uint32_t>(h, reqs, n, ws, ws_bytes, info, arena, arena_bytes);
    if (!p64 && v64) return batch_exec_t<int32_t, uint64_t>(h, reqs, n, ws, ws_bytes, info, arena, arena_bytes);
    if (p64 && !v64) return batch_exec_t<int64_t, uint32_t>(h, reqs, n, ws, ws_bytes, info, arena, arena_bytes);
    return batch_exec_t<int64_t, uint64_t>(h, reqs, n, ws, ws_bytes, info, arena, arena_bytes);
}
