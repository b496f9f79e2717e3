// spasgn: C = A with A(I, J) = B (paper Sec. 2.3; HipAssign, Sec. 4.7).
//
// B is expanded to B'[I[i], J[j]] = B[i, j] (stored entries only) and added
// to A with a user-chosen addition (the Add step of Sec. 4.7):
//   SECOND  where both hold an entry B's value wins (select-second),
//   PLUS    where both hold an entry the values are added,
//   REPLACE every A entry inside I x J is dropped first (block replace).
// On one GPU the Identify/Exchange/Build of B' collapses into per-row work:
//   plan : fill -1, scatter rowinv[I[i]] = i and colinv[J[j]] = j, check
//          that I and J repeat no index (Sec. 2.3 requires distinct ones);
//          count every output row: rows outside I keep A's length, rows in
//          I count the surviving A entries plus B's row; scan into rowptr.
//   exec : rows outside I  streaming copy, 64 rows per wavefront;
//          rows in I       one wavefront per row stages A's columns and B's
//                          mapped columns in LDS, resolves collisions and
//                          writes the row sorted (merge by co-rank when the
//                          mapped B row is increasing, rank by count
//                          otherwise).  Rows longer than AS_WCAP are written
//                          unsorted and sorted by the segmented sort.
#include "hp_internal.hpp"
#include "hp_segsort.hpp"
#include "hp_perm_tiles.hpp"

using namespace hp;

namespace {

constexpr int AS_WCAP = 256;   // A + B entries one wavefront resolves in LDS
// Rows of I whose mapped B columns do not increase (J out of order) are
// placed by counting, O(L) per entry, only up to this many A + B entries;
// longer ones are written unsorted and ordered by the class sorts (the
// count pass flags them).
constexpr int64_t AS_RANK_MAX = 64;
// Rows outside I longer than ASG_LONG are not copied by the wavefront that
// owns their 64-row group (hub rows at neighbouring ids would serialise on
// it) but by a workgroup of their own, and rows longer than ASG_HUGE by
// every workgroup together.
constexpr int64_t ASG_LONG = 512;
constexpr int64_t ASG_HUGE = 65536;

constexpr int FSUM_SLOTS = 64;   // spread partial sums of k_fused_counts (one 64-byte line each)
// The one-wavefront-a-row merge (k_asg_merge_row) holds B's row in AS_MQ
// 64-wide register slices; in the fused form it also sorts the merged row
// when it has at most AS_MQ * WAVE entries.
constexpr int AS_MQ = 4;

struct AsgLayout {
    DevHdr *hdr;
    uint64_t *tiles;
    int32_t *rowinv, *colinv, *cnt;
    int32_t *pinv, *qinv, *cnt_out;   // fused assign-and-permute only
    uint8_t *fflag;                   // fused: 2 merged row, 1 copied row the sort pass pulls, 0 done
    unsigned long long *fsum;         // fused: spread partial sums of the counts pass
    uint8_t *force;
    uint32_t *lists;
    int32_t *llist;        // rows of B whose A row is too long for the one-thread count
    uint32_t *lcount;      // [0]: llist entries, [1]: rlong entries, [2]: rhuge entries, [3]: hlist entries
    int32_t *hlist;        // rows of I with more than AS_HUGE A + B entries (the whole grid each)
    uint32_t *hcur;        // exec: placement cursor of the kept A entries of each hlist row
    int64_t hcap;
    int32_t *rlong;        // rows outside I of ASG_LONG+1..ASG_HUGE entries (a workgroup each)
    int32_t *rhuge;        // rows outside I longer than ASG_HUGE (the whole grid each)
};

// The fused form always reserves qinv, so its workspace size does not depend
// on q; the symmetric form (q null) then uses pinv for both maps.
// Rows of I with more than AS_HUGE A + B entries are merged (and counted) by
// every workgroup together instead of one wavefront: a single wavefront
// walking a hub row's tens of thousands of entries, each with a binary
// search of the other row, was the tail of the whole pass.  At most
// (nnz(A) + nnz(B)) / AS_HUGE rows qualify.
constexpr int64_t AS_HUGE = 4096;

AsgLayout asg_layout(Carve &c, int64_t m, int64_t n, int64_t nnzA, int64_t nnzB, bool fused = false,
                     bool sym = false) {
    AsgLayout L;
    L.pinv = L.qinv = L.cnt_out = nullptr;
    L.fflag = nullptr;
    L.fsum = nullptr;
    L.hdr = c.take<DevHdr>(1);
    L.tiles = c.take<uint64_t>(scan_tiles(m));
    L.rowinv = c.take<int32_t>(m + 1);
    L.colinv = c.take<int32_t>(n + 1);
    L.cnt = c.take<int32_t>(m + 1);
    L.force = c.take<uint8_t>(m + 16);
    L.lists = c.take<uint32_t>(seg_list_words(m));
    L.llist = c.take<int32_t>(m + 1);
    L.lcount = c.take<uint32_t>(64);
    L.rlong = c.take<int32_t>(std::min<int64_t>(m, nnzA / ASG_LONG) + 1);
    L.rhuge = c.take<int32_t>(std::min<int64_t>(m, nnzA / ASG_HUGE) + 1);
    L.hcap = std::min<int64_t>(m, (nnzA + nnzB) / AS_HUGE) + 1;
    L.hlist = c.take<int32_t>(L.hcap);
    L.hcur = c.take<uint32_t>(L.hcap);
    if (fused) {
        L.pinv = c.take<int32_t>(m + 1);
        L.qinv = c.take<int32_t>(n + 1);
        L.cnt_out = c.take<int32_t>(m + 1);
        L.fflag = c.take<uint8_t>(m + 16);
        L.fsum = c.take<unsigned long long>(FSUM_SLOTS * 2 * 8);
        if (sym) L.qinv = L.pinv;
    }
    return L;
}

// Fused form, after the counts: the rows of I get the top bit of their
// count (the sort pass must order them whatever their length), and
// selfs[r] = 1 when the exec's merge sorts the row itself: selfsort (the
// one-wavefront-a-row merge runs) and at most WAVE A entries and AS_MQ *
// WAVE entries after the merge, the rows that merge keeps in registers.
// selfs is the count pass's force array, which the fused form has no
// other use for.
template <typename PT>
__global__ __launch_bounds__(256) void k_fused_mark(const int32_t *__restrict__ I, int64_t nI, int64_t m,
                                                   const PT *__restrict__ arow, int32_t *cnt, uint8_t *selfs,
                                                   int selfsort, const DevHdr *hdr) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nI || hdr->err) return;
    const int32_t r = I[t];
    if (r >= 0 && r < m) {
        const int32_t c = cnt[r];
        cnt[r] = (int32_t)((uint32_t)c | 0x80000000u);
        selfs[r] = (selfsort && (int64_t)(arow[r + 1] - arow[r]) <= WAVE && c <= AS_MQ * WAVE) ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_fused_check(int64_t m, int64_t n, const int32_t *__restrict__ pinv,
                                                    const int32_t *__restrict__ qinv, bool general, DevHdr *hdr) {
    perm::perm_check4_tile(blockIdx.x, m, n, pinv, qinv, general, hdr);
}

// Output row i holds row p[i] of the assignment result: scatter the
// inverse permutations (pinv[p[i]] = i, qinv[q[i]] = i) and take the row's
// count.  The sort pass orders the merged rows (rows of I, flag 2) in place
// and fills rows outside I longer than THREAD_MAX (flag 1) straight from A;
// shorter rows outside I (flag 0) are pulled by k_fused_fill_short; merged
// rows the merge sorts itself (flag 3) are left alone.
__global__ __launch_bounds__(256) void k_fused_counts(const int32_t *__restrict__ p, const int32_t *__restrict__ q,
                                                     int64_t m, int64_t n, const int32_t *__restrict__ cnt,
                                                     const uint8_t *__restrict__ selfs, int32_t *pinv,
                                                     int32_t *qinv, int32_t *cnt_out, uint8_t *fflag,
                                                     unsigned long long *fsum, DevHdr *hdr) {
    __shared__ uint64_t s_part[2][256 / WAVE];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    uint64_t rest = 0, shrt = 0;
    if (i < m) {
        const int32_t r = p[i];
        const bool ok = r >= 0 && r < m;
        if (!ok) atomicOr(&hdr->err, E_RANGE);   // error path only
        else pinv[r] = (int32_t)i;
        const uint32_t c = ok ? (uint32_t)cnt[r] : 0u;
        const int32_t len = (int32_t)(c & 0x7FFFFFFFu);
        cnt_out[i] = len;
        const uint8_t f = (c >> 31) ? (selfs[r] ? 3 : 2) : (len > (int32_t)THREAD_MAX ? 1 : 0);
        fflag[i] = f;
        if (f < 2) rest = (uint64_t)len;
        if (f == 0 && len <= 4) shrt = (uint64_t)len;
    }
    // entries of the rows outside I and of those with at most 4 entries
    // (whether the exec's row slots pay): one partial per workgroup, added
    // into one of FSUM_SLOTS spread slots (a single counter for every
    // workgroup would serialise them), summed by k_fused_sum
    rest = wave_sum(rest);
    shrt = wave_sum(shrt);
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        s_part[0][w] = rest;
        s_part[1][w] = shrt;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint64_t t = 0;
        for (int k = 0; k < 256 / WAVE; k++) t += s_part[threadIdx.x][k];
        if (t) atomicAdd(&fsum[((blockIdx.x % FSUM_SLOTS) * 2 + threadIdx.x) * 8], (unsigned long long)t);
    }
    if (q && i < n) {
        const int32_t c = q[i];
        if (c < 0 || c >= n) atomicOr(&hdr->err, E_RANGE);
        else qinv[c] = (int32_t)i;
    }
}

// hdr->aux[0] and aux[1]: the sums of the spread partials of k_fused_counts
// (one wavefront).
__global__ __launch_bounds__(64) void k_fused_sum(const unsigned long long *__restrict__ fsum, DevHdr *hdr) {
    const int l = threadIdx.x;
    uint64_t a = 0, b = 0;
    if (l < FSUM_SLOTS) {
        a = fsum[(l * 2 + 0) * 8];
        b = fsum[(l * 2 + 1) * 8];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (l == 0) {
        hdr->aux[0] = a;
        hdr->aux[1] = b;
    }
}

// qinv[q[j]] = j, a launch of its own (mixing this scatter with the row
// gathers of k_fused_counts in one kernel is slower than the two apart).
__global__ __launch_bounds__(256) void k_fused_qinv(const int32_t *__restrict__ q, int64_t n, int32_t *qinv,
                                                   DevHdr *hdr) {
    perm::perm_qinv_tile(blockIdx.x, q, n, qinv, hdr);
}

__global__ __launch_bounds__(256) void k_asg_inv(const int32_t *__restrict__ I, int64_t nI,
                                                const int32_t *__restrict__ J, int64_t nJ, int64_t m,
                                                int64_t n, int32_t *rowinv, int32_t *colinv,
                                                DevHdr *hdr) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < nI) {
        const int32_t r = I[t];
        if (r < 0 || r >= m) atomicOr(&hdr->err, E_RANGE);   // error path only
        else rowinv[r] = (int32_t)t;
    }
    bool gap = false;
    if (t < nJ) {
        const int32_t c = J[t];
        if (c < 0 || c >= n) atomicOr(&hdr->err, E_RANGE);
        else colinv[c] = (int32_t)t;
        gap = t + 1 < nJ && J[t + 1] != c + 1;
    }
    // J a contiguous range? (then the merge maps B's columns without a
    // lookup); the flag is read first so that few blocks write it
    if (__syncthreads_or(gap) && threadIdx.x == 0 && !(ld_agent(&hdr->flags) & F_NOT_RANGE))
        atomicOr(&hdr->flags, F_NOT_RANGE);
}

// A repeated index leaves one of its positions unrecorded.
__global__ __launch_bounds__(256) void k_asg_dup(const int32_t *__restrict__ I, int64_t nI,
                                                const int32_t *__restrict__ J, int64_t nJ, int64_t m,
                                                int64_t n, const int32_t *__restrict__ rowinv,
                                                const int32_t *__restrict__ colinv, DevHdr *hdr) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool dup = false;
    if (t < nI) {
        const int32_t r = I[t];
        dup |= r >= 0 && r < m && rowinv[r] != (int32_t)t;
    }
    if (t < nJ) {
        const int32_t c = J[t];
        dup |= c >= 0 && c < n && colinv[c] != (int32_t)t;
    }
    if (dup) atomicOr(&hdr->err, E_DUP);   // error path only
}

template <typename PT>
__global__ __launch_bounds__(256) void k_asg_count_rest(const PT *__restrict__ arow, int64_t m,
                                                       const int32_t *__restrict__ rowinv, int32_t *cnt,
                                                       uint8_t *force, int32_t *rlong, int32_t *rhuge,
                                                       uint32_t *nlong, const DevHdr *hdr) {
    if (hdr->err) return;
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool rest = r < m && rowinv[r] < 0;
    const int64_t len = rest ? (int64_t)(arow[r + 1] - arow[r]) : 0;
    if (rest) {
        cnt[r] = (int32_t)len;
        force[r] = 0;
    }
    // at most nnz(A) / ASG_LONG (ASG_HUGE) rows qualify: the lists cannot overflow
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const bool lng = k == 0 ? (len > ASG_LONG && len <= ASG_HUGE) : len > ASG_HUGE;
        const uint64_t lm = ballot(lng);
        if (lm) {
            uint32_t base = 0;
            if (lane_id() == 0) base = atomicAdd(nlong + k, (uint32_t)__popcll(lm));
            base = __shfl(base, 0, WAVE);
            if (lng) (k == 0 ? rlong : rhuge)[base + __popcll(lm & lanemask_lt())] = (int32_t)r;
        }
    }
}

// Count pass for the rows of B, 16 lanes per row i (row I[i] of A), four
// rows per wavefront: the group loads B's row (<= 256 columns) into
// registers with coalesced loads, then tests each of the <= 16 A columns
// against it with one ballot.  Rows with longer A or B rows go to llist for
// the one-wavefront count.
constexpr int AS_G = 16;   // lanes per row; also the A and B/16 limits

template <typename PT>
__global__ __launch_bounds__(256) void k_asg_count_I(const PT *__restrict__ arow, const int32_t *__restrict__ acol,
                                                    const PT *__restrict__ brow, const int32_t *__restrict__ bcol,
                                                    const int32_t *__restrict__ I, int64_t nI,
                                                    const int32_t *__restrict__ J, int64_t nJ,
                                                    const int32_t *__restrict__ colinv, int64_t n, int op,
                                                    int32_t *cnt, uint8_t *force, int32_t *llist, uint32_t *lcount,
                                                    const DevHdr *hdr) {
    if (hdr->err) return;
    const bool jrange = !(ld_agent(&hdr->flags) & F_NOT_RANGE);   // set by the table pass
    const int l = lane_id(), g = l / AS_G, x = l % AS_G;
    const int64_t i = (int64_t)blockIdx.x * (256 / AS_G) + (threadIdx.x / WAVE) * (WAVE / AS_G) + g;
    const bool valid = i < nI;
    int64_t r = 0, as = 0, La = 0, bs = 0, Lb = 0;
    if (valid) {
        r = I[i];
        as = arow[r];
        La = arow[r + 1] - as;
        bs = brow[i];
        Lb = brow[i + 1] - bs;
    }
    const bool small = valid && La <= AS_G && Lb <= AS_G * AS_G;
    // rare: rows for the wavefront count (one atomic per wavefront)
    const bool lng = valid && !small && x == 0;
    const uint64_t lm = ballot(lng);
    if (lm) {
        uint32_t base = 0;
        if (l == 0) base = atomicAdd(lcount, (uint32_t)__popcll(lm));
        base = __shfl(base, 0, WAVE);
        if (lng) llist[base + __popcll(lm & lanemask_lt())] = (int32_t)i;
    }
    // B's columns: for the collision test, and (J not a range) to check
    // their mapped order; REPLACE over a range of J needs neither
    const bool replace = op == HP_OP_REPLACE;
    const bool needb = !replace || !jrange;
    int32_t bc[AS_G];
#pragma unroll
    for (int q = 0; q < AS_G; q++) {
        const int64_t t = q * AS_G + x;
        bc[q] = needb && small && t < Lb ? bcol[bs + t] : INT32_MIN;
    }
    int32_t jb = -1;
    if (small && x < La) jb = colinv[clampc(acol[as + x], n)];
    // the loop stops at the longest A row among the wavefront's four rows;
    // REPLACE keeps exactly the A entries outside J, whatever B holds
    int amax = small ? (int)La : 0;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) amax = max(amax, __shfl_xor(amax, off, WAVE));
    int nak = 0;
    for (int a = 0; a < amax; a++) {
        const int32_t ja = __shfl(jb, g * AS_G + a, WAVE);
        bool hit = false;
        if (!replace) {
#pragma unroll
            for (int q = 0; q < AS_G; q++) hit |= bc[q] == ja;
        }
        const bool ghit = ((ballot(hit) >> (g * AS_G)) & 0xffffull) != 0;
        const bool kept = ja < 0 || (!replace && !ghit);
        nak += (small && a < La && kept) ? 1 : 0;
    }
    // do the mapped B columns increase along the row (t order: q major,
    // lane minor)?  Always when J is a range.
    bool bad = false;
    if (!jrange) {
        int32_t bk[AS_G];
#pragma unroll
        for (int q = 0; q < AS_G; q++) bk[q] = bc[q] == INT32_MIN ? INT32_MAX : J[clampc(bc[q], nJ)];
#pragma unroll
        for (int q = 0; q < AS_G; q++) {
            const int32_t nx_same = __shfl_down(bk[q], 1, AS_G);
            const int32_t nx_wrap = q + 1 < AS_G ? __shfl(bk[q + 1], g * AS_G, WAVE) : INT32_MAX;
            const int32_t nxt = x < AS_G - 1 ? nx_same : nx_wrap;
            const int64_t t = q * AS_G + x;
            bad |= t + 1 < Lb && bk[q] >= nxt;
        }
    }
    const bool inc = ((ballot(bad) >> (g * AS_G)) & 0xffffull) == 0;
    if (small && x == 0) {
        cnt[r] = (int32_t)(nak + Lb);
        force[r] = (La + Lb > AS_WCAP || (!inc && La + Lb > AS_RANK_MAX)) ? 1 : 0;
    }
}

__device__ __forceinline__ uint32_t vadd(uint32_t a, uint32_t b) {
    return __float_as_uint(__uint_as_float(a) + __uint_as_float(b));
}
__device__ __forceinline__ uint64_t vadd(uint64_t a, uint64_t b) {
    return (uint64_t)__double_as_longlong(__longlong_as_double((long long)a) +
                                          __longlong_as_double((long long)b));
}

// Number of elements < key in the sorted array a[0, len).
template <typename T>
__device__ __forceinline__ int lower_bound_n(const T *a, int64_t len, int64_t key) {
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (int)lo;
}

template <typename T>
__device__ __forceinline__ int64_t find_n(const T *a, int64_t len, int64_t key) {
    const int64_t p = lower_bound_n(a, len, key);
    return (p < len && (int64_t)a[p] == key) ? p : -1;
}

// Number of entries of the (unsorted) array a[0, len) below key.
__device__ __forceinline__ int count_less(const int32_t *a, int len, int32_t key) {
    int c = 0;
    for (int x = 0; x < len; x++) c += a[x] < key;
    return c;
}

// Where the rows of A (+) B' go: row r of the assignment result is written
// to output row dest[r] with every column c stored as cmap[c] (the fused
// assign-and-permute; null maps = the plain assignment, rows in place).
struct OutMap {
    const int32_t *dest;
    const int32_t *cmap;
    int64_t n;   // cmap entries; a column outside [0, n) is clamped, never read out of bounds
    __device__ __forceinline__ int64_t row(int64_t r) const { return dest ? dest[r] : r; }
    __device__ __forceinline__ int32_t col(int32_t c) const { return cmap ? cmap[clampc(c, n)] : c; }
};

struct RowSmem {
    int32_t a[AS_WCAP];    // A's columns
    int32_t b[AS_WCAP];    // B's columns (indices into J)
    int32_t k[AS_WCAP];    // B's mapped columns J[b]
    int32_t ak[AS_WCAP];   // surviving A columns, compacted
    int32_t o[AS_WCAP];    // all output keys (unsorted case)
};

// One wavefront for row i of B (row I[i] of A).  COUNT: write cnt and the
// sort flag.  Otherwise write the merged row of C.
template <typename PT, typename VT, bool COUNT>
__device__ void asg_row_I(
    int64_t i, RowSmem &sm, const PT *__restrict__ arow, const int32_t *__restrict__ acol,
    const VT *__restrict__ aval, const PT *__restrict__ brow, const int32_t *__restrict__ bcol,
    const VT *__restrict__ bval, const int32_t *__restrict__ I, const int32_t *__restrict__ J, int64_t nJ,
    const int32_t *__restrict__ colinv, int64_t n, int op, const PT *__restrict__ crow, int32_t *ccol,
    VT *cval, int32_t *cnt, uint8_t *force, OutMap om = OutMap{nullptr, nullptr, 0}, int32_t *hlist = nullptr,
    uint32_t *hcount = nullptr) {
    const int l = lane_id();
    const int64_t r = I[i];
    const int64_t as = arow[r], La = arow[r + 1] - as;
    const int64_t bs = brow[i], Lb = brow[i + 1] - bs;
    const bool replace = op == HP_OP_REPLACE, plus = op == HP_OP_PLUS;
    if (hlist && La + Lb > AS_HUGE) {
        // left to k_asg_rows_huge (every workgroup on the row); the count
        // starts at B's entries, the kept A entries are added there
        if (l == 0) {
            hlist[atomicAdd(hcount, 1u)] = (int32_t)i;
            if (COUNT) {
                cnt[r] = (int32_t)Lb;
                force[r] = 1;
            }
        }
        return;
    }

    if (COUNT && La * 16 <= Lb && La + Lb > AS_WCAP) {
        // few A entries against a long B row: binary-search B in memory
        // instead of staging it (the count pass then reads little of B)
        const int32_t *bc = bcol + bs;
        int nak = 0;
        for (int64_t a0 = 0; a0 < La; a0 += WAVE) {
            const int64_t a = a0 + l;
            bool kept = false;
            if (a < La) {
                const int32_t jb = colinv[clampc(acol[as + a], n)];
                kept = replace ? jb < 0 : (jb < 0 || find_n(bc, Lb, jb) < 0);
            }
            nak += __popcll(ballot(kept));
        }
        if (l == 0) {
            cnt[r] = (int32_t)(nak + Lb);
            force[r] = La + Lb > AS_WCAP ? 1 : 0;
        }
        return;
    }
    // fused form (exec): the sort pass orders the row, so it is written in
    // any order, straight from memory as for a long row
    if (La + Lb <= AS_WCAP && (COUNT || om.cmap == nullptr)) {
        for (int x = l; x < La; x += WAVE) sm.a[x] = acol[as + x];
        for (int x = l; x < Lb; x += WAVE) {
            const int32_t cb = bcol[bs + x];
            sm.b[x] = cb;
            sm.k[x] = J[clampc(cb, nJ)];
        }
        __builtin_amdgcn_wave_barrier();
        // surviving A entries, compacted in A order
        int nak = 0;
        for (int a0 = 0; a0 < La; a0 += WAVE) {
            const int a = a0 + l;
            bool kept = false;
            if (a < La) {
                const int32_t jb = colinv[clampc(sm.a[a], n)];
                kept = replace ? jb < 0 : (jb < 0 || find_n(sm.b, Lb, jb) < 0);
            }
            const uint64_t msk = ballot(kept);
            if (!COUNT && kept) sm.ak[nak + __popcll(msk & lanemask_lt())] = sm.a[a];
            nak += __popcll(msk);
        }
        bool inc = true;
        for (int t0 = 0; t0 + 1 < Lb; t0 += WAVE) {
            const int t = t0 + l;
            const bool bad = t + 1 < Lb && sm.k[t] >= sm.k[t + 1];
            inc = inc && ballot(bad) == 0;
        }
        // a long row out of J's order is left to the class sorts
        const bool unsorted = !inc && La + Lb > AS_RANK_MAX;
        if (COUNT) {
            if (l == 0) {
                cnt[r] = (int32_t)(nak + Lb);
                force[r] = unsorted ? 1 : 0;
            }
            return;
        }
        __builtin_amdgcn_wave_barrier();
        if (!unsorted) {
            const int64_t d = crow[om.row(r)];
            const int L = nak + (int)Lb;
            if (!inc) {
                for (int x = l; x < nak; x += WAVE) sm.o[x] = sm.ak[x];
                for (int x = l; x < Lb; x += WAVE) sm.o[nak + x] = sm.k[x];
                __builtin_amdgcn_wave_barrier();
            }
            // surviving A entries
            int rank = 0;
            for (int a0 = 0; a0 < La; a0 += WAVE) {
                const int a = a0 + l;
                bool kept = false;
                int32_t key = 0;
                if (a < La) {
                    key = sm.a[a];
                    const int32_t jb = colinv[clampc(key, n)];
                    kept = replace ? jb < 0 : (jb < 0 || find_n(sm.b, Lb, jb) < 0);
                }
                const uint64_t msk = ballot(kept);
                if (kept) {
                    const int own = rank + __popcll(msk & lanemask_lt());
                    int pos;
                    if (inc) pos = own + lower_bound_n(sm.k, Lb, key);
                    else pos = count_less(sm.o, L, key);
                    ccol[d + pos] = om.col(key);
                    cval[d + pos] = aval[as + a];
                }
                rank += __popcll(msk);
            }
            // B' entries (values combined with A's where both exist for PLUS)
            for (int t = l; t < Lb; t += WAVE) {
                const int32_t key = sm.k[t];
                VT v = bval[bs + t];
                if (plus) {
                    const int64_t p = find_n(sm.a, La, key);
                    if (p >= 0) v = vadd(aval[as + p], v);
                }
                const int pos = inc ? t + lower_bound_n(sm.ak, nak, key) : count_less(sm.o, L, key);
                ccol[d + pos] = om.col(key);
                cval[d + pos] = v;
            }
            return;
        }
    }

    // Long row, a row out of J's order longer than AS_RANK_MAX, or any row
    // of the fused form: resolve collisions against the rows in global
    // memory, write surviving A entries then B' entries, and leave the order
    // to the segmented sort (force flag set by the count pass; every merged
    // row of the fused form is sorted).
    const int32_t *ac = acol + as;
    const int32_t *bc = bcol + bs;
    int nak = 0;
    for (int64_t a0 = 0; a0 < La; a0 += WAVE) {
        const int64_t a = a0 + l;
        bool kept = false;
        if (a < La) {
            const int32_t jb = colinv[clampc(ac[a], n)];
            kept = replace ? jb < 0 : (jb < 0 || find_n(bc, Lb, jb) < 0);
        }
        const uint64_t msk = ballot(kept);
        if (!COUNT && kept) {
            const int64_t pos = (int64_t)crow[om.row(r)] + nak + __popcll(msk & lanemask_lt());
            ccol[pos] = om.col(ac[a]);
            cval[pos] = aval[as + a];
        }
        nak += __popcll(msk);
    }
    if (COUNT) {
        if (l == 0) {
            cnt[r] = (int32_t)(nak + Lb);
            force[r] = 1;
        }
        return;
    }
    for (int64_t t = l; t < Lb; t += WAVE) {
        const int32_t key = J[clampc(bc[t], nJ)];
        VT v = bval[bs + t];
        if (plus) {
            const int64_t p = find_n(ac, La, key);
            if (p >= 0) v = vadd(aval[as + p], v);
        }
        const int64_t pos = (int64_t)crow[om.row(r)] + nak + t;
        ccol[pos] = om.col(key);
        cval[pos] = v;
    }
}

template <typename PT, typename VT, bool COUNT>
__global__ __launch_bounds__(256) void k_asg_rows_I(
    const PT *__restrict__ arow, const int32_t *__restrict__ acol, const VT *__restrict__ aval,
    const PT *__restrict__ brow, const int32_t *__restrict__ bcol, const VT *__restrict__ bval,
    const int32_t *__restrict__ I, int64_t nI, const int32_t *__restrict__ J, int64_t nJ,
    const int32_t *__restrict__ colinv, int64_t n, int op, const PT *__restrict__ crow, int32_t *ccol,
    VT *cval, int32_t *cnt, uint8_t *force, const DevHdr *hdr) {
    __shared__ __align__(16) RowSmem sm_all[4];
    if (hdr->err) return;
    const int w = threadIdx.x / WAVE;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    if (i >= nI) return;
    asg_row_I<PT, VT, COUNT>(i, sm_all[w], arow, acol, aval, brow, bcol, bval, I, J, nJ, colinv, n, op, crow,
                             ccol, cval, cnt, force);
}

// The rows the 16-lane kernels left in llist: persistent wavefronts, one
// row at a time (count or merge).
template <typename PT, typename VT, bool COUNT>
__global__ __launch_bounds__(256) void k_asg_rows_list(
    const PT *__restrict__ arow, const int32_t *__restrict__ acol, const VT *__restrict__ aval,
    const PT *__restrict__ brow, const int32_t *__restrict__ bcol, const VT *__restrict__ bval,
    const int32_t *__restrict__ I, const int32_t *__restrict__ J, int64_t nJ,
    const int32_t *__restrict__ colinv, int64_t n, int op, const PT *__restrict__ crow, int32_t *ccol,
    VT *cval, int32_t *cnt, uint8_t *force, const int32_t *__restrict__ llist, const uint32_t *__restrict__ lcount,
    const DevHdr *hdr, OutMap om = OutMap{nullptr, nullptr, 0}, int32_t *hlist = nullptr,
    uint32_t *hcount = nullptr) {
    __shared__ __align__(16) RowSmem sm_all[4];
    if (hdr->err) return;
    const int w = threadIdx.x / WAVE;
    const uint32_t nl = *lcount;
    for (uint32_t t = blockIdx.x * 4 + w; t < nl; t += gridDim.x * 4)
        asg_row_I<PT, VT, COUNT>(llist[t], sm_all[w], arow, acol, aval, brow, bcol, bval, I, J, nJ, colinv, n, op,
                                 crow, ccol, cval, cnt, force, om, hlist, hcount);
}

// Rows of hlist (more than AS_HUGE A + B entries), one after another, each
// spread over every wavefront of the grid: A's entries are tested against
// B's row by binary search as in the long-row path, kept ones counted into
// cnt[r] (COUNT) or placed through the row's cursor hcur[h] in any order
// (the row is sorted afterwards, its force flag set); B' entries go after
// the kept A entries, at their own offset.  Wave-uniform loop bounds keep
// every lane in the ballots.
template <typename PT, typename VT, bool COUNT>
__global__ __launch_bounds__(256) void k_asg_rows_huge(
    const PT *__restrict__ arow, const int32_t *__restrict__ acol, const VT *__restrict__ aval,
    const PT *__restrict__ brow, const int32_t *__restrict__ bcol, const VT *__restrict__ bval,
    const int32_t *__restrict__ I, const int32_t *__restrict__ J, int64_t nJ,
    const int32_t *__restrict__ colinv, int64_t n, int op, const PT *__restrict__ crow, int32_t *ccol,
    VT *cval, int32_t *cnt, const int32_t *__restrict__ hlist, const uint32_t *__restrict__ hcount,
    uint32_t *hcur, const DevHdr *hdr, OutMap om = OutMap{nullptr, nullptr, 0}) {
    if (hdr->err) return;
    const int l = lane_id();
    const int64_t gw = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    const int64_t nw = (int64_t)gridDim.x * (256 / WAVE);
    const bool replace = op == HP_OP_REPLACE, plus = op == HP_OP_PLUS;
    const uint32_t nh = *hcount;
    for (uint32_t h = 0; h < nh; h++) {
        const int64_t i = hlist[h];
        const int64_t r = I[i];
        const int64_t as = arow[r], La = arow[r + 1] - as;
        const int64_t bs = brow[i], Lb = brow[i + 1] - bs;
        const int32_t *ac = acol + as;
        const int32_t *bc = bcol + bs;
        int64_t d = 0, nak = 0;
        if (!COUNT) {
            const int64_t orow = om.row(r);
            d = (int64_t)crow[orow];
            nak = (int64_t)crow[orow + 1] - d - Lb;   // kept A entries, from the plan's count
        }
        for (int64_t a0 = gw * WAVE; a0 < La; a0 += nw * WAVE) {
            const int64_t a = a0 + l;
            bool kept = false;
            if (a < La) {
                const int32_t jb = colinv[clampc(ac[a], n)];
                kept = replace ? jb < 0 : (jb < 0 || find_n(bc, Lb, jb) < 0);
            }
            const uint64_t msk = ballot(kept);
            if (!msk) continue;
            if (COUNT) {
                if (l == 0) atomicAdd(&cnt[r], (int32_t)__popcll(msk));
            } else {
                uint32_t base = 0;
                if (l == 0) base = atomicAdd(&hcur[h], (uint32_t)__popcll(msk));
                base = __shfl(base, 0, WAVE);
                const int64_t pos = base + __popcll(msk & lanemask_lt());
                if (kept && pos < nak) {   // within the planned count
                    ccol[d + pos] = om.col(ac[a]);
                    cval[d + pos] = aval[as + a];
                }
            }
        }
        if (COUNT) continue;
        for (int64_t t = gw * WAVE + l; t < Lb; t += nw * WAVE) {
            const int32_t key = J[clampc(bc[t], nJ)];
            VT v = bval[bs + t];
            if (plus) {
                const int64_t p = find_n(ac, La, key);
                if (p >= 0) v = vadd(aval[as + p], v);
            }
            ccol[d + nak + t] = om.col(key);
            cval[d + nak + t] = v;
        }
    }
}

// Merge pass, 16 lanes per row of B as in the count: the group holds B's
// row in registers (columns, values, mapped columns J[b]) and A's <= 16
// entries one per lane.  When the mapped columns increase along the row,
// a B' entry goes to t + (kept A entries below it) and a kept A entry to
// its rank among the kept ones + (B' entries below it); collisions drop
// the A entry (PLUS adds its value to B's first).  Other rows go to llist.
template <typename PT, typename VT>
__global__ __launch_bounds__(256) void k_asg_merge_I(
    const PT *__restrict__ arow, const int32_t *__restrict__ acol, const VT *__restrict__ aval,
    const PT *__restrict__ brow, const int32_t *__restrict__ bcol, const VT *__restrict__ bval,
    const int32_t *__restrict__ I, int64_t nI, const int32_t *__restrict__ J, int64_t nJ,
    const int32_t *__restrict__ colinv, int64_t n, int op, const PT *__restrict__ crow, int32_t *ccol, VT *cval,
    int32_t *llist, uint32_t *lcount, int jrange, const DevHdr *hdr, OutMap om = OutMap{nullptr, nullptr, 0}) {
    if (hdr->err) return;
    const int32_t j0 = nJ > 0 ? J[0] : 0;
    const int l = lane_id(), g = l / AS_G, x = l % AS_G;
    const int64_t i = (int64_t)blockIdx.x * (256 / AS_G) + (threadIdx.x / WAVE) * (WAVE / AS_G) + g;
    const bool valid = i < nI;
    int64_t r = 0, as = 0, La = 0, bs = 0, Lb = 0;
    if (valid) {
        r = I[i];
        as = arow[r];
        La = arow[r + 1] - as;
        bs = brow[i];
        Lb = brow[i + 1] - bs;
    }
    bool small = valid && La <= AS_G && Lb <= AS_G * AS_G;
    int32_t bc[AS_G], bk[AS_G];
    VT bv[AS_G];
#pragma unroll
    for (int q = 0; q < AS_G; q++) {
        const int64_t t = q * AS_G + x;
        const bool in = small && t < Lb;
        bc[q] = in ? bcol[bs + t] : INT32_MIN;
        bv[q] = in ? bval[bs + t] : VT(0);
    }
#pragma unroll
    for (int q = 0; q < AS_G; q++)
        bk[q] = bc[q] == INT32_MIN ? INT32_MAX : (jrange ? j0 + (int32_t)clampc(bc[q], nJ) : J[clampc(bc[q], nJ)]);
    int32_t ak = INT32_MAX, jb = -1;
    VT av = VT(0);
    if (small && x < La) {
        ak = acol[as + x];
        av = aval[as + x];
        jb = colinv[clampc(ak, n)];
    }
    // mapped columns increasing along the row? (t order: q major, lane minor)
    bool bad = false;
#pragma unroll
    for (int q = 0; q < AS_G; q++) {
        const int32_t nx_same = __shfl_down(bk[q], 1, AS_G);
        const int32_t nx_wrap = q + 1 < AS_G ? __shfl(bk[q + 1], g * AS_G, WAVE) : INT32_MAX;
        const int32_t nxt = x < AS_G - 1 ? nx_same : nx_wrap;
        const int64_t t = q * AS_G + x;
        bad |= t + 1 < Lb && bk[q] >= nxt;
    }
    const bool inc = ((ballot(bad) >> (g * AS_G)) & 0xffffull) == 0;
    // fused form: the sort pass orders every merged row, so any placement
    // works and the mapped columns need not increase
    const bool fused = om.cmap != nullptr;
    const bool mine = small && (inc || fused);
    const bool lng = valid && !mine && x == 0;
    const uint64_t lm = ballot(lng);
    if (lm) {
        uint32_t base = 0;
        if (l == 0) base = atomicAdd(lcount, (uint32_t)__popcll(lm));
        base = __shfl(base, 0, WAVE);
        if (lng) llist[base + __popcll(lm & lanemask_lt())] = (int32_t)i;
    }
    // collisions: drop the A entry; PLUS adds its value into B's.  The loops
    // over A entries stop at the longest A row among the wave's groups.
    int amax = small ? (int)La : 0;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) amax = max(amax, __shfl_xor(amax, off, WAVE));
    const bool replace = op == HP_OP_REPLACE, plus = op == HP_OP_PLUS;
    uint32_t kept = 0;   // bit a: A entry a survives
    for (int a = 0; a < amax; a++) {
        const int32_t ja = __shfl(jb, g * AS_G + a, WAVE);
        const VT va = __shfl(av, g * AS_G + a, WAVE);
        bool hit = false;
#pragma unroll
        for (int q = 0; q < AS_G; q++) {
            const bool h = ja >= 0 && bc[q] == ja;
            hit |= h;
            if (h && plus) bv[q] = vadd(va, bv[q]);
        }
        const bool ghit = ((ballot(hit) >> (g * AS_G)) & 0xffffull) != 0;
        if (a < La && (ja < 0 || (!replace && !ghit))) kept |= 1u << a;
    }
    if (!mine) return;
    const int64_t d = crow[om.row(r)];
    if (fused) {
        // B' entries in B's order, then the kept A entries in A's order; the
        // column lookups all go out together (idle lanes look up column 0)
#pragma unroll
        for (int q = 0; q < AS_G; q++) bk[q] = om.col(q * AS_G + x < Lb ? bk[q] : 0);
        const bool mk = x < La && ((kept >> x) & 1u);
        const int32_t ma = om.col(mk ? ak : 0);
#pragma unroll
        for (int q = 0; q < AS_G; q++) {
            const int64_t t = q * AS_G + x;
            if (t < Lb) {
                ccol[d + t] = bk[q];
                cval[d + t] = bv[q];
            }
        }
        if (mk) {
            const int64_t pos = d + Lb + __popc(kept & ((1u << x) - 1u));
            ccol[pos] = ma;
            cval[pos] = av;
        }
        return;
    }
    // B' entries, each shifted by the kept A entries with smaller columns
    int below[AS_G];
#pragma unroll
    for (int q = 0; q < AS_G; q++) below[q] = 0;
    for (int a = 0; a < amax; a++) {
        int32_t ka = __shfl(ak, g * AS_G + a, WAVE);
        if (!((kept >> a) & 1u)) ka = INT32_MAX;
#pragma unroll
        for (int q = 0; q < AS_G; q++) below[q] += ka < bk[q];
    }
#pragma unroll
    for (int q = 0; q < AS_G; q++) {
        const int64_t t = q * AS_G + x;
        if (t < Lb) {
            ccol[d + t + below[q]] = om.col(bk[q]);
            cval[d + t + below[q]] = bv[q];
        }
    }
    // kept A entries
    for (int a = 0; a < amax; a++) {
        if (!((kept >> a) & 1u)) continue;   // uniform within the group
        const int32_t ka = __shfl(ak, g * AS_G + a, WAVE);
        int cntb = 0;
#pragma unroll
        for (int q = 0; q < AS_G; q++) cntb += bk[q] < ka;
#pragma unroll
        for (int off = AS_G / 2; off > 0; off >>= 1) cntb += __shfl_xor(cntb, off, AS_G);
        if (x == a) {
            const int64_t pos = d + __popc(kept & ((1u << a) - 1u)) + cntb;
            ccol[pos] = om.col(ka);
            cval[pos] = av;
        }
    }
}

// Lane a's value, for a wave-uniform a (32- or 64-bit).
template <typename T>
__device__ __forceinline__ T read_lane(T x, int a) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = (uint64_t)x;
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, a);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), a);
        return (T)(((uint64_t)hi << 32) | lo);
    } else {
        return (T)__builtin_amdgcn_readlane((uint32_t)x, a);
    }
}

// The same merge for long B rows (taken when B averages more than WAVE
// entries a row): one wavefront per row of I, four rows per workgroup, B's
// row in AS_MQ 64-wide slices of registers (each load 64 consecutive
// entries) and A's row one entry per lane, so the collision tests and the
// placement counts are ballots and the row's values wave-uniform.  About
// 40 VGPRs (eight wavefronts a SIMD) where the 16-lane merge needs 155.
// Rows with more than WAVE A entries or AS_MQ * WAVE B entries, or (plain
// form) mapped B columns out of order, go to llist.
template <typename PT, typename VT>
__global__ __launch_bounds__(256) void k_asg_merge_row(
    const PT *__restrict__ arow, const int32_t *__restrict__ acol, const VT *__restrict__ aval,
    const PT *__restrict__ brow, const int32_t *__restrict__ bcol, const VT *__restrict__ bval,
    const int32_t *__restrict__ I, int64_t nI, const int32_t *__restrict__ J, int64_t nJ,
    const int32_t *__restrict__ colinv, int64_t n, int op, const PT *__restrict__ crow, int32_t *ccol, VT *cval,
    int32_t *llist, uint32_t *lcount, int jrange, const DevHdr *hdr, OutMap om = OutMap{nullptr, nullptr, 0}) {
    __shared__ __align__(16) SegSmemWave sm;   // the fused form's row sort
    if (hdr->err) return;
    const int l = lane_id();
    const int64_t i = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    if (i >= nI) return;   // the whole wavefront
    const int32_t j0 = nJ > 0 ? J[0] : 0;
    const int64_t r = I[i];
    const int64_t as = arow[r], La = arow[r + 1] - as;
    const int64_t bs = brow[i], Lb = brow[i + 1] - bs;
    const bool small = La <= WAVE && Lb <= AS_MQ * WAVE;
    int32_t bc[AS_MQ], bk[AS_MQ];
    VT bv[AS_MQ];
#pragma unroll
    for (int q = 0; q < AS_MQ; q++) {
        const int64_t t = q * WAVE + l;
        const bool in = small && t < Lb;
        bc[q] = in ? bcol[bs + t] : INT32_MIN;
        bv[q] = in ? bval[bs + t] : VT(0);
    }
#pragma unroll
    for (int q = 0; q < AS_MQ; q++)
        bk[q] = bc[q] == INT32_MIN ? INT32_MAX : (jrange ? j0 + (int32_t)clampc(bc[q], nJ) : J[clampc(bc[q], nJ)]);
    int32_t ak = INT32_MAX, jb = -1;
    VT av = VT(0);
    if (small && l < La) {
        ak = acol[as + l];
        av = aval[as + l];
        jb = colinv[clampc(ak, n)];
    }
    // mapped columns increasing along the row (t = q * WAVE + lane)?
    bool bad = false;
#pragma unroll
    for (int q = 0; q < AS_MQ; q++) {
        const int32_t nx_same = __shfl_down(bk[q], 1, WAVE);
        const int32_t nx_wrap = q + 1 < AS_MQ ? __shfl(bk[q + 1], 0, WAVE) : INT32_MAX;
        const int32_t nxt = l < WAVE - 1 ? nx_same : nx_wrap;
        const int64_t t = q * WAVE + l;
        bad |= t + 1 < Lb && bk[q] >= nxt;
    }
    const bool inc = ballot(bad) == 0;
    const bool fused = om.cmap != nullptr;
    if (!(small && (inc || fused))) {
        if (l == 0) llist[atomicAdd(lcount, 1u)] = (int32_t)i;   // rare: the one-wavefront merge
        return;
    }
    const bool replace = op == HP_OP_REPLACE, plus = op == HP_OP_PLUS;
    const int na = (int)La;
    uint64_t kept = 0;   // bit a: A entry a survives (wave-uniform)
    for (int a = 0; a < na; a++) {
        const int32_t ja = read_lane(jb, a);
        const VT va = read_lane(av, a);
        bool hit = false;
#pragma unroll
        for (int q = 0; q < AS_MQ; q++) {
            const bool h = ja >= 0 && bc[q] == ja;
            hit |= h;
            if (h && plus) bv[q] = vadd(va, bv[q]);
        }
        const bool ghit = ballot(hit) != 0;
        if (ja < 0 || (!replace && !ghit)) kept |= 1ull << a;
    }
    const int64_t d = crow[om.row(r)];
    const bool mykept = l < na && ((kept >> l) & 1ull);
    if (fused) {
        // B' entries in B's order, then the kept A entries in A's order; the
        // column lookups all go out together (idle lanes look up column 0)
        int32_t mc[AS_MQ];
#pragma unroll
        for (int q = 0; q < AS_MQ; q++) mc[q] = om.col(q * WAVE + l < Lb ? bk[q] : 0);
        const int32_t ma = om.col(mykept ? ak : 0);
        const int nout = (int)Lb + __popcll(kept);
        if (nout <= AS_MQ * WAVE) {
            // the whole merged row fits this wavefront's sort (the plan
            // flagged it 3, so the sort pass leaves it alone): stage it in
            // LDS in merged order, take it back four entries a lane, sort
            int32_t *s_k = sm.k[threadIdx.x / WAVE];
            VT *s_v = reinterpret_cast<VT *>(sm.v[threadIdx.x / WAVE]);
#pragma unroll
            for (int q = 0; q < AS_MQ; q++) {
                const int t = q * WAVE + l;
                if (t < Lb) {
                    s_k[t] = mc[q];
                    s_v[t] = bv[q];
                }
            }
            if (mykept) {
                const int pos = (int)Lb + __popcll(kept & lanemask_lt());
                s_k[pos] = ma;
                s_v[pos] = av;
            }
            __builtin_amdgcn_wave_barrier();
            int32_t mk[AS_MQ];
            VT mv[AS_MQ];
#pragma unroll
            for (int q = 0; q < AS_MQ; q++) {
                const int e = q * WAVE + l;
                mk[q] = e < nout ? s_k[e] : INT32_MAX;
                mv[q] = e < nout ? s_v[e] : VT(0);
            }
            __builtin_amdgcn_wave_barrier();
            wave_sort_regs<VT>(mk, mv, nout, ccol + d, cval + d, s_k, s_v);
            return;
        }
#pragma unroll
        for (int q = 0; q < AS_MQ; q++) {
            const int64_t t = q * WAVE + l;
            if (t < Lb) {
                ccol[d + t] = mc[q];
                cval[d + t] = bv[q];
            }
        }
        if (mykept) {
            const int64_t pos = d + Lb + __popcll(kept & lanemask_lt());
            ccol[pos] = ma;
            cval[pos] = av;
        }
        return;
    }
    // B' entries, each shifted by the kept A entries with smaller columns;
    // a kept A entry goes to its rank among the kept ones plus the B'
    // entries below it
    int below[AS_MQ];
#pragma unroll
    for (int q = 0; q < AS_MQ; q++) below[q] = 0;
    int cntb_mine = 0;
    for (int a = 0; a < na; a++) {
        if (!((kept >> a) & 1ull)) continue;   // uniform
        const int32_t ka = read_lane(ak, a);
        int cb = 0;
#pragma unroll
        for (int q = 0; q < AS_MQ; q++) {
            below[q] += ka < bk[q];
            cb += __popcll(ballot(bk[q] < ka));
        }
        if (l == a) cntb_mine = cb;
    }
#pragma unroll
    for (int q = 0; q < AS_MQ; q++) {
        const int64_t t = q * WAVE + l;
        if (t < Lb) {
            ccol[d + t + below[q]] = om.col(bk[q]);
            cval[d + t + below[q]] = bv[q];
        }
    }
    if (mykept) {
        const int64_t pos = d + __popcll(kept & lanemask_lt()) + cntb_mine;
        ccol[pos] = om.col(ak);
        cval[pos] = av;
    }
}

// Entry k of a row of A with its column mapped (fused form).
template <typename VT>
struct LoadMapped {
    const int32_t *acol;
    const VT *aval;
    OutMap om;
    __device__ __forceinline__ void get(int64_t b, int64_t k, int32_t &kk, VT &vv) const {
        kk = om.col(acol[b + k]);
        vv = aval[b + k];
    }
};

// Rows outside I: copy A's row to C's row, 64 rows per wavefront, entries
// spread over lanes (coalesced reads and writes).  SORT_SHORT (fused form):
// a row of at most THREAD_MAX entries is instead mapped, sorted in its own
// lane's registers and stored there, and longer rows are left to the sort
// pass, which reads them from A (LoadFused).
template <typename PT, typename VT, bool SORT_SHORT = false>
__global__ __launch_bounds__(256) void k_asg_copy_rest(const PT *__restrict__ arow,
                                                      const int32_t *__restrict__ acol,
                                                      const VT *__restrict__ aval, int64_t m,
                                                      const int32_t *__restrict__ rowinv,
                                                      const PT *__restrict__ crow, int32_t *ccol,
                                                      VT *cval, const DevHdr *hdr,
                                                      OutMap om = OutMap{nullptr, nullptr, 0}) {
    __shared__ int32_t s_start[4][WAVE];
    __shared__ int64_t s_as[4][WAVE], s_cs[4][WAVE];
    if (hdr->err) return;
    const int w = threadIdx.x / WAVE, l = lane_id();
    const int64_t r = ((int64_t)blockIdx.x * 4 + w) * WAVE + l;
    int len = 0;
    if (r < m && rowinv[r] < 0) {
        const int64_t a = arow[r];
        len = (int)(arow[r + 1] - a);
        if (len > ASG_LONG) len = 0;   // k_asg_copy_long
        const int64_t d = crow[om.row(r)];
        if (SORT_SHORT) {
            if (len > 0 && len <= (int)THREAD_MAX)
                lane_sort_row<VT>(LoadMapped<VT>{acol, aval, om}, a, len, false, ccol + d, cval + d);
            len = 0;
        }
        s_as[w][l] = a;
        s_cs[w][l] = d;
    }
    const int incl = wave_incl_scan(len);
    const int E = __shfl(incl, WAVE - 1, WAVE);
    s_start[w][l] = incl - len;
    __builtin_amdgcn_wave_barrier();
    for (int e0 = 0; e0 < E; e0 += WAVE * 8) {
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int e = e0 + u * WAVE + l;
            if (e < E) {
                int lo = 0, hi = WAVE;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_start[w][mid] <= e) lo = mid;
                    else hi = mid;
                }
                const int off = e - s_start[w][lo];
                ccol[s_cs[w][lo] + off] = om.col(acol[s_as[w][lo] + off]);
                cval[s_cs[w][lo] + off] = aval[s_as[w][lo] + off];
            }
        }
    }
}

// Fused form: rows of at most 4 entries renamed, sorted and packed into
// their row slots (rows of I too; their slots are never read).
template <typename PT, typename VT>
__global__ __launch_bounds__(256) void k_fused_pack(const PT *__restrict__ arow, const int32_t *__restrict__ acol,
                                                   const VT *__restrict__ aval, const int32_t *__restrict__ qinv,
                                                   int64_t n, int64_t m, char *__restrict__ slots) {
    __shared__ int32_t lk[4 * perm::PACK_STAGE];
    __shared__ VT lv[4 * perm::PACK_STAGE];
    perm::perm_pack_tile<PT, VT>(blockIdx.x, arow, acol, aval, qinv, n, m, slots, lk, lv);
}

// Fused form, output rows outside I of at most THREAD_MAX entries (flag 0),
// one lane per output row i in order: row p[i] of A, columns renamed by
// qinv and sorted, from its row slot (perm_pack_tile, rows of at most 4
// entries) when slots are given, else straight from A.
template <typename PT, typename VT>
__global__ __launch_bounds__(256) void k_fused_fill_short(const int32_t *__restrict__ p,
                                                         const uint8_t *__restrict__ fflag,
                                                         const PT *__restrict__ arow, const int32_t *__restrict__ acol,
                                                         const VT *__restrict__ aval, const int32_t *__restrict__ qinv,
                                                         int64_t n, const char *__restrict__ slots,
                                                         const PT *__restrict__ crow, int32_t *ccol, VT *cval,
                                                         int64_t m, const DevHdr *hdr) {
    if (hdr->err) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    // the flag, the row bounds and p[i] in one round of loads (the asm
    // keeps the compiler from sinking each load below the branch before it)
    const uint8_t f = fflag[i];
    const int64_t d = crow[i];
    const int64_t e = crow[i + 1];
    const int32_t pr = p[i];
    asm volatile("" ::"v"(d), "v"(e), "v"(pr));
    if (f != 0) return;
    const int len = (int)(e - d);
    if (len == 0) return;
    const int64_t r = (uint32_t)pr < (uint64_t)m ? (int64_t)pr : 0;   // p was checked by the plan
    if (slots && len <= 4) {
        perm::perm_slot_copy<VT>(slots, r, len, d, ccol, cval);
        return;
    }
    lane_sort_row<VT>(LoadMapped<VT>{acol, aval, OutMap{nullptr, qinv, n}}, (int64_t)arow[r], len, false, ccol + d,
                      cval + d);
}

// Rows outside I longer than ASG_LONG, coalesced reads and writes: a
// workgroup per row of the rlong list, then every workgroup together on each
// row of the rhuge list.
template <typename PT, typename VT>
__global__ __launch_bounds__(256) void k_asg_copy_long(const PT *__restrict__ arow, const int32_t *__restrict__ acol,
                                                      const VT *__restrict__ aval, const int32_t *__restrict__ rlong,
                                                      const int32_t *__restrict__ rhuge,
                                                      const uint32_t *__restrict__ nlong, const PT *__restrict__ crow,
                                                      int32_t *ccol, VT *cval, const DevHdr *hdr, OutMap om) {
    if (hdr->err) return;
    const uint32_t nl = nlong[0], nh = nlong[1];
    for (uint32_t i = blockIdx.x; i < nl; i += gridDim.x) {
        const int64_t r = rlong[i];
        const int64_t a = arow[r], len = arow[r + 1] - a;
        const int64_t d = crow[om.row(r)];
        // eight entries a thread per round, the loads (and lookups) issued
        // together (len > ASG_LONG >= 1)
        for (int64_t e0 = 0; e0 < len; e0 += 8 * 256) {
            int32_t kc[8];
            VT kv[8];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int64_t e = e0 + u * 256 + threadIdx.x;
                const int64_t ec = e < len ? e : len - 1;
                kc[u] = acol[a + ec];
                kv[u] = aval[a + ec];
            }
#pragma unroll
            for (int u = 0; u < 8; u++) kc[u] = om.col(kc[u]);
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const int64_t e = e0 + u * 256 + threadIdx.x;
                if (e < len) {
                    ccol[d + e] = kc[u];
                    cval[d + e] = kv[u];
                }
            }
        }
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (uint32_t i = 0; i < nh; i++) {
        const int64_t r = rhuge[i];
        const int64_t a = arow[r], len = arow[r + 1] - a;
        const int64_t d = crow[om.row(r)];
        for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < len; e += stride) {
            ccol[d + e] = om.col(acol[a + e]);
            cval[d + e] = aval[a + e];
        }
    }
}

// Sort-pass loader of the fused form: a merged row (flag 2) is read back
// from C in place; any other listed row i is row p[i] of A with its columns
// mapped through qinv (bit 62 of the base tells the two apart).
template <typename PT, typename VT>
struct LoadFused {
    static constexpr int64_t IN_C = int64_t(1) << 62;
    const PT *arow;
    const int32_t *acol;
    const VT *aval;
    const int32_t *p;
    const int32_t *qinv;
    int64_t n;
    const PT *crow;
    const int32_t *ccol;
    const VT *cval;
    const uint8_t *fflag;
    __device__ __forceinline__ int64_t base(int64_t row) const {
        return fflag[row] == 2 ? ((int64_t)crow[row] | IN_C) : (int64_t)arow[p[row]];
    }
    __device__ __forceinline__ void get(int64_t b, int64_t k, int32_t &kk, VT &vv) const {
        if (b & IN_C) {
            b &= ~IN_C;
            kk = ccol[b + k];
            vv = cval[b + k];
        } else {
            kk = qinv[clampc(acol[b + k], n)];
            vv = aval[b + k];
        }
    }
};

hp_status_t asg_check_args(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B, const int32_t *I,
                           const int32_t *J, hp_asgn_op_t op, const hp_csr_t *C) {
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    st = check_csr_args(h, B, "B");
    if (st) return st;
    if (!C) return fail(h, HP_ERR_INVALID_ARG, "C is NULL");
    if (op != HP_OP_SECOND && op != HP_OP_PLUS && op != HP_OP_REPLACE)
        return fail(h, HP_ERR_INVALID_ARG, "unknown assignment operator");
    if (B->ptr_type != A->ptr_type || B->val_type != A->val_type)
        return fail(h, HP_ERR_INVALID_ARG, "B must have A's ptr_type and val_type");
    if ((B->nrows > 0 && !I) || (B->ncols > 0 && !J)) return fail(h, HP_ERR_INVALID_ARG, "I or J is NULL");
    if (C->nrows != A->nrows || C->ncols != A->ncols) return fail(h, HP_ERR_SHAPE, "C must have A's shape");
    if (C->ptr_type != A->ptr_type || C->val_type != A->val_type)
        return fail(h, HP_ERR_INVALID_ARG, "C must have A's ptr_type and val_type");
    if (!C->rowptr) return fail(h, HP_ERR_INVALID_ARG, "C->rowptr is NULL");
    return HP_OK;
}

inline int gridn(int64_t n, int per = 256) { return (int)std::max<int64_t>(1, (n + per - 1) / per); }

// Fused exec workspace with row slots: the sort temporaries, then m slots
// from the first 256-byte boundary after them, wherever the workspace starts.
size_t fused_xws_bytes(size_t seg_bytes, int64_t m, int vs) {
    const size_t sb = vs == 8 ? perm::perm_slot_bytes<uint64_t>() : perm::perm_slot_bytes<uint32_t>();
    return ((seg_bytes + 255) & ~size_t(255)) + 256 + (((size_t)m * sb + 255) & ~size_t(255));
}

// Plan of the assignment; with fused, also of the permutation of its result
// (C = P (A (+) B') Q^T, p non-null, q null for the symmetric form).
template <typename PT, typename VT>
hp_status_t asg_plan_t(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B, const int32_t *I,
                       const int32_t *J, hp_asgn_op_t op, hp_csr_t *C, void *ws, size_t ws_bytes,
                       hp_plan_info_t *info, bool fused = false, const int32_t *p = nullptr,
                       const int32_t *q = nullptr) {
    const int64_t m = A->nrows, n = A->ncols, nI = B->nrows, nJ = B->ncols;
    const bool sym = fused && q == nullptr;
    Carve need(nullptr);
    asg_layout(need, m, n, A->nnz, B->nnz, fused, sym);
    if (!ws || ws_bytes < need.size()) return fail(h, HP_ERR_WORKSPACE, "spasgn plan workspace too small");
    const size_t ps = sizeof(PT), vs = sizeof(VT);
    const void *ins[] = {A->rowptr, A->col, A->val, B->rowptr, B->col, B->val, I, J, p, q};
    const size_t insz[] = {(size_t)(m + 1) * ps, (size_t)A->nnz * 4, (size_t)A->nnz * vs,
                           (size_t)(nI + 1) * ps, (size_t)B->nnz * 4, (size_t)B->nnz * vs,
                           (size_t)nI * 4, (size_t)nJ * 4, p ? (size_t)m * 4 : 0, q ? (size_t)n * 4 : 0};
    for (int k = 0; k < 10; k++)
        if (overlaps(C->rowptr, (m + 1) * ps, ins[k], insz[k]) || overlaps(ws, ws_bytes, ins[k], insz[k]))
            return fail(h, HP_ERR_ALIAS, "output or workspace overlaps an input");
    if (overlaps(C->rowptr, (m + 1) * ps, ws, ws_bytes))
        return fail(h, HP_ERR_ALIAS, "C->rowptr overlaps the workspace");
    Carve c(ws);
    AsgLayout L = asg_layout(c, m, n, A->nnz, B->nnz, fused, sym);
    hipStream_t s = h->stream;
    if (hp_status_t v = validate_input(h, A, L.hdr, "spasgn plan: A")) return v;
    if (hp_status_t v = validate_input(h, B, L.hdr, "spasgn plan: B")) return v;
    stage_begin(h);
    hipError_t e = launch_init_hdr(s, L.hdr, L.tiles, scan_tiles(m));
    if (e == hipSuccess) e = launch_fill_words(s, L.rowinv, (size_t)m, 0xFFFFFFFFu);
    if (e == hipSuccess) e = launch_fill_words(s, L.colinv, (size_t)n, 0xFFFFFFFFu);
    if (fused) {
        if (e == hipSuccess) e = launch_fill_words(s, L.pinv, (size_t)m, 0xFFFFFFFFu);
        if (e == hipSuccess && !sym) e = launch_fill_words(s, L.qinv, (size_t)n, 0xFFFFFFFFu);
    }
    if (e == hipSuccess) {
        const int64_t hi = std::max(nI, nJ);
        hipLaunchKernelGGL(k_asg_inv, dim3(gridn(hi)), dim3(256), 0, s, I, nI, J, nJ, m, n, L.rowinv,
                           L.colinv, L.hdr);
        hipLaunchKernelGGL(k_asg_dup, dim3(gridn(hi)), dim3(256), 0, s, I, nI, J, nJ, m, n, L.rowinv,
                           L.colinv, L.hdr);
        stage_mark(h, "asgn.tables");
        e = launch_clear_words(s, L.lcount, 4);   // llist, rlong, rhuge and hlist counts
        hipLaunchKernelGGL(k_asg_count_rest<PT>, dim3(gridn(m)), dim3(256), 0, s, (const PT *)A->rowptr, m,
                           L.rowinv, L.cnt, L.force, L.rlong, L.rhuge, L.lcount + 1, L.hdr);
        if (nI > 0) {
            hipLaunchKernelGGL(k_asg_count_I<PT>, dim3(gridn(nI, 256 / AS_G)), dim3(256), 0, s,
                               (const PT *)A->rowptr, A->col, (const PT *)B->rowptr, B->col, I, nI, J, nJ, L.colinv,
                               n, (int)op, L.cnt, L.force, L.llist, L.lcount, L.hdr);
            hipLaunchKernelGGL((k_asg_rows_list<PT, VT, true>), dim3((unsigned)std::min<int64_t>(gridn(nI, 4), 1024)),
                               dim3(256), 0, s, (const PT *)A->rowptr, A->col, (const VT *)A->val,
                               (const PT *)B->rowptr, B->col, (const VT *)B->val, I, J, nJ, L.colinv, n, (int)op,
                               (const PT *)nullptr, (int32_t *)nullptr, (VT *)nullptr, L.cnt, L.force, L.llist,
                               L.lcount, L.hdr, OutMap{nullptr, nullptr, 0}, L.hlist, L.lcount + 3);
            hipLaunchKernelGGL((k_asg_rows_huge<PT, VT, true>), dim3(1024), dim3(256), 0, s, (const PT *)A->rowptr,
                               A->col, (const VT *)A->val, (const PT *)B->rowptr, B->col, (const VT *)B->val, I, J,
                               nJ, L.colinv, n, (int)op, (const PT *)nullptr, (int32_t *)nullptr, (VT *)nullptr,
                               L.cnt, (const int32_t *)L.hlist, (const uint32_t *)(L.lcount + 3), L.hcur, L.hdr,
                               OutMap{nullptr, nullptr, 0});
        }
        stage_mark(h, "asgn.count");
        e = hipGetLastError();
    }
    if (e == hipSuccess && fused) {
        const int64_t hi = std::max(m, n);
        if (nI > 0)
            hipLaunchKernelGGL(k_fused_mark<PT>, dim3(gridn(nI)), dim3(256), 0, s, I, nI, m, (const PT *)A->rowptr,
                               L.cnt, L.force, (int)(B->nnz > (int64_t)WAVE * nI), L.hdr);
        launch_clear_words(s, L.fsum, FSUM_SLOTS * 2 * 8 * 2);
        hipLaunchKernelGGL(k_fused_counts, dim3(gridn(m)), dim3(256), 0, s, p, nullptr, m, n, L.cnt,
                           (const uint8_t *)L.force, L.pinv, L.qinv,
                           L.cnt_out, L.fflag, L.fsum, L.hdr);
        hipLaunchKernelGGL(k_fused_sum, dim3(1), dim3(64), 0, s, (const unsigned long long *)L.fsum, L.hdr);
        if (!sym) hipLaunchKernelGGL(k_fused_qinv, dim3(gridn(n)), dim3(256), 0, s, q, n, L.qinv, L.hdr);
        hipLaunchKernelGGL(k_fused_check, dim3(gridn(hi, 1024)), dim3(256), 0, s, m, n, L.pinv, L.qinv, !sym, L.hdr);
        // flagged output rows only: classification mode 4
        e = launch_scan_counts<PT>(s, L.cnt_out, (PT *)C->rowptr, m, L.hdr, 0, L.tiles, 4, L.lists, m, L.fflag);
        stage_mark(h, "asgn.scan");
    } else if (e == hipSuccess) {
        e = launch_scan_counts<PT>(s, L.cnt, (PT *)C->rowptr, m, L.hdr, 0, L.tiles, 4, L.lists, m, L.force);
        stage_mark(h, "asgn.scan");
    }
    if (e != hipSuccess) return hip_check(h, e, "spasgn plan");
    if (hp_status_t rb = readback_hdr(h, L.hdr, "spasgn plan")) return rb;
    stage_end(h);
    const DevHdr &H = *h->host_hdr;
    hp_status_t stt = status_from_err(h, H.err, "spasgn");
    if (stt) return stt;
    C->nnz = (int64_t)H.total[0];
    if (info) {
        *info = hp_plan_info_t{};
        info->nnz_out = C->nnz;
        info->op = fused ? 4 : 3;
        for (int b = 0; b < NBINS; b++) {
            info->rows_sorted[b] = H.bin_cnt[b];
            info->class_elems[b] = (int64_t)H.bin_elems[b];
        }
        info->aux[0] = (int64_t)op;
        info->aux[1] = (H.flags & F_NOT_RANGE) ? 0 : 1;   // J contiguous
        info->aux[2] = sym ? 1 : 0;
        info->exec_ws_bytes = seg_tmp_bytes(H.bin_elems[BIN_GLOBAL], H.bin_cnt[BIN_GLOBAL], vs, n);
        // fused: aux[3] the smallest exec workspace; exec_ws_bytes adds the
        // row slots when rows outside I of at most 4 entries hold at least
        // half of the entries outside I
        info->aux[3] = (int64_t)info->exec_ws_bytes;
        if (fused && H.aux[1] > 0 && 2 * H.aux[1] >= H.aux[0])
            info->exec_ws_bytes = fused_xws_bytes(info->exec_ws_bytes, m, (int)vs);
    }
    return HP_OK;
}

template <typename PT, typename VT>
hp_status_t asg_exec_t(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B, const int32_t *I,
                       const int32_t *J, hp_asgn_op_t op, hp_csr_t *C, void *ws, size_t ws_bytes,
                       const hp_plan_info_t *info, void *xws, size_t xws_bytes, bool fused = false,
                       const int32_t *p = nullptr, const int32_t *q = nullptr) {
    const int64_t m = A->nrows, n = A->ncols, nI = B->nrows, nJ = B->ncols;
    const bool sym = fused && q == nullptr;
    Carve need(nullptr);
    asg_layout(need, m, n, A->nnz, B->nnz, fused, sym);
    if (!ws || ws_bytes < need.size()) return fail(h, HP_ERR_WORKSPACE, "spasgn workspace too small");
    if (!info || info->op != (fused ? 4 : 3) || info->aux[0] != (int64_t)op)
        return fail(h, HP_ERR_INVALID_ARG,
                    fused ? "info is not from hp_spasgn_permute_plan with this operator"
                          : "info is not from hp_spasgn_plan with this operator");
    if (fused && info->aux[2] != (q ? 0 : 1))
        return fail(h, HP_ERR_INVALID_ARG, "q differs in nullness from the plan");
    const size_t xmin = fused ? (size_t)info->aux[3] : info->exec_ws_bytes;
    if (xws_bytes < xmin || (xmin && !xws)) return fail(h, HP_ERR_WORKSPACE, "spasgn exec workspace too small");
    if (C->nnz != info->nnz_out) return fail(h, HP_ERR_INVALID_ARG, "C->nnz differs from the plan");
    if (C->nnz > 0 && (!C->col || !C->val)) return fail(h, HP_ERR_INVALID_ARG, "C->col/val is NULL");
    const size_t vs = sizeof(VT), ps = sizeof(PT);
    const void *ins[] = {A->rowptr, A->col, A->val, B->rowptr, B->col, B->val, I, J, ws, xws, C->rowptr, p, q};
    const size_t insz[] = {(size_t)(m + 1) * ps, (size_t)A->nnz * 4, (size_t)A->nnz * vs,
                           (size_t)(nI + 1) * ps, (size_t)B->nnz * 4, (size_t)B->nnz * vs,
                           (size_t)nI * 4, (size_t)nJ * 4, ws_bytes, xws_bytes, (size_t)(m + 1) * ps,
                           p ? (size_t)m * 4 : 0, q ? (size_t)n * 4 : 0};
    for (int k = 0; k < 13; k++)
        if (overlaps(C->col, (size_t)C->nnz * 4, ins[k], insz[k]) ||
            overlaps(C->val, (size_t)C->nnz * vs, ins[k], insz[k]))
            return fail(h, HP_ERR_ALIAS, "C->col/val overlaps an input or workspace");
    Carve c(ws);
    AsgLayout L = asg_layout(c, m, n, A->nnz, B->nnz, fused, sym);
    const OutMap om{L.pinv, L.qinv, n};   // null maps for the plain assignment
    hipStream_t s = h->stream;
    stage_begin(h);
    if (fused) {
        // row slots when the plan asked for them and the workspace holds them
        const bool slots = info->exec_ws_bytes > xmin && xws_bytes >= info->exec_ws_bytes;
        char *sl = nullptr;
        if (slots) {
            const uintptr_t at = (uintptr_t)xws + ((xmin + 255) & ~size_t(255));
            sl = (char *)((at + 255) & ~uintptr_t(255));
            hipLaunchKernelGGL((k_fused_pack<PT, VT>), dim3(gridn(m)), dim3(256), 0, s, (const PT *)A->rowptr,
                               A->col, (const VT *)A->val, L.qinv, n, m, sl);
        }
        hipLaunchKernelGGL((k_fused_fill_short<PT, VT>), dim3(gridn(m)), dim3(256), 0, s, p, L.fflag,
                           (const PT *)A->rowptr, A->col, (const VT *)A->val, L.qinv, n, (const char *)sl,
                           (const PT *)C->rowptr, C->col, (VT *)C->val, m, L.hdr);
    } else
        hipLaunchKernelGGL((k_asg_copy_rest<PT, VT>), dim3(gridn(m)), dim3(256), 0, s, (const PT *)A->rowptr,
                           A->col, (const VT *)A->val, m, L.rowinv, (const PT *)C->rowptr, C->col, (VT *)C->val,
                           L.hdr, om);
    if (!fused)   // the fused sort pass fills long rows outside I from A
        hipLaunchKernelGGL((k_asg_copy_long<PT, VT>), dim3(2048), dim3(256), 0, s, (const PT *)A->rowptr, A->col,
                           (const VT *)A->val, L.rlong, L.rhuge, L.lcount + 1, (const PT *)C->rowptr, C->col,
                           (VT *)C->val, L.hdr, om);
    stage_mark(h, "asgn.copy");
    if (nI > 0) {
        launch_clear_words(s, L.lcount, 1);       // llist (rlong/rhuge counts stay from the plan)
        launch_clear_words(s, L.lcount + 3, 1);   // hlist
        launch_clear_words(s, L.hcur, (size_t)L.hcap);
        if (B->nnz > (int64_t)WAVE * nI)   // long B rows: one wavefront per row
            hipLaunchKernelGGL((k_asg_merge_row<PT, VT>), dim3(gridn(nI, 256 / WAVE)), dim3(256), 0, s,
                               (const PT *)A->rowptr, A->col, (const VT *)A->val, (const PT *)B->rowptr, B->col,
                               (const VT *)B->val, I, nI, J, nJ, L.colinv, n, (int)op, (const PT *)C->rowptr, C->col,
                               (VT *)C->val, L.llist, L.lcount, (int)info->aux[1], L.hdr, om);
        else
            hipLaunchKernelGGL((k_asg_merge_I<PT, VT>), dim3(gridn(nI, 256 / AS_G)), dim3(256), 0, s,
                               (const PT *)A->rowptr, A->col, (const VT *)A->val, (const PT *)B->rowptr, B->col,
                               (const VT *)B->val, I, nI, J, nJ, L.colinv, n, (int)op, (const PT *)C->rowptr, C->col,
                               (VT *)C->val, L.llist, L.lcount, (int)info->aux[1], L.hdr, om);
        hipLaunchKernelGGL((k_asg_rows_list<PT, VT, false>), dim3((unsigned)std::min<int64_t>(gridn(nI, 4), 1024)),
                           dim3(256), 0, s, (const PT *)A->rowptr, A->col, (const VT *)A->val, (const PT *)B->rowptr,
                           B->col, (const VT *)B->val, I, J, nJ, L.colinv, n, (int)op, (const PT *)C->rowptr, C->col,
                           (VT *)C->val, L.cnt, L.force, L.llist, L.lcount, L.hdr, om, L.hlist, L.lcount + 3);
        hipLaunchKernelGGL((k_asg_rows_huge<PT, VT, false>), dim3(1024), dim3(256), 0, s, (const PT *)A->rowptr,
                           A->col, (const VT *)A->val, (const PT *)B->rowptr, B->col, (const VT *)B->val, I, J, nJ,
                           L.colinv, n, (int)op, (const PT *)C->rowptr, C->col, (VT *)C->val, L.cnt,
                           (const int32_t *)L.hlist, (const uint32_t *)(L.lcount + 3), L.hcur, L.hdr, om);
    }
    stage_mark(h, "asgn.merge");
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        uint32_t cnt[NBINS];
        for (int b = 0; b < NBINS; b++) cnt[b] = (uint32_t)info->rows_sorted[b];
        if (fused) {
            LoadFused<PT, VT> ld{(const PT *)A->rowptr, A->col, (const VT *)A->val, p, L.qinv, n,
                                 (const PT *)C->rowptr, C->col, (const VT *)C->val, L.fflag};
            e = launch_seg_classes<PT, VT, LoadFused<PT, VT>>(s, (const PT *)C->rowptr, C->col, (VT *)C->val,
                                                              L.lists, m, cnt, ld, false, n, true, xws,
                                                              (uint64_t)info->class_elems[BIN_GLOBAL], L.hdr, true);
        } else {
            LoadInPlace<PT, VT> ld{(const PT *)C->rowptr, C->col, (const VT *)C->val};
            e = launch_seg_classes<PT, VT, LoadInPlace<PT, VT>>(s, (const PT *)C->rowptr, C->col, (VT *)C->val,
                                                                L.lists, m, cnt, ld, false, n, true, xws,
                                                                (uint64_t)info->class_elems[BIN_GLOBAL], L.hdr,
                                                                true);
        }
        stage_mark(h, "asgn.sort");
    }
    stage_end(h);
    return hip_check(h, e == hipSuccess ? hipGetLastError() : e, "spasgn exec");
}

}  // namespace

extern "C" hp_status_t hp_spasgn_workspace(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                           size_t *bytes) {
    if (!h || !bytes) return HP_ERR_INVALID_ARG;
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    if (!B) return fail(h, HP_ERR_INVALID_ARG, "B is NULL (the workspace depends on nnz(B))");
    Carve c(nullptr);
    asg_layout(c, A->nrows, A->ncols, A->nnz, B->nnz);
    *bytes = c.size();
    return HP_OK;
}

extern "C" hp_status_t hp_spasgn_plan(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                      const int32_t *I, const int32_t *J, hp_asgn_op_t op, hp_csr_t *C,
                                      void *ws, size_t ws_bytes, hp_plan_info_t *info) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = asg_check_args(h, A, B, I, J, op, C);
    if (st) return st;
    const bool p64 = A->ptr_type == HP_IDX_I64, v64 = A->val_type == HP_VAL_F64;
    if (!p64 && !v64) return asg_plan_t<int32_t, uint32_t>(h, A, B, I, J, op, C, ws, ws_bytes, info);
    if (!p64 && v64) return asg_plan_t<int32_t, uint64_t>(h, A, B, I, J, op, C, ws, ws_bytes, info);
    if (p64 && !v64) return asg_plan_t<int64_t, uint32_t>(h, A, B, I, J, op, C, ws, ws_bytes, info);
    return asg_plan_t<int64_t, uint64_t>(h, A, B, I, J, op, C, ws, ws_bytes, info);
}

extern "C" hp_status_t hp_spasgn_exec(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                      const int32_t *I, const int32_t *J, hp_asgn_op_t op, hp_csr_t *C,
                                      void *ws, size_t ws_bytes, const hp_plan_info_t *info, void *xws,
                                      size_t xws_bytes) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = asg_check_args(h, A, B, I, J, op, C);
    if (st) return st;
    const bool p64 = A->ptr_type == HP_IDX_I64, v64 = A->val_type == HP_VAL_F64;
    if (!p64 && !v64) return asg_exec_t<int32_t, uint32_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, xws, xws_bytes);
    if (!p64 && v64) return asg_exec_t<int32_t, uint64_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, xws, xws_bytes);
    if (p64 && !v64) return asg_exec_t<int64_t, uint32_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, xws, xws_bytes);
    return asg_exec_t<int64_t, uint64_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, xws, xws_bytes);
}

namespace {
hp_status_t fused_check_args(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B, const int32_t *I,
                             const int32_t *J, hp_asgn_op_t op, const int32_t *p, const int32_t *q,
                             const hp_csr_t *C) {
    hp_status_t st = asg_check_args(h, A, B, I, J, op, C);
    if (st) return st;
    if (!q && A->nrows != A->ncols) return fail(h, HP_ERR_SHAPE, "symmetric permute needs a square A");
    if (A->nrows > 0 && !p) return fail(h, HP_ERR_INVALID_ARG, "p is NULL");
    return HP_OK;
}
}  // namespace

extern "C" hp_status_t hp_spasgn_permute_workspace(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                                   size_t *bytes) {
    if (!h || !bytes) return HP_ERR_INVALID_ARG;
    hp_status_t st = check_csr_args(h, A, "A");
    if (st) return st;
    if (!B) return fail(h, HP_ERR_INVALID_ARG, "B is NULL (the workspace depends on nnz(B))");
    Carve c(nullptr);
    asg_layout(c, A->nrows, A->ncols, A->nnz, B->nnz, true, false);
    *bytes = c.size();
    return HP_OK;
}

extern "C" hp_status_t hp_spasgn_permute_plan(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                              const int32_t *I, const int32_t *J, hp_asgn_op_t op,
                                              const int32_t *p, const int32_t *q, hp_csr_t *C, void *ws,
                                              size_t ws_bytes, hp_plan_info_t *info) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = fused_check_args(h, A, B, I, J, op, p, q, C);
    if (st) return st;
    const bool p64 = A->ptr_type == HP_IDX_I64, v64 = A->val_type == HP_VAL_F64;
    if (!p64 && !v64) return asg_plan_t<int32_t, uint32_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, true, p, q);
    if (!p64 && v64) return asg_plan_t<int32_t, uint64_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, true, p, q);
    if (p64 && !v64) return asg_plan_t<int64_t, uint32_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, true, p, q);
    return asg_plan_t<int64_t, uint64_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, true, p, q);
}

extern "C" hp_status_t hp_spasgn_permute_exec(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                              const int32_t *I, const int32_t *J, hp_asgn_op_t op,
                                              const int32_t *p, const int32_t *q, hp_csr_t *C, void *ws,
                                              size_t ws_bytes, const hp_plan_info_t *info, void *xws,
                                              size_t xws_bytes) {
    if (!h) return HP_ERR_INVALID_ARG;
    hp_status_t st = fused_check_args(h, A, B, I, J, op, p, q, C);
    if (st) return st;
    const bool p64 = A->ptr_type == HP_IDX_I64, v64 = A->val_type == HP_VAL_F64;
    if (!p64 && !v64)
        return asg_exec_t<int32_t, uint32_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, xws, xws_bytes, true, p, q);
    if (!p64 && v64)
        return asg_exec_t<int32_t, uint64_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, xws, xws_bytes, true, p, q);
    if (p64 && !v64)
        return asg_exec_t<int64_t, uint32_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, xws, xws_bytes, true, p, q);
    return asg_exec_t<int64_t, uint64_t>(h, A, B, I, J, op, C, ws, ws_bytes, info, xws, xws_bytes, true, p, q);
}
