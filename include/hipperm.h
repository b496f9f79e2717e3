/*
 * hipperm.h -- C ABI of an MI355X (gfx950) library for sparse-matrix
 * permutation, submatrix extraction and submatrix assignment on CSR
 * matrices held in one GPU's HBM.
 *
 * Operations (definitions from the problem formulation of the paper
 * "Distributed-memory Algorithms for Sparse Matrix Permutation, Extraction,
 * and Assignment", Sec. 2):
 *   permute : C[i,j] = A[p[i], q[j]]          (Sec. 2.1; C = P A Q^T)
 *   spref   : C[i,j] = A[I[i], J[j]]  for (i,j) in I x J   (Sec. 2.2; C = R A Q^T)
 *   spasgn  : C = A (+) B', B'[I[i], J[j]] = B[i,j] for stored B entries
 *             (Sec. 2.3 and the Add step of Sec. 4.7; user-chosen addition)
 *
 * Conventions for every call:
 *   - All matrix and index arrays are DEVICE pointers on the handle's
 *     device.  The caller owns every buffer: inputs, outputs, workspaces.
 *     The library never allocates or frees caller memory; it owns only the
 *     handle (a stream, events and one pinned host scalar block).
 *   - Indices are 0-based (the paper counts from 1).
 *   - CSR is canonical: rowptr[0] = 0, non-decreasing; columns strictly
 *     ascending inside a row.  rowptr is int32 or int64 (hp_idx_t); columns
 *     are int32; values are fp32 or fp64 (hp_val_t) and are moved as raw
 *     bits, never re-rounded (except the one addition of HP_OP_PLUS).
 *   - Outputs are out-of-place: output arrays must not overlap inputs
 *     (HP_ERR_ALIAS when they share an address).
 *   - Work is enqueued on the handle's stream in order.  The plan calls end
 *     with one blocking readback of a few scalars (output size, error
 *     flags, bin statistics); exec calls never block.  The readback wait is
 *     a bounded poll: past the host wait limit (environment variable
 *     HP_HOST_WAIT_MS, default ten minutes) the plan returns HP_ERR_TIMEOUT,
 *     and the work it enqueued may still be running, so the stream must be
 *     synchronised before the buffers it uses are freed.
 *   - Errors are returned as hp_status_t; no exception crosses the ABI.
 *     hp_last_error() gives a message for the last failing call.
 *
 * Each operation is split in two:
 *   plan : validates indices, builds the inverse index tables, counts the
 *          nonzeros of every output row and scans them into C->rowptr;
 *          sets C->nnz and fills *info (blocking: one scalar readback).
 *   exec : writes C->col and C->val (sized C->nnz by the caller after plan).
 *          It must get the same arguments, the same plan workspace (untouched
 *          in between) and the info struct of a plan call that returned
 *          HP_OK, plus an exec workspace of at least info->exec_ws_bytes
 *          (may be NULL when that is 0).  Exec trusts the plan: the inputs
 *          (A, B, the index vectors) must hold the same values as at plan
 *          time, otherwise the behaviour is undefined.
 */
#ifndef HIPPERM_H
#define HIPPERM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HP_OK = 0,
    HP_ERR_INVALID_ARG = 1,      /* NULL pointer, negative size, bad enum          */
    HP_ERR_INDEX_RANGE = 2,      /* an index outside [0, nrows) or [0, ncols)      */
    HP_ERR_NOT_PERMUTATION = 3,  /* permute: p or q repeats a value                */
    HP_ERR_DUPLICATE_INDEX = 4,  /* spasgn: I or J repeats a value (Sec. 2.3)      */
    HP_ERR_NOT_CANONICAL = 5,    /* hp_validate_csr: unsorted/duplicate columns    */
    HP_ERR_SHAPE = 6,            /* B is not |I| x |J|; symmetric permute on m != n */
    HP_ERR_OVERFLOW = 7,         /* output nnz does not fit an int32 rowptr        */
    HP_ERR_WORKSPACE = 8,        /* workspace smaller than the queried size        */
    HP_ERR_CAPACITY = 9,         /* batched: an output exceeded its arena slot     */
    HP_ERR_HIP = 10,             /* a HIP runtime call failed                      */
    HP_ERR_ALIAS = 11,           /* an output array overlaps an input array        */
    HP_ERR_TIMEOUT = 12,         /* a bounded wait (device or host side) gave up   */
    HP_ERR_REJECTED = 13         /* served form: request can never fit the budget  */
} hp_status_t;

typedef enum { HP_IDX_I32 = 0, HP_IDX_I64 = 1 } hp_idx_t;
typedef enum { HP_VAL_F32 = 0, HP_VAL_F64 = 1 } hp_val_t;

/* Addition used by spasgn where A and B' both hold an entry (Sec. 2.3):
 *   SECOND  : B's value overwrites A's (select-second, the common variant);
 *   PLUS    : A + B in the value type, IEEE-754 round-to-nearest-even;
 *   REPLACE : block replace -- every A entry inside I x J is removed first,
 *             then B' is inserted (so A(I,J) == B afterwards). */
typedef enum { HP_OP_SECOND = 0, HP_OP_PLUS = 1, HP_OP_REPLACE = 2 } hp_asgn_op_t;

typedef struct {
    int64_t nrows, ncols, nnz;
    int32_t ptr_type;   /* hp_idx_t */
    int32_t val_type;   /* hp_val_t */
    void *rowptr;       /* device, nrows+1 entries of ptr_type   */
    int32_t *col;       /* device, nnz entries                   */
    void *val;          /* device, nnz entries of val_type       */
} hp_csr_t;

/* Column-compressed matrix (Sec. 4.1 of the paper stores local blocks this
 * way).  dcsc == 0: CSC, colptr holds ncols+1 entries; jc and nzc are
 * ignored.  dcsc == 1: DCSC (doubly compressed, for hypersparse matrices):
 * only the nzc stored columns are kept, jc[k] is the column id of stored
 * column k (strictly increasing; jc may be NULL only when nzc == 0), colptr
 * holds nzc+1 entries.  Row indices are strictly increasing within each
 * column.  All arrays are device memory owned by the caller. */
typedef struct {
    int64_t nrows, ncols, nnz, nzc;
    int32_t ptr_type;   /* hp_idx_t, of colptr  */
    int32_t val_type;   /* hp_val_t             */
    int32_t dcsc;       /* 0: CSC, 1: DCSC      */
    int32_t pad;
    const int32_t *jc;  /* nzc entries (DCSC)   */
    void *colptr;       /* nzc+1 (DCSC) or ncols+1 (CSC) entries of ptr_type */
    int32_t *row;       /* nnz entries          */
    void *val;          /* nnz entries of val_type */
} hp_dcsc_t;

/* Filled by every plan call and passed unchanged to the matching exec call
 * (exec needs the class sizes to size its launches without a readback). */
typedef struct {
    int64_t nnz_out;          /* nonzeros of C (also stored in C->nnz)              */
    size_t exec_ws_bytes;     /* exec workspace the following exec call needs       */
    int32_t map_monotone;     /* 1 when the column map keeps order (no row sort)    */
    int32_t op;               /* which operation produced it (internal check)       */
    int64_t rows_sorted[4];   /* output rows per sort class: <=16, <=64, <=4096, >  */
    int64_t class_elems[4];   /* entries per sort class                             */
    int64_t aux[4];           /* operation-specific counts (permute: aux[0], fused
                                 assign-and-permute: aux[3] is the smallest exec
                                 workspace exec accepts)                            */
} hp_plan_info_t;

typedef struct hp_handle_s *hp_handle_t;

/* ---- handle ------------------------------------------------------------ */

/* Create a handle bound to HIP device `device`, using the default (null)
 * stream.  *h is set only on success. */
hp_status_t hp_create(hp_handle_t *h, int device);
hp_status_t hp_destroy(hp_handle_t h);
/* Enqueue all later work of this handle on `stream` (a hipStream_t). */
hp_status_t hp_set_stream(hp_handle_t h, void *stream);
const char *hp_status_string(hp_status_t s);
/* Message for the last failing call on h (static storage in the handle). */
const char *hp_last_error(hp_handle_t h);

/* Per-stage device timing: when enabled, every plan/exec records HIP events
 * on the handle's stream around each kernel stage (no extra synchronisation).
 * hp_stage_times waits for the last recorded event, then reports for up to
 * `cap` distinct stage names the total milliseconds and the number of
 * launches since the previous call, and clears the record.  Returns the
 * number of stages written; names point to static strings. */
hp_status_t hp_enable_timing(hp_handle_t h, int enable);
int hp_stage_times(hp_handle_t h, float *ms_total, int *count, const char **names, int cap);

/* Canonical-CSR check (rowptr monotone, columns in range, strictly
 * ascending in each row).  Returns HP_OK, HP_ERR_NOT_CANONICAL or
 * HP_ERR_INDEX_RANGE.  ws must hold hp_validate_workspace() bytes. */
/* Input validation inside the plans: when enabled, every plan on CSR input
 * (permute, spref, spasgn and the fused form; A, and B for assignments)
 * first runs the canonical-CSR check above on its inputs, with one extra
 * blocking readback, and returns HP_ERR_NOT_CANONICAL or HP_ERR_INDEX_RANGE
 * before launching anything else.  Off by default (non-canonical input is
 * then undefined behaviour); hp_create switches it on when the environment
 * variable HP_VALIDATE is set to anything but "0". */
hp_status_t hp_set_validate(hp_handle_t h, int enable);
hp_status_t hp_validate_workspace(hp_handle_t h, const hp_csr_t *A, size_t *bytes);
hp_status_t hp_validate_csr(hp_handle_t h, const hp_csr_t *A, void *ws, size_t ws_bytes);

/* ---- permute: C = P A Q^T, C[i,j] = A[p[i], q[j]] (Sec. 2.1) ----------- */
/* p: m entries, a permutation of [0, m); q: n entries, a permutation of
 * [0, n), or NULL for the symmetric form P A P^T (requires m == n).
 * C: caller sets nrows=m, ncols=n, ptr_type/val_type equal to A's and
 * rowptr (m+1 entries); plan writes rowptr and nnz (= nnz(A)).
 * Exec workspace: info->exec_ws_bytes is the workspace of the fastest form;
 * when rows of at most 4 entries hold at least half of the entries it
 * includes one fixed slot per row of A (32 bytes for 4-byte values, 64 for
 * 8-byte ones) into which exec first packs those rows.  info->aux[0] is the
 * smallest exec workspace exec accepts: given less than exec_ws_bytes (but
 * at least aux[0]) bytes, exec runs without the slots; the result is the
 * same.  The workspace may start at any address.
 * Errors: INDEX_RANGE, NOT_PERMUTATION, SHAPE, WORKSPACE, ALIAS. */
hp_status_t hp_permute_workspace(hp_handle_t h, const hp_csr_t *A, size_t *bytes);
hp_status_t hp_permute_plan(hp_handle_t h, const hp_csr_t *A, const int32_t *p, const int32_t *q,
                            hp_csr_t *C, void *ws, size_t ws_bytes, hp_plan_info_t *info);
hp_status_t hp_permute_exec(hp_handle_t h, const hp_csr_t *A, const int32_t *p, const int32_t *q,
                            hp_csr_t *C, void *ws, size_t ws_bytes, const hp_plan_info_t *info,
                            void *xws, size_t xws_bytes);

/* ---- permute that allocates nothing --------------------------------------- */
/* For callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  hp_permute_plan and
 * hp_permute_exec in one call, with both workspaces taken from a fixed
 * device array inside the library (HP_NOALLOC_SCRATCH_BYTES on every device
 * the library runs on, held until the process ends) instead of caller
 * workspaces.  The call allocates nothing (no hipMalloc or hipFree, no
 * event or stream creation); like the plan it blocks once, on the readback
 * of the output's row classes.
 * A, p, q: as hp_permute_plan.  C: as hp_permute_plan, and C->col and
 * C->val must hold nnz(A) entries (a permutation keeps nnz); plan writes
 * C->rowptr and C->nnz, exec C->col and C->val.
 * Limit: the plan workspace (hp_permute_workspace: about 33 bytes per row
 * of a square matrix) and the smallest exec workspace (info->aux[0] of the
 * plan: temporaries for rows longer than 2048 entries only) must fit the
 * array together, e.g. 1M rows with rows of up to 2048 entries; otherwise
 * HP_ERR_WORKSPACE (when only the exec part does not fit, C->rowptr has
 * already been written).  The exec runs with the row slots of
 * hp_permute_exec when the array holds them too.
 * Stage timing must be off (HP_ERR_INVALID_ARG).
 * Every call on one device shares that device's array, which keeps the
 * last call's contents; each call clears what it needs cleared (status
 * block, scan tiles, inverse maps) before use.  Calls that overlap on one
 * device (other threads, other streams or handles) race on the array and
 * give undefined results: serialise them.
 * Errors: as hp_permute_plan and hp_permute_exec, plus WORKSPACE. */
#define HP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
hp_status_t hp_permute_noalloc(hp_handle_t h, const hp_csr_t *A, const int32_t *p, const int32_t *q,
                               hp_csr_t *C);

/* ---- spref: C = A(I, J), C[i,j] = A[I[i], J[j]] (Sec. 2.2) -------------- */
/* I (nI entries) and J (nJ entries) may repeat values and be in any order:
 * a repeated row (column) is replicated, order follows I and J.
 * C: caller sets nrows=nI, ncols=nJ, types equal to A's, rowptr (nI+1).
 * Errors: INDEX_RANGE, OVERFLOW (int32 rowptr and nnz(C) >= 2^31),
 * WORKSPACE, ALIAS. */
hp_status_t hp_spref_workspace(hp_handle_t h, const hp_csr_t *A, int64_t nI, int64_t nJ,
                               size_t *bytes);
hp_status_t hp_spref_plan(hp_handle_t h, const hp_csr_t *A, const int32_t *I, int64_t nI,
                          const int32_t *J, int64_t nJ, hp_csr_t *C, void *ws, size_t ws_bytes,
                          hp_plan_info_t *info);
hp_status_t hp_spref_exec(hp_handle_t h, const hp_csr_t *A, const int32_t *I, int64_t nI,
                          const int32_t *J, int64_t nJ, hp_csr_t *C, void *ws, size_t ws_bytes,
                          const hp_plan_info_t *info, void *xws, size_t xws_bytes);

/* ---- spref on column-compressed input (Sec. 2.2; Alg. 5 of the appendix) -- */
/* C = A(I, J) for A in CSC or DCSC, with C returned in CSC: column j of C is
 * column J[j] of A restricted to the rows of I, in the order of I.  This is
 * the column-oriented form of the extraction (the appendix's algorithm
 * walks the selected columns and looks each selected row up in them); a
 * column of J that a DCSC matrix does not store gives an empty column of C.
 * I, J: as hp_spref (repeats and any order allowed).
 * C: caller sets nrows=nI, ncols=nJ, ptr_type/val_type equal to A's,
 * dcsc=0, colptr (nJ+1 entries); plan writes colptr and nnz, exec writes
 * row and val.  ws from hp_spref_dcsc_workspace, kept from plan to exec.
 * Errors: INDEX_RANGE, OVERFLOW, SHAPE, WORKSPACE, ALIAS. */
hp_status_t hp_spref_dcsc_workspace(hp_handle_t h, const hp_dcsc_t *A, int64_t nI, int64_t nJ,
                                    size_t *bytes);
hp_status_t hp_spref_dcsc_plan(hp_handle_t h, const hp_dcsc_t *A, const int32_t *I, int64_t nI,
                               const int32_t *J, int64_t nJ, hp_dcsc_t *C, void *ws, size_t ws_bytes,
                               hp_plan_info_t *info);
hp_status_t hp_spref_dcsc_exec(hp_handle_t h, const hp_dcsc_t *A, const int32_t *I, int64_t nI,
                               const int32_t *J, int64_t nJ, hp_dcsc_t *C, void *ws, size_t ws_bytes,
                               const hp_plan_info_t *info, void *xws, size_t xws_bytes);

/* ---- spasgn: C = A with A(I, J) = B (Sec. 2.3, Sec. 4.7) ------------------ */
/* I, J: distinct indices (Sec. 2.3) of lengths B->nrows and B->ncols.
 * A and B share ptr_type and val_type.  C: caller sets nrows=m, ncols=n,
 * types equal to A's, rowptr (m+1).
 * The workspace size depends on A's shape and nnz and on nnz(B) (B must be
 * given; its arrays are not read).
 * Errors: INDEX_RANGE, DUPLICATE_INDEX, SHAPE, OVERFLOW, WORKSPACE, ALIAS. */
hp_status_t hp_spasgn_workspace(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                size_t *bytes);
hp_status_t hp_spasgn_plan(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B, const int32_t *I,
                           const int32_t *J, hp_asgn_op_t op, hp_csr_t *C, void *ws,
                           size_t ws_bytes, hp_plan_info_t *info);
hp_status_t hp_spasgn_exec(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B, const int32_t *I,
                           const int32_t *J, hp_asgn_op_t op, hp_csr_t *C, void *ws,
                           size_t ws_bytes, const hp_plan_info_t *info, void *xws,
                           size_t xws_bytes);

/* ---- fused assign and permute: C = P (A (+) B') Q^T (Sec. 5.8, Sec. 5.9) -- */
/* One pass that both assigns B into A(I, J) with operator op (as
 * hp_spasgn) and permutes the result (as hp_permute):
 *   C[i, j] = X[p[i], q[j]],  X = A with A(I, J) = B under op.
 * The paper fuses the two by changing only where entries are sent; here the
 * merge of each row of I writes straight to output row pinv[r] with its
 * columns mapped through qinv and a sort pass orders those rows (when B's
 * rows average over 64 entries, the merge sorts a row of at most 256
 * entries itself), while the
 * output rows outside I pull row p[i] of A (renamed, sorted in registers;
 * rows of at most 4 entries from fixed row slots packed first, as in
 * hp_permute_exec, when they hold at least half of the entries outside I).
 * The result is bit-identical to hp_spasgn followed by hp_permute.
 * I, J, op, B: as hp_spasgn.  p, q: as hp_permute (q NULL = symmetric form,
 * needs m == n; exec must get q NULL exactly when plan did).
 * C: caller sets nrows=m, ncols=n, types equal to A's, rowptr (m+1); plan
 * writes rowptr and nnz, exec writes col and val.  ws (size from
 * hp_spasgn_permute_workspace, independent of q; like hp_spasgn_workspace
 * it needs B for nnz(B)) must be kept unchanged
 * from plan to exec; xws holds info->exec_ws_bytes (with the row slots),
 * or at least info->aux[3] bytes (then exec runs without them; the result
 * is the same); it may start at any address.
 * Errors: INDEX_RANGE, DUPLICATE_INDEX, NOT_PERMUTATION, SHAPE, OVERFLOW,
 * WORKSPACE, ALIAS. */
hp_status_t hp_spasgn_permute_workspace(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                        size_t *bytes);
hp_status_t hp_spasgn_permute_plan(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                   const int32_t *I, const int32_t *J, hp_asgn_op_t op,
                                   const int32_t *p, const int32_t *q, hp_csr_t *C, void *ws,
                                   size_t ws_bytes, hp_plan_info_t *info);
hp_status_t hp_spasgn_permute_exec(hp_handle_t h, const hp_csr_t *A, const hp_csr_t *B,
                                   const int32_t *I, const int32_t *J, hp_asgn_op_t op,
                                   const int32_t *p, const int32_t *q, hp_csr_t *C, void *ws,
                                   size_t ws_bytes, const hp_plan_info_t *info, void *xws,
                                   size_t xws_bytes);

/* ---- incremental-update bookkeeping (Sec. 5.9) ----------------------------- */
/* The paper's incremental experiment rebuilds a graph from a large part by
 * assigning small parts back, one per step, each fused with a random
 * permutation, and tracks the load imbalance over a process grid.  These
 * three non-blocking calls are what a driver of that workload needs between
 * steps; all arrays are device int32 unless stated.
 *
 * hp_gather_index: out[t] = map[idx[t]] for t < n (relabels a part's
 *   original indices, or composes permutations); an idx entry outside
 *   [0, nmap) gives -1.  out may be idx itself (in place) but must not
 *   overlap map (ALIAS).
 * hp_invert_perm: pinv[p[t]] = t for t < n (p a permutation of [0, n);
 *   entries outside [0, n) are skipped, other slots of pinv are left as
 *   they were).  pinv must not overlap p (ALIAS).
 * hp_block_nnz: counts[bi * gc + bj] (uint64, gr * gc entries, overwritten)
 *   = stored entries of A in grid block (bi, bj), where row r belongs to
 *   grid row r * gr / nrows and column c to grid column c * gc / ncols.
 *   1 <= gr * gc <= 4096, gr, gc >= 1.  The load imbalance is the largest
 *   count over the mean. */
hp_status_t hp_gather_index(hp_handle_t h, const int32_t *map, int64_t nmap, const int32_t *idx,
                            int64_t n, int32_t *out);
hp_status_t hp_invert_perm(hp_handle_t h, const int32_t *p, int64_t n, int32_t *pinv);
hp_status_t hp_block_nnz(hp_handle_t h, const hp_csr_t *A, int32_t gr, int32_t gc, uint64_t *counts);

/* ---- batched form -------------------------------------------------------- */
/* Many extraction (paper Sec. 2.2, Alg. 3), permutation (Sec. 2.1, Alg. 1)
 * and assignment (Sec. 2.3, Alg. 4) requests run together.  The plan half
 * of the extractions and permutations (J tables / inverse permutations,
 * counts, rowptr scans of every request) is a short sequence of stage
 * launches, each running the tiles of every request on persistent
 * workgroups, followed by one readback of all output sizes.  The exec half
 * (fill and row sort of every request) is a second sequence of stage
 * launches, captured once in a hipGraph and replayed for any later batch
 * with the same workspace, arena, launch shapes and stage shapes.  Stream
 * order between the stages is the only inter-tile dependency.  Each stage's
 * launch shape (persistent workgroups, and consecutive tiles a workgroup
 * takes per ticket) is picked per size class by timing candidates the
 * first time the class is seen (the halves are idempotent; choices persist
 * in a cache file: HP_TUNE_CACHE, else ~/.cache/hipperm).  Assignment
 * requests (streaming merges of whole matrices) run the assignment's own
 * plan and exec kernels on the same stream, inside the same captured graph
 * for exec; their row pointers and plan tables live in the batch workspace.
 * Results are identical, bit for bit, to separate plain calls.
 * All requests of one batch share ptr_type and val_type.
 * Ownership: the caller owns the workspace and the arena; results point
 * into the arena.  hp_batch_exec must follow the hp_batch_plan of the same
 * batch on the same handle and workspace. */
typedef enum { HP_REQ_SPREF = 0, HP_REQ_PERMUTE = 1, HP_REQ_SPASGN = 2 } hp_req_kind_t;

typedef struct {
    int32_t kind;          /* hp_req_kind_t                                        */
    int32_t status;        /* out: hp_status_t of this request after plan/exec     */
    hp_csr_t A;            /* input matrix (device arrays)                         */
    const int32_t *I, *J;  /* spref, spasgn: row / column index vectors (device)   */
    int64_t nI, nJ;        /* lengths of I and J (spasgn: equal B's shape)         */
    const int32_t *p, *q;  /* permute: permutations (device); q NULL = symmetric    */
    hp_csr_t C;            /* out: shape/types/nnz after plan; rowptr/col/val point
                              into the arena after exec                            */
    hp_csr_t B;            /* spasgn: the |I| x |J| block                          */
    int32_t op;            /* spasgn: hp_asgn_op_t                                 */
    int32_t pad;
    void *ready;           /* served form only (the batched calls ignore it): a
                              hipEvent_t the caller recorded on its stream after
                              writing the inputs; the worker's stream waits for it
                              before reading them.  NULL: the inputs are complete
                              at submit.  Must stay valid until the request
                              completes.                                          */
} hp_request_t;

typedef struct {
    size_t arena_bytes;    /* arena the exec call needs                            */
    int64_t nnz_total;     /* sum of the requests' output nnz                       */
    int32_t failed;        /* requests whose plan status is not HP_OK               */
    int32_t grid_plan;     /* largest persistent grid of the plan stages (tuned)   */
    int64_t tiles_plan;    /* tiles over all plan stages                            */
    int64_t tiles_exec;    /* tiles over all exec stages (set by exec)              */
    int32_t grid_exec;     /* largest persistent grid of the exec stages (by exec) */
    int32_t flags;         /* in: HP_BATCH_NO_GRAPH, HP_BATCH_NO_TUNE               */
} hp_batch_info_t;

#define HP_BATCH_NO_GRAPH 1   /* launch exec directly instead of a captured graph   */
#define HP_BATCH_NO_TUNE 2    /* fixed launch shapes, no timing runs               */

/* Workspace for a batch (tables, counters and rowptrs of every request). */
hp_status_t hp_batch_workspace(hp_handle_t h, const hp_request_t *reqs, int n, size_t *bytes);
/* Plan every request: per-request status and C.nnz; info->arena_bytes.
 * Returns HP_OK even when single requests fail (see reqs[k].status). */
hp_status_t hp_batch_plan(hp_handle_t h, hp_request_t *reqs, int n, void *ws, size_t ws_bytes,
                          hp_batch_info_t *info);
/* Exec the planned requests into the caller's arena (rowptr, col, val of
 * every request with status HP_OK; failed requests are skipped). */
hp_status_t hp_batch_exec(hp_handle_t h, hp_request_t *reqs, int n, void *ws, size_t ws_bytes,
                          hp_batch_info_t *info, void *arena, size_t arena_bytes);

/* ---- served form ---------------------------------------------------------- */
/* A request server on one device.  Requests (extraction, assignment,
 * permutation) on caller-owned, resident, immutable matrices are submitted
 * as they arrive and complete asynchronously.  Worker threads, each with its
 * own handle and stream, take whatever requests are pending when they become
 * free (continuous batching): extraction and permutation requests of one
 * index/value type go through the batched calls above (up to max_batch per
 * batch), assignment requests and requests over matrices of more than 2^22
 * stored entries (which fill the GPU by themselves) through the plain
 * calls.  Up to max_inflight batches run at once on separate streams.
 * Memory: every workspace and every result is carved from the caller's
 * device buffer `pool` (pool_bytes, the HBM budget).  A batch is admitted
 * when its workspace fits the free pool space; after its plan, its exact
 * output arena must fit too.  While memory is short a batch waits for
 * running batches to finish; a batch that cannot fit while no other batch
 * runs waits (up to release_wait_ms) for the caller to release results, is
 * then split into single requests, and a single request that still cannot
 * fit completes with HP_ERR_REJECTED (unreleased results count as used).
 * Results stay in the pool until hp_server_release; the caller must have
 * finished every use of a result (synchronised the streams that read it)
 * before releasing it, since its pool space is then reused.
 * Stream order: the workers run on their own streams.  A request whose
 * inputs were written by asynchronous work carries a `ready` event (see
 * hp_request_t); a completion is reported only after the request's work has
 * finished on the device.
 * Waits: workers poll the device with the bounded wait of the plan calls; a
 * request whose work does not finish within the host wait limit
 * (HP_HOST_WAIT_MS, default ten minutes) completes with HP_ERR_TIMEOUT, and
 * its pool space is never reused.
 * Latency is measured on the host: submit, start of the request's batch,
 * and the end of its exec (stream synchronised), in ns of a monotonic clock. */
typedef struct hp_server_s *hp_server_t;

typedef struct {
    int32_t max_inflight;    /* worker threads / streams (1..16; 0 = 4)            */
    int32_t max_batch;       /* requests per batch (0 = 256)                       */
    int32_t release_wait_ms; /* a request that does not fit while no other batch
                                runs waits this long for the caller to release
                                results before it is rejected (0 = 1000 ms;
                                negative: rejected at once)                        */
    int32_t reserved;        /* set to 0                                           */
} hp_server_config_t;

typedef struct {
    uint64_t id;           /* from hp_server_submit                                */
    int32_t status;        /* hp_status_t of the request                           */
    int32_t batch_size;    /* requests in the batch it ran in                      */
    hp_csr_t C;            /* the result (arrays inside the pool) when status OK   */
    int64_t t_submit_ns, t_start_ns, t_done_ns;
} hp_completion_t;

hp_status_t hp_server_create(hp_server_t *out, int device, void *pool, size_t pool_bytes,
                             const hp_server_config_t *cfg);
/* Copies *req (the matrices and index vectors it points to must stay valid
 * and unchanged until the request completes); *id receives its id. */
hp_status_t hp_server_submit(hp_server_t s, const hp_request_t *req, uint64_t *id);
/* Moves up to cap completions into out (*n of them); never blocks. */
hp_status_t hp_server_poll(hp_server_t s, hp_completion_t *out, int cap, int *n);
/* Blocks until every submitted request has completed. */
hp_status_t hp_server_drain(hp_server_t s);
/* Returns the pool space of a completed request's result. */
hp_status_t hp_server_release(hp_server_t s, uint64_t id);
/* Pool bytes in use (workspaces and unreleased results) and the peak. */
hp_status_t hp_server_memory(hp_server_t s, size_t *in_use, size_t *peak);
/* Drains, stops the workers and frees the server (not the pool). */
hp_status_t hp_server_destroy(hp_server_t s);

#ifdef __cplusplus
}
#endif
#endif /* HIPPERM_H */
