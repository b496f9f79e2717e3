// Served form: a request server on one device (continuous batching with an
// HBM budget).  Host code only; the GPU work is the batched and plain calls.
//
// Workers (one thread, handle and non-blocking stream each) loop:
//   1. under the lock, take pending requests: an assignment alone, a request
//      over a large matrix alone, or up to max_batch extraction/permutation
//      requests of the first one's index and value types (FIFO order
//      otherwise);
//   2. admit: carve the batch workspace from the pool, waiting while it does
//      not fit and other batches run; a batch that cannot fit even with
//      nothing else running is split, a single request is rejected;
//   3. plan on the worker's stream (one readback), then carve the exact
//      output arena the same way (an assignment reserves its output bound,
//      nnz(A) + nnz(B), at admission instead);
//   4. exec, synchronise the stream, publish completions, return the
//      workspace; result blocks stay until every result in them is released.
// A batch that still holds its workspace while waiting for an arena can
// block others; when every running batch is waiting, the waiting batch gives
// its requests back (split into single requests) instead of waiting.
#include "hp_internal.hpp"
#include "hp_alloc.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace hp;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Pending {
    uint64_t id;
    hp_request_t r;
    int64_t t_submit;
    bool solo;   // run in a batch of its own (after a split)
};

// Extraction and permutation requests over matrices with more stored
// entries than this run alone through the plain calls, never in a batch.
constexpr int64_t BATCH_MAX_NNZ = int64_t(1) << 22;

size_t ptr_bytes(int32_t t) { return t == HP_IDX_I64 ? 8 : 4; }
size_t val_bytes(int32_t t) { return t == HP_VAL_F64 ? 8 : 4; }

}  // namespace

struct hp_server_s {
    int device = 0;
    char *pool = nullptr;
    hp_server_config_t cfg{};
    RangeAlloc alloc;
    hp_handle_t ctl = nullptr;   // validation and workspace queries (under mu)
    std::mutex mu;
    std::condition_variable cv_work, cv_mem, cv_idle;
    std::deque<Pending> pending;
    std::vector<hp_completion_t> done;
    std::unordered_map<uint64_t, size_t> result_block;   // request id -> block offset
    std::unordered_map<size_t, int> block_refs;           // block offset -> unreleased results
    uint64_t next_id = 1;
    int64_t submitted = 0, completed = 0;
    int running = 0;   // batches that hold pool memory
    int waiting = 0;   // of those, batches waiting for their output arena
    bool stop = false;
    std::vector<std::thread> workers;
};

namespace {

using Lock = std::unique_lock<std::mutex>;

void complete_locked(hp_server_s *S, const Pending &p, hp_status_t st, int bsize, const hp_csr_t *C,
                     int64_t t_start, size_t block) {
    hp_completion_t c{};
    c.id = p.id;
    c.status = st;
    c.batch_size = bsize;
    if (C && st == HP_OK) {
        c.C = *C;
        S->result_block[p.id] = block;
    }
    c.t_submit_ns = p.t_submit;
    c.t_start_ns = t_start;
    c.t_done_ns = now_ns();
    S->done.push_back(c);
    S->completed++;
}

void release_block_locked(hp_server_s *S, size_t off) {
    auto it = S->block_refs.find(off);
    if (it == S->block_refs.end()) return;
    if (--it->second <= 0) {
        S->block_refs.erase(it);
        S->alloc.release(off);
    }
}

// Wait (under the lock) until a block of n bytes can be carved; returns its
// offset, or NONE when waiting cannot help: the block is larger than the
// pool, or no other batch is running that could return memory and the
// caller has not released results within the release wait (only a single
// request waits for releases: a batch is split instead).  A caller
// that already counts in `running` (it holds a workspace and waits for its
// output arena) passes holder = true and is counted as waiting meanwhile.
size_t carve_locked(hp_server_s *S, Lock &lk, size_t n, bool holder, bool single) {
    const int64_t wait = single ? (int64_t)std::max(0, S->cfg.release_wait_ms) * 1000000 : 0;
    const int64_t deadline = now_ns() + wait;
    for (;;) {
        const size_t off = S->alloc.alloc(n);
        if (off != RangeAlloc::NONE) return off;
        if (!S->alloc.fits_empty(n)) return RangeAlloc::NONE;
        const int others = S->running - S->waiting - (holder ? 1 : 0);
        // nothing running will return memory: only the caller's releases of
        // results can, and they are waited for up to the release wait
        if (others <= 0 && (S->result_block.empty() || now_ns() >= deadline)) return RangeAlloc::NONE;
        if (holder) S->waiting++;
        S->cv_mem.wait_for(lk, std::chrono::milliseconds(20));
        if (holder) S->waiting--;
    }
}

void run_spasgn(hp_server_s *S, hp_handle_t h, hipStream_t st, Pending p) {
    hp_request_t &r = p.r;
    const int64_t t0 = now_ns();
    const size_t ps = ptr_bytes(r.A.ptr_type), vs = val_bytes(r.A.val_type);
    size_t wsb = 0;
    hp_status_t s;
    size_t ws_off = RangeAlloc::NONE, out_off = RangeAlloc::NONE;
    const int64_t bound = r.A.nnz + r.B.nnz;
    const size_t rp_bytes = RangeAlloc::round((size_t)(r.A.nrows + 1) * ps);
    const size_t col_bytes = RangeAlloc::round((size_t)bound * 4);
    const size_t out_bytes = rp_bytes + col_bytes + (size_t)bound * vs;
    {
        Lock lk(S->mu);
        s = hp_spasgn_workspace(S->ctl, &r.A, &r.B, &wsb);
        if (s == HP_OK) {
            ws_off = carve_locked(S, lk, wsb, false, true);
            if (ws_off != RangeAlloc::NONE) {
                out_off = carve_locked(S, lk, out_bytes, false, true);
                if (out_off == RangeAlloc::NONE) {
                    S->alloc.release(ws_off);
                    ws_off = RangeAlloc::NONE;
                }
            }
            if (ws_off == RangeAlloc::NONE) s = HP_ERR_REJECTED;
        }
        if (s != HP_OK) {
            complete_locked(S, p, s, 1, nullptr, t0, 0);
            S->cv_idle.notify_all();
            return;
        }
        S->running++;
    }
    hp_csr_t C{};
    C.nrows = r.A.nrows;
    C.ncols = r.A.ncols;
    C.ptr_type = r.A.ptr_type;
    C.val_type = r.A.val_type;
    C.rowptr = S->pool + out_off;
    hp_plan_info_t info{};
    s = hp_spasgn_plan(h, &r.A, &r.B, r.I, r.J, (hp_asgn_op_t)r.op, &C, S->pool + ws_off, wsb, &info);
    size_t x_off = RangeAlloc::NONE;
    if (s == HP_OK && info.exec_ws_bytes) {
        Lock lk(S->mu);
        x_off = carve_locked(S, lk, info.exec_ws_bytes, true, true);
        if (x_off == RangeAlloc::NONE) s = HP_ERR_REJECTED;
    }
    if (s == HP_OK) {
        C.col = (int32_t *)(S->pool + out_off + rp_bytes);
        C.val = S->pool + out_off + rp_bytes + col_bytes;
        s = hp_spasgn_exec(h, &r.A, &r.B, r.I, r.J, (hp_asgn_op_t)r.op, &C, S->pool + ws_off, wsb, &info,
                           x_off == RangeAlloc::NONE ? nullptr : S->pool + x_off, info.exec_ws_bytes);
        if (s == HP_OK) s = wait_stream(h, "server");
    }
    Lock lk(S->mu);
    if (s != HP_ERR_TIMEOUT) {   // after a timeout the stream may still use the blocks: never reuse them
        S->alloc.release(ws_off);
        if (x_off != RangeAlloc::NONE) S->alloc.release(x_off);
        if (s == HP_OK) S->block_refs[out_off] = 1;
        else S->alloc.release(out_off);
    }
    complete_locked(S, p, s, 1, &C, t0, out_off);
    S->running--;
    S->cv_mem.notify_all();
    S->cv_idle.notify_all();
}

// Run one batch of extraction / permutation requests.  Returns the requests
// to give back to the queue (after a split), empty otherwise.
std::vector<Pending> run_batch(hp_server_s *S, hp_handle_t h, hipStream_t st,
                               std::vector<Pending> &B, size_t ws_off, size_t wsb) {
    const int n = (int)B.size();
    const int64_t t0 = now_ns();
    std::vector<hp_request_t> reqs(n);
    for (int k = 0; k < n; k++) reqs[k] = B[k].r;
    hp_batch_info_t info{};
    // every batch has its own shape: launch directly, with the fixed grid
    // (timing runs would add to the latency of the first batch of a class)
    info.flags = HP_BATCH_NO_GRAPH | HP_BATCH_NO_TUNE;
    hp_status_t s = hp_batch_plan(h, reqs.data(), n, S->pool + ws_off, wsb, &info);
    size_t a_off = RangeAlloc::NONE;
    std::vector<Pending> back;
    if (s == HP_OK && info.arena_bytes) {
        Lock lk(S->mu);
        a_off = carve_locked(S, lk, info.arena_bytes, true, n == 1);
        if (a_off == RangeAlloc::NONE) {
            if (n > 1) {
                // give the requests back to run one at a time
                S->alloc.release(ws_off);
                S->running--;
                for (auto &p : B) {
                    p.solo = true;
                    back.push_back(p);
                }
                S->cv_mem.notify_all();
                return back;
            }
            s = HP_ERR_REJECTED;
        }
    }
    if (s == HP_OK) {
        s = hp_batch_exec(h, reqs.data(), n, S->pool + ws_off, wsb, &info,
                          a_off == RangeAlloc::NONE ? nullptr : S->pool + a_off, info.arena_bytes);
        if (s == HP_OK) s = wait_stream(h, "server");
    }
    Lock lk(S->mu);
    if (s == HP_ERR_TIMEOUT) a_off = RangeAlloc::NONE;   // the stream may still use the blocks: never reuse them
    else S->alloc.release(ws_off);
    int live = 0;
    for (int k = 0; k < n; k++) {
        const hp_status_t rs = s != HP_OK ? s : (hp_status_t)reqs[k].status;
        if (rs == HP_OK && a_off != RangeAlloc::NONE) live++;
        complete_locked(S, B[k], rs, n, &reqs[k].C, t0, a_off);
    }
    if (a_off != RangeAlloc::NONE) {
        if (live) S->block_refs[a_off] = live;
        else S->alloc.release(a_off);
    }
    S->running--;
    S->cv_mem.notify_all();
    S->cv_idle.notify_all();
    return back;
}

// A lone extraction or permutation runs through the plain calls, which cost
// less per request than the batched stage launches.  The admission carved
// [plan workspace | row-pointer staging] as one block at ws_off; the output
// block (row pointers, columns, values) is carved after the plan, when the
// output size is known (for a permutation it is nnz(A) and the row pointers
// go there directly).
size_t solo_ws_bytes(hp_server_s *S, const hp_request_t &r, size_t *plan_ws) {
    size_t b = 0;
    hp_status_t s = r.kind == HP_REQ_SPREF ? hp_spref_workspace(S->ctl, &r.A, r.nI, r.nJ, &b)
                                           : hp_permute_workspace(S->ctl, &r.A, &b);
    if (s != HP_OK) return 0;
    *plan_ws = RangeAlloc::round(b);
    const int64_t rows = r.kind == HP_REQ_SPREF ? r.nI : r.A.nrows;
    return *plan_ws + RangeAlloc::round((size_t)(rows + 1) * ptr_bytes(r.A.ptr_type));
}

void run_solo(hp_server_s *S, hp_handle_t h, hipStream_t st, Pending &p, size_t ws_off,
              size_t plan_ws, size_t wsb) {
    hp_request_t &r = p.r;
    const int64_t t0 = now_ns();
    const bool spref = r.kind == HP_REQ_SPREF;
    const size_t ps = ptr_bytes(r.A.ptr_type), vs = val_bytes(r.A.val_type);
    const int64_t rows = spref ? r.nI : r.A.nrows;
    const size_t rp_bytes = RangeAlloc::round((size_t)(rows + 1) * ps);
    hp_csr_t C{};
    C.nrows = rows;
    C.ncols = spref ? r.nJ : r.A.ncols;
    C.ptr_type = r.A.ptr_type;
    C.val_type = r.A.val_type;
    C.rowptr = S->pool + ws_off + plan_ws;   // staging
    hp_plan_info_t info{};
    hp_status_t s = spref ? hp_spref_plan(h, &r.A, r.I, r.nI, r.J, r.nJ, &C, S->pool + ws_off, plan_ws, &info)
                          : hp_permute_plan(h, &r.A, r.p, r.q, &C, S->pool + ws_off, plan_ws, &info);
    size_t out_off = RangeAlloc::NONE, x_off = RangeAlloc::NONE;
    if (s == HP_OK) {
        const size_t col_bytes = RangeAlloc::round((size_t)C.nnz * 4);
        Lock lk(S->mu);
        out_off = carve_locked(S, lk, rp_bytes + col_bytes + (size_t)C.nnz * vs, true, true);
        if (out_off != RangeAlloc::NONE && info.exec_ws_bytes) {
            x_off = carve_locked(S, lk, info.exec_ws_bytes, true, true);
            if (x_off == RangeAlloc::NONE) {
                S->alloc.release(out_off);
                out_off = RangeAlloc::NONE;
            }
        }
        if (out_off == RangeAlloc::NONE) s = HP_ERR_REJECTED;
    }
    if (s == HP_OK) {
        char *ob = S->pool + out_off;
        if (hipMemcpyAsync(ob, C.rowptr, (size_t)(rows + 1) * ps, hipMemcpyDeviceToDevice, st) != hipSuccess)
            s = HP_ERR_HIP;
        C.rowptr = ob;
        C.col = (int32_t *)(ob + rp_bytes);
        C.val = ob + rp_bytes + RangeAlloc::round((size_t)C.nnz * 4);
        void *xw = x_off == RangeAlloc::NONE ? nullptr : S->pool + x_off;
        if (s == HP_OK)
            s = spref ? hp_spref_exec(h, &r.A, r.I, r.nI, r.J, r.nJ, &C, S->pool + ws_off, plan_ws, &info, xw,
                                      info.exec_ws_bytes)
                      : hp_permute_exec(h, &r.A, r.p, r.q, &C, S->pool + ws_off, plan_ws, &info, xw,
                                        info.exec_ws_bytes);
        if (s == HP_OK) s = wait_stream(h, "server");
    }
    (void)wsb;
    Lock lk(S->mu);
    if (s == HP_ERR_TIMEOUT) {   // the stream may still use the blocks: never reuse them
        x_off = out_off = RangeAlloc::NONE;
    } else {
        S->alloc.release(ws_off);
    }
    if (x_off != RangeAlloc::NONE) S->alloc.release(x_off);
    if (out_off != RangeAlloc::NONE) {
        if (s == HP_OK) S->block_refs[out_off] = 1;
        else S->alloc.release(out_off);
    }
    complete_locked(S, p, s, 1, &C, t0, out_off);
    S->running--;
    S->cv_mem.notify_all();
    S->cv_idle.notify_all();
}

void worker_main(hp_server_s *S) {
    hipSetDevice(S->device);
    hp_handle_t h = nullptr;
    hipStream_t st = nullptr;
    bool ok = hp_create(&h, S->device) == HP_OK &&
              hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
              hp_set_stream(h, st) == HP_OK;
    for (;;) {
        std::vector<Pending> B;
        size_t wsb = 0, ws_off = RangeAlloc::NONE, plan_ws = 0;
        bool asgn = false, solo = false;
        {
            Lock lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
            if (S->pending.empty()) break;
            if (!ok) {   // no device resources: fail what is queued
                while (!S->pending.empty()) {
                    complete_locked(S, S->pending.front(), HP_ERR_HIP, 1, nullptr, now_ns(), 0);
                    S->pending.pop_front();
                }
                S->cv_idle.notify_all();
                continue;
            }
            Pending first = S->pending.front();
            S->pending.pop_front();
            if (first.r.kind == HP_REQ_SPASGN) {
                asgn = true;
                B.push_back(first);
            } else {
                B.push_back(first);
                if (!first.solo) {
                    // continuous batching: whatever compatible work is waiting
                    for (auto it = S->pending.begin(); it != S->pending.end() && (int)B.size() < S->cfg.max_batch;) {
                        const hp_request_t &r = it->r;
                        if (!it->solo && r.kind != HP_REQ_SPASGN && r.A.ptr_type == first.r.A.ptr_type &&
                            r.A.val_type == first.r.A.val_type) {
                            B.push_back(*it);
                            it = S->pending.erase(it);
                        } else {
                            ++it;
                        }
                    }
                }
                solo = B.size() == 1;
                if (solo) {
                    wsb = solo_ws_bytes(S, B[0].r, &plan_ws);
                } else {
                    std::vector<hp_request_t> tmp(B.size());
                    for (size_t k = 0; k < B.size(); k++) tmp[k] = B[k].r;
                    if (hp_batch_workspace(S->ctl, tmp.data(), (int)tmp.size(), &wsb) != HP_OK) wsb = 0;
                }
                ws_off = carve_locked(S, lk, wsb, false, B.size() == 1);
                if (ws_off == RangeAlloc::NONE) {
                    if (B.size() > 1) {
                        for (auto it = B.rbegin(); it != B.rend(); ++it) {
                            it->solo = true;
                            S->pending.push_front(*it);
                        }
                        S->cv_work.notify_all();
                        continue;
                    }
                    complete_locked(S, B[0], HP_ERR_REJECTED, 1, nullptr, now_ns(), 0);
                    S->cv_idle.notify_all();
                    continue;
                }
                S->running++;
            }
        }
        // the worker's stream waits for the caller's writes of each input
        for (auto &pb : B)
            if (pb.r.ready) hipStreamWaitEvent(st, (hipEvent_t)pb.r.ready, 0);
        if (asgn) {
            run_spasgn(S, h, st, B[0]);
        } else if (solo) {
            run_solo(S, h, st, B[0], ws_off, plan_ws, wsb);
        } else {
            std::vector<Pending> back = run_batch(S, h, st, B, ws_off, wsb);
            if (!back.empty()) {
                Lock lk(S->mu);
                for (auto it = back.rbegin(); it != back.rend(); ++it) S->pending.push_front(*it);
                S->cv_work.notify_all();
            }
        }
    }
    if (st) hipStreamDestroy(st);
    if (h) hp_destroy(h);
}

}  // namespace

extern "C" hp_status_t hp_server_create(hp_server_t *out, int device, void *pool, size_t pool_bytes,
                                        const hp_server_config_t *cfg) {
    if (!out || !pool || pool_bytes < RangeAlloc::ALIGN) return HP_ERR_INVALID_ARG;
    hp_server_s *S = new hp_server_s();
    S->device = device;
    S->pool = (char *)pool;
    S->alloc.reset(pool_bytes);
    if (cfg) S->cfg = *cfg;
    if (S->cfg.max_inflight <= 0) S->cfg.max_inflight = 4;
    if (S->cfg.max_inflight > 16) S->cfg.max_inflight = 16;
    if (S->cfg.max_batch <= 0) S->cfg.max_batch = 256;
    if (S->cfg.release_wait_ms == 0) S->cfg.release_wait_ms = 1000;
    if (hp_create(&S->ctl, device) != HP_OK) {
        delete S;
        return HP_ERR_HIP;
    }
    for (int k = 0; k < S->cfg.max_inflight; k++) S->workers.emplace_back(worker_main, S);
    *out = S;
    return HP_OK;
}

extern "C" hp_status_t hp_server_submit(hp_server_t S, const hp_request_t *req, uint64_t *id) {
    if (!S || !req || !id) return HP_ERR_INVALID_ARG;
    Lock lk(S->mu);
    if (S->stop) return HP_ERR_INVALID_ARG;
    hp_request_t r = *req;
    r.status = HP_OK;
    r.C = hp_csr_t{};
    hp_status_t s;
    size_t bytes = 0;
    if (r.kind == HP_REQ_SPASGN) {
        s = hp_spasgn_workspace(S->ctl, &r.A, &r.B, &bytes);
        if (s == HP_OK && (r.op < HP_OP_SECOND || r.op > HP_OP_REPLACE))
            s = fail(S->ctl, HP_ERR_INVALID_ARG, "server: bad assignment op");
        if (s == HP_OK && (!r.I || !r.J) && (r.B.nrows > 0 || r.B.ncols > 0))
            s = fail(S->ctl, HP_ERR_INVALID_ARG, "server: I or J is NULL");
    } else {
        s = hp_batch_workspace(S->ctl, &r, 1, &bytes);   // validates the request
    }
    if (s != HP_OK) return s;
    // a request over a large matrix fills the GPU by itself and runs faster
    // through the plain calls than through the batched stage launches
    const bool big = r.kind != HP_REQ_SPASGN && r.A.nnz > BATCH_MAX_NNZ;
    Pending p{S->next_id++, r, now_ns(), big};
    *id = p.id;
    S->pending.push_back(p);
    S->submitted++;
    S->cv_work.notify_one();
    return HP_OK;
}

extern "C" hp_status_t hp_server_poll(hp_server_t S, hp_completion_t *out, int cap, int *n) {
    if (!S || !n || cap < 0 || (cap > 0 && !out)) return HP_ERR_INVALID_ARG;
    Lock lk(S->mu);
    const int k = std::min<int>(cap, (int)S->done.size());
    for (int i = 0; i < k; i++) out[i] = S->done[i];
    S->done.erase(S->done.begin(), S->done.begin() + k);
    *n = k;
    return HP_OK;
}

extern "C" hp_status_t hp_server_drain(hp_server_t S) {
    if (!S) return HP_ERR_INVALID_ARG;
    Lock lk(S->mu);
    S->cv_idle.wait(lk, [&] { return S->completed == S->submitted; });
    return HP_OK;
}

extern "C" hp_status_t hp_server_release(hp_server_t S, uint64_t id) {
    if (!S) return HP_ERR_INVALID_ARG;
    Lock lk(S->mu);
    auto it = S->result_block.find(id);
    if (it == S->result_block.end()) return HP_ERR_INVALID_ARG;
    const size_t off = it->second;
    S->result_block.erase(it);
    release_block_locked(S, off);
    S->cv_mem.notify_all();
    return HP_OK;
}

extern "C" hp_status_t hp_server_memory(hp_server_t S, size_t *in_use, size_t *peak) {
    if (!S) return HP_ERR_INVALID_ARG;
    Lock lk(S->mu);
    if (in_use) *in_use = S->alloc.in_use();
    if (peak) *peak = S->alloc.peak();
    return HP_OK;
}

extern "C" hp_status_t hp_server_destroy(hp_server_t S) {
    if (!S) return HP_ERR_INVALID_ARG;
    {
        Lock lk(S->mu);
        S->cv_idle.wait(lk, [&] { return S->completed == S->submitted; });
        S->stop = true;
        S->cv_work.notify_all();
        S->cv_mem.notify_all();
    }
    for (auto &t : S->workers) t.join();
    if (S->ctl) hp_destroy(S->ctl);
    delete S;
    return HP_OK;
}
