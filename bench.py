#!/usr/bin/env python3
"""Benchmark of the sparse indexing hot path on one MI355X.

One step = one complete extraction C = A(I, J) (plan + exec: J tables,
selected-row scan, counts, rowptr scan, gather, row sort) on the R-MAT
workload: scale 22, edge factor 16, symmetrised, int32 CSR, fp32 values,
I and J random 25% subsets, unsorted, with 1% repeated indices.  Inputs are
generated on the device before timing; outputs are allocated by the
caching allocator inside the step.  `value` is scanned nonzeros (entries
of the selected rows of A) per second over the timed steps.

The same JSON line carries the roofline of the step's dominant kernel
(algorithmic bytes per launch / its HIP-event-timed average duration), the
oracle timed on a bounded sample of the same workload on the host cores,
and secondary workloads (grid permutation, assignment, fused assignment and
permutation, batched and served forms) under "also".

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "nnz/s & % HBM peak for A(I,J)/P·A·Qᵀ at 1 GPU; batched p50/p99 latency"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _sync():
    torch.cuda.synchronize()


def _timed(step, steps, warmup):
    for _ in range(warmup):
        step()
    _sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    _sync()
    return (time.perf_counter() - t0) / steps


def _timed_then_staged(h, step, steps):
    """Seconds per step with stage timing off, then the per-stage device
    times from as many more steps with timing on.  Stage events cost the
    GPU a few microseconds each, so the step time is taken without them;
    the roofline durations come from the events around each stage."""
    sec = _timed(step, steps, 0)
    h.timing(True)
    _timed(step, steps, 0)
    stages = h.stage_times()
    h.timing(False)
    return sec, stages


def _esize(t):
    return t.element_size()


# ---------------------------------------------------------------------------
# Algorithmic bytes: what the method must read once and write once
# (auxiliary tables such as bitmaps and inverse maps are not counted).
# ---------------------------------------------------------------------------

def spref_bytes(A, nI, nJ, S, nnz_out):
    sp, sv = _esize(A.rowptr), _esize(A.val)
    return dict(
        total=4 * (nI + nJ) + 2 * nI * sp + 4 * S + sv * nnz_out + (nI + 1) * sp + nnz_out * (4 + sv),
        # per-kernel figures (one launch each per step)
        gather=4 * S + sv * nnz_out + (nI + 1) * sp + nnz_out * (4 + sv),
        count=4 * S + 4 * nI,
    )


def permute_bytes(A):
    m, n, nnz = A.nrows, A.ncols, A.nnz
    sp, sv = _esize(A.rowptr), _esize(A.val)
    return dict(total=4 * (m + n) + 2 * (m + 1) * sp + 2 * nnz * (4 + sv),
                fill_short=2 * nnz * (4 + sv) + (m + 1) * sp + m * sp)


def spasgn_bytes(A, B, nI, nJ, nnz_out):
    sp, sv = _esize(A.rowptr), _esize(A.val)
    rd = (A.nrows + 1) * sp + A.nnz * (4 + sv) + (B.nrows + 1) * sp + B.nnz * (4 + sv)
    return dict(total=4 * (nI + nJ) + rd + (A.nrows + 1) * sp + nnz_out * (4 + sv))


def merge_bytes(A, B, I, nnz_out):
    """Bytes the assignment merge of the rows of I must move once: I, A's row
    bounds and entries of those rows, B, and the merged rows written."""
    sp, sv = _esize(A.rowptr), _esize(A.val)
    nI = I.numel()
    Il = I.long()
    na_i = int((A.rowptr[Il + 1] - A.rowptr[Il]).sum())
    nout_i = nnz_out - (A.nnz - na_i)
    return (4 * nI + 2 * nI * sp + na_i * (4 + sv) + (nI + 1) * sp + B.nnz * (4 + sv) + nI * sp
            + nout_i * (4 + sv))


def _source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(stage, workload):
    """HBM bytes per launch of `stage` on `workload` from a committed counter
    summary in profiles/ (rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs,
    scaled by the counters of a 1 GiB device copy).  None when there is no
    summary or the kernel's sources changed since the counters were taken."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".txt"):
            continue
        with open(os.path.join(pdir, name)) as fh:
            for line in fh:
                if not line.startswith("traffic-json: "):
                    continue
                rec = json.loads(line[len("traffic-json: "):])
                if rec.get("stage") != stage or rec.get("workload") != workload:
                    continue
                try:
                    if _source_digest(rec["sources"]) != rec["sources_sha256_16"]:
                        return None
                except OSError:
                    return None
                return int(rec["traffic_bytes_per_launch"])
    return None


def roofline(stages, name, bytes_per_launch, workload=None):
    tot_ms, cnt = stages[name]
    avg_s = tot_ms / 1e3 / max(cnt, 1)
    ach = bytes_per_launch / avg_s / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic(name, workload) if workload else None,
            "avg_us": round(avg_s * 1e6, 2), "bytes_per_launch": int(bytes_per_launch)}


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def run_rmat_extract(hp, args):
    t = time.time()
    w = synth.workload_rmat_extract(scale=args.scale, device="cuda")
    A, I, J = w["A"], w["I"], w["J"]
    _sync()
    log(f"[bench] rmat scale {args.scale}: {A.nrows} rows, {A.nnz} nnz, generated in {time.time()-t:.1f}s")
    h = hp.handle(0)
    C, ws, info = h.spref_plan(A, I, J)
    h.spref_exec(A, I, J, C, ws, info)
    xws = [None]

    def step():
        C, _, inf = h.spref_plan(A, I, J, ws=ws)
        if inf.exec_ws_bytes and (xws[0] is None or xws[0].numel() < inf.exec_ws_bytes):
            xws[0] = torch.empty(inf.exec_ws_bytes, dtype=torch.uint8, device="cuda")
        h.spref_exec(A, I, J, C, ws, inf, xws[0])

    rp = A.rowptr.long()
    S = int((rp[I.long() + 1] - rp[I.long()]).sum())
    nnz_out = C.nnz
    for _ in range(args.warmup):
        step()
    _sync()
    sec, stages = _timed_then_staged(h, step, args.steps)
    b = spref_bytes(A, I.numel(), J.numel(), S, nnz_out)
    res = dict(value=S / sec, unit="nnz/s", ms_per_step=sec * 1e3,
               config={"workload": "rmat-extract", "desc": "C = A(I,J); R-MAT scale %d ef16 symmetrised, "
                       "int32 CSR, fp32; I,J 25%% unsorted subsets with 1%% repeats" % args.scale,
                       "nrows": A.nrows, "nnz": A.nnz, "nI": I.numel(), "nJ": J.numel(),
                       "scanned_nnz": S, "nnz_out": nnz_out},
               out_nnz_per_s=nnz_out / sec, algorithmic_GBps=b["total"] / sec / 1e9,
               hbm_frac_step=b["total"] / sec / 1e9 / HBM_PEAK_GBPS,
               stages_us={k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in stages.items()})
    # the dominant kernel of the step is the gather (one launch per step; the
    # sort stage is several smaller kernels)
    res["roofline"] = roofline(stages, "spref.gather", b["gather"], "rmat-extract")
    if args.cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_spref(A, I, J, args.cpu_reps)
    return res


def _host_cpus():
    """(threads the oracle may use here, CPU model name).  The thread count
    is the CPUs this process may run on, capped by OMP_NUM_THREADS when set."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(1, n), model


def cpu_baseline_spref(A, I, J, reps=3):
    """The oracle's extraction through the column multimap (its routine whose
    cost is the entries read) on the whole headline workload, inputs already
    in host memory: single-threaded and row-parallel over the host's CPUs,
    median of `reps` runs each."""
    import numpy as np
    import oracle
    Ah = (A.nrows, A.ncols, A.rowptr.cpu().numpy().astype(np.int64), A.col.cpu().numpy(), A.val.cpu().numpy())
    Ih, Jh = I.cpu().numpy().astype(np.int32), J.cpu().numpy().astype(np.int32)
    rp = Ah[2]
    Il = Ih.astype(np.int64)
    scanned = int((rp[Il + 1] - rp[Il]).sum())
    nt, model = _host_cpus()

    def med(threads):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.spref_map(Ah, Ih, Jh, threads=threads)
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2]

    t1 = med(1)
    tn = med(nt)
    return {"value": scanned / tn, "unit": "nnz/s", "cores": nt, "kind": "oracle",
            "sample": f"the whole extraction ({len(Ih)} rows of I, {scanned} scanned nnz), oracle routine through the "
                      f"column multimap, row-parallel over {nt} threads, median of {reps} runs ({tn:.2f} s)",
            "single_thread": {"value": scanned / t1, "unit": "nnz/s", "cores": 1, "seconds": round(t1, 3)},
            "cpu_model": model}


def run_er_small_latency(hp, args):
    """Latency of single small calls: P A P^T and A(I, I) on the Erdos-Renyi
    4096 x 4096 matrix (average degree 8, int32 CSR, fp64; I 1024 sorted
    unique rows), each call plan + exec with reused workspaces, timed on the
    host from the call to the end of its device work; p10 / p50 / p90 over
    `lat_reps` calls.  The permutation through the no-allocation entry point
    is timed beside it."""
    import numpy as np
    w = synth.workload_er_small(device="cuda")
    A, p, I = w["A"], w["p"], w["I"]
    h = hp.handle(0)
    _, wsp, _ = h.permute_plan(A, p)
    _, wss, _ = h.spref_plan(A, I, I)
    out = hp.CSR(A.nrows, A.ncols, torch.empty_like(A.rowptr), torch.empty_like(A.col), torch.empty_like(A.val))

    def perm():
        C, _, inf = h.permute_plan(A, p, ws=wsp)
        h.permute_exec(A, p, None, C, wsp, inf)

    def sp():
        C, _, inf = h.spref_plan(A, I, I, ws=wss)
        h.spref_exec(A, I, I, C, wss, inf)

    def noalloc():
        h.permute_noalloc(A, p, out=out)

    res = {}
    for name, fn in (("permute", perm), ("spref", sp), ("permute_noalloc", noalloc)):
        for _ in range(10):
            fn()
        _sync()
        ts = []
        for _ in range(args.lat_reps):
            t0 = time.perf_counter()
            fn()
            _sync()
            ts.append((time.perf_counter() - t0) * 1e6)
        q = np.percentile(np.asarray(ts), [10, 50, 90])
        res[name] = {"p10_us": round(float(q[0]), 1), "p50_us": round(float(q[1]), 1), "p90_us": round(float(q[2]), 1)}
    return dict(value=res["permute"]["p50_us"], unit="us", higher_is_better=False,
                ms_per_step=res["permute"]["p50_us"] / 1e3, latency=res,
                config={"workload": "er-small-latency", "desc": "single calls, plan + exec, host-timed to completion: "
                        "P A P^T and A(I,I) on ER 4096^2 avg degree 8 (int32, fp64), I = 1024 sorted unique rows; "
                        "p10/p50/p90 over %d calls" % args.lat_reps, "nnz": A.nnz, "reps": args.lat_reps})


def run_grid_permute(hp, args):
    w = synth.workload_grid(side=args.side, with_block=False, device="cuda")
    A, p, q = w["A"], w["p"], w["q"]
    h = hp.handle(0)
    C, ws, info = h.permute_plan(A, p, q)
    h.permute_exec(A, p, q, C, ws, info)

    def step():
        C, _, inf = h.permute_plan(A, p, q, ws=ws)
        h.permute_exec(A, p, q, C, ws, inf)

    for _ in range(args.warmup):
        step()
    _sync()
    sec, stages = _timed_then_staged(h, step, args.steps)
    b = permute_bytes(A)
    res = dict(value=A.nnz / sec, unit="nnz/s", ms_per_step=sec * 1e3,
               config={"workload": "grid-permute", "desc": "P A Q^T; %dx%d 5-point grid, int64 rowptr, "
                       "fp64, independent random P, Q" % (args.side, args.side), "nrows": A.nrows, "nnz": A.nnz},
               algorithmic_GBps=b["total"] / sec / 1e9, hbm_frac_step=b["total"] / sec / 1e9 / HBM_PEAK_GBPS,
               stages_us={k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in stages.items()})
    res["roofline"] = roofline(stages, "perm.fill_short", b["fill_short"], "grid-permute")
    return res


def run_grid_assign(hp, args):
    w = synth.workload_grid(side=args.side, device="cuda")
    A, B, I, J = w["A"], w["B"], w["I"], w["J"]
    h = hp.handle(0)
    C, ws, info = h.spasgn_plan(A, B, I, J, "second")
    h.spasgn_exec(A, B, I, J, C, ws, info, "second")
    nnz_out = C.nnz
    del C

    def step():
        C, _, inf = h.spasgn_plan(A, B, I, J, "second", ws=ws)
        h.spasgn_exec(A, B, I, J, C, ws, inf, "second")

    for _ in range(args.warmup):
        step()
    _sync()
    sec, stages = _timed_then_staged(h, step, max(3, args.steps // 4))
    b = spasgn_bytes(A, B, I.numel(), J.numel(), nnz_out)
    res = dict(value=(A.nnz + B.nnz) / sec, unit="nnz/s", ms_per_step=sec * 1e3,
               config={"workload": "grid-assign", "desc": "A(I,J) = B (select-second); %dx%d grid, int64 "
                       "rowptr, fp64; I = J contiguous 10%% range; B density 1e-4" % (args.side, args.side),
                       "nnz_A": A.nnz, "nnz_B": B.nnz, "nnz_out": nnz_out},
               algorithmic_GBps=b["total"] / sec / 1e9, hbm_frac_step=b["total"] / sec / 1e9 / HBM_PEAK_GBPS,
               stages_us={k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in stages.items()})
    res["roofline"] = roofline(stages, "asgn.merge", merge_bytes(A, B, I, nnz_out), "grid-assign")
    return res


def run_grid_assign_permute(hp, args):
    """Fused C = P (A (+) B') Q^T against the two separate calls, same inputs."""
    w = synth.workload_grid(side=args.side, device="cuda")
    A, B, I, J, p, q = w["A"], w["B"], w["I"], w["J"], w["p"], w["q"]
    h = hp.handle(0)
    C, ws, info = h.spasgn_permute_plan(A, B, I, J, p, q, "second")
    h.spasgn_permute_exec(A, B, I, J, p, q, C, ws, info, "second")
    nnz_out = C.nnz
    del C
    _, wsa, _ = h.spasgn_plan(A, B, I, J, "second")
    _, wsp, _ = h.permute_plan(A, p, q)

    def step():
        C, _, inf = h.spasgn_permute_plan(A, B, I, J, p, q, "second", ws=ws)
        h.spasgn_permute_exec(A, B, I, J, p, q, C, ws, inf, "second")

    def step_separate():
        X, _, inf = h.spasgn_plan(A, B, I, J, "second", ws=wsa)
        h.spasgn_exec(A, B, I, J, X, wsa, inf, "second")
        C, _, inf2 = h.permute_plan(X, p, q, ws=wsp)
        h.permute_exec(X, p, q, C, wsp, inf2)

    nsteps = max(3, args.steps // 4)
    sec_sep = _timed(step_separate, nsteps, args.warmup) if args.fused_separate else None
    for _ in range(args.warmup):
        step()
    _sync()
    sec, stages = _timed_then_staged(h, step, nsteps)
    b = spasgn_bytes(A, B, I.numel(), J.numel(), nnz_out)
    b["total"] += 4 * (A.nrows + A.ncols)
    res = dict(value=(A.nnz + B.nnz) / sec, unit="nnz/s", ms_per_step=sec * 1e3,
               config={"workload": "grid-assign-permute",
                       "desc": "P (A with A(I,J) = B) Q^T fused (select-second); %dx%d grid, int64 rowptr, "
                       "fp64; I = J contiguous 10%% range; B density 1e-4; independent random P, Q"
                       % (args.side, args.side), "nnz_A": A.nnz, "nnz_B": B.nnz, "nnz_out": nnz_out},
               separate_ms_per_step=sec_sep * 1e3 if sec_sep else None,
               speedup_vs_separate=sec_sep / sec if sec_sep else None,
               algorithmic_GBps=b["total"] / sec / 1e9, hbm_frac_step=b["total"] / sec / 1e9 / HBM_PEAK_GBPS,
               stages_us={k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in stages.items()})
    res["roofline"] = roofline(stages, "asgn.merge", merge_bytes(A, B, I, nnz_out), "grid-assign-permute")
    return res


def run_incremental(hp, args):
    """Nine ~2% blocks assigned back into the ~80% part of an R-MAT graph, one
    per step, with a symmetric random permutation fused into every step;
    beside it the same steps as separate calls, assignment only, and one
    permutation before the first step.  Load imbalance on an 8 x 8 grid."""
    from paper_2509_20776_amd import incremental as inc
    w = synth.workload_incremental(scale=args.incr_scale, device="cuda")
    A = w["A"]
    h = hp.handle(0)
    sp = inc.split(h, A, w["I"], w["J"])
    perms = [(p, None) for p in w["P"]]
    inc.run(h, sp, "fused", perms, measure=False)      # warm-up
    out = {}
    for mode in inc.MODES:
        r = inc.run(h, sp, mode, perms)
        out[mode] = r
        log(f"[bench] incremental {mode}: " + " ".join(f"{t:.2f}" for t in r.step_ms) + " ms; imbalance "
            + " ".join(f"{x:.2f}" for x in r.imbalance))
    f = out["fused"]
    moved = sum(f.nnz[k] + sp.B[k].nnz for k in range(len(sp.B)))
    sec = sum(f.step_ms) / 1e3
    mean = lambda r: sum(r.step_ms) / len(r.step_ms)
    return dict(value=moved / sec, unit="nnz/s", ms_per_step=mean(f),
                config={"workload": "incremental", "desc": "R-MAT scale %d ef 16 symmetrised (int32, fp32); 9 "
                        "blocks of ~2%% of the entries (disjoint 4%% row sets x random 50%% column sets) assigned "
                        "back into the rest, one per step, select-second, symmetric random permutation per step"
                        % args.incr_scale, "nnz_A": A.nnz, "nnz_large": sp.large.nnz,
                        "nnz_blocks": [b.nnz for b in sp.B]},
                step_ms={m: [round(t, 3) for t in r.step_ms] for m, r in out.items()},
                ms_per_step_by_mode={m: round(mean(r), 3) for m, r in out.items()},
                speedup_fused_vs_separate=mean(out["separate"]) / mean(f),
                imbalance_8x8={m: [round(x, 3) for x in r.imbalance] for m, r in out.items()})


def run_hypersparse_extract(hp, args):
    """C = A(I, J) on a hypersparse matrix in DCSC (appendix Alg. 5 walks the
    selected columns): 2^26 x 2^26, 2^24 uniform nonzeros, I and J 25% with
    1% repeats; beside it the same matrix in plain CSC."""
    w = synth.workload_hypersparse(scale=args.hyper_scale, device="cuda")
    A, I, J = w["A"], w["I"], w["J"]
    h = hp.handle(0)
    cnt = A.colptr[1:] - A.colptr[:-1]
    cp = torch.zeros(A.ncols + 1, dtype=torch.int64, device="cuda")
    cp.index_add_(0, A.jc.long() + 1, cnt)
    Acsc = synth.DCSC(A.nrows, A.ncols, None, torch.cumsum(cp, 0), A.row, A.val)
    full = torch.zeros(A.ncols, dtype=torch.int64, device="cuda")
    full[A.jc.long()] = cnt
    S = int(full[J.long()].sum())     # entries of the selected columns
    out = {}
    for name, M in (("dcsc", A), ("csc", Acsc)):
        C, ws, info = h.spref_dcsc_plan(M, I, J)
        h.spref_dcsc_exec(M, I, J, C, ws, info)
        nnz_out = C.nnz
        del C
        xws = [None]

        def step(M=M, ws=ws):
            C, _, inf = h.spref_dcsc_plan(M, I, J, ws=ws)
            if inf.exec_ws_bytes and (xws[0] is None or xws[0].numel() < inf.exec_ws_bytes):
                xws[0] = torch.empty(inf.exec_ws_bytes, dtype=torch.uint8, device="cuda")
            h.spref_dcsc_exec(M, I, J, C, ws, inf, xws[0])

        for _ in range(args.warmup):
            step()
        _sync()
        sec, st = _timed_then_staged(h, step, args.steps)
        out[name] = (sec, st, nnz_out)
    sec, stages, nnz_out = out["dcsc"]
    return dict(value=S / sec, unit="nnz/s", ms_per_step=sec * 1e3,
                config={"workload": "hypersparse-extract", "desc": "C = A(I,J), A in DCSC (int64 colptr, fp64), "
                        "2^%d x 2^%d, %d uniform nonzeros (%d stored columns); I, J 25%% unsorted with 1%% repeats; "
                        "C in CSC" % (args.hyper_scale, args.hyper_scale, A.nnz, A.jc.numel()),
                        "scanned_nnz": S, "nnz_out": nnz_out},
                csc_ms_per_step=out["csc"][0] * 1e3,
                csc_stages_us={k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in out["csc"][1].items()},
                stages_us={k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in stages.items()})


def copy_calibration(mib):
    """A plain device-to-device copy of known size: under rocprofv3 --pmc its
    FETCH_SIZE / WRITE_SIZE per dispatch give the factor that turns counter
    readings into HBM bytes."""
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    _sync()
    log(f"[bench] copy calibration: {n} bytes read and {n} bytes written per copy")
    del src, dst


def stream_copy_gbps(mib=1024, reps=5):
    """Practical HBM ceiling: a plain device-to-device copy (bytes read +
    written per second), timed with events on the current stream."""
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return round(2 * n / sec / 1e9, 1)


def random_access_ceiling(mib=64, count=1 << 24, reps=5):
    """Practical rate of random 4-byte accesses, the bound of a permutation
    of a matrix whose rows move to random places: `count` random reads
    (gather) and, separately, `count` random writes (scatter, distinct
    targets) into a table of `mib` MiB, with torch's indexing kernels,
    timed with events.  Returns accesses per second of each."""
    n = (mib << 20) // 4
    table = torch.arange(n, dtype=torch.int32, device="cuda")
    key = synth.stream_key(0, "random-ceiling")
    idx = synth.randperm(key, n, "cuda")[:count].long()
    vals = torch.ones(count, dtype=torch.int32, device="cuda")
    out = torch.empty(count, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for name, fn in (("gather", lambda: torch.index_select(table, 0, idx, out=out)),
                     ("scatter", lambda: table.index_copy_(0, idx, vals))):
        fn()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        res[name + "_per_s"] = round(count / sec / 1e9, 2) * 1e9
    res["table_MiB"] = mib
    res["accesses"] = count
    del table, idx, vals, out
    return res


def run_served_sweep(hp, args):
    """The served trace at a series of arrival rates, beside the plain
    per-call replay of each: where each path saturates."""
    pool = _served_pool(args)
    var = _served_variants(pool)
    _sync()
    pts = []
    for rate in [float(x) for x in args.served_sweep.split(",")]:
        r = _served_at(hp, args, pool, var, rate)
        pts.append({"rate": rate, "req_per_s": round(r["value"], 1), "p50_ms": round(r["p50_ms"], 3),
                    "p99_ms": round(r["p99_ms"], 3), "mean_batch": round(r["mean_batch"], 2),
                    "plain_req_per_s": round(r["plain"]["req_per_s"], 1),
                    "plain_p50_ms": round(r["plain"]["p50_ms"], 3), "plain_p99_ms": round(r["plain"]["p99_ms"], 3)})
        log(f"[bench] served sweep {rate:g} req/s: {pts[-1]}")
    last = pts[-1]
    return dict(value=last["req_per_s"], unit="req/s", ms_per_step=1e3 / max(last["req_per_s"], 1e-9),
                sweep=pts, config={"workload": "served-sweep", "rates": args.served_sweep})


def _scanned(A, I):
    rp = A.rowptr.long()
    Il = I.long()
    return int((rp[Il + 1] - rp[Il]).sum())


def run_batched(hp, args):
    """512 extraction / permutation requests (50/50) over a pool of 64 directed
    R-MAT matrices (scale U{12..20}, edge factor U{8..32}, int32 CSR, fp32),
    index subsets of 5-50%: one batched plan + graph-replayed exec per step,
    against the same 512 requests as plain calls back-to-back on one stream."""
    t = time.time()
    pool = synth.batched_pool(count=args.batch_pool, device="cuda")
    reqs = synth.batched_requests(pool, count=args.batch_requests, device="cuda")
    for r in reqs:
        r["A"] = pool[r["mat"]]
    _sync()
    log(f"[bench] batched: {len(pool)} matrices ({sum(A.nnz for A in pool)} nnz), {len(reqs)} requests, "
        f"generated in {time.time()-t:.1f}s")
    h = hp.handle(0)
    b = hp.Batch(h, reqs)
    st = b.plan()
    assert all(x == 0 for x in st), st
    b.exec()
    _sync()
    # every batched result is byte-identical to its plain call
    bits = lambda t: t.view(torch.int64 if t.element_size() == 8 else torch.int32)
    for k, (r, C) in enumerate(zip(reqs, b.results())):
        P = hp.spref(r["A"], r["I"], r["J"]) if r["kind"] == "spref" else hp.permute(r["A"], r["p"], r["q"])
        if not (torch.equal(C.rowptr, P.rowptr) and torch.equal(C.col, P.col) and torch.equal(bits(C.val), bits(P.val))):
            raise AssertionError(f"batched request {k} ({r['kind']}) differs from its plain call")
    del P
    log(f"[bench] batched: all {len(reqs)} results equal their plain calls")
    nbytes, scanned = 0, 0
    for k, r in enumerate(reqs):
        A = r["A"]
        if r["kind"] == "spref":
            S = _scanned(A, r["I"])
            scanned += S
            nbytes += spref_bytes(A, r["I"].numel(), r["J"].numel(), S, int(b.arr[k].C.nnz))["total"]
        else:
            scanned += A.nnz
            nbytes += permute_bytes(A)["total"]

    def step_batched():
        b.plan()
        b.exec()

    def step_plain():
        for r in reqs:
            if r["kind"] == "spref":
                hp.spref(r["A"], r["I"], r["J"])
            else:
                hp.permute(r["A"], r["p"], r["q"])

    steps = max(2, args.steps // 5)
    sec_b = _timed(step_batched, steps, 1)
    sec_p = _timed(step_plain, steps, 1)
    return dict(value=scanned / sec_b, unit="nnz/s", ms_per_step=sec_b * 1e3,
                plain_ms_per_step=sec_p * 1e3, speedup_vs_plain=sec_p / sec_b,
                algorithmic_GBps=nbytes / sec_b / 1e9, plain_algorithmic_GBps=nbytes / sec_p / 1e9,
                equal_to_plain=True, grid_plan=int(b.info.grid_plan), grid_exec=int(b.info.grid_exec),
                tiles_plan=int(b.info.tiles_plan), tiles_exec=int(b.info.tiles_exec),
                config={"workload": "batched", "desc": "%d spref/permute requests (50/50) on a pool of %d R-MAT "
                        "(scale U{12..20}, ef U{8..32}), int32 CSR, fp32, subsets 5-50%%; value = scanned nnz/s "
                        "of one batched plan+exec (exec replayed from a hipGraph)" % (len(reqs), len(pool)),
                        "requests": len(reqs), "pool": len(pool), "scanned_nnz": scanned})


def _served_pool(args):
    """Resident pool: R-MAT (ef 16, symmetrised) and Erdos-Renyi (degree 16)
    matrices alternating, scale U{16..hi}, int32 / int64 rowptr alternating,
    fp32 values."""
    return synth.served_pool(0, args.served_pool, 16, args.served_scale_hi, device="cuda")


def _served_variants(pool, per=4):
    """Per matrix: `per` extraction index pairs (5-50%, 1% repeats), `per`
    permutation pairs, `per` assignment blocks (I, J 1-10%, nnz(B) ~ 1% of
    nnz(A), ops cycling select-second / plus / replace)."""
    return synth.served_variants(pool, 0, per, device="cuda")


def _pctl(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def run_served(hp, args):
    """Poisson arrivals (2,000 req/s by default), mix 60/20/20 spref / spasgn /
    permute over a resident pool; latency = completion - arrival.  The same
    trace is replayed through the plain per-call path (one stream, FIFO).
    With --served-rate2, the same at a second (overload) rate under
    "overload"."""
    t = time.time()
    pool = _served_pool(args)
    var = _served_variants(pool)
    _sync()
    log(f"[bench] served: pool of {len(pool)} ({sum(A.nnz for A in pool)} nnz), generated in {time.time()-t:.1f}s")
    res = _served_at(hp, args, pool, var, args.served_rate)
    if args.served_rate2 > 0:
        o = _served_at(hp, args, pool, var, args.served_rate2)
        res["overload"] = {k: o[k] for k in ("value", "p50_ms", "p99_ms", "mean_batch", "failed", "plain")}
        res["overload"]["rate"] = args.served_rate2
    return res


def _served_at(hp, args, pool, var, rate):
    import numpy as np
    arr, trace = synth.served_trace(var, rate, args.served_seconds, 0)
    arr = arr.numpy()
    n = len(arr)

    def submit(srv, r):
        if r["kind"] == "spref":
            return srv.submit("spref", r["A"], I=r["I"], J=r["J"])
        if r["kind"] == "permute":
            return srv.submit("permute", r["A"], p=r["p"], q=r["q"])
        return srv.submit("spasgn", r["A"], I=r["I"], J=r["J"], B=r["B"], op=r["op"])

    def out_nnz(C):
        return int(C.col.numel())

    # warm the kernels and the tuner once per kind and type
    srv = hp.Server(args.served_budget_gb << 30, max_inflight=args.served_streams, max_batch=args.served_max_batch)
    for v in var[:4]:
        for kind in ("spref", "spasgn", "permute"):
            submit(srv, v[kind][0])
    srv.drain()
    for c in srv.poll():
        if c["status"] == 0:
            srv.release(c["id"])
    # served run: a collector thread takes completions and releases their
    # results as soon as they arrive, while this thread submits on schedule
    import threading
    lat, bsz = [], []
    stats = {"nnz": 0, "bad": 0}
    ns0 = time.monotonic_ns()
    pend = {}
    submitted_all = threading.Event()
    lock = threading.Lock()          # a completion's id is in pend before it can be polled

    def collect_loop():
        while True:
            with lock:
                got = srv.poll()
            for c in got:
                k = pend.pop(c["id"])
                if c["status"] != 0:
                    stats["bad"] += 1
                else:
                    stats["nnz"] += out_nnz(c["C"])
                    srv.release(c["id"])
                lat.append((c["t_done_ns"] - (ns0 + int(arr[k] * 1e9))) / 1e6)
                bsz.append(c["batch_size"])
            if not got:
                if submitted_all.is_set() and not pend:
                    return
                time.sleep(0.0005)

    t0 = time.perf_counter()
    ns0 = time.monotonic_ns()
    collector = threading.Thread(target=collect_loop, daemon=True)
    collector.start()
    for k in range(n):
        dt = arr[k] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        with lock:
            pend[submit(srv, trace[k])] = k
    submitted_all.set()
    srv.drain()
    collector.join()
    nnz_done, status_bad = stats["nnz"], stats["bad"]
    wall = time.perf_counter() - t0
    in_use, peak = srv.memory()
    srv.close()
    # the same trace through plain calls, FIFO on one stream
    lat_p, nnz_p = [], 0
    t0 = time.perf_counter()
    for k in range(n if args.served_plain else 0):
        dt = arr[k] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        r = trace[k]
        if r["kind"] == "spref":
            C = hp.spref(r["A"], r["I"], r["J"])
        elif r["kind"] == "permute":
            C = hp.permute(r["A"], r["p"], r["q"])
        else:
            C = hp.spasgn(r["A"], r["B"], r["I"], r["J"], r["op"])
        _sync()
        nnz_p += out_nnz(C)
        lat_p.append((time.perf_counter() - t0 - arr[k]) * 1e3)
        if time.perf_counter() - t0 > args.served_seconds * args.served_plain_cap:
            log(f"[bench] plain replay stopped after {k+1} of {n} requests (time cap)")
            break
    wall_p = max(time.perf_counter() - t0, 1e-9)
    done_rate = (len(lat) - status_bad) / wall
    return dict(value=len(lat) / wall, unit="req/s", ms_per_step=wall * 1e3 / max(1, len(lat)),
                offered_req_per_s=rate, overloaded=bool(done_rate < 0.95 * rate),
                p50_ms=_pctl(lat, 50), p99_ms=_pctl(lat, 99), out_nnz_per_s=nnz_done / wall,
                failed=status_bad, mean_batch=float(np.mean(bsz)) if bsz else 0.0,
                pool_peak_bytes=int(peak),
                plain={"req_per_s": len(lat_p) / wall_p, "p50_ms": _pctl(lat_p, 50), "p99_ms": _pctl(lat_p, 99),
                       "out_nnz_per_s": nnz_p / wall_p, "completed": len(lat_p)},
                config={"workload": "served", "desc": "Poisson %g req/s for %g s, 60/20/20 spref/spasgn/permute "
                        "on %d resident matrices (R-MAT ef16 sym / ER deg 16, scale U{16..%d}, int32/int64 "
                        "rowptr, fp32), %d streams, batches of at most %d, pool budget %d GB"
                        % (rate, args.served_seconds, len(pool), args.served_scale_hi,
                           args.served_streams, args.served_max_batch, args.served_budget_gb),
                        "requests": n})


WORKLOADS = {"rmat-extract": run_rmat_extract, "er-small-latency": run_er_small_latency,
             "grid-permute": run_grid_permute,
             "grid-assign": run_grid_assign, "grid-assign-permute": run_grid_assign_permute,
             "incremental": run_incremental, "hypersparse-extract": run_hypersparse_extract,
             "batched": run_batched, "served": run_served, "served-sweep": run_served_sweep}
EXTRAS_SKIP = {"served-sweep"}   # on request only (--workload served-sweep)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat-extract", choices=sorted(WORKLOADS))
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--side", type=int, default=4096)
    ap.add_argument("--incr-scale", type=int, default=22)
    ap.add_argument("--hyper-scale", type=int, default=26)
    ap.add_argument("--cpu-reps", type=int, default=3, help="oracle runs per thread count (median reported)")
    ap.add_argument("--lat-reps", type=int, default=100, help="calls per latency measurement")
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--no-extras", dest="extras", action="store_false")
    ap.add_argument("--batch-pool", type=int, default=64)
    ap.add_argument("--batch-requests", type=int, default=512)
    ap.add_argument("--served-pool", type=int, default=32)
    ap.add_argument("--served-scale-hi", type=int, default=24)
    ap.add_argument("--served-rate", type=float, default=2000.0)
    ap.add_argument("--served-sweep", default="1000,2000,3000,4000,6000",
                    help="arrival rates of --workload served-sweep")
    ap.add_argument("--served-rate2", type=float, default=0.0,
                    help="second arrival rate for the served leg (0: skip)")
    ap.add_argument("--served-seconds", type=float, default=10.0)
    ap.add_argument("--served-plain-cap", type=float, default=3.0,
                    help="the plain replay stops after this many times the trace length")
    ap.add_argument("--served-streams", type=int, default=4)
    ap.add_argument("--served-budget-gb", type=int, default=64)
    ap.add_argument("--served-max-batch", type=int, default=16)
    ap.add_argument("--no-served-plain", dest="served_plain", action="store_false")
    ap.add_argument("--no-fused-separate", dest="fused_separate", action="store_false",
                    help="grid-assign-permute: skip timing the two separate calls (for per-kernel profiles)")
    ap.add_argument("--copy-cal-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); "
              "the multi-GPU row-block design is documented but not built", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2509_20776_amd import hipperm as hp
    if args.copy_cal_mb > 0:
        copy_calibration(args.copy_cal_mb)
    head = WORKLOADS[args.workload](hp, args)
    also = {}
    if args.extras:
        for name, fn in WORKLOADS.items():
            if name == args.workload or name in EXTRAS_SKIP:
                continue
            a2 = argparse.Namespace(**vars(args))
            a2.cpu_baseline = False
            r = fn(hp, a2)
            also[name] = {k: v for k, v in r.items() if k != "cpu_baseline"}
            log(f"[bench] {name}: {r['value']:.3e} {r['unit']}, {r['ms_per_step']:.3f} ms/step")
    copy_gbps = stream_copy_gbps()
    rand = random_access_ceiling()
    out = {"metric": METRIC, "value": head["value"], "unit": head["unit"], "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic", "config": head["config"], "roofline": head.get("roofline"),
           "cpu_baseline": head.get("cpu_baseline"), "stream_copy_GBps": copy_gbps,
           "random_access_ceiling": rand}
    for k, v in head.items():
        if k not in out and k not in ("cpu_baseline",):
            out[k] = v
    if also:
        out["also"] = also
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
