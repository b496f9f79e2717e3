"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This module only *draws* inputs; it contains none of the indexing arithmetic
(no permutation, extraction or assignment).  Both the oracle and the HIP path
receive exactly the same arrays from here.

Random numbers come from a counter-based generator: the i-th draw of stream
``key`` is the (i+1)-th output of SplitMix64 (Steele, Lea, Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014; constants as in
Vigna's public-domain reference) seeded with ``key``, i.e.
``mix64(key + (i+1)*GAMMA)``.  It is written with torch int64 tensor ops
(two's-complement wraparound), so the same draw is produced on the CPU and on
the GPU; large inputs are generated on the device and copied to the host for
the oracle.

Workload shapes follow the paper's inputs (social/web graphs -> R-MAT, road
networks -> 2D grid, GAP-urand -> Erdos-Renyi; dataset table of the
experimental setup section).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import torch

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def _s64(x: int) -> int:
    """Python int (mod 2^64) -> signed int64 value with the same bits."""
    x &= MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


def mix64_int(z: int) -> int:
    """SplitMix64 output function on a Python int (reference, exact)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def splitmix64_ref(state: int, count: int) -> list:
    """Plain SplitMix64 sequence (state += GAMMA; output mix(state))."""
    out = []
    for _ in range(count):
        state = (state + GAMMA) & MASK64
        out.append(mix64_int(state))
    return out


def stream_key(seed: int, *labels) -> int:
    """Derive an independent 64-bit stream key from a seed and labels."""
    z = mix64_int(seed + GAMMA)
    for lab in labels:
        if isinstance(lab, str):
            v = 0
            for ch in lab.encode():
                v = (v * 131 + ch) & MASK64
        else:
            v = int(lab) & MASK64
        z = mix64_int(z ^ mix64_int(v + GAMMA))
    return z


def _srl(x: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def _mix64(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _s64(M1)
    z = (z ^ _srl(z, 27)) * _s64(M2)
    return z ^ _srl(z, 31)


def hash64(key: int, idx: torch.Tensor) -> torch.Tensor:
    """Draw idx of stream key: int64 tensor holding uint64 bit patterns."""
    return _mix64(idx.to(torch.int64) * _s64(GAMMA) + _s64(key + GAMMA))


def draws(key: int, n: int, device="cpu", start: int = 0) -> torch.Tensor:
    return hash64(key, torch.arange(start, start + n, dtype=torch.int64, device=device))


def randint_below(key: int, n: int, hi, device="cpu") -> torch.Tensor:
    """n draws uniform on [0, hi) (63-bit modulo; bias < hi/2^63)."""
    h = _srl(draws(key, n, device), 1)
    return h % hi


def randperm(key: int, n: int, device="cpu") -> torch.Tensor:
    """Uniform random permutation of [0, n) as int32 (argsort of distinct draws).

    mix64 is a bijection and key+(i+1)*GAMMA is distinct for distinct i, so the
    sort keys never tie and the result is device independent."""
    h = draws(key, n, device)
    return torch.argsort(h, stable=True).to(torch.int32)


def values(key: int, n: int, dtype: torch.dtype, device="cpu") -> torch.Tensor:
    """Values in (0, 1] with no exact zeros: k/2^53 (fp64) or k/2^24 (fp32)."""
    h = draws(key, n, device)
    if dtype == torch.float64:
        k = _srl(h, 11) + 1
        return k.to(torch.float64) * (2.0 ** -53)
    if dtype == torch.float32:
        k = _srl(h, 40) + 1
        return (k.to(torch.float64) * (2.0 ** -24)).to(torch.float32)
    raise ValueError(dtype)


@dataclass
class CSR:
    """Canonical CSR: rowptr (int32/int64, nrows+1), col int32 (ascending,
    unique within a row), val fp32/fp64; 0-based."""
    nrows: int
    ncols: int
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def to(self, device) -> "CSR":
        return CSR(self.nrows, self.ncols, self.rowptr.to(device), self.col.to(device), self.val.to(device))

    def numpy(self):
        return (self.rowptr.cpu().numpy(), self.col.cpu().numpy(), self.val.cpu().numpy())


def csr_from_sorted_keys(keys: torch.Tensor, nrows: int, ncols: int, vkey: int,
                         ptr_dtype=torch.int32, val_dtype=torch.float64) -> CSR:
    """Build CSR from sorted unique linear keys r*ncols+c; values drawn in CSR order."""
    rows = keys // ncols
    cols = (keys - rows * ncols).to(torch.int32)
    counts = torch.bincount(rows, minlength=nrows)
    rowptr = torch.zeros(nrows + 1, dtype=torch.int64, device=keys.device)
    rowptr[1:] = torch.cumsum(counts, 0)
    if ptr_dtype == torch.int32:
        assert int(rowptr[-1]) < 2 ** 31
    return CSR(nrows, ncols, rowptr.to(ptr_dtype), cols.contiguous(),
               values(vkey, int(keys.numel()), val_dtype, keys.device))


@dataclass
class DCSC:
    """Column-compressed matrix: CSC when jc is None (colptr has ncols+1
    entries), else doubly compressed (only the columns jc are stored)."""
    nrows: int
    ncols: int
    jc: Optional[torch.Tensor]
    colptr: torch.Tensor
    row: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.row.numel())


def dcsc_uniform(m: int, n: int, nnz: int, seed: int = 0, label="hyper", ptr_dtype=torch.int64,
                 val_dtype=torch.float64, compress: bool = True, device="cpu") -> DCSC:
    """nnz positions drawn uniformly (with replacement, duplicates removed)
    over the m x n grid, stored by column; compress keeps only the non-empty
    columns (DCSC).  With nnz below n most columns are empty (hypersparse)."""
    key = stream_key(seed, label, m, n)
    lin = torch.unique(randint_below(stream_key(key, "pos"), nnz, m * n, device), sorted=True)
    cols = lin // m
    rows = (lin - cols * m).to(torch.int32)
    if compress:
        jc, cnt = torch.unique_consecutive(cols, return_counts=True)
        jc = jc.to(torch.int32)
    else:
        jc, cnt = None, torch.bincount(cols, minlength=n)
    colptr = torch.zeros(cnt.numel() + 1, dtype=torch.int64, device=lin.device)
    colptr[1:] = torch.cumsum(cnt, 0)
    return DCSC(m, n, jc, colptr.to(ptr_dtype), rows.contiguous(),
                values(stream_key(key, "val"), int(lin.numel()), val_dtype, lin.device))


def erdos_renyi(m: int, n: int, avg_deg: float, seed: int = 0, label="er",
                ptr_dtype=torch.int32, val_dtype=torch.float64, device="cpu") -> CSR:
    """round(m*avg_deg) positions drawn uniformly (with replacement) over the
    m x n grid, duplicates removed: the uniform random (GAP-urand-like) graph."""
    key = stream_key(seed, label, m, n)
    t = int(round(m * avg_deg))
    lin = randint_below(stream_key(key, "pos"), t, m * n, device)
    lin = torch.unique(lin, sorted=True)
    return csr_from_sorted_keys(lin, m, n, stream_key(key, "val"), ptr_dtype, val_dtype)


RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def rmat(scale: int, edge_factor: int, seed: int = 0, label="rmat", abcd=RMAT_ABCD,
         symmetric: bool = True, ptr_dtype=torch.int32, val_dtype=torch.float32,
         device="cpu") -> CSR:
    """R-MAT power-law matrix (social/web stand-in).

    edge_factor * 2^scale edges; each level picks a quadrant with
    probabilities (a, b, c, d) from a 32-bit draw against thresholds
    floor(p * 2^32).  No noise, no relabelling (hubs sit at low ids),
    self-loops kept.  symmetric=True adds the transpose; duplicates removed.
    Values are drawn after de-duplication, in CSR order."""
    n = 1 << scale
    e = edge_factor * n
    key = stream_key(seed, label, scale, edge_factor, int(symmetric))
    a, b, c, _ = abcd
    ta = int(a * 2 ** 32)
    tab = int((a + b) * 2 ** 32)
    tabc = int((a + b + c) * 2 ** 32)
    rows = torch.zeros(e, dtype=torch.int64, device=device)
    cols = torch.zeros(e, dtype=torch.int64, device=device)
    idx = torch.arange(e, dtype=torch.int64, device=device)
    for lvl in range(0, scale, 2):
        h = hash64(stream_key(key, "lvl", lvl), idx)
        for sub in range(2):
            level = lvl + sub
            if level >= scale:
                break
            u = _srl(h, 32) if sub == 0 else (h & 0xFFFFFFFF)
            rbit = (u >= tab).to(torch.int64)
            cbit = (((u >= ta) & (u < tab)) | (u >= tabc)).to(torch.int64)
            shift = scale - 1 - level
            rows |= rbit << shift
            cols |= cbit << shift
        del h
    del idx
    if symmetric:
        lin = torch.cat([rows * n + cols, cols * n + rows])
    else:
        lin = rows * n + cols
    del rows, cols
    lin = torch.unique(lin, sorted=True)
    return csr_from_sorted_keys(lin, n, n, stream_key(key, "val"), ptr_dtype, val_dtype)


def grid5(nx: int, ny: int, seed: int = 0, label="grid", ptr_dtype=torch.int64,
          val_dtype=torch.float64, device="cpu") -> CSR:
    """2D 5-point-stencil graph (road-network stand-in): vertex r = x*ny + y,
    joined to its 4 grid neighbours; no diagonal.  nnz = 4*nx*ny - 2*nx - 2*ny."""
    key = stream_key(seed, label, nx, ny)
    nv = nx * ny
    r = torch.arange(nv, dtype=torch.int64, device=device)
    x = r // ny
    y = r - x * ny
    cand = torch.stack([r - ny, r - 1, r + 1, r + ny], 1)
    ok = torch.stack([x > 0, y > 0, y < ny - 1, x < nx - 1], 1)
    counts = ok.sum(1)
    rowptr = torch.zeros(nv + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(counts, 0)
    col = cand[ok].to(torch.int32)
    return CSR(nv, nv, rowptr.to(ptr_dtype), col.contiguous(),
               values(stream_key(key, "val"), int(col.numel()), val_dtype, device))


def subset(key: int, n: int, k: int, sort: bool = False, repeat_frac: float = 0.0,
           device="cpu") -> torch.Tensor:
    """k indices from [0, n): (k - r) distinct uniform indices plus
    r = round(repeat_frac * k) copies of uniformly chosen ones among them,
    in random order (or sorted)."""
    r = int(round(repeat_frac * k))
    d = k - r
    assert 0 <= d <= n
    base = randperm(stream_key(key, "base"), n, device)[:d].to(torch.int64)
    if r > 0:
        pick = randint_below(stream_key(key, "rep"), r, d, device)
        allv = torch.cat([base, base[pick]])
    else:
        allv = base
    if sort:
        allv = torch.sort(allv).values
    else:
        allv = allv[randperm(stream_key(key, "shuf"), k, device).to(torch.int64)]
    return allv.to(torch.int32).contiguous()


def contiguous_range(key: int, n: int, k: int, device="cpu") -> torch.Tensor:
    """[s, s+k) with s uniform on [0, n-k]."""
    s = int(randint_below(key, 1, n - k + 1)[0])
    return torch.arange(s, s + k, dtype=torch.int32, device=device)


def bernoulli_block(nrows: int, ncols: int, density: float, seed: int = 0, label="blk",
                    ptr_dtype=torch.int64, val_dtype=torch.float64, device="cpu") -> CSR:
    """Random sparse block: round(density*nrows*ncols) uniform positions drawn
    with replacement, duplicates removed."""
    key = stream_key(seed, label, nrows, ncols)
    t = int(round(density * nrows * ncols))
    lin = randint_below(stream_key(key, "pos"), t, nrows * ncols, device)
    lin = torch.unique(lin, sorted=True)
    return csr_from_sorted_keys(lin, nrows, ncols, stream_key(key, "val"), ptr_dtype, val_dtype)


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int = 0, label="arr") -> torch.Tensor:
    """Arrival times (s) of a Poisson process: cumulative exponential gaps
    from inverse-CDF of 53-bit uniforms (host, float64)."""
    key = stream_key(seed, label)
    n = int(rate_hz * duration_s * 1.5) + 64
    u = values(key, n, torch.float64)           # (0, 1]
    gaps = -torch.log(u) / rate_hz
    t = torch.cumsum(gaps, 0)
    return t[t < duration_s]


# --------------------------------------------------------------------------
# Workloads.  Sizes default to the full benchmark shapes; tests pass smaller.
# --------------------------------------------------------------------------

def workload_er_small(seed: int = 0, n: int = 4096, device="cpu"):
    """ER n x n, avg degree 8, int32 CSR, fp64; random P; I = 1024-of-n rows
    sorted and unique (extraction A(I, I))."""
    A = erdos_renyi(n, n, 8.0, seed, "cfg-er", torch.int32, torch.float64, device)
    p = randperm(stream_key(seed, "cfg-er", "p"), n, device)
    k = max(1, n // 4)
    I = subset(stream_key(seed, "cfg-er", "I"), n, k, sort=True, device=device)
    return dict(A=A, p=p, I=I)


def workload_rmat_extract(seed: int = 0, scale: int = 22, edge_factor: int = 16,
                          frac: float = 0.25, repeat_frac: float = 0.01, device="cpu"):
    """R-MAT scale/ef symmetrised, int32 CSR, fp32; I, J random 25% unsorted
    subsets with 1% repeated indices."""
    A = rmat(scale, edge_factor, seed, "cfg-rmat", symmetric=True,
             ptr_dtype=torch.int32, val_dtype=torch.float32, device=device)
    n = A.nrows
    k = int(n * frac)
    I = subset(stream_key(seed, "cfg-rmat", "I"), n, k, False, repeat_frac, device)
    J = subset(stream_key(seed, "cfg-rmat", "J"), n, k, False, repeat_frac, device)
    return dict(A=A, I=I, J=J)


def workload_hypersparse(seed: int = 0, scale: int = 26, per_col: float = 0.25, frac: float = 0.25,
                         repeat_frac: float = 0.01, compress: bool = True, device="cpu"):
    """2^scale x 2^scale matrix with per_col * 2^scale uniform nonzeros in
    DCSC (int64 colptr, fp64), most columns empty; I, J random `frac`
    unsorted subsets with `repeat_frac` repeated indices."""
    n = 1 << scale
    A = dcsc_uniform(n, n, int(per_col * n), seed, "cfg-hyper", torch.int64, torch.float64, compress, device)
    k = int(n * frac)
    I = subset(stream_key(seed, "cfg-hyper", "I"), n, k, False, repeat_frac, device)
    J = subset(stream_key(seed, "cfg-hyper", "J"), n, k, False, repeat_frac, device)
    return dict(A=A, I=I, J=J)


def workload_grid(seed: int = 0, side: int = 4096, frac: float = 0.10, density: float = 1e-4,
                  with_block: bool = True, device="cpu"):
    """side x side 5-point grid, int64 rowptr, fp64; independent random P, Q;
    I = J a contiguous 10% range; B random |I| x |J| block at the density."""
    A = grid5(side, side, seed, "cfg-grid", torch.int64, torch.float64, device)
    n = A.nrows
    p = randperm(stream_key(seed, "cfg-grid", "p"), n, device)
    q = randperm(stream_key(seed, "cfg-grid", "q"), n, device)
    k = int(frac * n)
    I = contiguous_range(stream_key(seed, "cfg-grid", "I"), n, k, device)
    J = I.clone()
    out = dict(A=A, p=p, q=q, I=I, J=J)
    if with_block:
        out["B"] = bernoulli_block(k, k, density, seed, "cfg-grid-B", torch.int64, torch.float64, device)
    return out


def workload_incremental(seed: int = 0, scale: int = 22, edge_factor: int = 16, parts: int = 9,
                         part_frac: float = 0.02, col_frac: float = 0.5, device="cpu"):
    """Incremental update: R-MAT scale/ef symmetrised (int32 CSR, fp32, hubs at
    low ids); `parts` disjoint random row sets of part_frac/col_frac of the
    rows each, each with an independent random (unsorted, distinct) column
    set of col_frac of the columns, so every block holds about part_frac of
    the entries; one symmetric random permutation per step."""
    A = rmat(scale, edge_factor, seed, "cfg-incr", symmetric=True,
             ptr_dtype=torch.int32, val_dtype=torch.float32, device=device)
    n = A.nrows
    kr = max(1, int(n * part_frac / col_frac))
    if kr * parts > n:
        raise ValueError("row sets do not fit")
    rows = randperm(stream_key(seed, "cfg-incr", "rows"), n, device)
    I = [rows[k * kr:(k + 1) * kr].clone() for k in range(parts)]
    J = [subset(stream_key(seed, "cfg-incr", "J", k), n, max(1, int(n * col_frac)), device=device)
         for k in range(parts)]
    P = [randperm(stream_key(seed, "cfg-incr", "p", k), n, device) for k in range(parts)]
    return dict(A=A, I=I, J=J, P=P)


def batched_pool(seed: int = 0, count: int = 64, scale_lo: int = 12, scale_hi: int = 20,
                 ef_lo: int = 8, ef_hi: int = 32, device="cpu"):
    """Pool of directed R-MAT matrices (int32 CSR, fp32) with scale and edge
    factor drawn uniformly per matrix."""
    key = stream_key(seed, "batch-pool")
    sc = randint_below(stream_key(key, "scale"), count, scale_hi - scale_lo + 1) + scale_lo
    ef = randint_below(stream_key(key, "ef"), count, ef_hi - ef_lo + 1) + ef_lo
    pool = []
    for t in range(count):
        pool.append(rmat(int(sc[t]), int(ef[t]), seed, f"batch-{t}", symmetric=False,
                         ptr_dtype=torch.int32, val_dtype=torch.float32, device=device))
    return pool


def batched_requests(pool, seed: int = 0, count: int = 512, kinds=("spref", "permute"),
                     frac_lo: float = 0.05, frac_hi: float = 0.50, device="cpu"):
    """count requests over the pool: kind uniform over `kinds`, matrix uniform
    over the pool, index subsets of 5-50% of rows/cols (unsorted, unique) or
    full random permutations."""
    key = stream_key(seed, "batch-req")
    mat = randint_below(stream_key(key, "mat"), count, len(pool))
    kind = randint_below(stream_key(key, "kind"), count, len(kinds))
    fr = values(stream_key(key, "frac"), 2 * count, torch.float64)
    reqs = []
    for t in range(count):
        A = pool[int(mat[t])]
        k = kinds[int(kind[t])]
        rk = stream_key(key, "r", t)
        if k == "permute":
            reqs.append(dict(kind=k, mat=int(mat[t]),
                             p=randperm(stream_key(rk, "p"), A.nrows, device),
                             q=randperm(stream_key(rk, "q"), A.ncols, device)))
        else:
            f1 = frac_lo + (frac_hi - frac_lo) * float(fr[2 * t])
            f2 = frac_lo + (frac_hi - frac_lo) * float(fr[2 * t + 1])
            ki = max(1, int(f1 * A.nrows))
            kj = max(1, int(f2 * A.ncols))
            reqs.append(dict(kind=k, mat=int(mat[t]),
                             I=subset(stream_key(rk, "I"), A.nrows, ki, device=device),
                             J=subset(stream_key(rk, "J"), A.ncols, kj, device=device)))
    return reqs


def served_pool(seed: int = 0, count: int = 32, scale_lo: int = 16, scale_hi: int = 24, scales=None,
                device="cpu"):
    """Resident pool of the served workload: R-MAT (edge factor 16,
    symmetrised) and Erdos-Renyi (degree 16) matrices alternating, scale
    uniform in [scale_lo, scale_hi] (or the given list), int32 / int64 row
    pointers alternating in pairs, fp32 values."""
    key = stream_key(seed, "served-pool")
    if scales is None:
        sc = randint_below(stream_key(key, "scale"), count, scale_hi - scale_lo + 1) + scale_lo
        scales = [int(x) for x in sc]
    pool = []
    for t, s in enumerate(scales):
        ptr = torch.int32 if t % 4 < 2 else torch.int64
        if t % 2 == 0:
            A = rmat(s, 16, seed, f"served-rmat-{t}", symmetric=True, ptr_dtype=ptr, device=device)
        else:
            A = erdos_renyi(1 << s, 1 << s, 16.0, seed, f"served-er-{t}", ptr_dtype=ptr,
                            val_dtype=torch.float32, device=device)
        pool.append(A)
    return pool


def served_variants(pool, seed: int = 0, per: int = 4, device="cpu"):
    """Per pool matrix: `per` extraction index pairs (5-50% of rows and
    columns, 1% repeats, unsorted), `per` permutation pairs, and `per`
    assignment blocks (distinct I, J of 1-10%, nnz(B) about 1% of nnz(A),
    operators cycling select-second / plus / replace)."""
    out = []
    for m, A in enumerate(pool):
        key = stream_key(seed, "served-var", m)
        fr = values(stream_key(key, "fr"), 4 * per, torch.float64)
        v = {"spref": [], "permute": [], "spasgn": []}
        for k in range(per):
            f1 = 0.05 + 0.45 * float(fr[4 * k])
            f2 = 0.05 + 0.45 * float(fr[4 * k + 1])
            I = subset(stream_key(key, "I", k), A.nrows, max(1, int(f1 * A.nrows)), repeat_frac=0.01, device=device)
            J = subset(stream_key(key, "J", k), A.ncols, max(1, int(f2 * A.ncols)), repeat_frac=0.01, device=device)
            v["spref"].append(dict(kind="spref", A=A, I=I, J=J))
            v["permute"].append(dict(kind="permute", A=A, p=randperm(stream_key(key, "p", k), A.nrows, device),
                                     q=randperm(stream_key(key, "q", k), A.ncols, device)))
            g1 = 0.01 + 0.09 * float(fr[4 * k + 2])
            g2 = 0.01 + 0.09 * float(fr[4 * k + 3])
            nI, nJ = max(1, int(g1 * A.nrows)), max(1, int(g2 * A.ncols))
            aI = subset(stream_key(key, "aI", k), A.nrows, nI, device=device)
            aJ = subset(stream_key(key, "aJ", k), A.ncols, nJ, device=device)
            B = bernoulli_block(nI, nJ, min(1.0, 0.01 * A.nnz / (nI * nJ)), seed, f"served-B-{m}-{k}",
                                ptr_dtype=A.rowptr.dtype, val_dtype=torch.float32, device=device)
            v["spasgn"].append(dict(kind="spasgn", A=A, I=aI, J=aJ, B=B, op=["second", "plus", "replace"][k % 3]))
        out.append(v)
    return out


def served_trace(variants, rate_hz: float, duration_s: float, seed: int = 0):
    """Poisson arrivals with a 60/20/20 extraction / assignment / permutation
    mix over the pool's variants: (arrival times in s, list of requests)."""
    arr = poisson_arrivals(rate_hz, duration_s, seed, "served-arrivals")
    key = stream_key(seed, "served-trace")
    n = int(arr.numel())
    u = values(stream_key(key, "kind"), n, torch.float64)
    mi = randint_below(stream_key(key, "mat"), n, len(variants))
    per = len(variants[0]["spref"]) if variants else 1
    vi = randint_below(stream_key(key, "var"), n, per)
    trace = []
    for k in range(n):
        kind = "spref" if u[k] <= 0.6 else ("spasgn" if u[k] <= 0.8 else "permute")
        trace.append(variants[int(mi[k])][kind][int(vi[k])])
    return arr, trace
