"""Incremental graph update with a permutation fused into every step
(paper Sec. 5.9).

A matrix is split into a large part and `len(parts)` small non-overlapping
blocks A(I_k, J_k): the row sets I_k are disjoint, so the blocks are too.
The large part is A with every block's entries removed (a block assignment
of an empty matrix).  Step k assigns block k back.  With a permutation mode
every step also relabels rows and columns by a fresh permutation, so after
the last step the matrix is P A Q^T for the composed permutations (A itself
when nothing is permuted).  The paper's figure of merit is the load
imbalance of the matrix over a process grid after each step (largest block
nonzero count over the mean), which stays near 1 only when every step
permutes.

Modes:
  "fused"      hp_spasgn_permute per step (C = P_k (C (+) B_k') Q_k^T),
  "separate"   hp_spasgn then hp_permute per step (same result),
  "assign"     hp_spasgn only,
  "perm-once"  hp_permute with the first permutation before step 1, then
               hp_spasgn only.

Index sets, blocks and permutations are the caller's device tensors; every
array operation (extraction, assignment, permutation, relabelling of the
blocks' indices, composition of the permutations, block counts) runs in
the library's kernels, and this module only sequences the calls.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import torch

from . import hipperm as hp

MODES = ("fused", "separate", "assign", "perm-once")


@dataclass
class Split:
    large: hp.CSR                    # A without the blocks
    I: List[torch.Tensor]            # row sets, disjoint
    J: List[torch.Tensor]            # column sets
    B: List[hp.CSR]                  # B_k = A(I_k, J_k)


@dataclass
class Result:
    C: hp.CSR                        # final matrix
    p_total: torch.Tensor            # row i of C is row p_total[i] of A
    q_total: Optional[torch.Tensor]  # column j of C is column q_total[j] of A (None: same as rows)
    step_ms: List[float] = field(default_factory=list)
    imbalance: List[float] = field(default_factory=list)   # before step 1, then after each step
    nnz: List[int] = field(default_factory=list)


def _empty_block(A: hp.CSR, nI: int, nJ: int) -> hp.CSR:
    dev = A.col.device
    return hp.CSR(nI, nJ, torch.zeros(nI + 1, dtype=A.rowptr.dtype, device=dev),
                  torch.zeros(0, dtype=torch.int32, device=dev), torch.zeros(0, dtype=A.val.dtype, device=dev))


def split(hd: hp.Handle, A: hp.CSR, I: Sequence[torch.Tensor], J: Sequence[torch.Tensor]) -> Split:
    """Extract B_k = A(I_k, J_k) and remove every block from A."""
    if len(I) != len(J):
        raise ValueError("one column set per row set")
    B = [hd.spref(A, Ik, Jk) for Ik, Jk in zip(I, J)]
    L = A
    for Ik, Jk in zip(I, J):
        L = hd.spasgn(L, _empty_block(A, int(Ik.numel()), int(Jk.numel())), Ik, Jk, "replace")
    return Split(L, list(I), list(J), B)


def imbalance(hd: hp.Handle, C: hp.CSR, grid: Tuple[int, int]) -> float:
    """Largest block nonzero count over the mean, on a gr x gc grid."""
    cnt = hd.block_nnz(C, grid[0], grid[1]).double()
    mean = float(cnt.mean())
    return float(cnt.max()) / mean if mean > 0 else 1.0


def run(hd: hp.Handle, sp: Split, mode: str, perms: Sequence[Tuple[torch.Tensor, Optional[torch.Tensor]]] = (),
        op: str = "second", grid: Tuple[int, int] = (8, 8), measure: bool = True) -> Result:
    """Assign the blocks back one per step.  perms[k] = (p_k, q_k) is the
    permutation of step k (q_k None: symmetric, needs a square matrix); the
    permuting modes need one per block ("perm-once" uses perms[0] only)."""
    if mode not in MODES:
        raise ValueError(f"mode must be one of {MODES}")
    permuting = mode in ("fused", "separate")
    if (permuting and len(perms) < len(sp.B)) or (mode == "perm-once" and not perms):
        raise ValueError("not enough permutations for this mode")
    C = sp.large
    m, n = C.nrows, C.ncols
    dev = C.col.device
    sym = bool(perms) and perms[0][1] is None
    pos_r = torch.arange(m, dtype=torch.int32, device=dev)          # current row of original row r
    pos_c = pos_r if sym else torch.arange(n, dtype=torch.int32, device=dev)
    moved = False
    res = Result(C, pos_r, None if sym else pos_c)

    def relabel(p, q):
        nonlocal pos_r, pos_c, moved
        pos_r = hd.gather_index(hd.invert_perm(p), pos_r)
        pos_c = pos_r if sym else hd.gather_index(hd.invert_perm(q), pos_c)
        moved = True

    if measure:
        res.imbalance.append(imbalance(hd, C, grid))
        res.nnz.append(C.nnz)
    if mode == "perm-once":
        p0, q0 = perms[0]
        C = hd.permute(C, p0, q0)
        relabel(p0, q0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)] if measure else None
    for k, (Ik, Jk, Bk) in enumerate(zip(sp.I, sp.J, sp.B)):
        if measure:
            ev[0].record()
        Ic = hd.gather_index(pos_r, Ik) if moved else Ik
        Jc = hd.gather_index(pos_c, Jk) if moved else Jk
        if mode == "fused":
            p, q = perms[k]
            C = hd.spasgn_permute(C, Bk, Ic, Jc, p, q, op)
            relabel(p, q)
        elif mode == "separate":
            p, q = perms[k]
            C = hd.permute(hd.spasgn(C, Bk, Ic, Jc, op), p, q)
            relabel(p, q)
        else:
            C = hd.spasgn(C, Bk, Ic, Jc, op)
        if measure:
            ev[1].record()
            ev[1].synchronize()
            res.step_ms.append(ev[0].elapsed_time(ev[1]))
            res.imbalance.append(imbalance(hd, C, grid))
            res.nnz.append(C.nnz)
    res.C = C
    res.p_total = hd.invert_perm(pos_r)
    res.q_total = None if sym else hd.invert_perm(pos_c)
    return res
