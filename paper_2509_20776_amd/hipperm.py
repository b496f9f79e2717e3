"""Thin ctypes binding of libhipperm.so (include/hipperm.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch provides device memory (torch.empty on the GPU) and the stream
(torch.cuda.current_stream()).  When the built library is missing this
module raises at import time; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhipperm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_20776_amd.build` "
                      "(the library has no non-GPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

STATUS = {0: "HP_OK", 1: "HP_ERR_INVALID_ARG", 2: "HP_ERR_INDEX_RANGE", 3: "HP_ERR_NOT_PERMUTATION",
          4: "HP_ERR_DUPLICATE_INDEX", 5: "HP_ERR_NOT_CANONICAL", 6: "HP_ERR_SHAPE",
          7: "HP_ERR_OVERFLOW", 8: "HP_ERR_WORKSPACE", 9: "HP_ERR_CAPACITY", 10: "HP_ERR_HIP",
          11: "HP_ERR_ALIAS", 12: "HP_ERR_TIMEOUT", 13: "HP_ERR_REJECTED"}
OPS = {"second": 0, "plus": 1, "replace": 2}


class HPError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"{self.name}: {msg}")


class hp_csr_t(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("ptr_type", ctypes.c_int32), ("val_type", ctypes.c_int32),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class hp_dcsc_t(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("nzc", ctypes.c_int64), ("ptr_type", ctypes.c_int32), ("val_type", ctypes.c_int32),
                ("dcsc", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("jc", ctypes.c_void_p), ("colptr", ctypes.c_void_p), ("row", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class hp_plan_info_t(ctypes.Structure):
    _fields_ = [("nnz_out", ctypes.c_int64), ("exec_ws_bytes", ctypes.c_size_t),
                ("map_monotone", ctypes.c_int32), ("op", ctypes.c_int32),
                ("rows_sorted", ctypes.c_int64 * 4), ("class_elems", ctypes.c_int64 * 4),
                ("aux", ctypes.c_int64 * 4)]


class hp_request_t(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("status", ctypes.c_int32), ("A", hp_csr_t),
                ("I", ctypes.c_void_p), ("J", ctypes.c_void_p), ("nI", ctypes.c_int64),
                ("nJ", ctypes.c_int64), ("p", ctypes.c_void_p), ("q", ctypes.c_void_p), ("C", hp_csr_t),
                ("B", hp_csr_t), ("op", ctypes.c_int32), ("pad", ctypes.c_int32), ("ready", ctypes.c_void_p)]


class hp_batch_info_t(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("nnz_total", ctypes.c_int64), ("failed", ctypes.c_int32),
                ("grid_plan", ctypes.c_int32), ("tiles_plan", ctypes.c_int64), ("tiles_exec", ctypes.c_int64),
                ("grid_exec", ctypes.c_int32), ("flags", ctypes.c_int32)]


class hp_server_config_t(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("release_wait_ms", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class hp_completion_t(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("C", hp_csr_t), ("t_submit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


BATCH_NO_GRAPH = 1
BATCH_NO_TUNE = 2


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_CSRP = ctypes.POINTER(hp_csr_t)
_INFOP = ctypes.POINTER(hp_plan_info_t)


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


hp_create = _sig("hp_create", [ctypes.POINTER(_P), ctypes.c_int])
hp_destroy = _sig("hp_destroy", [_P])
hp_set_stream = _sig("hp_set_stream", [_P, _P])
hp_status_string = _sig("hp_status_string", [ctypes.c_int], ctypes.c_char_p)
hp_last_error = _sig("hp_last_error", [_P], ctypes.c_char_p)
hp_enable_timing = _sig("hp_enable_timing", [_P, ctypes.c_int])
hp_stage_times = _sig("hp_stage_times", [_P, ctypes.POINTER(ctypes.c_float),
                                         ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_char_p), ctypes.c_int])
hp_permute_workspace = _sig("hp_permute_workspace", [_P, _CSRP, ctypes.POINTER(_SZ)])
hp_permute_plan = _sig("hp_permute_plan", [_P, _CSRP, _P, _P, _CSRP, _P, _SZ, _INFOP])
hp_permute_exec = _sig("hp_permute_exec", [_P, _CSRP, _P, _P, _CSRP, _P, _SZ, _INFOP, _P, _SZ])
hp_spref_workspace = _sig("hp_spref_workspace", [_P, _CSRP, _I64, _I64, ctypes.POINTER(_SZ)])
hp_spref_plan = _sig("hp_spref_plan", [_P, _CSRP, _P, _I64, _P, _I64, _CSRP, _P, _SZ, _INFOP])
hp_spref_exec = _sig("hp_spref_exec", [_P, _CSRP, _P, _I64, _P, _I64, _CSRP, _P, _SZ, _INFOP, _P, _SZ])
_REQP = ctypes.POINTER(hp_request_t)
_BINFOP = ctypes.POINTER(hp_batch_info_t)
hp_batch_workspace = _sig("hp_batch_workspace", [_P, _REQP, ctypes.c_int, ctypes.POINTER(_SZ)])
hp_batch_plan = _sig("hp_batch_plan", [_P, _REQP, ctypes.c_int, _P, _SZ, _BINFOP])
hp_batch_exec = _sig("hp_batch_exec", [_P, _REQP, ctypes.c_int, _P, _SZ, _BINFOP, _P, _SZ])
hp_validate_workspace = _sig("hp_validate_workspace", [_P, _CSRP, ctypes.POINTER(_SZ)])
hp_validate_csr = _sig("hp_validate_csr", [_P, _CSRP, _P, _SZ])
hp_set_validate = _sig("hp_set_validate", [_P, ctypes.c_int])
hp_spasgn_workspace = _sig("hp_spasgn_workspace", [_P, _CSRP, _CSRP, ctypes.POINTER(_SZ)])
hp_spasgn_plan = _sig("hp_spasgn_plan", [_P, _CSRP, _CSRP, _P, _P, ctypes.c_int, _CSRP, _P, _SZ, _INFOP])
hp_spasgn_exec = _sig("hp_spasgn_exec", [_P, _CSRP, _CSRP, _P, _P, ctypes.c_int, _CSRP, _P, _SZ, _INFOP,
                                         _P, _SZ])
hp_spasgn_permute_workspace = _sig("hp_spasgn_permute_workspace", [_P, _CSRP, _CSRP, ctypes.POINTER(_SZ)])
hp_spasgn_permute_plan = _sig("hp_spasgn_permute_plan", [_P, _CSRP, _CSRP, _P, _P, ctypes.c_int, _P, _P, _CSRP,
                                                         _P, _SZ, _INFOP])
hp_spasgn_permute_exec = _sig("hp_spasgn_permute_exec", [_P, _CSRP, _CSRP, _P, _P, ctypes.c_int, _P, _P, _CSRP,
                                                         _P, _SZ, _INFOP, _P, _SZ])
_DCSCP = ctypes.POINTER(hp_dcsc_t)
hp_spref_dcsc_workspace = _sig("hp_spref_dcsc_workspace", [_P, _DCSCP, _I64, _I64, ctypes.POINTER(_SZ)])
hp_spref_dcsc_plan = _sig("hp_spref_dcsc_plan", [_P, _DCSCP, _P, _I64, _P, _I64, _DCSCP, _P, _SZ, _INFOP])
hp_spref_dcsc_exec = _sig("hp_spref_dcsc_exec", [_P, _DCSCP, _P, _I64, _P, _I64, _DCSCP, _P, _SZ, _INFOP,
                                                 _P, _SZ])
hp_permute_noalloc = _sig("hp_permute_noalloc", [_P, _CSRP, _P, _P, _CSRP])
hp_gather_index = _sig("hp_gather_index", [_P, _P, _I64, _P, _I64, _P])
hp_invert_perm = _sig("hp_invert_perm", [_P, _P, _I64, _P])
hp_block_nnz = _sig("hp_block_nnz", [_P, _CSRP, ctypes.c_int32, ctypes.c_int32, _P])
hp_server_create = _sig("hp_server_create", [ctypes.POINTER(_P), ctypes.c_int, _P, _SZ,
                                             ctypes.POINTER(hp_server_config_t)])
hp_server_submit = _sig("hp_server_submit", [_P, _REQP, ctypes.POINTER(ctypes.c_uint64)])
hp_server_poll = _sig("hp_server_poll", [_P, ctypes.POINTER(hp_completion_t), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)])
hp_server_drain = _sig("hp_server_drain", [_P])
hp_server_release = _sig("hp_server_release", [_P, ctypes.c_uint64])
hp_server_memory = _sig("hp_server_memory", [_P, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ)])
hp_server_destroy = _sig("hp_server_destroy", [_P])

@dataclass
class CSR:
    nrows: int
    ncols: int
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col.numel())


@dataclass
class DCSC:
    """Column-compressed matrix: CSC when jc is None (colptr has ncols+1
    entries), else doubly compressed (only the columns jc are stored,
    colptr has len(jc)+1 entries)."""
    nrows: int
    ncols: int
    jc: Optional[torch.Tensor]
    colptr: torch.Tensor
    row: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.row.numel())


def _ptr_type(t):
    if t.dtype == torch.int32:
        return 0
    if t.dtype == torch.int64:
        return 1
    raise HPError(1, f"rowptr dtype {t.dtype} not int32/int64")


def _val_type(t):
    if t.dtype == torch.float32:
        return 0
    if t.dtype == torch.float64:
        return 1
    raise HPError(1, f"value dtype {t.dtype} not float32/float64")


def _dptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise HPError(1, "tensor is not on the GPU")
    if not t.is_contiguous():
        raise HPError(1, "tensor is not contiguous")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() > 0 else ctypes.c_void_p(t.data_ptr() or 0)


def to_csr_t(A) -> hp_csr_t:
    return hp_csr_t(A.nrows, A.ncols, int(A.col.numel()), _ptr_type(A.rowptr), _val_type(A.val),
                    _dptr(A.rowptr), _dptr(A.col), _dptr(A.val))


def to_dcsc_t(A) -> hp_dcsc_t:
    dc = A.jc is not None
    nzc = int(A.jc.numel()) if dc else int(A.ncols)
    return hp_dcsc_t(A.nrows, A.ncols, int(A.row.numel()), nzc, _ptr_type(A.colptr), _val_type(A.val),
                     1 if dc else 0, 0, _idx(A.jc) if dc else None, _dptr(A.colptr), _dptr(A.row), _dptr(A.val))


def _idx(x: Optional[torch.Tensor]):
    if x is None:
        return None
    if x.dtype != torch.int32:
        raise HPError(1, "index vectors must be int32")
    return _dptr(x)


class Handle:
    """One library handle on one device; work goes on torch's current stream."""

    def __init__(self, device: int = 0):
        self.device = device
        h = _P()
        st = hp_create(ctypes.byref(h), device)
        if st != 0:
            raise HPError(st, "hp_create failed")
        self.h = h

    def close(self):
        if self.h:
            hp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        hp_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def check(self, st):
        if st != 0:
            raise HPError(st, (hp_last_error(self.h) or b"").decode())

    def timing(self, on: bool):
        self.check(hp_enable_timing(self.h, 1 if on else 0))

    def stage_times(self):
        """{stage: (total_ms, launches)} since the previous call."""
        ms = (ctypes.c_float * 64)()
        cnt = (ctypes.c_int * 64)()
        nm = (ctypes.c_char_p * 64)()
        k = hp_stage_times(self.h, ms, cnt, nm, 64)
        return {nm[i].decode(): (float(ms[i]), int(cnt[i])) for i in range(k)}

    def _alloc(self, nbytes):
        return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=f"cuda:{self.device}")

    def set_validate(self, on: bool):
        """Plans check their CSR inputs first (hp_set_validate)."""
        self.check(hp_set_validate(self.h, 1 if on else 0))

    def validate(self, A):
        """Raise HPError unless A is canonical CSR (hp_validate_csr)."""
        self._stream()
        Ac = to_csr_t(A)
        need = _SZ(0)
        self.check(hp_validate_workspace(self.h, ctypes.byref(Ac), ctypes.byref(need)))
        ws = self._alloc(need.value)
        self.check(hp_validate_csr(self.h, ctypes.byref(Ac), _dptr(ws), ws.numel()))

    # ---- permute -----------------------------------------------------------
    def permute_plan(self, A, p, q=None, ws=None):
        """Plan C = P A Q^T; returns (C with rowptr filled, ws, info)."""
        self._stream()
        Ac = to_csr_t(A)
        need = _SZ(0)
        self.check(hp_permute_workspace(self.h, ctypes.byref(Ac), ctypes.byref(need)))
        if ws is None or ws.numel() < need.value:
            ws = self._alloc(need.value)
        rowptr = torch.empty(A.nrows + 1, dtype=A.rowptr.dtype, device=A.rowptr.device)
        Cc = hp_csr_t(A.nrows, A.ncols, 0, Ac.ptr_type, Ac.val_type, _dptr(rowptr), None, None)
        info = hp_plan_info_t()
        self.check(hp_permute_plan(self.h, ctypes.byref(Ac), _idx(p), _idx(q), ctypes.byref(Cc),
                                   _dptr(ws), ws.numel(), ctypes.byref(info)))
        C = CSR(A.nrows, A.ncols, rowptr,
                torch.empty(Cc.nnz, dtype=torch.int32, device=A.col.device),
                torch.empty(Cc.nnz, dtype=A.val.dtype, device=A.val.device))
        return C, ws, info

    def permute_exec(self, A, p, q, C, ws, info, xws=None):
        """Exec of a permute plan.  Without `xws` one of info.exec_ws_bytes
        is allocated; a caller's `xws` goes to the library as it is (it
        needs at least info.aux[0] bytes: the row-slot form runs when it
        holds info.exec_ws_bytes)."""
        self._stream()
        Ac = to_csr_t(A)
        Cc = to_csr_t(C)
        if xws is None and info.exec_ws_bytes:
            xws = self._alloc(info.exec_ws_bytes)
        self.check(hp_permute_exec(self.h, ctypes.byref(Ac), _idx(p), _idx(q), ctypes.byref(Cc),
                                   _dptr(ws), ws.numel(), ctypes.byref(info),
                                   _dptr(xws) if xws is not None else None,
                                   xws.numel() if xws is not None else 0))
        return C

    def permute(self, A, p, q=None):
        C, ws, info = self.permute_plan(A, p, q)
        return self.permute_exec(A, p, q, C, ws, info)

    def permute_noalloc(self, A, p, q=None, out=None):
        """C = P A Q^T through hp_permute_noalloc: the library takes its
        workspaces from its fixed scratch array.  `out` (a CSR of A's shape
        and types with nnz(A) entries) receives the result; without it one
        is allocated here, before the call."""
        self._stream()
        Ac = to_csr_t(A)
        if out is None:
            out = CSR(A.nrows, A.ncols, torch.empty(A.nrows + 1, dtype=A.rowptr.dtype, device=A.rowptr.device),
                      torch.empty(A.nnz, dtype=torch.int32, device=A.col.device),
                      torch.empty(A.nnz, dtype=A.val.dtype, device=A.val.device))
        Cc = to_csr_t(out)
        self.check(hp_permute_noalloc(self.h, ctypes.byref(Ac), _idx(p), _idx(q), ctypes.byref(Cc)))
        return out

    # ---- spref -------------------------------------------------------------
    def spref_plan(self, A, I, J, ws=None):
        """Plan C = A(I, J); returns (C with rowptr filled, ws, info)."""
        self._stream()
        Ac = to_csr_t(A)
        nI, nJ = int(I.numel()), int(J.numel())
        need = _SZ(0)
        self.check(hp_spref_workspace(self.h, ctypes.byref(Ac), nI, nJ, ctypes.byref(need)))
        if ws is None or ws.numel() < need.value:
            ws = self._alloc(need.value)
        rowptr = torch.empty(nI + 1, dtype=A.rowptr.dtype, device=A.rowptr.device)
        Cc = hp_csr_t(nI, nJ, 0, Ac.ptr_type, Ac.val_type, _dptr(rowptr), None, None)
        info = hp_plan_info_t()
        self.check(hp_spref_plan(self.h, ctypes.byref(Ac), _idx(I), nI, _idx(J), nJ, ctypes.byref(Cc),
                                 _dptr(ws), ws.numel(), ctypes.byref(info)))
        C = CSR(nI, nJ, rowptr, torch.empty(Cc.nnz, dtype=torch.int32, device=A.col.device),
                torch.empty(Cc.nnz, dtype=A.val.dtype, device=A.val.device))
        return C, ws, info

    def spref_exec(self, A, I, J, C, ws, info, xws=None):
        self._stream()
        Ac = to_csr_t(A)
        Cc = to_csr_t(C)
        if info.exec_ws_bytes and (xws is None or xws.numel() < info.exec_ws_bytes):
            xws = self._alloc(info.exec_ws_bytes)
        self.check(hp_spref_exec(self.h, ctypes.byref(Ac), _idx(I), int(I.numel()), _idx(J),
                                 int(J.numel()), ctypes.byref(Cc), _dptr(ws), ws.numel(),
                                 ctypes.byref(info), _dptr(xws) if xws is not None else None,
                                 xws.numel() if xws is not None else 0))
        return C

    def spref(self, A, I, J):
        C, ws, info = self.spref_plan(A, I, J)
        return self.spref_exec(A, I, J, C, ws, info)

    # ---- spref on CSC / DCSC -------------------------------------------------
    def spref_dcsc_plan(self, A, I, J, ws=None):
        """Plan C = A(I, J) for column-compressed A; C comes back in CSC."""
        self._stream()
        Ac = to_dcsc_t(A)
        nI, nJ = int(I.numel()), int(J.numel())
        need = _SZ(0)
        self.check(hp_spref_dcsc_workspace(self.h, ctypes.byref(Ac), nI, nJ, ctypes.byref(need)))
        if ws is None or ws.numel() < need.value:
            ws = self._alloc(need.value)
        colptr = torch.empty(nJ + 1, dtype=A.colptr.dtype, device=A.colptr.device)
        Cc = hp_dcsc_t(nI, nJ, 0, nJ, Ac.ptr_type, Ac.val_type, 0, 0, None, _dptr(colptr), None, None)
        info = hp_plan_info_t()
        self.check(hp_spref_dcsc_plan(self.h, ctypes.byref(Ac), _idx(I), nI, _idx(J), nJ, ctypes.byref(Cc),
                                      _dptr(ws), ws.numel(), ctypes.byref(info)))
        C = DCSC(nI, nJ, None, colptr, torch.empty(Cc.nnz, dtype=torch.int32, device=A.row.device),
                 torch.empty(Cc.nnz, dtype=A.val.dtype, device=A.val.device))
        return C, ws, info

    def spref_dcsc_exec(self, A, I, J, C, ws, info, xws=None):
        self._stream()
        Ac, Cc = to_dcsc_t(A), to_dcsc_t(C)
        if info.exec_ws_bytes and (xws is None or xws.numel() < info.exec_ws_bytes):
            xws = self._alloc(info.exec_ws_bytes)
        self.check(hp_spref_dcsc_exec(self.h, ctypes.byref(Ac), _idx(I), int(I.numel()), _idx(J), int(J.numel()),
                                      ctypes.byref(Cc), _dptr(ws), ws.numel(), ctypes.byref(info),
                                      _dptr(xws) if xws is not None else None,
                                      xws.numel() if xws is not None else 0))
        return C

    def spref_dcsc(self, A, I, J):
        C, ws, info = self.spref_dcsc_plan(A, I, J)
        return self.spref_dcsc_exec(A, I, J, C, ws, info)

    # ---- spasgn ------------------------------------------------------------
    @staticmethod
    def _op(op):
        if isinstance(op, str):
            if op not in OPS:
                raise HPError(1, f"unknown operator {op!r}")
            return OPS[op]
        return int(op)

    def spasgn_plan(self, A, B, I, J, op="second", ws=None):
        """Plan C = A with A(I, J) = B; returns (C with rowptr filled, ws, info)."""
        self._stream()
        if int(I.numel()) != B.nrows or int(J.numel()) != B.ncols:
            raise HPError(6, "B must be |I| x |J|")
        Ac, Bc = to_csr_t(A), to_csr_t(B)
        need = _SZ(0)
        self.check(hp_spasgn_workspace(self.h, ctypes.byref(Ac), ctypes.byref(Bc), ctypes.byref(need)))
        if ws is None or ws.numel() < need.value:
            ws = self._alloc(need.value)
        rowptr = torch.empty(A.nrows + 1, dtype=A.rowptr.dtype, device=A.rowptr.device)
        Cc = hp_csr_t(A.nrows, A.ncols, 0, Ac.ptr_type, Ac.val_type, _dptr(rowptr), None, None)
        info = hp_plan_info_t()
        self.check(hp_spasgn_plan(self.h, ctypes.byref(Ac), ctypes.byref(Bc), _idx(I), _idx(J),
                                  self._op(op), ctypes.byref(Cc), _dptr(ws), ws.numel(), ctypes.byref(info)))
        C = CSR(A.nrows, A.ncols, rowptr, torch.empty(Cc.nnz, dtype=torch.int32, device=A.col.device),
                torch.empty(Cc.nnz, dtype=A.val.dtype, device=A.val.device))
        return C, ws, info

    def spasgn_exec(self, A, B, I, J, C, ws, info, op="second", xws=None):
        self._stream()
        Ac, Bc, Cc = to_csr_t(A), to_csr_t(B), to_csr_t(C)
        if info.exec_ws_bytes and (xws is None or xws.numel() < info.exec_ws_bytes):
            xws = self._alloc(info.exec_ws_bytes)
        self.check(hp_spasgn_exec(self.h, ctypes.byref(Ac), ctypes.byref(Bc), _idx(I), _idx(J),
                                  self._op(op), ctypes.byref(Cc), _dptr(ws), ws.numel(), ctypes.byref(info),
                                  _dptr(xws) if xws is not None else None,
                                  xws.numel() if xws is not None else 0))
        return C

    def spasgn(self, A, B, I, J, op="second"):
        C, ws, info = self.spasgn_plan(A, B, I, J, op)
        return self.spasgn_exec(A, B, I, J, C, ws, info, op)

    # ---- incremental-update bookkeeping -------------------------------------
    def gather_index(self, map_, idx, out=None):
        """out[t] = map_[idx[t]] (-1 where idx[t] is outside map_)."""
        self._stream()
        if out is None:
            out = torch.empty_like(idx)
        self.check(hp_gather_index(self.h, _idx(map_), int(map_.numel()), _idx(idx), int(idx.numel()), _idx(out)))
        return out

    def invert_perm(self, p, out=None):
        """pinv with pinv[p[t]] = t."""
        self._stream()
        if out is None:
            out = torch.empty_like(p)
        self.check(hp_invert_perm(self.h, _idx(p), int(p.numel()), _idx(out)))
        return out

    def block_nnz(self, A, gr, gc, out=None):
        """Stored entries of A per block of a gr x gc grid (device int64, row-major)."""
        self._stream()
        if out is None:
            out = torch.empty(gr * gc, dtype=torch.int64, device=A.col.device)
        Ac = to_csr_t(A)
        self.check(hp_block_nnz(self.h, ctypes.byref(Ac), gr, gc, _dptr(out)))
        return out

    # ---- fused assign + permute -------------------------------------------
    def spasgn_permute_plan(self, A, B, I, J, p, q=None, op="second", ws=None):
        """Plan C = P (A with A(I, J) = B) Q^T; returns (C with rowptr filled, ws, info)."""
        self._stream()
        if int(I.numel()) != B.nrows or int(J.numel()) != B.ncols:
            raise HPError(6, "B must be |I| x |J|")
        Ac, Bc = to_csr_t(A), to_csr_t(B)
        need = _SZ(0)
        self.check(hp_spasgn_permute_workspace(self.h, ctypes.byref(Ac), ctypes.byref(Bc), ctypes.byref(need)))
        if ws is None or ws.numel() < need.value:
            ws = self._alloc(need.value)
        rowptr = torch.empty(A.nrows + 1, dtype=A.rowptr.dtype, device=A.rowptr.device)
        Cc = hp_csr_t(A.nrows, A.ncols, 0, Ac.ptr_type, Ac.val_type, _dptr(rowptr), None, None)
        info = hp_plan_info_t()
        self.check(hp_spasgn_permute_plan(self.h, ctypes.byref(Ac), ctypes.byref(Bc), _idx(I), _idx(J),
                                          self._op(op), _idx(p), _idx(q), ctypes.byref(Cc), _dptr(ws),
                                          ws.numel(), ctypes.byref(info)))
        C = CSR(A.nrows, A.ncols, rowptr, torch.empty(Cc.nnz, dtype=torch.int32, device=A.col.device),
                torch.empty(Cc.nnz, dtype=A.val.dtype, device=A.val.device))
        return C, ws, info

    def spasgn_permute_exec(self, A, B, I, J, p, q, C, ws, info, op="second", xws=None):
        """Exec of a fused plan.  Without `xws` one of info.exec_ws_bytes is
        allocated; a caller's `xws` goes to the library as it is (at least
        info.aux[3] bytes; the row-slot form runs when it holds
        info.exec_ws_bytes)."""
        self._stream()
        Ac, Bc, Cc = to_csr_t(A), to_csr_t(B), to_csr_t(C)
        if xws is None and info.exec_ws_bytes:
            xws = self._alloc(info.exec_ws_bytes)
        self.check(hp_spasgn_permute_exec(self.h, ctypes.byref(Ac), ctypes.byref(Bc), _idx(I), _idx(J),
                                          self._op(op), _idx(p), _idx(q), ctypes.byref(Cc), _dptr(ws),
                                          ws.numel(), ctypes.byref(info),
                                          _dptr(xws) if xws is not None else None,
                                          xws.numel() if xws is not None else 0))
        return C

    def spasgn_permute(self, A, B, I, J, p, q=None, op="second"):
        C, ws, info = self.spasgn_permute_plan(A, B, I, J, p, q, op)
        return self.spasgn_permute_exec(A, B, I, J, p, q, C, ws, info, op)


KINDS = {"spref": 0, "permute": 1, "spasgn": 2}


class Batch:
    """Many requests planned and executed together (hp_batch_plan /
    hp_batch_exec).  Each request is a dict with kind="spref" (A, I, J),
    kind="permute" (A, p, q=None) or kind="spasgn" (A, B, I, J, op)."""

    def __init__(self, handle: "Handle", requests):
        self.hd = handle
        self.requests = list(requests)
        n = len(self.requests)
        self.arr = (hp_request_t * max(n, 1))()
        for k, r in enumerate(self.requests):
            rq = self.arr[k]
            rq.kind = KINDS[r["kind"]]
            rq.A = to_csr_t(r["A"])
            if r["kind"] == "spref":
                rq.I, rq.J = _idx(r["I"]), _idx(r["J"])
                rq.nI, rq.nJ = int(r["I"].numel()), int(r["J"].numel())
            elif r["kind"] == "spasgn":
                rq.B = to_csr_t(r["B"])
                rq.I, rq.J = _idx(r["I"]), _idx(r["J"])
                rq.nI, rq.nJ = int(r["I"].numel()), int(r["J"].numel())
                rq.op = Handle._op(r.get("op", "second"))
            else:
                rq.p, rq.q = _idx(r["p"]), _idx(r.get("q"))
        self.ws = None
        self.arena = None
        self.info = hp_batch_info_t()

    def plan(self):
        self.hd._stream()
        n = len(self.requests)
        need = _SZ(0)
        self.hd.check(hp_batch_workspace(self.hd.h, self.arr, n, ctypes.byref(need)))
        if self.ws is None or self.ws.numel() < need.value:
            self.ws = self.hd._alloc(need.value)
        self.hd.check(hp_batch_plan(self.hd.h, self.arr, n, _dptr(self.ws), self.ws.numel(),
                                    ctypes.byref(self.info)))
        return [int(self.arr[k].status) for k in range(n)]

    def exec(self, graph: bool = True):
        """Run the exec half: replayed from a captured hipGraph (graph=True)
        or launched directly."""
        self.hd._stream()
        self.info.flags = 0 if graph else BATCH_NO_GRAPH
        n = len(self.requests)
        if self.arena is None or self.arena.numel() < self.info.arena_bytes:
            self.arena = self.hd._alloc(self.info.arena_bytes)
        self.hd.check(hp_batch_exec(self.hd.h, self.arr, n, _dptr(self.ws), self.ws.numel(),
                                    ctypes.byref(self.info), _dptr(self.arena), self.arena.numel()))

    def results(self):
        """CSR views into the arena (None for requests that failed)."""
        return [_csr_view(self.arena, self.arr[k].C) if self.arr[k].status == 0 else None
                for k in range(len(self.requests))]

    def run(self):
        self.plan()
        self.exec()
        return self.results()


def _csr_view(buf: torch.Tensor, C: hp_csr_t) -> CSR:
    """CSR whose arrays are views into the device buffer `buf` that holds them."""
    base = buf.data_ptr()
    pt = torch.int64 if C.ptr_type == 1 else torch.int32
    vt = torch.float64 if C.val_type == 1 else torch.float32

    def view(ptr, count, dt):
        if count == 0:
            return torch.empty(0, dtype=dt, device=buf.device)
        es = torch.empty(0, dtype=dt).element_size()
        off = ptr - base
        return buf[off:off + count * es].view(dt)
    return CSR(int(C.nrows), int(C.ncols), view(C.rowptr, int(C.nrows) + 1, pt),
               view(C.col or base, int(C.nnz), torch.int32), view(C.val or base, int(C.nnz), vt))


class Server:
    """Served form (hp_server_*): submit requests as they arrive; workers run
    them in continuous batches on their own streams inside an HBM budget of
    `pool_bytes` (a device buffer this object allocates once).

    submit(kind, A, ...) -> id; poll() -> list of completion dicts with the
    result as CSR views into the pool (valid until release(id))."""

    def __init__(self, pool_bytes: int, device: int = 0, max_inflight: int = 4, max_batch: int = 256,
                 release_wait_ms: int = 0):
        torch.cuda.set_device(device)
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        cfg = hp_server_config_t(max_inflight, max_batch, release_wait_ms, 0)
        h = _P()
        code = hp_server_create(ctypes.byref(h), device, _dptr(self.pool), pool_bytes, ctypes.byref(cfg))
        if code != 0:
            raise HPError(code, "hp_server_create failed")
        self.h = h
        self._keep = {}        # id -> tensors the request points to
        self.device = device

    def submit(self, kind: str, A: CSR, I=None, J=None, p=None, q=None, B: Optional[CSR] = None,
               op: str = "second") -> int:
        rq = hp_request_t()
        rq.kind = KINDS[kind]
        rq.A = to_csr_t(A)
        keep = [A, I, J, p, q, B]
        if kind == "spref":
            rq.I, rq.J = _idx(I), _idx(J)
            rq.nI, rq.nJ = int(I.numel()), int(J.numel())
        elif kind == "permute":
            rq.p, rq.q = _idx(p), _idx(q)
        else:
            if int(I.numel()) != B.nrows or int(J.numel()) != B.ncols:
                raise HPError(6, "B must be |I| x |J|")
            rq.B = to_csr_t(B)
            rq.I, rq.J = _idx(I), _idx(J)
            rq.nI, rq.nJ = int(I.numel()), int(J.numel())
            rq.op = OPS[op]
        # the inputs may still be being written on the caller's stream: the
        # worker's stream waits for this event before it reads them
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(self.device))
        rq.ready = ctypes.c_void_p(ev.cuda_event)
        keep.append(ev)
        rid = ctypes.c_uint64(0)
        code = hp_server_submit(self.h, ctypes.byref(rq), ctypes.byref(rid))
        if code != 0:
            raise HPError(code, "hp_server_submit rejected the request")
        self._keep[rid.value] = keep
        return rid.value

    def poll(self, cap: int = 4096):
        buf = (hp_completion_t * cap)()
        n = ctypes.c_int(0)
        code = hp_server_poll(self.h, buf, cap, ctypes.byref(n))
        if code != 0:
            raise HPError(code, "hp_server_poll")
        out = []
        for k in range(n.value):
            c = buf[k]
            self._keep.pop(c.id, None)
            out.append(dict(id=c.id, status=c.status, batch_size=c.batch_size,
                            C=_csr_view(self.pool, c.C) if c.status == 0 else None,
                            t_submit_ns=c.t_submit_ns, t_start_ns=c.t_start_ns, t_done_ns=c.t_done_ns))
        return out

    def drain(self):
        code = hp_server_drain(self.h)
        if code != 0:
            raise HPError(code, "hp_server_drain")

    def release(self, rid: int):
        """Return a result's pool space.  Work already queued on the current
        stream may still read the result, so that stream is synchronised
        first (the space is reused by later requests at once)."""
        torch.cuda.current_stream(self.device).synchronize()
        code = hp_server_release(self.h, rid)
        if code != 0:
            raise HPError(code, f"hp_server_release({rid})")

    def memory(self):
        a, b = _SZ(0), _SZ(0)
        hp_server_memory(self.h, ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def close(self):
        if self.h:
            hp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def handle(device: int = 0) -> Handle:
    if device not in _default:
        _default[device] = Handle(device)
    return _default[device]


def permute(A, p, q=None, device: int = 0) -> CSR:
    """C = P A Q^T with C[i, j] = A[p[i], q[j]]; q=None gives P A P^T."""
    return handle(device).permute(A, p, q)


def spref(A, I, J, device: int = 0) -> CSR:
    """C = A(I, J) with C[i, j] = A[I[i], J[j]]; repeated/unordered indices allowed."""
    return handle(device).spref(A, I, J)


def spref_dcsc(A, I, J, device: int = 0) -> DCSC:
    """C = A(I, J) for A in CSC/DCSC (a DCSC); C in CSC."""
    return handle(device).spref_dcsc(A, I, J)


def spasgn(A, B, I, J, op="second", device: int = 0) -> CSR:
    """C = A with A(I, J) = B; op: "second" (overwrite), "plus" or "replace" (block)."""
    return handle(device).spasgn(A, B, I, J, op)


def spasgn_permute(A, B, I, J, p, q=None, op="second", device: int = 0) -> CSR:
    """C = P X Q^T with X = A after A(I, J) = B under op, in one fused pass."""
    return handle(device).spasgn_permute(A, B, I, J, p, q, op)
