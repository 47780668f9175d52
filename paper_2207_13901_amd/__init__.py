"""spleaf: sparse tensor algebra leaf kernels for one MI355X (gfx950).

A thin binding of libspleaf's C ABI (include/spleaf.h): the functions below
only marshal torch tensors (device memory) and the current HIP stream into
the C structs; every step of every operation runs in the library's HIP
kernels.  The names follow the C entry points without the ``spl_`` prefix.

Sparse operands are ``CSR`` (Dense, Compressed), ``CSF`` (Dense,
Compressed, Compressed) and ``DDC`` (Dense, Dense, Compressed) objects
holding int32 pos/crd and a value tensor, all on the same GPU.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _native as N
from ._native import SpleafError

__all__ = [
    "CSR", "CSF", "Context", "schedule", "spmv", "spmm", "tile_bounds",
    "validate", "op_parse", "op_tin", "workspace_query", "workspace", "SpleafError",
    "timing_enable", "timing_read", "probe", "spttv", "mttkrp", "inner", "sddmm",
    "spadd3", "autotune", "mlp_load", "mlp_save", "mlp_predict", "mlp_train_step",
    "schedule_dict", "coord_partition", "spmv_window", "DDC", "csf_tile_bounds",
    "spmv_noalloc", "tin", "tin_source", "transpose", "CSC",
]

_DT = {torch.float64: N.F64, torch.float32: N.F32, torch.bfloat16: N.BF16}
_KIND = {"default": N.SCHED_DEFAULT, "row": N.ROW, "nnz": N.NNZ, "merge": N.MERGE,
         "learned": N.SCHED_LEARNED, "autotune": N.SCHED_AUTOTUNE}
_KIND_NAME = {v: k for k, v in _KIND.items()}


def _dtype_code(t: torch.Tensor) -> int:
    try:
        return _DT[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}") from None


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


@dataclass
class CSR:
    """CSR matrix: pos int32[n+1] (or int64[n+1], accepted by spmv with the
    merge schedule), crd int32[nnz], vals[nnz]; shape (n, m)."""
    pos: torch.Tensor
    crd: torch.Tensor
    vals: torch.Tensor
    shape: tuple

    def struct(self) -> N.SplSparse:
        s = N.SplSparse()
        s.order = 2
        s.vtype = _dtype_code(self.vals)
        s.dims[0], s.dims[1], s.dims[2] = self.shape[0], self.shape[1], 0
        s.level[0], s.level[1] = N.DENSE, N.COMPRESSED
        s.pos[1] = _ptr(self.pos)
        s.crd[1] = _ptr(self.crd)
        s.vals = _ptr(self.vals)
        s.nnz = self.crd.numel()
        s.pos_type = N.I64 if self.pos.dtype == torch.int64 else N.I32
        return s

    def with_vals(self, vals: torch.Tensor) -> "CSR":
        return CSR(self.pos, self.crd, vals, self.shape)


@dataclass
class CSF:
    """CSF 3-tensor: pos1 int32[I+1], crd1 int32[F] (j per fiber),
    pos2 int32[F+1], crd2 int32[nnz] (k per value), vals[nnz]."""
    pos1: torch.Tensor
    crd1: torch.Tensor
    pos2: torch.Tensor
    crd2: torch.Tensor
    vals: torch.Tensor
    shape: tuple

    def struct(self) -> N.SplSparse:
        s = N.SplSparse()
        s.order = 3
        s.vtype = _dtype_code(self.vals)
        for d in range(3):
            s.dims[d] = self.shape[d]
        s.level[0], s.level[1], s.level[2] = N.DENSE, N.COMPRESSED, N.COMPRESSED
        s.pos[1], s.crd[1] = _ptr(self.pos1), _ptr(self.crd1)
        s.pos[2], s.crd[2] = _ptr(self.pos2), _ptr(self.crd2)
        s.vals = _ptr(self.vals)
        s.nnz = self.crd2.numel()
        s.nfibers = self.crd1.numel()
        if self.pos2.dtype == torch.int64:
            if self.pos1.dtype != torch.int64:
                raise ValueError("int64 positions: pos1 and pos2 both int64")
            s.pos_type = N.I64
        return s

    def with_vals(self, vals: torch.Tensor) -> "CSF":
        return CSF(self.pos1, self.crd1, self.pos2, self.crd2, vals, self.shape)

    @property
    def nfibers(self) -> int:
        return self.crd1.numel()


@dataclass
class DDC:
    """(Dense, Dense, Compressed) 3-tensor I x J x K: fiber f = i*J + j owns
    positions [pos2[f], pos2[f+1]); pos2 int32[I*J+1], crd2 int32[nnz] (k per
    value), vals[nnz]."""
    pos2: torch.Tensor
    crd2: torch.Tensor
    vals: torch.Tensor
    shape: tuple

    def struct(self) -> N.SplSparse:
        s = N.SplSparse()
        s.order = 3
        s.vtype = _dtype_code(self.vals)
        for d in range(3):
            s.dims[d] = self.shape[d]
        s.level[0], s.level[1], s.level[2] = N.DENSE, N.DENSE, N.COMPRESSED
        s.pos[2], s.crd[2] = _ptr(self.pos2), _ptr(self.crd2)
        s.vals = _ptr(self.vals)
        s.nnz = self.crd2.numel()
        s.nfibers = self.shape[0] * self.shape[1]
        s.pos_type = N.I64 if self.pos2.dtype == torch.int64 else N.I32
        return s

    def with_vals(self, vals: torch.Tensor) -> "DDC":
        return DDC(self.pos2, self.crd2, vals, self.shape)

    @property
    def nfibers(self) -> int:
        return self.shape[0] * self.shape[1]


def _dense(t: torch.Tensor) -> N.SplDense:
    d = N.SplDense()
    d.data = t.data_ptr()
    d.dtype = _dtype_code(t)
    d.ndim = t.dim()
    if t.dim() == 1:
        if t.numel() and t.stride(0) != 1:
            raise ValueError("dense vector must be contiguous")
        d.dims[0], d.dims[1], d.ld = t.shape[0], 1, 1
    elif t.dim() == 2:
        if t.numel() and t.stride(1) != 1:
            raise ValueError("dense matrix must be row-major (unit column stride)")
        d.dims[0], d.dims[1] = t.shape
        d.ld = t.stride(0) if t.shape[0] > 1 else t.shape[1]
    else:
        raise ValueError("dense operand must have 1 or 2 dimensions")
    return d


def schedule(kind: str = "default", lanes_per_row: int = 0, tile: int = 0,
             items_per_lane: int = 0, col_tile: int = 0, variant: int = 0) -> N.SplSchedule:
    """Build a spl_schedule; zero fields take the library default."""
    s = N.SplSchedule()
    s.kind = _KIND[kind] if isinstance(kind, str) else int(kind)
    s.lanes_per_row, s.tile, s.items_per_lane = lanes_per_row, tile, items_per_lane
    s.col_tile, s.variant = col_tile, variant
    return s


class Context:
    """Owns one spl_context for a device."""

    _per_device: dict = {}

    def __init__(self, device: int = 0):
        self.lib = N.load()
        self.device = device
        h = ctypes.c_void_p()
        st = self.lib.spl_context_create(device, ctypes.byref(h))
        if st != N.OK:
            raise SpleafError(st, f"spl_context_create({device})")
        self.h = h

    @classmethod
    def get(cls, device: Optional[int] = None) -> "Context":
        if device is None:
            device = torch.cuda.current_device()
        if device not in cls._per_device:
            cls._per_device[device] = cls(device)
        return cls._per_device[device]

    def check(self, st: int, what: str):
        if st != N.OK:
            raise SpleafError(st, f"{what}: {self.lib.spl_last_error(self.h).decode()}")

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.spl_context_destroy(self.h)
        except Exception:
            pass


def _ctx_stream(t: torch.Tensor, ctx: Optional[Context]):
    ctx = ctx or Context.get(t.device.index)
    stream = torch.cuda.current_stream(t.device).cuda_stream
    return ctx, stream


def workspace_query(op: int, B, ncols: int = 1, sched=None,
                    ctx: Optional[Context] = None) -> int:
    ctx = ctx or Context.get()
    nbytes = ctypes.c_size_t()
    s = B.struct()
    ctx.check(ctx.lib.spl_workspace_query(ctx.h, op, ctypes.byref(s), ncols,
                                          ctypes.byref(sched) if sched else None,
                                          ctypes.byref(nbytes)), "spl_workspace_query")
    return nbytes.value


def _workspace(op, B, ncols, sched, ctx, device, given=None):
    if given is not None:
        return given, given.numel()
    nbytes = workspace_query(op, B, ncols, sched, ctx)
    if nbytes == 0:
        return None, 0
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def workspace(op: int, B, ncols: int = 1, sched=None, ctx: Optional[Context] = None):
    """A uint8 device tensor large enough for one call of `op` (or None)."""
    dev = B.vals.device
    ws, _ = _workspace(op, B, ncols, sched, ctx or Context.get(dev.index), dev)
    return ws


def spmv(B: CSR, c: torch.Tensor, a: Optional[torch.Tensor] = None, sched=None,
         ctx: Optional[Context] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """a(i) = B(i,j) * c(j)."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    if a is None:
        a = torch.empty(B.shape[0], dtype=B.vals.dtype, device=B.vals.device)
    s = B.struct()
    ws, nb = _workspace(N.OP_SPMV, B, 1, sched, ctx, B.vals.device, ws)
    ctx.check(ctx.lib.spl_spmv(ctx.h, ctypes.byref(s), ctypes.byref(_dense(c)),
                               ctypes.byref(_dense(a)),
                               ctypes.byref(sched) if sched else None,
                               _ptr(ws), nb, stream), "spl_spmv")
    return a


def spmv_noalloc(B: CSR, c: torch.Tensor, a: torch.Tensor, sched=None,
                 ctx: Optional[Context] = None) -> torch.Tensor:
    """a(i) = B(i,j) * c(j) through spl_spmv_noalloc: the library allocates
    nothing (tile bounds and carries in its static device scratch), so `a`
    must be given."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    s = B.struct()
    ctx.check(ctx.lib.spl_spmv_noalloc(ctx.h, ctypes.byref(s), ctypes.byref(_dense(c)),
                                       ctypes.byref(_dense(a)),
                                       ctypes.byref(sched) if sched else None, stream),
              "spl_spmv_noalloc")
    return a


def coord_partition(B: CSR, bounds: torch.Tensor, out: Optional[torch.Tensor] = None,
                    ctx: Optional[Context] = None) -> torch.Tensor:
    """Value-range partition of B's columns: bounds int32[ncolors+1] on the
    device; returns out int32[ncolors+1, n] with color c of row i at
    positions [out[c, i], out[c+1, i])."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    ncolors = bounds.numel() - 1
    if out is None:
        out = torch.empty(ncolors + 1, B.shape[0], dtype=torch.int32, device=B.vals.device)
    s = B.struct()
    ctx.check(ctx.lib.spl_coord_partition(ctx.h, ctypes.byref(s), ncolors, _ptr(bounds),
                                          _ptr(out), stream), "spl_coord_partition")
    return out


def spmv_window(B: CSR, begin: torch.Tensor, end: torch.Tensor, c: torch.Tensor,
                a: Optional[torch.Tensor] = None, sched=None,
                ctx: Optional[Context] = None) -> torch.Tensor:
    """a(i) = sum of B's values times c over positions [begin[i], end[i])."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    if a is None:
        a = torch.empty(B.shape[0], dtype=B.vals.dtype, device=B.vals.device)
    s = B.struct()
    ctx.check(ctx.lib.spl_spmv_window(ctx.h, ctypes.byref(s), _ptr(begin), _ptr(end),
                                      ctypes.byref(_dense(c)), ctypes.byref(_dense(a)),
                                      _sched_ptr(sched), stream), "spl_spmv_window")
    return a


def spmm(B: CSR, C: torch.Tensor, A: Optional[torch.Tensor] = None, sched=None,
         ctx: Optional[Context] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A(i,j) = B(i,k) * C(k,j); BF16 inputs give an FP32 output."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    if A is None:
        odt = torch.float32 if C.dtype == torch.bfloat16 else C.dtype
        A = torch.empty(B.shape[0], C.shape[1], dtype=odt, device=C.device)
    s = B.struct()
    ws, nb = _workspace(N.OP_SPMM, B, C.shape[1], sched, ctx, B.vals.device, ws)
    ctx.check(ctx.lib.spl_spmm(ctx.h, ctypes.byref(s), ctypes.byref(_dense(C)),
                               ctypes.byref(_dense(A)),
                               ctypes.byref(sched) if sched else None,
                               _ptr(ws), nb, stream), "spl_spmm")
    return A


def tile_bounds(B, sched, ctx: Optional[Context] = None):
    """The level partition of B for `sched` (ROW, NNZ or MERGE with a tile
    size): returns (tile_row, tile_pos) int32 tensors of ntiles + 1."""
    dev = (B.pos if isinstance(B, CSR) else B.pos2).device
    ctx, stream = _ctx_stream(B.vals, ctx)
    s = B.struct()
    rows = B.shape[0] if isinstance(B, CSR) else B.nfibers
    items = rows + s.nnz
    cap = items // max(sched.tile, 1) + 3
    tr = torch.empty(cap, dtype=torch.int32, device=dev)
    tp = torch.empty(cap, dtype=torch.int32, device=dev)
    nt = ctypes.c_int64()
    ctx.check(ctx.lib.spl_tile_bounds(ctx.h, ctypes.byref(s), ctypes.byref(sched),
                                      tr.data_ptr(), tp.data_ptr(), cap, ctypes.byref(nt),
                                      stream), "spl_tile_bounds")
    return tr[:nt.value + 1], tp[:nt.value + 1]


def csf_tile_bounds(B: CSF, T: int, ctx: Optional[Context] = None):
    """The fiber-aligned non-zero partition of a CSF tensor in blocks of T
    positions: returns (tile_slice, tile_fiber) int32 tensors of ntiles + 1
    (tile t covers positions [pos2[tile_fiber[t]], pos2[tile_fiber[t+1]]))."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    s = B.struct()
    cap = s.nnz // max(T, 1) + 3
    ts = torch.empty(cap, dtype=torch.int32, device=B.pos2.device)
    tf = torch.empty(cap, dtype=torch.int32, device=B.pos2.device)
    nt = ctypes.c_int64()
    ctx.check(ctx.lib.spl_csf_tile_bounds(ctx.h, ctypes.byref(s), T, ts.data_ptr(),
                                          tf.data_ptr(), cap, ctypes.byref(nt), stream),
              "spl_csf_tile_bounds")
    return ts[:nt.value + 1], tf[:nt.value + 1]


def validate(B, ctx: Optional[Context] = None) -> None:
    """Raise SpleafError(ERR_INVALID) if B's pos/crd contents are malformed."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    s = B.struct()
    ctx.check(ctx.lib.spl_validate(ctx.h, ctypes.byref(s), stream), "spl_validate")


def op_tin(op: int) -> str:
    return N.load().spl_op_tin(op).decode()


def op_parse(tin: str) -> int:
    out = ctypes.c_int32()
    st = N.load().spl_op_parse(tin.encode(), ctypes.byref(out))
    if st != N.OK:
        raise SpleafError(st, f"not one of the supported statements: {tin!r}")
    return out.value


def timing_enable(enable: bool = True, ctx: Optional[Context] = None) -> None:
    """Bracket every subsequent leaf kernel with HIP events on its stream."""
    ctx = ctx or Context.get()
    ctx.check(ctx.lib.spl_timing_enable(ctx.h, int(enable)), "spl_timing_enable")


def timing_read(op: int, ctx: Optional[Context] = None):
    """(launches, total_ms) of the leaf kernels of `op` recorded so far."""
    ctx = ctx or Context.get()
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    ctx.check(ctx.lib.spl_timing_read(ctx.h, op, ctypes.byref(n), ctypes.byref(ms)),
              "spl_timing_read")
    return n.value, ms.value


def probe(kind: int, buf: torch.Tensor, row_bytes: int = 128, count: int = 0,
          blocks: int = 4096, ctx: Optional[Context] = None) -> torch.Tensor:
    """Memory-system probe (kind 0: stream-read `buf`; kind 1: `count`
    random `row_bytes` reads from table `buf`, 4-byte lanes; kind 2: the
    same with 16-byte lanes).  Returns the per-workgroup partial sums
    (device)."""
    ctx, stream = _ctx_stream(buf, ctx)
    out = torch.empty(blocks, dtype=torch.float64, device=buf.device)
    nbytes = buf.numel() * buf.element_size()
    ctx.check(ctx.lib.spl_probe(ctx.h, kind, buf.data_ptr(), nbytes, row_bytes, count,
                                out.data_ptr(), blocks, stream), "spl_probe")
    return out


def _sched_ptr(sched):
    return ctypes.byref(sched) if sched else None


def spttv(B: CSF, c: torch.Tensor, A: Optional[torch.Tensor] = None, sched=None,
          ctx: Optional[Context] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A(i,j) = B(i,j,k) * c(k): returns the values of A, one per fiber of B
    (for CSF, A's pos/crd are B's pos1/crd1; for DDC, A is dense I x J,
    flattened row-major)."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    if A is None:
        A = torch.empty(B.nfibers, dtype=B.vals.dtype, device=B.vals.device)
    s = B.struct()
    ws, nb = _workspace(N.OP_SPTTV, B, 1, sched, ctx, B.vals.device, ws)
    ctx.check(ctx.lib.spl_spttv(ctx.h, ctypes.byref(s), ctypes.byref(_dense(c)),
                                ctypes.byref(_dense(A)), _sched_ptr(sched), _ptr(ws), nb,
                                stream), "spl_spttv")
    return A


def mttkrp(B: CSF, C: torch.Tensor, D: torch.Tensor, A: Optional[torch.Tensor] = None,
           sched=None, ctx: Optional[Context] = None,
           ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A(i,l) = B(i,j,k) * C(j,l) * D(k,l); FP32 output."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    if A is None:
        A = torch.empty(B.shape[0], C.shape[1], dtype=torch.float32, device=C.device)
    s = B.struct()
    ws, nb = _workspace(N.OP_MTTKRP, B, C.shape[1], sched, ctx, B.vals.device, ws)
    ctx.check(ctx.lib.spl_mttkrp(ctx.h, ctypes.byref(s), ctypes.byref(_dense(C)),
                                 ctypes.byref(_dense(D)), ctypes.byref(_dense(A)),
                                 _sched_ptr(sched), _ptr(ws), nb, stream), "spl_mttkrp")
    return A


def inner(B, C, out: Optional[torch.Tensor] = None, ctx: Optional[Context] = None,
          ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """a = sum of B * C over the shared pattern; a one-element float64 tensor."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=B.vals.device)
    sb, sc = B.struct(), C.struct()
    if ws is None and isinstance(C, DDC):
        # a Dense middle level of C is written out in the workspace as well
        nbytes = (workspace_query(N.OP_INNER, B, 1, None, ctx) +
                  workspace_query(N.OP_INNER, C, 1, None, ctx))
        ws = torch.empty(nbytes, dtype=torch.uint8, device=B.vals.device)
    ws, nb = _workspace(N.OP_INNER, B, 1, None, ctx, B.vals.device, ws)
    ctx.check(ctx.lib.spl_inner(ctx.h, ctypes.byref(sb), ctypes.byref(sc), out.data_ptr(),
                                None, _ptr(ws), nb, stream), "spl_inner")
    return out


def sddmm(B: CSR, C: torch.Tensor, D: torch.Tensor, A: Optional[torch.Tensor] = None,
          sched=None, ctx: Optional[Context] = None,
          ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A(i,j) = B(i,j) * C(i,k) * D(j,k) on B's pattern: returns A's values."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    if A is None:
        A = torch.empty(B.crd.numel(), dtype=B.vals.dtype, device=B.vals.device)
    s = B.struct()
    ws, nb = _workspace(N.OP_SDDMM, B, C.shape[1], sched, ctx, B.vals.device, ws)
    ctx.check(ctx.lib.spl_sddmm(ctx.h, ctypes.byref(s), ctypes.byref(_dense(C)),
                                ctypes.byref(_dense(D)), ctypes.byref(_dense(A)),
                                _sched_ptr(sched), _ptr(ws), nb, stream), "spl_sddmm")
    return A


def spadd3(B: CSR, C: CSR, D: CSR, sched=None, ctx: Optional[Context] = None) -> CSR:
    """A = B + C + D, assembled in two phases (the symbolic phase reads the
    output size back to the host to allocate A)."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    dev = B.vals.device
    n = B.shape[0]
    sb, sc, sd = B.struct(), C.struct(), D.struct()
    apos = torch.empty(n + 1, dtype=torch.int32, device=dev)
    ws, nb = _workspace(N.OP_SPADD3, B, 1, None, ctx, dev)
    nnz = ctypes.c_int64()
    ctx.check(ctx.lib.spl_spadd3_symbolic(ctx.h, ctypes.byref(sb), ctypes.byref(sc),
                                          ctypes.byref(sd), apos.data_ptr(), ctypes.byref(nnz),
                                          _sched_ptr(sched), _ptr(ws), nb, stream),
              "spl_spadd3_symbolic")
    acrd = torch.empty(nnz.value, dtype=torch.int32, device=dev)
    avals = torch.empty(nnz.value, dtype=B.vals.dtype, device=dev)
    ctx.check(ctx.lib.spl_spadd3_numeric(ctx.h, ctypes.byref(sb), ctypes.byref(sc),
                                         ctypes.byref(sd), apos.data_ptr(), _ptr(acrd),
                                         _ptr(avals), _sched_ptr(sched), stream),
              "spl_spadd3_numeric")
    return CSR(apos, acrd, avals, B.shape)


# ---------------------------------------------------------- transposition

def transpose(B: CSR, ctx: Optional[Context] = None) -> CSR:
    """The CSR of B^T (spl_transpose)."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    dev = B.vals.device
    n, m = B.shape
    nnz = B.crd.numel()
    s = B.struct()
    nb = ctypes.c_size_t()
    ctx.check(ctx.lib.spl_transpose_workspace_query(ctx.h, ctypes.byref(s), ctypes.byref(nb)),
              "spl_transpose_workspace_query")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    tpos = torch.empty(m + 1, dtype=torch.int32, device=dev)
    tcrd = torch.empty(nnz, dtype=torch.int32, device=dev)
    tvals = torch.empty(nnz, dtype=B.vals.dtype, device=dev)
    ctx.check(ctx.lib.spl_transpose(ctx.h, ctypes.byref(s), tpos.data_ptr(), _ptr(tcrd),
                                    _ptr(tvals), ws.data_ptr(), nb.value, stream), "spl_transpose")
    return CSR(tpos, tcrd, tvals, (m, n))


@dataclass
class CSC:
    """CSC matrix n x m: pos int32[m+1] over columns, crd int32[nnz] row
    coordinates (increasing within a column), vals[nnz] -- the
    (Dense, Compressed) format over the dimension order (j, i), i.e. the CSR
    arrays of the transpose."""
    pos: torch.Tensor
    crd: torch.Tensor
    vals: torch.Tensor
    shape: tuple

    def as_transposed_csr(self) -> CSR:
        """The same arrays read as the CSR of the m x n transpose."""
        return CSR(self.pos, self.crd, self.vals, (self.shape[1], self.shape[0]))

    def to_csr(self, ctx: Optional[Context] = None) -> CSR:
        """This matrix in CSR, by the library's transposition."""
        return transpose(self.as_transposed_csr(), ctx)


# -------------------------------------------- general index-notation leaves

class _TinCall:
    """Marshals one index-notation call: operands by name (CSR/CSF/DDC or a
    dense torch vector/matrix), the output binding, and the structs that must
    outlive the call."""

    def __init__(self, stmt: str, operands: dict, out_name: str, out):
        self.stmt = stmt.encode()
        self.keep = []
        arr = (N.SplTinOperand * max(1, len(operands)))()
        for k, (name, t) in enumerate(operands.items()):
            arr[k] = self._bind(name, t)
        self.ops, self.nops = arr, len(operands)
        self.out = self._bind(out_name, out)

    def _bind(self, name, t):
        op = N.SplTinOperand()
        op.name = name.encode()
        self.keep.append(op.name)
        if isinstance(t, (CSR, CSF, DDC)):
            s = t.struct()
            self.keep.append(s)
            op.sparse = ctypes.pointer(s)
        else:
            d = _dense(t)
            self.keep.append(d)
            op.dense = ctypes.pointer(d)
        return op


def _lhs_name(stmt: str) -> str:
    head = stmt.split("=", 1)[0]
    return head.split("(", 1)[0].strip()


def tin_source(stmt: str, out, ctx: Optional[Context] = None, **operands) -> str:
    """The HIP source the library generates for `stmt` with these operand
    formats (nothing is compiled or run; no GPU needed without `ctx`)."""
    lib = N.load()
    h = ctx.h if ctx else None
    call = _TinCall(stmt, operands, _lhs_name(stmt), out)
    n = ctypes.c_size_t()

    def check(st):
        if st != N.OK:
            detail = lib.spl_last_error(h).decode() if h else ""
            raise SpleafError(st, f"spl_tin_source: {detail}")

    check(lib.spl_tin_source(h, call.stmt, call.nops, call.ops, ctypes.byref(call.out), None, 0,
                             ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    check(lib.spl_tin_source(h, call.stmt, call.nops, call.ops, ctypes.byref(call.out), buf,
                             n.value + 1, ctypes.byref(n)))
    return buf.value.decode()


def tin(stmt: str, out=None, shape=None, ctx: Optional[Context] = None, **operands):
    """Evaluate an index-notation statement with a generated leaf.

    out: a dense torch tensor (every entry written), or None with `shape`
    given for a CSR output (assembled in two phases and returned), or None
    with a scalar left side (returns a float64 tensor of one entry).
    Operands are passed by the names the statement uses."""
    first = next(iter(operands.values()))
    vals = first.vals if isinstance(first, (CSR, CSF, DDC)) else first
    ctx, stream = _ctx_stream(vals, ctx)
    dev = vals.device
    name = _lhs_name(stmt)
    lhs = stmt.split("=", 1)[0]
    scalar = "(" not in lhs or lhs[lhs.index("(") + 1:].strip().startswith(")")
    if out is None and scalar:
        out = torch.empty(1, dtype=torch.float64, device=dev)
    if out is not None:
        call = _TinCall(stmt, operands, name, out)
        nb = ctypes.c_size_t()
        ctx.check(ctx.lib.spl_tin_workspace_query(ctx.h, call.stmt, call.nops, call.ops,
                                                  ctypes.byref(call.out), ctypes.byref(nb)),
                  "spl_tin_workspace_query")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=dev) if nb.value else None
        ctx.check(ctx.lib.spl_tin_eval(ctx.h, call.stmt, call.nops, call.ops,
                                       ctypes.byref(call.out), _ptr(ws), nb.value, stream),
                  "spl_tin_eval")
        return out
    if shape is None:
        raise ValueError("a sparse output needs its shape")
    n = shape[0]
    apos = torch.empty(n + 1, dtype=torch.int32, device=dev)
    empty = torch.empty(0, dtype=torch.int32, device=dev)
    A = CSR(apos, empty, torch.empty(0, dtype=vals.dtype, device=dev), tuple(shape))
    call = _TinCall(stmt, operands, name, A)
    nb = ctypes.c_size_t()
    ctx.check(ctx.lib.spl_tin_workspace_query(ctx.h, call.stmt, call.nops, call.ops,
                                              ctypes.byref(call.out), ctypes.byref(nb)),
              "spl_tin_workspace_query")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev) if nb.value else None
    nnz = ctypes.c_int64()
    ctx.check(ctx.lib.spl_tin_symbolic(ctx.h, call.stmt, call.nops, call.ops,
                                       ctypes.byref(call.out), apos.data_ptr(), ctypes.byref(nnz),
                                       _ptr(ws), nb.value, stream), "spl_tin_symbolic")
    A = CSR(apos, torch.empty(nnz.value, dtype=torch.int32, device=dev),
            torch.empty(nnz.value, dtype=vals.dtype, device=dev), tuple(shape))
    call = _TinCall(stmt, operands, name, A)
    ctx.check(ctx.lib.spl_tin_eval(ctx.h, call.stmt, call.nops, call.ops, ctypes.byref(call.out),
                                   _ptr(ws), nb.value, stream), "spl_tin_eval")
    return A


# ------------------------------------------------------- schedule selection

_SCHED_FIELDS = ("lanes_per_row", "tile", "items_per_lane", "col_tile", "variant")


def schedule_dict(s: N.SplSchedule) -> dict:
    """A spl_schedule as the keyword dict `schedule()` takes (zero fields
    left out)."""
    d = {"kind": _KIND_NAME.get(s.kind, int(s.kind))}
    for f in _SCHED_FIELDS:
        v = int(getattr(s, f))
        if v:
            d[f] = v
    return d


def _sched_array(cands):
    arr = (N.SplSchedule * len(cands))()
    for i, c in enumerate(cands):
        arr[i] = c if isinstance(c, N.SplSchedule) else schedule(**c)
    return arr


def _selector_op(op) -> int:
    return {"spmv": N.OP_SPMV, "spmm": N.OP_SPMM}.get(op, op)


def autotune(op, B: CSR, X: torch.Tensor, Y: torch.Tensor, candidates=None, reps: int = 3,
             ctx: Optional[Context] = None):
    """spl_autotune: time every candidate (dicts or spl_schedule; None for
    the library's list) on these operands; returns (best dict, [ms, ...])."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    op = _selector_op(op)
    s = B.struct()
    arr = _sched_array(candidates) if candidates is not None else None
    n = len(arr) if arr is not None else 0
    times = (ctypes.c_float * max(n, 16))()
    best = N.SplSchedule()
    ctx.check(ctx.lib.spl_autotune(ctx.h, op, ctypes.byref(s), ctypes.byref(_dense(X)),
                                   ctypes.byref(_dense(Y)), arr, n, reps, ctypes.byref(best),
                                   times, stream), "spl_autotune")
    count = n if n else (12 if op == N.OP_SPMV else 9)
    return schedule_dict(best), [float(times[i]) for i in range(count)]


def mlp_load(op, candidates, params, norm=None, ctx: Optional[Context] = None) -> None:
    """spl_mlp_load: install a selector (host parameters and 7 means + 7
    inverse standard deviations) in the context."""
    ctx = ctx or Context.get()
    arr = _sched_array(candidates)
    P = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    nrm = None if norm is None else np.ascontiguousarray(np.asarray(norm, dtype=np.float32))
    ctx.check(ctx.lib.spl_mlp_load(ctx.h, _selector_op(op), len(arr), arr,
                                   P.ctypes.data, None if nrm is None else nrm.ctypes.data),
              "spl_mlp_load")


def mlp_save(op, ctx: Optional[Context] = None):
    """spl_mlp_save: (candidate dicts, parameters, standardization) of the
    installed selector, as numpy arrays."""
    ctx = ctx or Context.get()
    op = _selector_op(op)
    K = ctypes.c_int()
    ctx.check(ctx.lib.spl_mlp_save(ctx.h, op, ctypes.byref(K), 0, None, None, None),
              "spl_mlp_save")
    arr = (N.SplSchedule * K.value)()
    P = np.empty(int(ctx.lib.spl_mlp_param_count(K.value)), dtype=np.float32)
    nrm = np.empty(14, dtype=np.float32)
    ctx.check(ctx.lib.spl_mlp_save(ctx.h, op, ctypes.byref(K), K.value, arr, P.ctypes.data,
                                   nrm.ctypes.data), "spl_mlp_save")
    return [schedule_dict(a) for a in arr], P, nrm


def mlp_predict(op, B: CSR, ctx: Optional[Context] = None) -> dict:
    """spl_mlp_predict: the installed selector's schedule for B."""
    ctx, stream = _ctx_stream(B.vals, ctx)
    out = N.SplSchedule()
    s = B.struct()
    ctx.check(ctx.lib.spl_mlp_predict(ctx.h, _selector_op(op), ctypes.byref(s),
                                      ctypes.byref(out), stream), "spl_mlp_predict")
    return schedule_dict(out)


def mlp_train_step(op, X: torch.Tensor, T: torch.Tensor, lr: float,
                   loss: Optional[torch.Tensor] = None, ctx: Optional[Context] = None):
    """spl_mlp_train_step on a batch (X: batch x 7 raw features, T: batch x K,
    float32 on the GPU); returns the device loss tensor (loss before the
    step)."""
    ctx, stream = _ctx_stream(X, ctx)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    ctx.check(ctx.lib.spl_mlp_train_step(ctx.h, _selector_op(op), X.data_ptr(), T.data_ptr(),
                                         X.shape[0], lr, loss.data_ptr(), stream),
              "spl_mlp_train_step")
    return loss
