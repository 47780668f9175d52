"""CPU correctness oracle for the sparse leaf kernels (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library: the C loops in
``oracle.c`` are compiled into ``liboracle.so`` with gcc, and this module only
converts numpy arrays and calls them.  ``brute`` holds a second, independent
evaluation by dense ``numpy.einsum`` for tiny inputs, and ``mlp`` a float64
reference of the schedule-selection network.

Every value array is widened to float64 before the call (exact for FP32 and
BF16 inputs); the C side accumulates in long double and returns float64
results together with S, the per-entry sum of |term|.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


_OMP_SRC = os.path.join(_HERE, "cpu_baseline.c")
_OMP_LIB = os.path.join(_HERE, "libcpu_baseline.so")


def _gcc(src, lib, force, extra=()):
    stale = (not os.path.exists(lib)
             or os.path.getmtime(lib) < os.path.getmtime(src))
    if force or stale:
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-Wall", *extra, "-shared", "-fPIC",
                               "-o", tmp, src])
        os.replace(tmp, lib)
    return lib


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so and the OpenMP CPU baseline into
    libcpu_baseline.so with gcc (-O2, no fast-math)."""
    _gcc(_OMP_SRC, _OMP_LIB, force, ("-fopenmp",))
    return _gcc(_SRC, _LIB, force)


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_spadd3_symbolic.restype = _i64
        lib.orc_inner.restype = ctypes.c_double
        lib.orc_inner3.restype = ctypes.c_double
        for name in ("orc_row_split", "orc_nnz_split", "orc_merge_split",
                     "orc_csf_split", "orc_rows_finished_at"):
            getattr(lib, name).restype = _i64
        _lib = lib
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _f64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(_f64p)


def _rows(rows):
    if rows is None:
        return None, None, 0
    r = np.ascontiguousarray(rows, dtype=np.int64)
    return r, r.ctypes.data_as(_i64p), len(r)


def _out(shape):
    a = np.zeros(shape, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


def spmv(pos, crd, vals, c, rows=None):
    """a(i) = B(i,j) c(j) for CSR B; returns (a, S)."""
    lib = _load()
    n = len(pos) - 1
    pos, pp = _i32(pos)
    crd, cp = _i32(crd)
    vals, vp = _f64(vals)
    c, xp = _f64(c)
    r, rp, nr = _rows(rows)
    cnt = nr if rows is not None else n
    a, ap = _out(cnt)
    S, sp = _out(cnt)
    lib.orc_spmv(_i64(n), pp, cp, vp, xp, rp, _i64(nr), ap, sp)
    return a, S


def spmm(pos, crd, vals, C, rows=None):
    """A(i,j) = B(i,k) C(k,j); C is m x N row-major. Returns (A, S)."""
    lib = _load()
    n = len(pos) - 1
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    N = C.shape[1]
    pos, pp = _i32(pos)
    crd, cp = _i32(crd)
    vals, vp = _f64(vals)
    Cc, Cp = _f64(C)
    r, rp, nr = _rows(rows)
    cnt = nr if rows is not None else n
    A, Ap = _out((cnt, N))
    S, Sp = _out((cnt, N))
    lib.orc_spmm(_i64(n), _i64(N), pp, cp, vp, Cp, _i64(N), rp, _i64(nr),
                 Ap, _i64(N), Sp)
    return A, S


def spadd3(B, C, D):
    """A = B + C + D for CSR triples (pos, crd, vals), two-phase.

    Returns (pos, crd, vals, S, nnz_from_symbolic_phase)."""
    lib = _load()
    n = len(B[0]) - 1
    Bp, Bpp = _i32(B[0]); Bc, Bcp = _i32(B[1]); Bv, Bvp = _f64(B[2])
    Cp, Cpp = _i32(C[0]); Cc, Ccp = _i32(C[1]); Cv, Cvp = _f64(C[2])
    Dp, Dpp = _i32(D[0]); Dc, Dcp = _i32(D[1]); Dv, Dvp = _f64(D[2])
    Apos = np.zeros(n + 1, dtype=np.int32)
    nnz = lib.orc_spadd3_symbolic(_i64(n), Bpp, Bcp, Cpp, Ccp, Dpp, Dcp,
                                  Apos.ctypes.data_as(_i32p))
    Acrd = np.zeros(max(nnz, 1), dtype=np.int32)
    Av, Avp = _out(max(nnz, 1))
    AS, ASp = _out(max(nnz, 1))
    lib.orc_spadd3_numeric(_i64(n), Bpp, Bcp, Bvp, Cpp, Ccp, Cvp, Dpp, Dcp,
                           Dvp, Apos.ctypes.data_as(_i32p),
                           Acrd.ctypes.data_as(_i32p), Avp, ASp)
    return Apos, Acrd[:nnz], Av[:nnz], AS[:nnz], int(nnz)


def sddmm(pos, crd, Bvals, C, D):
    """A(i,j) = B(i,j) C(i,k) D(j,k) on B's pattern; returns (A_vals, S)."""
    lib = _load()
    n = len(pos) - 1
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    D = np.ascontiguousarray(np.asarray(D, dtype=np.float64))
    K = C.shape[1]
    pos, pp = _i32(pos)
    crd, cp = _i32(crd)
    Bv, Bvp = _f64(Bvals)
    Cc, Cp = _f64(C)
    Dd, Dp = _f64(D)
    nnz = len(crd)
    A, Ap = _out(nnz)
    S, Sp = _out(nnz)
    lib.orc_sddmm(_i64(n), _i64(K), pp, cp, Bvp, Cp, _i64(K), Dp, _i64(K),
                  Ap, Sp)
    return A, S


def spttv(pos1, pos2, crd2, vals, c):
    """A(i,j) = B(i,j,k) c(k) on B's (i,j) pattern; returns (A_vals[F], S)."""
    lib = _load()
    I = len(pos1) - 1
    F = int(pos1[-1])
    p1, p1p = _i32(pos1)
    p2, p2p = _i32(pos2)
    c2, c2p = _i32(crd2)
    v, vp = _f64(vals)
    cc, ccp = _f64(c)
    A, Ap = _out(F)
    S, Sp = _out(F)
    lib.orc_spttv(_i64(I), p1p, p2p, c2p, vp, ccp, Ap, Sp)
    return A, S


def mttkrp(pos1, crd1, pos2, crd2, vals, C, D, rows=None):
    """A(i,l) = B(i,j,k) C(j,l) D(k,l); returns (A, S)."""
    lib = _load()
    I = len(pos1) - 1
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    D = np.ascontiguousarray(np.asarray(D, dtype=np.float64))
    R = C.shape[1]
    p1, p1p = _i32(pos1)
    c1, c1p = _i32(crd1)
    p2, p2p = _i32(pos2)
    c2, c2p = _i32(crd2)
    v, vp = _f64(vals)
    Cc, Cp = _f64(C)
    Dd, Dp = _f64(D)
    r, rp, nr = _rows(rows)
    cnt = nr if rows is not None else I
    A, Ap = _out((cnt, R))
    S, Sp = _out((cnt, R))
    lib.orc_mttkrp(_i64(I), _i64(R), p1p, c1p, p2p, c2p, vp, Cp, _i64(R),
                   Dp, _i64(R), rp, _i64(nr), Ap, _i64(R), Sp)
    return A, S


def inner(B, C):
    """a = sum over coordinates stored in both B and C of B*C.

    B and C are (pos1, crd1, pos2, crd2, vals) for order 3, or
    (pos, crd, None, None, vals) for order 2.  Returns (a, S)."""
    lib = _load()
    I = len(B[0]) - 1
    keep = []

    def idx(a):
        if a is None:
            return None
        arr, p = _i32(a)
        keep.append(arr)
        return p

    bv, bvp = _f64(B[4])
    cv, cvp = _f64(C[4])
    S = ctypes.c_double(0.0)
    a = lib.orc_inner(_i64(I), idx(B[0]), idx(B[1]), idx(B[2]), idx(B[3]), bvp,
                      idx(C[0]), idx(C[1]), idx(C[2]), idx(C[3]), cvp,
                      ctypes.byref(S))
    return float(a), float(S.value)


def coord_partition(pos, crd, bounds):
    """Value-range partition of a CSR's columns: out int32[ncolors+1, n]."""
    lib = _load()
    n = len(pos) - 1
    p, pp = _i32(pos)
    c, cp = _i32(crd)
    b, bp = _i32(bounds)
    ncolors = len(bounds) - 1
    out = np.zeros((ncolors + 1) * max(n, 0), dtype=np.int32)
    lib.orc_coord_partition(_i64(n), pp, cp, _i64(ncolors), bp,
                            out.ctypes.data_as(_i32p))
    return out.reshape(ncolors + 1, n)


def spmv_window(begin, end, crd, vals, c):
    """a(i) over positions [begin[i], end[i]); returns (a, S)."""
    lib = _load()
    n = len(begin)
    b, bp = _i32(begin)
    e, ep = _i32(end)
    k, kp = _i32(crd)
    v, vp = _f64(vals)
    x, xp = _f64(c)
    a, ap = _out(n)
    S, Sp = _out(n)
    lib.orc_spmv_window(_i64(n), bp, ep, kp, vp, xp, ap, Sp)
    return a, S


def spttv_ddc(I, J, pos2, crd2, vals, c):
    """SpTTV of a (Dense, Dense, Compressed) tensor: A(i,j) for every (i,j),
    returned flattened row-major (I*J values) with S."""
    lib = _load()
    p2, p2p = _i32(pos2)
    c2, c2p = _i32(crd2)
    v, vp = _f64(vals)
    cc, ccp = _f64(c)
    A, Ap = _out(I * J)
    S, Sp = _out(I * J)
    lib.orc_spttv_ddc(_i64(I), _i64(J), p2p, c2p, vp, ccp, Ap, Sp)
    return A, S


def mttkrp_ddc(I, J, pos2, crd2, vals, C, D, rows=None):
    """SpMTTKRP of a (Dense, Dense, Compressed) tensor; returns (A, S)."""
    lib = _load()
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    D = np.ascontiguousarray(np.asarray(D, dtype=np.float64))
    R = C.shape[1]
    p2, p2p = _i32(pos2)
    c2, c2p = _i32(crd2)
    v, vp = _f64(vals)
    Cc, Cp = _f64(C)
    Dd, Dp = _f64(D)
    r, rp, nr = _rows(rows)
    cnt = nr if rows is not None else I
    A, Ap = _out((cnt, R))
    S, Sp = _out((cnt, R))
    lib.orc_mttkrp_ddc(_i64(I), _i64(J), _i64(R), p2p, c2p, vp, Cp, _i64(R), Dp, _i64(R),
                       rp, _i64(nr), Ap, _i64(R), Sp)
    return A, S


def inner3(I, J, B, C):
    """Inner product of two I x J x K tensors given as (pos1, crd1, pos2, crd2,
    vals); pos1 = crd1 = None marks a Dense middle level.  Returns (a, S)."""
    lib = _load()
    keep = []

    def idx(a):
        if a is None:
            return None
        arr, p = _i32(a)
        keep.append(arr)
        return p

    bv, bvp = _f64(B[4])
    cv, cvp = _f64(C[4])
    S = ctypes.c_double(0.0)
    a = lib.orc_inner3(_i64(I), _i64(J), idx(B[0]), idx(B[1]), idx(B[2]), idx(B[3]), bvp,
                       idx(C[0]), idx(C[1]), idx(C[2]), idx(C[3]), cvp, ctypes.byref(S))
    return float(a), float(S.value)


def _split(fn, n, pos, size, extra_len=0):
    pos_a, pp = _i32(pos)
    nnz = int(pos_a[-1]) if len(pos_a) else 0
    cap = (n + nnz) // max(size, 1) + 3
    tr = np.zeros(cap, dtype=np.int32)
    tp = np.zeros(cap, dtype=np.int32)
    nt = fn(_i64(n), pp, _i64(size), tr.ctypes.data_as(_i32p),
            tp.ctypes.data_as(_i32p))
    return tr[:nt + 1].copy(), tp[:nt + 1].copy()


def row_split(pos, R):
    """Universe partition of rows in blocks of R, image to positions."""
    return _split(_load().orc_row_split, len(pos) - 1, pos, R)


def nnz_split(pos, T):
    """Non-zero partition in blocks of T positions, rows by preimage."""
    return _split(_load().orc_nnz_split, len(pos) - 1, pos, T)


def merge_split(pos, Dm):
    """Equal split of the merged (row ends, positions) sequence."""
    return _split(_load().orc_merge_split, len(pos) - 1, pos, Dm)


def csf_split(pos1, pos2, T):
    """Fiber-aligned non-zero split of a CSF tensor; returns
    (tile_slice, tile_fiber, tile_pos)."""
    lib = _load()
    I = len(pos1) - 1
    p1, p1p = _i32(pos1)
    p2, p2p = _i32(pos2)
    nnz = int(p2[-1])
    cap = nnz // max(T, 1) + 3
    ts = np.zeros(cap, dtype=np.int32)
    tf = np.zeros(cap, dtype=np.int32)
    tp = np.zeros(cap, dtype=np.int32)
    nt = lib.orc_csf_split(_i64(I), p1p, p2p, _i64(T), ts.ctypes.data_as(_i32p),
                           tf.ctypes.data_as(_i32p), tp.ctypes.data_as(_i32p))
    return ts[:nt + 1].copy(), tf[:nt + 1].copy(), tp[:nt + 1].copy()


def rows_finished_at(pos, p):
    """Number of rows whose segment ends at or before position p."""
    pos_a, pp = _i32(pos)
    return int(_load().orc_rows_finished_at(_i64(len(pos_a) - 1), pp, _i64(p)))


def transpose(pos, crd, vals, shape):
    """CSR arrays (pos, crd, vals) of B^T for B = CSR (pos, crd, vals) of
    shape (n, m); a CSC matrix passed as the CSR of its transpose comes back
    as its CSR."""
    lib = _load()
    n, m = shape
    pos, pp = _i32(pos)
    crd, cp = _i32(crd)
    vals, vp = _f64(vals)
    nnz = int(pos[n]) if n else 0
    tpos = np.zeros(m + 1, dtype=np.int32)
    tcrd = np.zeros(max(nnz, 1), dtype=np.int32)
    tvals = np.zeros(max(nnz, 1), dtype=np.float64)
    lib.orc_transpose(_i64(n), _i64(m), pp, cp, vp, tpos.ctypes.data_as(_i32p),
                      tcrd.ctypes.data_as(_i32p), tvals.ctypes.data_as(_f64p))
    return tpos, tcrd[:nnz], tvals[:nnz]


def csc_spmv(cpos, crd, vals, x, n):
    """y(i) = A(i,j) x(j) for A n x m stored as CSC (cpos over columns,
    row coordinates in crd); returns (y, S)."""
    lib = _load()
    m = len(cpos) - 1
    cpos, pp = _i32(cpos)
    crd, cp = _i32(crd)
    vals, vp = _f64(vals)
    x, xp = _f64(x)
    y, yp = _out(n)
    S, sp = _out(n)
    lib.orc_csc_spmv(_i64(n), _i64(m), pp, cp, vp, xp, yp, sp)
    return y, S


def error_statement(got, ref, S):
    """Error of a result against an oracle reference, entrywise normwise:
    max and median of |got - ref| / S over the entries with S > 0 (S the
    oracle's sum of |term|), and ||got - ref||_2 / ||ref||_2 (0 when both are
    0).  Only statistics of the comparison: no arithmetic of the method."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    S = np.asarray(S, dtype=np.float64).ravel()
    err = np.abs(got - ref)
    pos = S > 0
    rel = err[pos] / S[pos] if pos.any() else np.zeros(1)
    nref = float(np.linalg.norm(ref))
    nerr = float(np.linalg.norm(got - ref))
    return {"max_err_over_S": float(rel.max()), "median_err_over_S": float(np.median(rel)),
            "rel_l2": nerr / nref if nref > 0 else (0.0 if nerr == 0 else float("inf")),
            "entries": int(got.size)}


class CpuBaseline:
    """The benchmark's CPU comparison: double-precision SpMV and SpMM loops
    with OpenMP over rows (dynamic, 1,024 rows a chunk), not the oracle."""

    def __init__(self):
        build()
        lib = ctypes.CDLL(_OMP_LIB)
        lib.cpu_threads.restype = ctypes.c_int
        self.lib = lib

    def threads(self) -> int:
        return int(self.lib.cpu_threads())

    def spmv(self, pos, crd, vals, c, a):
        n = len(pos) - 1
        self.lib.cpu_spmv(_i64(n), pos.ctypes.data_as(_i32p), crd.ctypes.data_as(_i32p),
                          vals.ctypes.data_as(_f64p), c.ctypes.data_as(_f64p),
                          a.ctypes.data_as(_f64p))

    def spmm(self, pos, crd, vals, C, A):
        n = len(pos) - 1
        self.lib.cpu_spmm(_i64(n), _i64(C.shape[1]), pos.ctypes.data_as(_i32p),
                          crd.ctypes.data_as(_i32p), vals.ctypes.data_as(_f64p),
                          C.ctypes.data_as(_f64p), _i64(C.shape[1]), A.ctypes.data_as(_f64p),
                          _i64(A.shape[1]))
