"""Counter-based generators for sparse matrices and CSF tensors.

Every random number is SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
applied to a 64-bit counter: draw ``idx`` of stream ``(seed, stream)`` is
``mix(key(seed, stream) + (idx + 1) * 0x9E3779B97F4A7C15)``.  A draw depends
only on its key and index, never on the device, thread count or batch size, so
the same call on CPU or GPU yields the same integers.  Per-row degree vectors
(at most a few million entries) are built on the host in float64; the per-
nonzero work (columns, values, sorting, de-duplication) runs with torch on the
requested device.

Uniform doubles are ``(h >> 11) * 2**-53``; uniform[-1, 1] is ``2u - 1``;
FP32 and BF16 values are the round-to-nearest-even narrowing of the FP64 (and
then FP32) stream; normal(0, 1) is Box-Muller.

Layouts: CSR is (pos int32[n+1], crd int32[nnz]) with strictly increasing
coordinates inside each row; CSF is (pos1, crd1, pos2, crd2).  Dense operands
are row-major.
"""
from __future__ import annotations

import math

import numpy as np
import torch

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
BASE_SEED = 220713901


def _s64(v: int) -> int:
    """Python int (mod 2**64) -> the int64 with the same bits."""
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _mix_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * _M1) & MASK64
    z = ((z ^ (z >> 27)) * _M2) & MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """64-bit key of stream ``stream`` under ``seed``."""
    return _mix_int(_mix_int(seed * GOLDEN + 0x632BE59BD9B4E019) + stream)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of an int64 tensor holding uint64 bits."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _s64(_M1)
    z = (z ^ _srl(z, 27)) * _s64(_M2)
    return z ^ _srl(z, 31)


def hash64(key: int, idx: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output for counters ``idx`` (int64 tensor) of ``key``."""
    z = (idx + 1) * _s64(GOLDEN) + _s64(key)
    return _mix(z)


def uniform(key: int, idx: torch.Tensor) -> torch.Tensor:
    """float64 uniform in [0, 1) with 53 random bits."""
    return _srl(hash64(key, idx), 11).to(torch.float64) * (2.0 ** -53)


def uniform_np(key: int, count: int) -> np.ndarray:
    """Host copy of ``uniform(key, arange(count))``."""
    return uniform(key, torch.arange(count, dtype=torch.int64)).numpy()


def key_for(config: int, array_id: int) -> int:
    return stream_key(BASE_SEED + 1000 * config + array_id, array_id)


# --------------------------------------------------------------------------
# degree vectors (host, float64)
# --------------------------------------------------------------------------

def powerlaw_degrees(n: int, alpha: float, target: int, cap: int, key: int,
                     dmin: int = 1) -> np.ndarray:
    """Pareto row degrees with an exact total.

    x_i = (1 - u_i) ** (-1 / (alpha - 1)) has density proportional to
    x ** -alpha on [1, inf).  d_i = min(cap, ceil(s * x_i)) with the largest
    s (found by bisection) such that sum(d) <= target; the remaining deficit
    is added one at a time to rows below the cap, in index order.  Rows keep
    their sampled order, so heavy rows are scattered.
    """
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    u = uniform_np(key, n)
    x = (1.0 - u) ** (-1.0 / (alpha - 1.0))

    def total(s):
        return int(np.minimum(cap, np.maximum(dmin, np.ceil(s * x))).sum())

    lo, hi = 0.0, 1.0
    while total(hi) <= target and hi < 1e18:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) <= target:
            lo = mid
        else:
            hi = mid
    d = np.minimum(cap, np.maximum(dmin, np.ceil(lo * x))).astype(np.int64)
    deficit = target - int(d.sum())
    while deficit > 0:
        room = np.nonzero(d < cap)[0]
        if len(room) == 0:
            break
        take = room[:deficit]
        d[take] += 1
        deficit -= len(take)
    return d


_POISSON_CACHE: dict = {}


def poisson_degrees(n: int, lam: float, key: int, kmax: int = 200) -> np.ndarray:
    """Poisson(lam) degrees by inverse CDF of one uniform per row."""
    if lam not in _POISSON_CACHE:
        k = np.arange(kmax + 1)
        logp = -lam + k * math.log(lam) - np.array([math.lgamma(v + 1) for v in k])
        _POISSON_CACHE[lam] = np.cumsum(np.exp(logp))
    cdf = _POISSON_CACHE[lam]
    u = uniform_np(key, n)
    return np.minimum(np.searchsorted(cdf, u, side="right"), kmax).astype(np.int64)


# --------------------------------------------------------------------------
# distinct sorted coordinates per row
# --------------------------------------------------------------------------

def _pos_from_deg(deg: torch.Tensor) -> torch.Tensor:
    pos = torch.zeros(deg.numel() + 1, dtype=torch.int64, device=deg.device)
    torch.cumsum(deg, 0, out=pos[1:])
    return pos


def distinct_keys(deg: torch.Tensor, lo: torch.Tensor, width: torch.Tensor,
                  stride: int, key: int) -> torch.Tensor:
    """Sorted int64 keys ``row * stride + col`` with deg[row] distinct cols.

    Columns of row r are uniform on [lo[r], lo[r] + width[r]).  Duplicates
    are dropped and redrawn from fresh counters (round r uses its own key)
    until every row holds exactly deg[r] distinct columns; requires
    deg <= width.
    """
    dev = deg.device
    n = deg.numel()
    if bool((deg > width).any()):
        raise ValueError("row degree exceeds the width of its column window")
    rows = torch.repeat_interleave(torch.arange(n, device=dev), deg)
    nnz = rows.numel()
    u = uniform(stream_key(key, 0), torch.arange(nnz, dtype=torch.int64, device=dev))
    cols = lo[rows] + torch.floor(u * width[rows].to(torch.float64)).to(torch.int64)
    keys = torch.unique(rows * stride + cols)  # sorted, duplicates removed
    rnd = 1
    while keys.numel() < nnz:
        have = torch.bincount(torch.div(keys, stride, rounding_mode="floor"),
                              minlength=n)
        need = deg - have
        nrows = torch.repeat_interleave(torch.arange(n, device=dev), need)
        u = uniform(stream_key(key, rnd),
                    torch.arange(nrows.numel(), dtype=torch.int64, device=dev))
        ncols = lo[nrows] + torch.floor(
            u * width[nrows].to(torch.float64)).to(torch.int64)
        keys = torch.unique(torch.cat([keys, nrows * stride + ncols]))
        rnd += 1
        if rnd > 10000:
            raise RuntimeError("column de-duplication did not converge")
    return keys


def csr_from_degrees(deg, m: int, key: int, device="cpu", lo=None, width=None):
    """CSR (pos int32, crd int32) with the given row degrees."""
    deg_t = torch.as_tensor(np.asarray(deg, dtype=np.int64), device=device)
    n = deg_t.numel()
    if lo is None:
        lo_t = torch.zeros(n, dtype=torch.int64, device=device)
        w_t = torch.full((n,), m, dtype=torch.int64, device=device)
    else:
        lo_t = torch.as_tensor(np.asarray(lo, dtype=np.int64), device=device)
        w_t = torch.as_tensor(np.asarray(width, dtype=np.int64), device=device)
    keys = distinct_keys(deg_t, lo_t, w_t, m, key)
    crd = (keys % m).to(torch.int32)
    pos = _pos_from_deg(deg_t).to(torch.int32)
    return pos, crd


def values(key: int, count: int, device="cpu", kind="sym") -> torch.Tensor:
    """float64 values: 'sym' uniform[-1,1], 'unit' uniform[0,1),
    'normal' N(0,1) (Box-Muller), 'int' integers in {-4..4}."""
    idx = torch.arange(count, dtype=torch.int64, device=device)
    if kind == "sym":
        return 2.0 * uniform(key, idx) - 1.0
    if kind == "unit":
        return uniform(key, idx)
    if kind == "normal":
        u1 = uniform(key, 2 * idx)
        u2 = uniform(key, 2 * idx + 1)
        return torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos(2.0 * math.pi * u2)
    if kind == "int":
        return torch.floor(uniform(key, idx) * 9.0) - 4.0
    raise ValueError(kind)


def narrow(v64: torch.Tensor, dtype: str) -> torch.Tensor:
    """Round-to-nearest-even narrowing: f64 -> f32 -> bf16."""
    if dtype == "f64":
        return v64
    v32 = v64.to(torch.float32)
    if dtype == "f32":
        return v32
    if dtype == "bf16":
        return v32.to(torch.bfloat16)
    raise ValueError(dtype)


# --------------------------------------------------------------------------
# CSF tensors
# --------------------------------------------------------------------------

def csf_from_slice_sizes(sizes, J: int, K: int, key: int, device="cpu"):
    """CSF (pos1, crd1, pos2, crd2) of an I x J x K tensor whose slice i
    stores sizes[i] distinct (j, k) pairs, uniform over J x K."""
    sz = torch.as_tensor(np.asarray(sizes, dtype=np.int64), device=device)
    I = sz.numel()
    JK = J * K
    zero = torch.zeros(I, dtype=torch.int64, device=device)
    width = torch.full((I,), JK, dtype=torch.int64, device=device)
    keys = distinct_keys(sz, zero, width, JK, key)
    i = torch.div(keys, JK, rounding_mode="floor")
    jk = keys - i * JK
    j = torch.div(jk, K, rounding_mode="floor")
    k = jk - j * K
    nnz = keys.numel()
    fiber_key = i * J + j
    if nnz:
        new_fiber = torch.ones(nnz, dtype=torch.bool, device=device)
        new_fiber[1:] = fiber_key[1:] != fiber_key[:-1]
        fstart = torch.nonzero(new_fiber).flatten()
    else:
        fstart = torch.zeros(0, dtype=torch.int64, device=device)
    F = fstart.numel()
    pos2 = torch.empty(F + 1, dtype=torch.int64, device=device)
    pos2[:F] = fstart
    pos2[F] = nnz
    crd1 = j[fstart]
    fslice = i[fstart]
    per_slice = torch.bincount(fslice, minlength=I)
    pos1 = _pos_from_deg(per_slice)
    return (pos1.to(torch.int32), crd1.to(torch.int32), pos2.to(torch.int32),
            k.to(torch.int32))
