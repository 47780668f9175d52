"""The five synthetic workloads, and scaled-down versions of them for tests.

1. CSR 4096 x 4096, exactly 10 distinct uniform columns per row; FP64 values
   and vector uniform[-1, 1].
2. CSR 2,000,000 x 2,000,000, Pareto(alpha = 2) row degrees with mean 16
   (32,000,000 nonzeros) and cap 50,000; distinct uniform columns; values
   uniform[-1, 1] in FP64 and FP32; a dense 2,000,000 x 32 row-major operand
   with the same distribution.
3. Three CSR 1,000,000 x 1,000,000 with Poisson(8) degrees; a Bernoulli(0.3)
   set of rows shares its degree and columns across the three matrices
   (drawn from a key that depends on the row only); FP32 values uniform
   [-1, 1]; SDDMM factors 1,000,000 x 128 uniform[-1, 1] in FP32 and BF16.
4. CSF 200,000^3 with exactly 1e8 nonzeros; Pareto(alpha = 1.8) slice sizes
   with mean 500 and cap 1,000,000; distinct uniform (j, k) pairs per slice;
   values uniform[0, 1]; c uniform[0, 1]; rank-32 factors N(0, 1); a second
   value array on the same pattern for the inner product.
5. Schedule-selection corpus (see ``corpus``).
6. The paper's weak-scaling SpMV matrix at one GPU's share: banded CSR
   20,000,000 x 20,000,000 whose row i holds columns max(0, i - 17) ..
   min(n - 1, i + 17) (35 per interior row, 699,999,694 nonzeros, about
   700 million); FP64 values and vector uniform[-1, 1].
7. (Dense, Dense, Compressed) 3-tensor shaped like the paper's "patents"
   tensor (a short dense first mode, two long modes): 46 x 239,172 x 239,172
   with exactly 1e8 nonzeros split evenly over the 46 slices, distinct
   uniform (j, k) pairs per slice (so every one of the 11,001,912 fibers
   holds about 9 values); values and c uniform[0, 1]; rank-32 factors
   N(0, 1).  Synthetic: only the shape and format stand in for the dataset.

``scale`` shrinks every size by the same factor for tests (the degree cap
shrinks with it), keeping the structure: power-law rows, ragged tails, and
rows longer than a tile.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gen


def _dev(device):
    return torch.device(device)


def config1(device="cpu", n=4096, deg=10, kind="sym"):
    dev = _dev(device)
    d = np.full(n, deg, dtype=np.int64)
    pos, crd = gen.csr_from_degrees(d, n, gen.key_for(1, 0), dev)
    vals = gen.values(gen.key_for(1, 1), int(crd.numel()), dev, kind)
    x = gen.values(gen.key_for(1, 2), n, dev, kind)
    return dict(n=n, m=n, pos=pos, crd=crd, vals=vals, x=x)


def config2(device="cpu", scale=1.0, N=32, kind="sym", with_dense=True):
    """Power-law CSR (and the dense SpMM operand); values in float64."""
    dev = _dev(device)
    n = max(1, int(round(2_000_000 * scale)))
    target = 16 * n
    cap = max(2, min(n, int(round(50_000 * math.sqrt(scale)))))
    deg = gen.powerlaw_degrees(n, 2.0, target, cap, gen.key_for(2, 0))
    pos, crd = gen.csr_from_degrees(deg, n, gen.key_for(2, 1), dev)
    nnz = int(crd.numel())
    out = dict(n=n, m=n, pos=pos, crd=crd,
               vals=gen.values(gen.key_for(2, 2), nnz, dev, kind),
               x=gen.values(gen.key_for(2, 3), n, dev, kind), cap=cap)
    if with_dense:
        out["B"] = gen.values(gen.key_for(2, 4), n * N, dev, kind).reshape(n, N)
    return out


def config3(device="cpu", scale=1.0, K=128, kind="sym", with_dense=True,
            overlap=0.3):
    """Three CSR with shared rows for SpAdd3, plus SDDMM factors."""
    dev = _dev(device)
    n = max(1, int(round(1_000_000 * scale)))
    shared = gen.uniform_np(gen.key_for(3, 0), n) < overlap
    deg_shared = gen.poisson_degrees(n, 8.0, gen.key_for(3, 1))
    deg_shared = np.minimum(deg_shared, n)
    sh_idx = np.nonzero(shared)[0]
    # shared rows: one pattern, drawn once from a key independent of the matrix
    sp, sc = gen.csr_from_degrees(deg_shared[sh_idx], n, gen.key_for(3, 2), dev)
    mats = []
    for mid in range(3):
        d_own = np.minimum(gen.poisson_degrees(n, 8.0, gen.key_for(3, 10 + mid)), n)
        d = np.where(shared, deg_shared, d_own)
        own_idx = np.nonzero(~shared)[0]
        op, oc = gen.csr_from_degrees(d[own_idx], n, gen.key_for(3, 20 + mid), dev)
        deg_t = torch.as_tensor(d, device=dev)
        pos = torch.zeros(n + 1, dtype=torch.int64, device=dev)
        torch.cumsum(deg_t, 0, out=pos[1:])
        nnz = int(pos[-1])
        crd = torch.empty(nnz, dtype=torch.int32, device=dev)
        for idx, ppos, pcrd in ((sh_idx, sp, sc), (own_idx, op, oc)):
            if len(idx) == 0:
                continue
            idx_t = torch.as_tensor(idx, device=dev)
            cnt = (ppos[1:] - ppos[:-1]).to(torch.int64)
            src_row = torch.repeat_interleave(torch.arange(len(idx), device=dev), cnt)
            within = torch.arange(pcrd.numel(), device=dev) - ppos[:-1].to(torch.int64)[src_row]
            dst = pos[idx_t][src_row] + within
            crd[dst] = pcrd
        vals = gen.values(gen.key_for(3, 30 + mid), nnz, dev, kind)
        mats.append(dict(pos=pos.to(torch.int32), crd=crd, vals=vals))
    out = dict(n=n, m=n, B=mats[0], C=mats[1], D=mats[2], shared=shared)
    if with_dense:
        out["Cd"] = gen.values(gen.key_for(3, 40), n * K, dev, kind).reshape(n, K)
        out["Dd"] = gen.values(gen.key_for(3, 41), n * K, dev, kind).reshape(n, K)
    return out


def config4(device="cpu", scale=1.0, R=32, kind_vals="unit", with_dense=True):
    """Power-law CSF tensor, TTV vector, MTTKRP factors, second values."""
    dev = _dev(device)
    I = max(1, int(round(200_000 * scale)))
    J = K = I
    target = int(round(1e8 * scale))
    cap = max(2, min(J * K, int(round(1_000_000 * scale))))
    sizes = gen.powerlaw_degrees(I, 1.8, target, cap, gen.key_for(4, 0))
    pos1, crd1, pos2, crd2 = gen.csf_from_slice_sizes(sizes, J, K,
                                                      gen.key_for(4, 1), dev)
    nnz = int(crd2.numel())
    out = dict(I=I, J=J, K=K, pos1=pos1, crd1=crd1, pos2=pos2, crd2=crd2,
               vals=gen.values(gen.key_for(4, 2), nnz, dev, kind_vals),
               vals2=gen.values(gen.key_for(4, 3), nnz, dev, kind_vals),
               c=gen.values(gen.key_for(4, 4), K, dev, "unit"))
    if with_dense:
        out["C"] = gen.values(gen.key_for(4, 5), J * R, dev, "normal").reshape(J, R)
        out["D"] = gen.values(gen.key_for(4, 6), K * R, dev, "normal").reshape(K, R)
    return out


def banded(device="cpu", n=20_000_000, half_width=17, kind="sym", pos_dtype=torch.int32):
    """Banded CSR (config 6): row i holds columns max(0, i - w) ..
    min(n - 1, i + w); values and the vector in float64.  pos_dtype
    torch.int64 keeps positions past 2^31 (n above about 61 million)."""
    dev = _dev(device)
    w = int(half_width)
    i = torch.arange(n, dtype=torch.int64, device=dev)
    lo = torch.clamp(i - w, min=0)
    deg = torch.clamp(i + w, max=n - 1) - lo + 1
    del i
    pos = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    pos[1:] = torch.cumsum(deg, 0)
    nnz = int(pos[-1].item())
    row = torch.repeat_interleave(torch.arange(n, dtype=torch.int64, device=dev), deg)
    crd = (lo[row] + torch.arange(nnz, dtype=torch.int64, device=dev) - pos[:-1][row])
    crd = crd.to(torch.int32)
    del row, lo, deg
    vals = gen.values(gen.key_for(6, 1), nnz, dev, kind)
    x = gen.values(gen.key_for(6, 2), n, dev, kind)
    return dict(n=n, m=n, pos=pos.to(pos_dtype), crd=crd, vals=vals, x=x, half_width=w)


def csf_int64(device="cpu", I=1 << 20, fibers=64, run=33, R=32, chunk=1 << 27):
    """A CSF tensor past 2^31 positions with a regular pattern (int64 pos1 and
    pos2): every slice holds `fibers` fibers at j = t * (J / fibers) + i mod
    (J / fibers), every fiber `run` positions at k = s * 32 + (7 f) mod 32, so
    nnz = I * fibers * run (2,214,592,512 by default); values uniform[0, 1)
    in FP32, factors N(0, 1) in FP32, all drawn in chunks."""
    dev = _dev(device)
    J = 65536
    K = 32 * run
    F = I * fibers
    nnz = F * run
    pos1 = torch.arange(I + 1, dtype=torch.int64, device=dev) * fibers
    f = torch.arange(F, dtype=torch.int64, device=dev)
    crd1 = ((f % fibers) * (J // fibers) + (f // fibers) % (J // fibers)).to(torch.int32)
    pos2 = torch.arange(F + 1, dtype=torch.int64, device=dev) * run
    del f
    crd2 = torch.empty(nnz, dtype=torch.int32, device=dev)
    vals = torch.empty(nnz, dtype=torch.float32, device=dev)
    key = gen.key_for(9, 1)
    for a in range(0, nnz, chunk):
        p = torch.arange(a, min(nnz, a + chunk), dtype=torch.int64, device=dev)
        crd2[a:a + p.numel()] = ((p % run) * 32 + ((p // run) * 7) % 32).to(torch.int32)
        vals[a:a + p.numel()] = gen.uniform(key, p).to(torch.float32)
        del p
    C = gen.values(gen.key_for(9, 2), J * R, dev, "normal").reshape(J, R).to(torch.float32)
    D = gen.values(gen.key_for(9, 3), K * R, dev, "normal").reshape(K, R).to(torch.float32)
    return dict(I=I, J=J, K=K, pos1=pos1, crd1=crd1, pos2=pos2, crd2=crd2, vals=vals, C=C, D=D)


def ddc(device="cpu", scale=1.0, R=32, I=46, with_dense=True):
    """Config 7: (Dense, Dense, Compressed) tensor; pos2 indexes all I*J
    fibers (fiber f = i*J + j)."""
    dev = _dev(device)
    J = K = max(1, int(round(239_172 * scale)))
    target = int(round(1e8 * scale))
    sizes = np.full(I, target // I, dtype=np.int64)
    sizes[: target % I] += 1
    pos1, crd1, pos2c, crd2 = gen.csf_from_slice_sizes(sizes, J, K, gen.key_for(7, 1), dev)
    # scatter the compressed fibers' lengths to their (i, j) slots
    fib_i = torch.repeat_interleave(torch.arange(I, device=dev), pos1[1:] - pos1[:-1])
    slot = fib_i.to(torch.int64) * J + crd1.to(torch.int64)
    count = torch.zeros(I * J, dtype=torch.int64, device=dev)
    count[slot] = (pos2c[1:] - pos2c[:-1]).to(torch.int64)
    pos2 = torch.zeros(I * J + 1, dtype=torch.int64, device=dev)
    pos2[1:] = torch.cumsum(count, 0)
    del count, slot, fib_i, pos2c
    nnz = int(crd2.numel())
    out = dict(I=I, J=J, K=K, pos2=pos2.to(torch.int32), crd2=crd2,
               vals=gen.values(gen.key_for(7, 2), nnz, dev, "unit"),
               vals2=gen.values(gen.key_for(7, 3), nnz, dev, "unit"),
               c=gen.values(gen.key_for(7, 4), K, dev, "unit"))
    if with_dense:
        out["C"] = gen.values(gen.key_for(7, 5), J * R, dev, "normal").reshape(J, R)
        out["D"] = gen.values(gen.key_for(7, 6), K * R, dev, "normal").reshape(K, R)
    return out
