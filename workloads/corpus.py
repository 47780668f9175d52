"""Seeded corpus of CSR matrices for schedule selection.

Matrix ``i`` of the corpus is fully determined by ``i``: its family is
``i % 4`` (uniform, power law, banded, block diagonal), its row count is
log-uniform on [1e4, 4e6] (square matrices), its nonzero count log-uniform on
[1e5, 1e8] clipped to a mean degree in [1, 2000] and to what the family can
hold, and the family parameter (power-law exponent in [1.5, 3.0], band
half-width log-uniform on [8, 512], block size log-uniform on [16, 256]) is
drawn from the same stream.  Degrees of the uniform, banded and block
families are a normal approximation of Poisson(mean), capped at half of the
row's column window so that distinct columns are cheap to draw; power-law
degrees are Pareto with an exact total.  Columns are uniform inside each
row's window (all columns, the band, or the block).  Values are uniform
[-1, 1] in FP32.  Everything after the per-matrix parameters runs on
`device` with torch.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gen

FAMILIES = ("uniform", "powerlaw", "banded", "block")
CORPUS_SEED = gen.BASE_SEED + 5000


def _logu(u, lo, hi):
    return math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))


def spec(i: int, max_nnz: float = 1e8) -> dict:
    u = gen.uniform_np(gen.stream_key(CORPUS_SEED, i), 6)
    fam = FAMILIES[i % 4]
    n = int(round(_logu(u[0], 1e4, 4e6)))
    nnz = int(round(_logu(u[1], 1e5, max_nnz)))
    s = dict(id=i, family=fam, n=n)
    if fam == "powerlaw":
        s["alpha"] = 1.5 + 1.5 * float(u[2])
        s["cap"] = min(n, 50_000)
        cap_total = n * s["cap"]
    elif fam == "banded":
        s["band"] = int(round(_logu(u[2], 8, 512)))
        cap_total = n * s["band"]           # half of the 2b+1 window
    elif fam == "block":
        s["block"] = int(round(_logu(u[2], 16, 256)))
        cap_total = n * (s["block"] // 2)
    else:
        cap_total = n * (n // 2)
    nnz = max(n, min(nnz, 2000 * n, cap_total))
    s["nnz_target"] = int(nnz)
    return s


def _windows(s, dev):
    n = s["n"]
    i = torch.arange(n, dtype=torch.int64, device=dev)
    if s["family"] == "banded":
        b = s["band"]
        lo = torch.clamp(i - b, min=0)
        hi = torch.clamp(i + b + 1, max=n)
    elif s["family"] == "block":
        bs = s["block"]
        lo = (i // bs) * bs
        hi = torch.clamp(lo + bs, max=n)
    else:
        lo = torch.zeros(n, dtype=torch.int64, device=dev)
        hi = torch.full((n,), n, dtype=torch.int64, device=dev)
    return lo, hi - lo


def _powerlaw_degrees(n, alpha, target, cap, key, dev):
    u = gen.uniform(key, torch.arange(n, dtype=torch.int64, device=dev))
    x = (1.0 - u) ** (-1.0 / (alpha - 1.0))

    def degs(scale):
        return torch.clamp(torch.ceil(scale * x), 1, cap)

    lo, hi = 0.0, 1.0
    while float(degs(hi).sum()) <= target and hi < 1e18:
        hi *= 2.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if float(degs(mid).sum()) <= target:
            lo = mid
        else:
            hi = mid
    d = degs(lo).to(torch.int64)
    deficit = int(target - int(d.sum()))
    if deficit > 0:
        room = torch.nonzero(d < cap).flatten()[:deficit]
        d[room] += 1
    return d


def generate(i: int, device="cuda", max_nnz: float = 1e8):
    """(spec, pos int32, crd int32, vals float32) of corpus matrix i."""
    s = spec(i, max_nnz)
    dev = torch.device(device)
    n = s["n"]
    key = gen.stream_key(CORPUS_SEED, 1000 + i)
    lo, width = _windows(s, dev)
    if s["family"] == "powerlaw":
        deg = _powerlaw_degrees(n, s["alpha"], s["nnz_target"], s["cap"], key, dev)
    else:
        mean = s["nnz_target"] / n
        idx = torch.arange(n, dtype=torch.int64, device=dev)
        u1 = gen.uniform(gen.stream_key(key, 1), idx)
        u2 = gen.uniform(gen.stream_key(key, 2), idx)
        z = torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos(2.0 * math.pi * u2)
        deg = torch.round(mean + math.sqrt(mean) * z).to(torch.int64)
        deg = torch.clamp(deg, min=0)
    deg = torch.minimum(deg, torch.clamp(width // 2, min=1))
    deg = torch.minimum(deg, width)
    keys = gen.distinct_keys(deg, lo, width, n, gen.stream_key(key, 3))
    crd = (keys % n).to(torch.int32)
    pos = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    torch.cumsum(deg, 0, out=pos[1:])
    nnz = int(pos[-1])
    vals = (2.0 * gen.uniform(gen.stream_key(key, 4),
                              torch.arange(nnz, dtype=torch.int64, device=dev)) - 1.0)
    s["nnz"] = nnz
    return s, pos.to(torch.int32), crd, vals.to(torch.float32)


def split(count: int, held_out: int):
    """Train / held-out ids, stratified by family with a seeded shuffle."""
    rs = np.random.RandomState(CORPUS_SEED % (2 ** 31))
    train, test = [], []
    per = held_out // 4
    for f in range(4):
        ids = np.arange(f, count, 4)
        ids = ids[rs.permutation(len(ids))]
        test.extend(ids[:per].tolist())
        train.extend(ids[per:].tolist())
    return sorted(train), sorted(test)
