"""spl_spmv_noalloc: the SpMV entry point that allocates nothing (tile bounds
and carries in the library's static device scratch) gives the same bits as
spl_spmv on the same operands and schedule, and stays within the oracle's
tolerance; two calls in a row, the second on a smaller matrix, so the
second call runs over scratch the first one left behind.  Sizes beyond the
scratch and the selection schedules are refused before anything runs."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import RTOL, assert_close, host64, need_gpu
from workloads import configs

pytestmark = pytest.mark.gpu

SCHEDULES = [dict(kind="default"), dict(kind="merge", tile=8192, items_per_lane=4),
             dict(kind="nnz", tile=1000), dict(kind="row", lanes_per_row=8),
             dict(kind="merge", variant=1)]


def _spl():
    need_gpu()
    import paper_2207_13901_amd as spl
    return spl


def _matrix(spl, scale, dtype):
    c = configs.config2(scale=scale, N=1)
    n = c["n"]
    d = torch.device("cuda", 0)
    B = spl.CSR(c["pos"].to(d), c["crd"].to(d), c["vals"].to(dtype).to(d), (n, n))
    return B, c["x"].to(dtype).to(d), c


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("sched", SCHEDULES, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
def test_noalloc_matches_spmv_twice(dtype, sched):
    spl = _spl()
    s = spl.schedule(**sched)
    # larger matrix first, then a smaller one over the scratch it left
    for scale in (0.01, 0.003):
        B, x, c = _matrix(spl, scale, dtype)
        print(f"noalloc: dtype={dtype} sched={sched} n={B.shape[0]} nnz={B.crd.numel()}",
              flush=True)
        want = spl.spmv(B, x, sched=s)
        got = torch.full_like(want, float("nan"))
        spl.spmv_noalloc(B, x, got, sched=s)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (scale, sched)
        ref, S = oracle.spmv(c["pos"].numpy(), c["crd"].numpy(), host64(B.vals), host64(x))
        assert_close(host64(got), ref, S, RTOL[dtype], f"noalloc {dtype} {sched} scale {scale}")


def test_noalloc_refuses_oversize_and_selection():
    spl = _spl()
    B, x, _ = _matrix(spl, 0.04, torch.float64)  # 1.28e6 nonzeros
    y = torch.zeros(B.shape[0], dtype=torch.float64, device=x.device)
    # one position per tile: 16 bytes of bounds and carries per position,
    # beyond the 16 MiB scratch
    with pytest.raises(spl.SpleafError) as e:
        spl.spmv_noalloc(B, x, y, sched=spl.schedule(kind="nnz", tile=1))
    assert "static scratch holds" in str(e.value)
    with pytest.raises(spl.SpleafError):
        spl.spmv_noalloc(B, x, y, sched=spl.schedule(kind="autotune"))
    torch.cuda.synchronize()
    assert not y.any()  # nothing ran
    # the same context still works afterwards
    want = spl.spmv(B, x)
    got = torch.empty_like(want)
    spl.spmv_noalloc(B, x, got)
    assert torch.equal(got, want)
