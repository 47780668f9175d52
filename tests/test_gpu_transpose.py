"""GPU parity of the transposition (spl_transpose) and of CSC operands read
through it: B^T's pos, crd and vals bit for bit against the oracle's
transposition (one, two and three radix passes; empty matrices, empty rows
and columns, one row or column; the 2,000,000-row power-law matrix at full
size), repeated calls identical, and SpMV of a CSC matrix against the
oracle's plain CSC definition."""
import numpy as np
import pytest
import torch

import oracle
from tests import tiny
from tests.gpu_util import assert_close, host64, need_gpu
from workloads import configs

pytestmark = pytest.mark.gpu


def _spl():
    need_gpu()
    import paper_2207_13901_amd as spl
    return spl


def _dev():
    return torch.device("cuda", 0)


def _csr(spl, pos, crd, vals, shape, dtype=torch.float64):
    d = _dev()
    return spl.CSR(torch.as_tensor(np.asarray(pos, np.int32), device=d),
                   torch.as_tensor(np.asarray(crd, np.int32), device=d),
                   torch.as_tensor(np.asarray(vals, np.float64)).to(dtype).to(d), shape)


def _check(spl, B, what):
    T = spl.transpose(B)
    n, m = B.shape
    rp, rc, rv = oracle.transpose(B.pos.cpu().numpy(), B.crd.cpu().numpy(), host64(B.vals),
                                  (n, m))
    assert T.shape == (m, n)
    assert np.array_equal(T.pos.cpu().numpy(), rp), what
    assert np.array_equal(T.crd.cpu().numpy(), rc), what
    assert np.array_equal(host64(T.vals), rv), what
    assert T.vals.dtype == B.vals.dtype
    return T


@pytest.mark.parametrize("n,m,density", [(50, 7, 0.4), (300, 256, 0.05), (300, 257, 0.05),
                                         (40, 3000, 0.01), (5000, 600, 0.01), (1, 900, 0.3),
                                         (700, 1, 0.5)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_transpose_bit_exact(n, m, density, dtype):
    spl = _spl()
    rs = np.random.RandomState(n + m)
    pos, crd, vals = tiny.csr(rs, n, m, density, empty_rows={0} if n > 1 else (),
                              full_rows={n // 2} if m < 1000 else ())
    print(f"transpose n={n} m={m} nnz={len(crd)} {dtype}", flush=True)
    _check(spl, _csr(spl, pos, crd, vals, (n, m), dtype), (n, m, dtype))


def test_transpose_empty_and_deterministic():
    spl = _spl()
    B = _csr(spl, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0), (5, 9))
    T = _check(spl, B, "empty")
    assert not T.pos.any()
    c = configs.config2(scale=0.01, N=1)
    B = spl.CSR(c["pos"].to(_dev()), c["crd"].to(_dev()), c["vals"].to(_dev()),
                (c["n"], c["n"]))
    T1 = _check(spl, B, "power law scale 0.01")
    T2 = spl.transpose(B)
    assert torch.equal(T1.pos, T2.pos) and torch.equal(T1.crd, T2.crd)
    assert torch.equal(T1.vals, T2.vals)


def test_transpose_full_size_power_law():
    # 2,000,000 columns: three radix passes over 32e6 entries
    spl = _spl()
    c = configs.config2(device="cuda", with_dense=False)
    n = c["n"]
    B = spl.CSR(c["pos"], c["crd"], c["vals"].to(torch.float32), (n, n))
    _check(spl, B, "power law full size")


@pytest.mark.parametrize("kind", ["float", "int"])
def test_csc_spmv(kind):
    # A (n x m) given by columns: its CSR comes from the transposition, then
    # the CSR SpMV leaf; against the oracle's plain CSC definition
    spl = _spl()
    rs = np.random.RandomState(21)
    n, m = 3000, 1700
    cpos, crd, vals = tiny.csr(rs, m, n, 0.004, empty_rows={5}, kind=kind)
    x = rs.randint(-4, 5, m).astype(np.float64) if kind == "int" else rs.uniform(-1, 1, m)
    A = spl.CSC(*(torch.as_tensor(a, device=_dev()) for a in (cpos, crd, vals)), (n, m))
    xd = torch.as_tensor(x, device=_dev())
    ref, S = oracle.csc_spmv(cpos, crd, vals, x, n)
    for sched in (dict(kind="default"), dict(kind="row", lanes_per_row=4),
                  dict(kind="nnz", tile=512)):
        y = spl.spmv(A.to_csr(), xd, sched=spl.schedule(**sched))
        if kind == "int":
            assert np.array_equal(host64(y), ref), sched
        else:
            assert_close(host64(y), ref, S, 1e-12, f"csc spmv {sched}")
