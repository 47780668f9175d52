"""GPU parity of the generated index-notation leaves (spl_tin_*) against the
general oracle (oracle/tin.py): CSR output patterns bit for bit, values
within 1e-12 S (FP64) or 1e-5 S (FP32) on sampled rows of the outermost index
(600 rows: three workgroups and a ragged tail), small-integer values bit for
bit, every dense output entry written, and repeated calls identical."""
import numpy as np
import pytest
import torch

from oracle import tin as T
from tests.gpu_util import RTOL, assert_close, host64, need_gpu
from tests.tin_cases import CASES, EXTENTS, SMALL, make

pytestmark = pytest.mark.gpu


def _spl():
    need_gpu()
    import paper_2207_13901_amd as spl
    return spl


def _rows(n, three_level):
    rs = np.random.RandomState(n)
    k = 12 if three_level else 40
    return np.unique(np.concatenate([[0, 1, 2, 3, 7, 255, 256, n - 1],
                                     rs.choice(n, k, replace=False)]))


def _run(spl, stmt, kind, lib, shape, dtype, dev):
    if kind == "csr":
        return spl.tin(stmt, shape=shape, **lib)
    if kind == "scalar":
        return spl.tin(stmt, **lib)
    out = torch.full(shape, float("nan"), dtype=dtype, device=dev)
    return spl.tin(stmt, out, **lib)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]} [{c[1]}]" for c in CASES])
def test_tin_matches_oracle(case, dtype):
    spl = _spl()
    stmt, kind, recipe = case
    dev = torch.device("cuda", 0)
    ext = SMALL if kind == "scalar" else EXTENTS
    lib, ref, shape = make(stmt, recipe, dtype, seed=11, extents=ext, device=dev)
    print(f"tin: {stmt} [{kind}] {dtype}", flush=True)
    got = _run(spl, stmt, kind, lib, shape, dtype, dev)
    torch.cuda.synchronize()
    rtol = RTOL[dtype]
    if kind == "scalar":
        want, S = T.evaluate(stmt, ref)
        assert_close(host64(got), np.reshape(want, 1), np.reshape(S, 1), rtol, stmt)
        return
    three = any(v == "csf" or v == "ddc" for v in recipe.values())
    rows = _rows(shape[0], three)
    want, S = T.evaluate(stmt, ref, out_shape=shape, rows=rows)
    if kind == "csr":
        pos, crd = T.pattern(stmt, ref, shape)
        assert np.array_equal(got.pos.cpu().numpy(), pos), stmt
        assert np.array_equal(got.crd.cpu().numpy(), crd), stmt
        vals = host64(got.vals)
        for r, i in enumerate(rows):
            cols = crd[pos[i]:pos[i + 1]]
            assert_close(vals[pos[i]:pos[i + 1]], want[r, cols], S[r, cols], rtol,
                         f"{stmt} row {i}")
        return
    host = host64(got)
    assert not np.isnan(host).any(), "every output entry is written"
    assert_close(host[rows], want, S, rtol, stmt)


@pytest.mark.parametrize("case", [c for c in CASES if c[1] != "scalar"],
                         ids=[f"{c[0]} [{c[1]}]" for c in CASES if c[1] != "scalar"])
def test_tin_integer_values_bit_exact_and_deterministic(case):
    spl = _spl()
    stmt, kind, recipe = case
    dev = torch.device("cuda", 0)
    lib, ref, shape = make(stmt, recipe, torch.float64, seed=12, kind="int", extents=EXTENTS,
                           device=dev)
    got = _run(spl, stmt, kind, lib, shape, torch.float64, dev)
    again = _run(spl, stmt, kind, lib, shape, torch.float64, dev)
    three = any(v == "csf" or v == "ddc" for v in recipe.values())
    rows = _rows(shape[0], three)
    want, _ = T.evaluate(stmt, ref, out_shape=shape, rows=rows)
    if kind == "csr":
        assert torch.equal(got.vals, again.vals) and torch.equal(got.crd, again.crd)
        pos = got.pos.cpu().numpy()
        crd = got.crd.cpu().numpy()
        vals = host64(got.vals)
        for r, i in enumerate(rows):
            assert np.array_equal(vals[pos[i]:pos[i + 1]], want[r, crd[pos[i]:pos[i + 1]]]), i
        return
    assert torch.equal(got, again)
    assert np.array_equal(host64(got)[rows], want), stmt


def test_tin_scalar_on_a_larger_pattern():
    # the co-iterated 2-D inner product over 600 rows (three workgroups of
    # partials and the fixed-order final sum)
    spl = _spl()
    stmt = "a = B(i,j) * C(i,j)"
    dev = torch.device("cuda", 0)
    lib, ref, _ = make(stmt, dict(B="csr", C="csr"), torch.float64, seed=13, extents=EXTENTS,
                       device=dev)
    got = spl.tin(stmt, **lib)
    want, S = T.evaluate(stmt, ref)
    assert_close(host64(got), np.reshape(want, 1), np.reshape(S, 1), 1e-12, stmt)
