"""GPU parity of SpMV, SpMM and the tile partition against the CPU oracle.

Every comparison runs through the C ABI (via the thin torch binding): tile
bounds are bit-exact integers; values satisfy |got - ref| <= rtol * S with
rtol 1e-12 (FP64) or 1e-5 (FP32, and BF16 inputs with FP32 accumulation,
against the oracle on the same BF16-rounded inputs); with small-integer
values every schedule is bit-identical to the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from tests import tiny
from tests.gpu_util import RTOL, assert_close, dev, host64, need_gpu
from workloads import configs

pytestmark = pytest.mark.gpu

SCHEDULES_SPMV = [
    dict(kind="row", lanes_per_row=1), dict(kind="row", lanes_per_row=4),
    dict(kind="row", lanes_per_row=64),
    dict(kind="nnz", tile=64, items_per_lane=4), dict(kind="nnz", tile=1000),
    dict(kind="nnz", tile=5000, items_per_lane=8),
    dict(kind="merge", tile=1024, items_per_lane=4), dict(kind="merge", tile=2048),
    dict(kind="merge", tile=777), dict(kind="default"),
    # several chunks per workgroup: the pipelined leaf's steady state
    dict(kind="merge", tile=8192, items_per_lane=4), dict(kind="merge", tile=6000, items_per_lane=8),
    # row-end search leaf: one chunk, several, ragged
    dict(kind="merge", variant=1), dict(kind="merge", tile=1024, items_per_lane=4, variant=1),
    dict(kind="merge", tile=9000, items_per_lane=8, variant=1),
    dict(kind="merge", tile=7777, items_per_lane=4, variant=1),
    # whole rows per lane (long rows by a wave): one chunk, several, ragged
    dict(kind="merge", variant=2), dict(kind="merge", tile=1024, items_per_lane=4, variant=2),
    dict(kind="merge", tile=9000, items_per_lane=8, variant=2),
    dict(kind="merge", tile=7777, items_per_lane=4, variant=2),
]
SCHEDULES_SPMM = [
    dict(kind="row", col_tile=32), dict(kind="row", col_tile=8),
    dict(kind="nnz", tile=100, col_tile=32, items_per_lane=8),
    dict(kind="nnz", tile=3000, col_tile=16, items_per_lane=16),
    dict(kind="merge", tile=128, col_tile=32, items_per_lane=16),
    dict(kind="merge", tile=2000, col_tile=64, items_per_lane=32),
    dict(kind="default"),
    # vector lanes (aligned operands) with 8 items and one chunk per tile,
    # 16 lanes per group; and the one-column-per-lane leaf forced
    dict(kind="merge", tile=64, col_tile=32, items_per_lane=8),
    dict(kind="merge", tile=4096, col_tile=64, items_per_lane=16),
    dict(kind="merge", tile=512, col_tile=32, items_per_lane=16, variant=1),
]


def _spl():
    need_gpu()
    import paper_2207_13901_amd as spl
    return spl


def _csr(spl, pos, crd, vals, shape, dtype):
    d = dev()
    return spl.CSR(torch.as_tensor(pos, dtype=torch.int32, device=d),
                   torch.as_tensor(crd, dtype=torch.int32, device=d),
                   torch.as_tensor(np.asarray(vals), dtype=torch.float64, device=d).to(dtype),
                   shape)


def _edge_cases():
    rs = np.random.RandomState(1)
    cases = {
        "all_empty": (np.zeros(9, np.int32), np.zeros(0, np.int32), np.zeros(0), (8, 5)),
        "one_by_one": (np.array([0, 1], np.int32), np.array([0], np.int32), np.array([0.5]), (1, 1)),
    }
    p, c, v = tiny.csr(rs, 40, 3000, 0.0, empty_rows={0, 1, 39}, full_rows={7})
    cases["long_row"] = (p, c, v, (40, 3000))
    p, c, v = tiny.csr(rs, 300, 200, 0.02, empty_rows=set(range(0, 300, 3)) | {299})
    cases["sparse_empty_tail"] = (p, c, v, (300, 200))
    p, c, v = tiny.csr(rs, 70, 70, 0.0, full_rows={3, 5, 69})
    cases["rows_65_plus"] = (p, c, v, (70, 70))
    return cases


@pytest.mark.parametrize("kind,size", [("row", 1), ("row", 7), ("nnz", 1), ("nnz", 13),
                                       ("nnz", 4096), ("merge", 1), ("merge", 10),
                                       ("merge", 2048)])
def test_tile_bounds_match_oracle(kind, size):
    spl = _spl()
    split = {"row": oracle.row_split, "nnz": oracle.nnz_split, "merge": oracle.merge_split}[kind]
    mats = list(_edge_cases().values())
    c2 = configs.config2(scale=0.002, with_dense=False)
    mats.append((c2["pos"].numpy(), c2["crd"].numpy(), c2["vals"].numpy(), (c2["n"], c2["n"])))
    for pos, crd, vals, shape in mats:
        B = _csr(spl, pos, crd, vals, shape, torch.float64)
        tr, tp = spl.tile_bounds(B, spl.schedule(kind, tile=size))
        rr, rp = split(pos, size)
        assert np.array_equal(tr.cpu().numpy(), rr)
        assert np.array_equal(tp.cpu().numpy(), rp)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_coord_partition_and_window_spmv(dtype):
    spl = _spl()
    cases = list(_edge_cases().values())
    c2 = configs.config2(scale=0.002, with_dense=False)
    cases.append((c2["pos"].numpy(), c2["crd"].numpy(), c2["vals"].numpy(), (c2["n"], c2["n"])))
    rs = np.random.RandomState(5)
    for pos, crd, vals, shape in cases:
        n, m = shape
        B = _csr(spl, pos, crd, vals, shape, dtype)
        x = torch.as_tensor(rs.uniform(-1, 1, m), device=dev()).to(dtype)
        for bounds in ([0, m], np.linspace(0, m, 9).astype(int).tolist(),
                       [-5, 0, m // 3, m // 3, m + 7], [m, m + 1]):
            bt = torch.tensor(bounds, dtype=torch.int32, device=dev())
            out = spl.coord_partition(B, bt)
            ref = oracle.coord_partition(pos, crd, np.array(bounds, dtype=np.int32))
            assert np.array_equal(out.cpu().numpy(), ref), (shape, bounds)
            for c in range(len(bounds) - 1):
                ra, S = oracle.spmv_window(ref[c], ref[c + 1], crd, host64(B.vals), host64(x))
                for sc in (None, dict(kind="row", lanes_per_row=1), dict(kind="row", lanes_per_row=8),
                           dict(kind="row", lanes_per_row=64),
                           dict(kind="merge", tile=1024, items_per_lane=4),
                           dict(kind="merge", tile=256 * 8 * 3, items_per_lane=8)):
                    a = spl.spmv_window(B, out[c], out[c + 1], x,
                                        sched=spl.schedule(**sc) if sc else None)
                    assert_close(host64(a), ra, S, RTOL[dtype], f"window {c} {bounds} {sc}")
                    # fixed reduction orders: a second call gives the same bits
                    a2 = spl.spmv_window(B, out[c], out[c + 1], x,
                                         sched=spl.schedule(**sc) if sc else None)
                    assert torch.equal(a, a2), (c, bounds, sc)
    B = _csr(spl, *cases[-1][:3], cases[-1][3], torch.float64)
    o = spl.coord_partition(B, torch.tensor([0, 10], dtype=torch.int32, device=dev()))
    for bad in (spl.schedule("nnz"), spl.schedule("merge", variant=1)):
        with pytest.raises(spl.SpleafError, match="ROW or MERGE"):
            spl.spmv_window(B, o[0], o[1],
                            torch.ones(B.shape[1], dtype=torch.float64, device=dev()), sched=bad)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spmv_int64_positions(dtype):
    # the same matrices with int64 pos: the merge split and the flag leaf
    # read 8-byte row ends and int64 tile positions
    spl = _spl()
    cases = list(_edge_cases().values())
    c2 = configs.config2(scale=0.002, with_dense=False)
    cases.append((c2["pos"].numpy(), c2["crd"].numpy(), c2["vals"].numpy(), (c2["n"], c2["n"])))
    scheds = [None, dict(kind="merge"), dict(kind="merge", tile=1024, items_per_lane=4),
              dict(kind="merge", tile=8192, items_per_lane=4),
              dict(kind="merge", tile=6000, items_per_lane=8)]
    rs = np.random.RandomState(8)
    for pos, crd, vals, shape in cases:
        B = _csr(spl, pos, crd, vals, shape, dtype)
        B64 = spl.CSR(B.pos.to(torch.int64), B.crd, B.vals, shape)
        x = torch.as_tensor(rs.uniform(-1, 1, shape[1]), device=dev()).to(dtype)
        ref, S = oracle.spmv(pos, crd, host64(B.vals), host64(x))
        for sc in scheds:
            y = spl.spmv(B64, x, sched=spl.schedule(**sc) if sc else None)
            assert_close(host64(y), ref, S, RTOL[dtype], f"int64 pos {shape} {sc}")
    x = torch.ones(B64.shape[1], dtype=dtype, device=dev())
    for bad in (dict(kind="row"), dict(kind="nnz"), dict(kind="merge", variant=1),
                dict(kind="merge", variant=2), dict(kind="learned")):
        with pytest.raises(spl.SpleafError, match="UNSUPPORTED"):
            spl.spmv(B64, x, sched=spl.schedule(**bad))
    # SpMM takes int64 positions with vector lanes only: 5 columns give none
    with pytest.raises(spl.SpleafError, match="UNSUPPORTED"):
        spl.spmm(B64, torch.ones(B64.shape[1], 5, dtype=dtype, device=dev()))


def test_merge_bounds_above_the_sweep_limit():
    # more than 8,000,000 rows: the merge split is found by a search per tile
    # (below, by a sweep over the rows); both must equal the oracle's split
    spl = _spl()
    rs = np.random.RandomState(17)
    for n in (8_000_000, 9_000_001):
        deg = (rs.random_sample(n) < 0.1).astype(np.int64) * rs.randint(1, 4, n)
        deg[n // 2] = 50_000  # one row across many tiles
        pos = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(deg, out=pos[1:])
        nnz = int(pos[-1])
        crd = np.zeros(nnz, dtype=np.int32)
        B = _csr(spl, pos.astype(np.int32), crd, np.ones(nnz), (n, 1), torch.float64)
        for size in (7, 2048):
            tr, tp = spl.tile_bounds(B, spl.schedule("merge", tile=size))
            rr, rp = oracle.merge_split(pos.astype(np.int32), size)
            assert np.array_equal(tr.cpu().numpy(), rr), (n, size)
            assert np.array_equal(tp.cpu().numpy(), rp), (n, size)
        # the windowed product's merge split (bounds reading the window total
        # on the device): every row without its first entry when it has two
        vals = rs.uniform(-1, 1, nnz)
        Bv = _csr(spl, pos.astype(np.int32), crd, vals, (n, 1), torch.float64)
        begin = (pos[:-1] + (deg >= 2)).astype(np.int32)
        end = pos[1:].astype(np.int32)
        x = torch.tensor([1.5], dtype=torch.float64, device=dev())
        ref, S = oracle.spmv_window(begin, end, crd, vals, np.array([1.5]))
        bt, et = torch.as_tensor(begin, device=dev()), torch.as_tensor(end, device=dev())
        for sc in (dict(kind="merge", tile=1024, items_per_lane=4),
                   dict(kind="merge", tile=8192, items_per_lane=8)):
            a = spl.spmv_window(Bv, bt, et, x, sched=spl.schedule(**sc))
            assert_close(host64(a), ref, S, RTOL[torch.float64], f"window {n} {sc}")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spmv_config1_all_schedules(dtype):
    spl = _spl()
    c1 = configs.config1()
    B = _csr(spl, c1["pos"], c1["crd"], c1["vals"], (4096, 4096), dtype)
    x = c1["x"].to(dtype).to(dev())
    ref, S = oracle.spmv(c1["pos"].numpy(), c1["crd"].numpy(), host64(B.vals), host64(x))
    for sc in SCHEDULES_SPMV:
        y = spl.spmv(B, x, sched=spl.schedule(**sc))
        assert_close(host64(y), ref, S, RTOL[dtype], str(sc))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spmv_powerlaw_scaled_all_schedules(dtype):
    spl = _spl()
    c2 = configs.config2(scale=0.01, with_dense=False)   # 20k rows, 320k nnz, cap 5000
    B = _csr(spl, c2["pos"], c2["crd"], c2["vals"], (c2["n"], c2["n"]), dtype)
    x = c2["x"].to(dtype).to(dev())
    ref, S = oracle.spmv(c2["pos"].numpy(), c2["crd"].numpy(), host64(B.vals), host64(x))
    for sc in SCHEDULES_SPMV:
        y = spl.spmv(B, x, sched=spl.schedule(**sc))
        assert_close(host64(y), ref, S, RTOL[dtype], str(sc))


@pytest.mark.parametrize("name", list(_edge_cases().keys()))
def test_spmv_edge_cases(name):
    spl = _spl()
    pos, crd, vals, shape = _edge_cases()[name]
    B = _csr(spl, pos, crd, vals, shape, torch.float64)
    x = torch.linspace(-1, 1, shape[1], dtype=torch.float64, device=dev())
    ref, S = oracle.spmv(pos, crd, vals, host64(x))
    for sc in SCHEDULES_SPMV:
        y = spl.spmv(B, x, sched=spl.schedule(**sc))
        assert_close(host64(y), ref, S, 1e-12, f"{name} {sc}")


def test_spmv_empty_matrix_and_zero_rows():
    spl = _spl()
    B = _csr(spl, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), (0, 4), torch.float64)
    y = spl.spmv(B, torch.ones(4, dtype=torch.float64, device=dev()))
    assert y.numel() == 0


def test_spmv_integer_values_bit_exact_across_schedules():
    spl = _spl()
    c2 = configs.config2(scale=0.01, with_dense=False, kind="int")
    for dtype in (torch.float64, torch.float32):
        B = _csr(spl, c2["pos"], c2["crd"], c2["vals"], (c2["n"], c2["n"]), dtype)
        x = c2["x"].to(dtype).to(dev())
        ref, _ = oracle.spmv(c2["pos"].numpy(), c2["crd"].numpy(), host64(B.vals), host64(x))
        for sc in SCHEDULES_SPMV:
            y = spl.spmv(B, x, sched=spl.schedule(**sc))
            assert np.array_equal(host64(y), ref), sc


def test_spmv_deterministic():
    spl = _spl()
    c2 = configs.config2(scale=0.01, with_dense=False)
    B = _csr(spl, c2["pos"], c2["crd"], c2["vals"], (c2["n"], c2["n"]), torch.float32)
    x = c2["x"].to(torch.float32).to(dev())
    for sc in SCHEDULES_SPMV:
        y1 = spl.spmv(B, x, sched=spl.schedule(**sc)).clone()
        y2 = spl.spmv(B, x, sched=spl.schedule(**sc))
        assert torch.equal(y1, y2), sc


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("N", [32, 5, 70])
def test_spmm_powerlaw_scaled(dtype, N):
    spl = _spl()
    c2 = configs.config2(scale=0.005, N=N)
    B = _csr(spl, c2["pos"], c2["crd"], c2["vals"], (c2["n"], c2["n"]), dtype)
    Bd = c2["B"].to(dtype).to(dev())
    ref, S = oracle.spmm(c2["pos"].numpy(), c2["crd"].numpy(), host64(B.vals), host64(Bd))
    for sc in SCHEDULES_SPMM:
        A = spl.spmm(B, Bd, sched=spl.schedule(**sc))
        assert A.dtype == (torch.float32 if dtype == torch.bfloat16 else dtype)
        assert_close(host64(A), ref, S, RTOL[dtype], f"{dtype} N={N} {sc}")


BF16_SCHEDULES = [
    dict(kind="default"), dict(kind="merge", tile=512, col_tile=32, items_per_lane=16),
    dict(kind="merge", tile=256, col_tile=32, items_per_lane=8),
    dict(kind="merge", tile=4096, col_tile=64, items_per_lane=8),
    dict(kind="merge", tile=1024, col_tile=16, items_per_lane=16),
    # 8-byte lanes (4 BF16 columns per lane)
    dict(kind="merge", tile=512, col_tile=32, items_per_lane=16, variant=2),
    dict(kind="merge", tile=3000, col_tile=16, items_per_lane=8, variant=2),
]


@pytest.mark.parametrize("N", [32, 24, 40, 16, 8, 72, 5])
def test_spmm_bf16_lane_widths(N):
    # 16-byte lanes (8 BF16 columns: 2 to 8 lanes per group) and 8-byte
    # lanes, N a multiple of 8 or not; small-integer values make every
    # product and sum exact, so every schedule matches the oracle bit for bit
    spl = _spl()
    c2 = configs.config2(scale=0.004, N=N, kind="int")
    B = _csr(spl, c2["pos"], c2["crd"], c2["vals"], (c2["n"], c2["n"]), torch.bfloat16)
    Bd = c2["B"].to(torch.bfloat16).to(dev())
    ref, _ = oracle.spmm(c2["pos"].numpy(), c2["crd"].numpy(), host64(B.vals), host64(Bd))
    for sc in BF16_SCHEDULES:
        A = spl.spmm(B, Bd, sched=spl.schedule(**sc))
        assert np.array_equal(host64(A), ref), (N, sc)
    c2 = configs.config2(scale=0.004, N=N)
    B = _csr(spl, c2["pos"], c2["crd"], c2["vals"], (c2["n"], c2["n"]), torch.bfloat16)
    Bd = c2["B"].to(torch.bfloat16).to(dev())
    ref, S = oracle.spmm(c2["pos"].numpy(), c2["crd"].numpy(), host64(B.vals), host64(Bd))
    for sc in BF16_SCHEDULES:
        A = spl.spmm(B, Bd, sched=spl.schedule(**sc))
        assert_close(host64(A), ref, S, 1e-5, f"bf16 N={N} {sc}")


@pytest.mark.parametrize("name", list(_edge_cases().keys()))
def test_spmm_edge_cases(name):
    spl = _spl()
    pos, crd, vals, shape = _edge_cases()[name]
    B = _csr(spl, pos, crd, vals, shape, torch.float32)
    Bd = torch.linspace(-1, 1, shape[1] * 33, dtype=torch.float32, device=dev()).reshape(shape[1], 33)
    ref, S = oracle.spmm(pos, crd, host64(B.vals), host64(Bd))
    for sc in SCHEDULES_SPMM:
        A = spl.spmm(B, Bd, sched=spl.schedule(**sc))
        assert_close(host64(A), ref, S, 1e-5, f"{name} {sc}")


def test_spmm_integer_values_bit_exact_and_strided_output():
    spl = _spl()
    c2 = configs.config2(scale=0.003, N=24, kind="int")
    B = _csr(spl, c2["pos"], c2["crd"], c2["vals"], (c2["n"], c2["n"]), torch.float32)
    Bd = c2["B"].to(torch.float32).to(dev())
    ref, _ = oracle.spmm(c2["pos"].numpy(), c2["crd"].numpy(), host64(B.vals), host64(Bd))
    big = torch.full((c2["n"], 40), 7.0, dtype=torch.float32, device=dev())
    for sc in SCHEDULES_SPMM:
        out = big[:, 3:27]
        spl.spmm(B, Bd, A=out, sched=spl.schedule(**sc))
        assert np.array_equal(host64(out), ref), sc
        assert torch.all(big[:, :3] == 7.0) and torch.all(big[:, 27:] == 7.0)


def test_spmm_deterministic():
    spl = _spl()
    c2 = configs.config2(scale=0.005)
    B = _csr(spl, c2["pos"], c2["crd"], c2["vals"], (c2["n"], c2["n"]), torch.float32)
    Bd = c2["B"].to(torch.float32).to(dev())
    for sc in SCHEDULES_SPMM:
        a1 = spl.spmm(B, Bd, sched=spl.schedule(**sc)).clone()
        a2 = spl.spmm(B, Bd, sched=spl.schedule(**sc))
        assert torch.equal(a1, a2), sc


def test_validate_catches_malformed_levels():
    spl = _spl()
    rs = np.random.RandomState(2)
    pos, crd, vals = tiny.csr(rs, 30, 30, 0.3)
    spl.validate(_csr(spl, pos, crd, vals, (30, 30), torch.float64))
    bad_crd = crd.copy()
    bad_crd[5] = 30
    with pytest.raises(spl.SpleafError, match="out of range"):
        spl.validate(_csr(spl, pos, bad_crd, vals, (30, 30), torch.float64))
    r = next(i for i in range(30) if pos[i + 1] - pos[i] >= 2)
    uns = crd.copy()
    uns[pos[r]], uns[pos[r] + 1] = uns[pos[r] + 1], uns[pos[r]]
    with pytest.raises(spl.SpleafError, match="increasing"):
        spl.validate(_csr(spl, pos, uns, vals, (30, 30), torch.float64))
    bpos = pos.copy()
    bpos[10] = bpos[11] + 1
    with pytest.raises(spl.SpleafError, match="decreases"):
        spl.validate(_csr(spl, bpos, crd, vals, (30, 30), torch.float64))


def test_host_errors_reported():
    spl = _spl()
    rs = np.random.RandomState(3)
    pos, crd, vals = tiny.csr(rs, 10, 10, 0.3)
    B = _csr(spl, pos, crd, vals, (10, 10), torch.float64)
    with pytest.raises(spl.SpleafError, match="SPL_ERR_SHAPE"):
        spl.spmv(B, torch.ones(9, dtype=torch.float64, device=dev()))
    with pytest.raises(spl.SpleafError, match="SPL_ERR_DTYPE"):
        spl.spmv(B, torch.ones(10, dtype=torch.float32, device=dev()))
    with pytest.raises(spl.SpleafError, match="SPL_ERR_ARG"):
        spl.spmv(B, torch.ones(10, dtype=torch.float64, device=dev()),
                 sched=spl.schedule("row", lanes_per_row=3))
    for bad in (dict(kind="nnz", variant=1), dict(kind="row", variant=1),
                dict(kind="nnz", variant=2), dict(kind="merge", variant=3)):
        with pytest.raises(spl.SpleafError, match="SPL_ERR_ARG"):
            spl.spmv(B, torch.ones(10, dtype=torch.float64, device=dev()),
                     sched=spl.schedule(**bad))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_spmm_int64_positions_match_int32(dtype):
    # the same matrix with int64 pos: the same kernel walk (row ends staged
    # relative to each chunk), so bit-identical results, and within the
    # oracle's tolerance
    spl = _spl()
    c2 = configs.config2(scale=0.005, N=32)
    B = _csr(spl, c2["pos"], c2["crd"], c2["vals"], (c2["n"], c2["n"]), dtype)
    B64 = spl.CSR(B.pos.to(torch.int64), B.crd, B.vals, B.shape)
    Bd = c2["B"].to(torch.float32).to(dtype).to(dev())
    ref, S = oracle.spmm(c2["pos"].numpy(), c2["crd"].numpy(), host64(B.vals), host64(Bd))
    for sc in (dict(kind="default"), dict(kind="merge", tile=4096, col_tile=32, items_per_lane=8),
               dict(kind="merge", tile=777, col_tile=32, items_per_lane=16)):
        a32 = spl.spmm(B, Bd, sched=spl.schedule(**sc))
        a64 = spl.spmm(B64, Bd, sched=spl.schedule(**sc))
        assert torch.equal(a32, a64), (dtype, sc)
        assert_close(host64(a64), ref, S, RTOL[dtype], f"int64 spmm {dtype} {sc}")
    for bad in (dict(kind="nnz", tile=512), dict(kind="row"), dict(kind="merge", variant=1)):
        with pytest.raises(spl.SpleafError, match="SPL_ERR_UNSUPPORTED"):
            spl.spmm(B64, Bd, sched=spl.schedule(**bad))
