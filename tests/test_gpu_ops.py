"""GPU parity of SpTTV, SpMTTKRP, the inner product, SDDMM and SpAdd3
against the CPU oracle, through the C ABI.

Output patterns (SpAdd3 pos/crd) are compared bit for bit; values satisfy
|got - ref| <= rtol * S with rtol 1e-12 (FP64) or 1e-5 (FP32, and BF16
inputs with FP32 accumulation compared with the oracle run on the same
BF16-rounded inputs); small-integer values are bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2207_13901_amd import _native as N
from tests import tiny
from tests.gpu_util import RTOL, assert_close, dev, host64, need_gpu
from workloads import configs

pytestmark = pytest.mark.gpu

TTV_SCHEDULES = [dict(kind="default"), dict(kind="row", lanes_per_row=2),
                 dict(kind="nnz", tile=500), dict(kind="merge", tile=4096, items_per_lane=4),
                 dict(kind="merge", tile=20000, items_per_lane=8), dict(kind="merge", variant=1),
                 dict(kind="merge", tile=5000, items_per_lane=4, variant=1),
                 dict(kind="merge", variant=2),
                 dict(kind="merge", tile=20000, items_per_lane=8, variant=2),
                 dict(kind="merge", tile=3000, items_per_lane=4, variant=2)]
MTTKRP_SCHEDULES = [dict(kind="default"), dict(kind="merge", tile=128, col_tile=32, items_per_lane=8),
                    dict(kind="nnz", tile=300), dict(kind="nnz", tile=4096, col_tile=16),
                    dict(kind="row", tile=3), dict(kind="merge", tile=5000, col_tile=64,
                                                   items_per_lane=16),
                    dict(kind="merge", tile=32, col_tile=32, items_per_lane=16),
                    dict(kind="merge", tile=1, col_tile=64, items_per_lane=8),
                    dict(kind="nnz", tile=700, col_tile=32, items_per_lane=8),
                    dict(kind="merge", tile=2048, col_tile=32, items_per_lane=8),
                    dict(kind="merge", tile=512, col_tile=32, items_per_lane=8, variant=1)]
# 4 items per lane group: the 4-column-lane leaf only (R and every ld multiples
# of 4); 5 items: 4-column lanes at col_tile 32 only; col_tile 32 with items
# and tile left to the library (5 items, tile 512 with 4-column lanes)
MTTKRP_VEC4 = [dict(kind="merge", tile=512, col_tile=32, items_per_lane=4),
               dict(kind="merge", tile=1, col_tile=64, items_per_lane=4),
               dict(kind="merge", tile=3000, col_tile=32, items_per_lane=4),
               dict(kind="merge", tile=512, col_tile=32, items_per_lane=5),
               dict(kind="merge", tile=1, col_tile=32, items_per_lane=5),
               dict(kind="merge", col_tile=32)]
# merge tiles of 2048 and 5000 items give the vector-ALU leaves several chunks
# per workgroup (their default is one)
SDDMM_SCHEDULES = [dict(kind="default"), dict(kind="nnz", tile=300), dict(kind="row", tile=7),
                   dict(kind="merge", tile=512), dict(kind="merge", tile=2048),
                   dict(kind="merge", tile=5000)]


def _spl():
    need_gpu()
    import paper_2207_13901_amd as spl
    return spl


def _t(a, dtype=torch.int32):
    return torch.as_tensor(np.asarray(a)).to(dtype).to(dev())


def _csf(spl, c, dtype, vals_key="vals"):
    shape = (c["I"], c["J"], c["K"])
    return spl.CSF(_t(c["pos1"]), _t(c["crd1"]), _t(c["pos2"]), _t(c["crd2"]),
                   _t(c[vals_key], torch.float64).to(dtype), shape)


def _tiny_csf(seed, kind="float"):
    rs = np.random.RandomState(seed)
    p1, c1, p2, c2, v = tiny.csf(rs, 40, 9, 300, 0.05, kind=kind, empty_slices={0, 5, 39})
    return dict(I=40, J=9, K=300, pos1=p1, crd1=c1, pos2=p2, crd2=c2, vals=v,
                vals2=rs.uniform(-1, 1, len(v)))


def _numpy(c):
    return {k: (v.numpy() if isinstance(v, torch.Tensor) else v) for k, v in c.items()}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spttv(dtype):
    spl = _spl()
    for c in (_numpy(configs.config4(scale=0.001, with_dense=False)), _tiny_csf(1)):
        B = _csf(spl, c, dtype)
        cv = _t(np.linspace(-1, 1, c["K"]), torch.float64).to(dtype)
        ref, S = oracle.spttv(c["pos1"], c["pos2"], c["crd2"], host64(B.vals), host64(cv))
        for sc in TTV_SCHEDULES:
            A = spl.spttv(B, cv, sched=spl.schedule(**sc))
            assert A.numel() == len(c["crd1"])
            assert_close(host64(A), ref, S, RTOL[dtype], f"spttv {sc}")


def test_spttv_unit_vector_extracts_entries():
    spl = _spl()
    c = _tiny_csf(2)
    B = _csf(spl, c, torch.float64)
    for k in (0, 17, 299):
        e = torch.zeros(c["K"], dtype=torch.float64, device=dev())
        e[k] = 1.0
        A = spl.spttv(B, e)
        ref, _ = oracle.spttv(c["pos1"], c["pos2"], c["crd2"], c["vals"], e.cpu().numpy())
        assert np.array_equal(host64(A), ref)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("R", [32, 5, 70])
def test_mttkrp(dtype, R):
    spl = _spl()
    c4 = _numpy(configs.config4(scale=0.001, R=R))
    for c in (c4, dict(_tiny_csf(3), C=np.random.RandomState(4).normal(size=(9, R)),
                       D=np.random.RandomState(5).normal(size=(300, R)))):
        B = _csf(spl, c, dtype)
        C = _t(c["C"], torch.float64).to(torch.float32).to(dtype)
        D = _t(c["D"], torch.float64).to(torch.float32).to(dtype)
        ref, S = oracle.mttkrp(c["pos1"], c["crd1"], c["pos2"], c["crd2"], host64(B.vals),
                               host64(C), host64(D))
        staged = [dict(sc, variant=3) for sc in MTTKRP_VEC4 if sc.get("items_per_lane") == 4] \
            if dtype == torch.float32 and R % 4 == 0 else []
        for sc in MTTKRP_SCHEDULES + (MTTKRP_VEC4 if R % 4 == 0 else []) + staged:
            A = spl.mttkrp(B, C, D, sched=spl.schedule(**sc))
            assert A.dtype == torch.float32
            assert_close(host64(A), ref, S, 1e-5, f"mttkrp {dtype} R={R} {sc}")
        if R % 4:
            with pytest.raises(spl.SpleafError, match="items_per_lane 4"):
                spl.mttkrp(B, C, D, sched=spl.schedule(**MTTKRP_VEC4[0]))
            with pytest.raises(spl.SpleafError, match="items_per_lane 5"):
                spl.mttkrp(B, C, D, sched=spl.schedule(**MTTKRP_VEC4[3]))
        else:
            # 5 items need col_tile 32; 3 items need 8-column BF16 lanes
            with pytest.raises(spl.SpleafError, match="items_per_lane 5"):
                spl.mttkrp(B, C, D, sched=spl.schedule(kind="merge", col_tile=64,
                                                       items_per_lane=5))
            if dtype == torch.float32:
                with pytest.raises(spl.SpleafError, match="items_per_lane 3"):
                    spl.mttkrp(B, C, D, sched=spl.schedule(kind="merge", col_tile=32,
                                                           items_per_lane=3))


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_mttkrp_caller_workspace_from_query(dtype):
    # the query cannot see the lane width (it depends on the factors'
    # pointers) and takes the largest size over the widths: a workspace of
    # exactly that size serves every schedule, including the defaults that
    # pick items and tile with the lane width
    spl = _spl()
    c = _numpy(configs.config4(scale=0.001, R=32))
    B = _csf(spl, c, dtype)
    C = _t(c["C"], torch.float64).to(torch.float32).to(dtype)
    D = _t(c["D"], torch.float64).to(torch.float32).to(dtype)
    ref, S = oracle.mttkrp(c["pos1"], c["crd1"], c["pos2"], c["crd2"], host64(B.vals),
                           host64(C), host64(D))
    scheds = [None, dict(kind="merge", col_tile=32), dict(kind="merge", tile=1, col_tile=32),
              dict(kind="merge", tile=1, col_tile=32, items_per_lane=4),
              dict(kind="nnz", tile=300), dict(kind="merge", tile=1, col_tile=64, items_per_lane=8)]
    scheds.append(dict(kind="merge", tile=1, col_tile=32, items_per_lane=3) if dtype == torch.bfloat16
                  else dict(kind="merge", tile=1, col_tile=32, items_per_lane=5))
    for sc in scheds:
        sched = spl.schedule(**sc) if sc else None
        ws = spl.workspace(N.OP_MTTKRP, B, 32, sched)
        A = spl.mttkrp(B, C, D, sched=sched, ws=ws)
        assert_close(host64(A), ref, S, 1e-5, f"mttkrp caller workspace {dtype} {sc}")


def test_mttkrp_integer_values_bit_exact():
    spl = _spl()
    c = _tiny_csf(6, kind="int")
    rs = np.random.RandomState(7)
    C = _t(rs.randint(-4, 5, (9, 32)), torch.float32)
    D = _t(rs.randint(-4, 5, (300, 32)), torch.float32)
    B = _csf(spl, c, torch.float32)
    ref, _ = oracle.mttkrp(c["pos1"], c["crd1"], c["pos2"], c["crd2"], c["vals"],
                           host64(C), host64(D))
    for sc in MTTKRP_SCHEDULES + MTTKRP_VEC4 + [dict(sc, variant=3) for sc in MTTKRP_VEC4
                                                if sc.get("items_per_lane") == 4]:
        A = spl.mttkrp(B, C, D, sched=spl.schedule(**sc))
        assert np.array_equal(host64(A), ref), sc


# 3 items: 8-column BF16 lanes at col_tile 32 only (R and every ld multiples of 8)
MTTKRP_BF16_ITEMS3 = [dict(kind="merge", tile=512, col_tile=32, items_per_lane=3),
                      dict(kind="merge", tile=1, col_tile=32, items_per_lane=3),
                      dict(kind="merge", tile=5000, col_tile=32, items_per_lane=3)]
MTTKRP_BF16 = MTTKRP_VEC4 + [
    dict(kind="merge", tile=256, col_tile=64, items_per_lane=8),
    dict(kind="merge", tile=4096, col_tile=64, items_per_lane=8),
    dict(kind="nnz", tile=1000, col_tile=32, items_per_lane=4),
    dict(kind="row", tile=5, col_tile=32, items_per_lane=4),
    # 8-byte lanes (4 BF16 rank columns per lane)
    dict(kind="merge", tile=512, col_tile=32, items_per_lane=4, variant=2),
    dict(kind="merge", tile=700, col_tile=32, items_per_lane=8, variant=2)]


@pytest.mark.parametrize("R", [32, 24, 16, 40, 8, 12])
def test_mttkrp_bf16_lane_widths(R):
    # 16-byte lanes of 8 BF16 rank columns (4 or 8 lanes per group) and
    # 8-byte lanes, R a multiple of 8 or only of 4; small-integer values make
    # every product and sum exact (bit-exact against the oracle), random
    # values stay within the tolerance
    spl = _spl()
    rs = np.random.RandomState(R)
    for kind in ("int", "sym"):
        c = _numpy(configs.config4(scale=0.001, R=R)) if kind == "sym" else \
            _tiny_csf(6, kind="int")
        J, K = c["J"], c["K"]
        if kind == "int":
            Cn, Dn = rs.randint(-4, 5, (J, R)), rs.randint(-4, 5, (K, R))
        else:
            Cn, Dn = c["C"], c["D"]
        B = _csf(spl, c, torch.bfloat16)
        C = _t(Cn, torch.float64).to(torch.float32).to(torch.bfloat16)
        D = _t(Dn, torch.float64).to(torch.float32).to(torch.bfloat16)
        ref, S = oracle.mttkrp(c["pos1"], c["crd1"], c["pos2"], c["crd2"], host64(B.vals),
                               host64(C), host64(D))
        for sc in MTTKRP_BF16 + (MTTKRP_BF16_ITEMS3 if R % 8 == 0 else []):
            A = spl.mttkrp(B, C, D, sched=spl.schedule(**sc))
            if kind == "int":
                assert np.array_equal(host64(A), ref), (R, sc)
            else:
                assert_close(host64(A), ref, S, 1e-5, f"mttkrp bf16 R={R} {sc}")
        if R % 8:
            with pytest.raises(spl.SpleafError, match="items_per_lane 3"):
                spl.mttkrp(B, C, D, sched=spl.schedule(**MTTKRP_BF16_ITEMS3[0]))
    with pytest.raises(spl.SpleafError, match="variant 2"):
        B32 = _csf(spl, c, torch.float32)
        spl.mttkrp(B32, C.float(), D.float(), sched=spl.schedule(**MTTKRP_BF16[-1]))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_inner_product(dtype):
    spl = _spl()
    for c in (_numpy(configs.config4(scale=0.001, with_dense=False)), _tiny_csf(8)):
        B = _csf(spl, c, dtype)
        C = B.with_vals(_t(c["vals2"], torch.float64).to(dtype))
        a = spl.inner(B, C)
        ref, S = oracle.inner((c["pos1"], c["crd1"], c["pos2"], c["crd2"], host64(B.vals)),
                              (c["pos1"], c["crd1"], c["pos2"], c["crd2"], host64(C.vals)))
        assert_close(host64(a), np.array([ref]), np.array([S]), 1e-12, "inner")
        # equal to the sum of the Hadamard product of the aligned values
        had = float(np.sum(host64(B.vals) * host64(C.vals)))
        assert abs(float(a.item()) - had) <= 1e-12 * S
        a2 = spl.inner(B, C)
        assert torch.equal(a, a2)  # fixed reduction order
    # the same pattern in other arrays takes the co-iteration path: same sum
    other = spl.CSF(B.pos1.clone(), B.crd1.clone(), B.pos2.clone(), B.crd2.clone(), C.vals,
                    B.shape)
    assert_close(host64(spl.inner(B, other)), np.array([ref]), np.array([S]), 1e-12,
                 "inner, same pattern in copies")


def _c3(scale=0.002, K=128, kind="sym"):
    return configs.config3(scale=scale, K=K, kind=kind)


@pytest.mark.parametrize("case", ["f64", "f32", "bf16_valu", "bf16_mfma"])
def test_sddmm(case):
    spl = _spl()
    c = _c3()
    Bm = c["B"]
    vdt = torch.float64 if case == "f64" else torch.float32
    fdt = {"f64": torch.float64, "f32": torch.float32}.get(case, torch.bfloat16)
    B = spl.CSR(Bm["pos"].to(dev()), Bm["crd"].to(dev()), Bm["vals"].to(vdt).to(dev()),
                (c["n"], c["m"]))
    C = c["Cd"].to(torch.float32 if fdt == torch.bfloat16 else fdt).to(fdt).to(dev())
    D = c["Dd"].to(torch.float32 if fdt == torch.bfloat16 else fdt).to(fdt).to(dev())
    ref, S = oracle.sddmm(Bm["pos"].numpy(), Bm["crd"].numpy(), host64(B.vals), host64(C),
                          host64(D))
    variant = 1 if case == "bf16_mfma" else 0
    for sc in SDDMM_SCHEDULES:
        A = spl.sddmm(B, C, D, sched=spl.schedule(**sc, variant=variant))
        assert_close(host64(A), ref, S, 1e-12 if case == "f64" else 1e-5, f"sddmm {case} {sc}")


def test_sddmm_edge_cases():
    spl = _spl()
    rs = np.random.RandomState(9)
    pos, crd, vals = tiny.csr(rs, 200, 150, 0.05, empty_rows={0, 1, 50, 199}, full_rows={3})
    B = spl.CSR(_t(pos), _t(crd), _t(vals, torch.float32), (200, 150))
    # K = 1 with unit factors gives A = B exactly
    A = spl.sddmm(B, torch.ones(200, 1, device=dev()), torch.ones(150, 1, device=dev()))
    assert np.array_equal(host64(A), host64(B.vals))
    # ragged K for the vector path, and K = 32 on the matrix cores
    for K, variant, dt in ((40, 0, torch.float32), (32, 1, torch.bfloat16), (96, 1, torch.bfloat16)):
        C = _t(rs.uniform(-1, 1, (200, K)), torch.float32).to(dt)
        D = _t(rs.uniform(-1, 1, (150, K)), torch.float32).to(dt)
        ref, S = oracle.sddmm(pos, crd, host64(B.vals), host64(C), host64(D))
        A = spl.sddmm(B, C, D, sched=spl.schedule(variant=variant))
        assert_close(host64(A), ref, S, 1e-5, f"K={K} variant={variant}")
    # factors whose leading dimension rules out 16-byte accesses (one element
    # per lane access), and a short FP64 K on the vector-lane path
    Cw = _t(rs.uniform(-1, 1, (200, 41)), torch.float32)[:, :40]
    Dw = _t(rs.uniform(-1, 1, (150, 41)), torch.float32)[:, :40]
    ref, S = oracle.sddmm(pos, crd, host64(B.vals), host64(Cw), host64(Dw))
    assert_close(host64(spl.sddmm(B, Cw, Dw)), ref, S, 1e-5, "strided factors")
    B64 = spl.CSR(B.pos, B.crd, B.vals.to(torch.float64), (200, 150))
    C6 = _t(rs.uniform(-1, 1, (200, 6)), torch.float64)
    D6 = _t(rs.uniform(-1, 1, (150, 6)), torch.float64)
    ref, S = oracle.sddmm(pos, crd, host64(B64.vals), host64(C6), host64(D6))
    assert_close(host64(spl.sddmm(B64, C6, D6)), ref, S, 1e-12, "K=6 FP64")
    with pytest.raises(spl.SpleafError, match="UNSUPPORTED"):
        spl.sddmm(B, _t(rs.uniform(-1, 1, (200, 40)), torch.bfloat16),
                  _t(rs.uniform(-1, 1, (150, 40)), torch.bfloat16),
                  sched=spl.schedule(variant=1))


def _csr_dev(spl, m, shape, dtype):
    return spl.CSR(m["pos"].to(dev()), m["crd"].to(dev()), m["vals"].to(dtype).to(dev()), shape)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spadd3(dtype):
    spl = _spl()
    c = configs.config3(scale=0.003, with_dense=False)
    shape = (c["n"], c["m"])
    ops = [_csr_dev(spl, c[k], shape, dtype) for k in "BCD"]
    A = spl.spadd3(*ops)
    host = [(c[k]["pos"].numpy(), c[k]["crd"].numpy(), host64(o.vals)) for k, o in zip("BCD", ops)]
    rpos, rcrd, rvals, rS, rnnz = oracle.spadd3(*host)
    assert np.array_equal(A.pos.cpu().numpy(), rpos)
    assert np.array_equal(A.crd.cpu().numpy(), rcrd)
    assert A.crd.numel() == rnnz
    assert_close(host64(A.vals), rvals, rS, RTOL[dtype], "spadd3")
    # the pattern does not depend on operand order; B and C swap exactly
    A2 = spl.spadd3(ops[1], ops[0], ops[2])
    assert torch.equal(A2.pos, A.pos) and torch.equal(A2.crd, A.crd)
    assert torch.equal(A2.vals, A.vals)
    A3 = spl.spadd3(ops[2], ops[1], ops[0])
    assert torch.equal(A3.crd, A.crd)
    assert_close(host64(A3.vals), rvals, rS, RTOL[dtype], "spadd3 permuted")


def test_spadd3_invariants_and_errors():
    spl = _spl()
    rs = np.random.RandomState(10)
    n, m = 300, 200
    pos, crd, vals = tiny.csr(rs, n, m, 0.05, empty_rows={0, 7, 299}, kind="int")
    B = spl.CSR(_t(pos), _t(crd), _t(vals, torch.float32), (n, m))
    E = spl.CSR(_t(np.zeros(n + 1)), _t(np.zeros(0)), _t(np.zeros(0), torch.float32), (n, m))
    A = spl.spadd3(B, E, E)
    assert torch.equal(A.pos, B.pos) and torch.equal(A.crd, B.crd) and torch.equal(A.vals, B.vals)
    A3 = spl.spadd3(B, B, B)
    assert torch.equal(A3.pos, B.pos) and torch.equal(A3.crd, B.crd)
    assert torch.equal(A3.vals, 3 * B.vals)
    negB = B.with_vals(-B.vals)
    A0 = spl.spadd3(B, negB, E)
    assert torch.equal(A0.crd, B.crd) and bool(torch.all(A0.vals == 0))
    with pytest.raises(spl.SpleafError, match="UNSUPPORTED"):
        spl.spadd3(B, B, B, sched=spl.schedule("nnz", tile=64))
    # integer values: bit-exact against the oracle
    p2, c2, v2 = tiny.csr(rs, n, m, 0.05, kind="int")
    p3, c3, v3 = tiny.csr(rs, n, m, 0.05, kind="int")
    C = spl.CSR(_t(p2), _t(c2), _t(v2, torch.float32), (n, m))
    D = spl.CSR(_t(p3), _t(c3), _t(v3, torch.float32), (n, m))
    A = spl.spadd3(B, C, D)
    rpos, rcrd, rvals, _, _ = oracle.spadd3((pos, crd, vals), (p2, c2, v2), (p3, c3, v3))
    assert np.array_equal(A.pos.cpu().numpy(), rpos)
    assert np.array_equal(A.crd.cpu().numpy(), rcrd)
    assert np.array_equal(host64(A.vals), rvals)


def test_spadd3_long_rows_span_output_windows():
    # rows whose union alone fills several LDS output windows, next to short
    # and empty rows in the same workgroup and in the next one
    spl = _spl()
    rs = np.random.RandomState(11)
    n, m = 700, 9000
    pos, crd, vals = tiny.csr(rs, n, m, 0.002, empty_rows={0, 255, 256}, full_rows={5, 300},
                              kind="int")
    p2, c2, v2 = tiny.csr(rs, n, m, 0.3, empty_rows={5}, full_rows={254}, kind="int")
    p3, c3, v3 = tiny.csr(rs, n, m, 0.001, full_rows={699}, kind="int")
    ops = [spl.CSR(_t(p), _t(c), _t(v, torch.float32), (n, m))
           for p, c, v in ((pos, crd, vals), (p2, c2, v2), (p3, c3, v3))]
    rpos, rcrd, rvals, _, _ = oracle.spadd3((pos, crd, vals), (p2, c2, v2), (p3, c3, v3))
    # every form of both phases (merges reading directly, with coordinates
    # in LDS, with coordinates and values in LDS; ranks; workgroups whose runs
    # exceed the stage read directly)
    for variant in (0, 1, 2, 3, 4):
        A = spl.spadd3(*ops, sched=spl.schedule("row", variant=variant))
        assert np.array_equal(A.pos.cpu().numpy(), rpos), variant
        assert np.array_equal(A.crd.cpu().numpy(), rcrd), variant
        assert np.array_equal(host64(A.vals), rvals), variant


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spadd3_staged_fill_variants(dtype):
    spl = _spl()
    c = configs.config3(scale=0.003, with_dense=False)
    shape = (c["n"], c["m"])
    ops = [_csr_dev(spl, c[k], shape, dtype) for k in "BCD"]
    host = [(c[k]["pos"].numpy(), c[k]["crd"].numpy(), host64(o.vals)) for k, o in zip("BCD", ops)]
    rpos, rcrd, rvals, rS, _ = oracle.spadd3(*host)
    first = None
    for variant in (1, 2, 3, 4):
        A = spl.spadd3(*ops, sched=spl.schedule("row", variant=variant))
        assert np.array_equal(A.pos.cpu().numpy(), rpos) and np.array_equal(A.crd.cpu().numpy(), rcrd)
        assert_close(host64(A.vals), rvals, rS, RTOL[dtype], f"spadd3 variant {variant}")
        if first is None:
            first = A.vals.clone()
        assert torch.equal(A.vals, first), variant  # same sums in the same order
    with pytest.raises(spl.SpleafError, match="SPL_ERR_ARG"):
        spl.spadd3(*ops, sched=spl.schedule("row", variant=5))


def test_spadd3_rank_form_rows_within_the_stage():
    # the rank forms on workgroups whose runs fit the stage but whose rows
    # are long, overlap wholly or partly, or are empty: coordinates held by
    # one, two or three operands, duplicates at the first and last entries,
    # a full row next to empty ones, and signed zeros; the merge forms give
    # the same pattern and bits
    spl = _spl()
    rs = np.random.RandomState(12)
    n, m = 600, 1000
    pos, crd, vals = tiny.csr(rs, n, m, 0.001, empty_rows={0, 1, 191, 192, 255, 256, 599},
                              full_rows={3}, kind="int")
    p2, c2, v2 = tiny.csr(rs, n, m, 0.001, empty_rows={3, 192, 256}, full_rows={300}, kind="int")
    # D repeats B's coordinates in rows 0..299 and C's in the rest, plus a few
    rows = []
    for i in range(n):
        src = (crd[pos[i]:pos[i + 1]] if i < 300 else c2[p2[i]:p2[i + 1]]).tolist()
        extra = rs.choice(m, rs.randint(0, 3), replace=False).tolist()
        rows.append(sorted(set(src) | set(extra)))
    p3 = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    c3 = np.array([c for r in rows for c in r], dtype=np.int64)
    v3 = rs.randint(-4, 5, c3.size).astype(np.float64)
    v2[:5] = -0.0
    ops = [spl.CSR(_t(p), _t(c), _t(v, torch.float32), (n, m))
           for p, c, v in ((pos, crd, vals), (p2, c2, v2), (p3, c3, v3))]
    rpos, rcrd, rvals, _, _ = oracle.spadd3((pos, crd, vals), (p2, c2, v2), (p3, c3, v3))
    # the rank fill's workgroups: 128 rows, at most 1,280 entries per operand
    per_wg = [max(int(p[min(w + 128, n)] - p[w]) for p in (pos, p2, p3)) for w in range(0, n, 128)]
    assert 1000 <= max(per_wg) <= 1280  # long rows, yet every workgroup fits the stage
    A1 = spl.spadd3(*ops, sched=spl.schedule("row", variant=1))
    A4 = spl.spadd3(*ops, sched=spl.schedule("row", variant=4))
    for A in (A1, A4):
        assert np.array_equal(A.pos.cpu().numpy(), rpos)
        assert np.array_equal(A.crd.cpu().numpy(), rcrd)
        assert np.array_equal(host64(A.vals), rvals)
    assert torch.equal(A4.vals.view(torch.int32), A1.vals.view(torch.int32))  # bits, signs of zero


def _perturbed_csf(c, rs, drop=0.3, extra=0.3):
    """A second CSF pattern: c's coordinates with a fraction dropped and
    random ones added (sorted, distinct), new values."""
    I, J, K = c["I"], c["J"], c["K"]
    p1, c1, p2, c2 = c["pos1"], c["crd1"], c["pos2"], c["crd2"]
    coords = set()
    for i in range(I):
        for f in range(p1[i], p1[i + 1]):
            for p in range(p2[f], p2[f + 1]):
                if rs.rand() >= drop:
                    coords.add((i, int(c1[f]), int(c2[p])))
    nnz = len(c2)
    for _ in range(int(extra * nnz)):
        coords.add((int(rs.randint(I)), int(rs.randint(J)), int(rs.randint(K))))
    coords = sorted(coords)
    crd1, pos2, crd2 = [], [0], []
    last = None
    counts = np.zeros(I, dtype=np.int64)
    for (i, j, k) in coords:
        if (i, j) != last:
            crd1.append(j)
            pos2.append(pos2[-1])
            counts[i] += 1
            last = (i, j)
        crd2.append(k)
        pos2[-1] += 1
    pos1 = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    vals = rs.uniform(-1, 1, len(crd2))
    return (pos1, np.array(crd1, np.int32), np.array(pos2, np.int32), np.array(crd2, np.int32),
            vals)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_inner_product_general_patterns(dtype):
    spl = _spl()
    rs = np.random.RandomState(21)
    for c in (_tiny_csf(9), _numpy(configs.config4(scale=0.0005, with_dense=False))):
        B = _csf(spl, c, dtype)
        hp = _perturbed_csf(c, rs)
        Cc = spl.CSF(_t(hp[0]), _t(hp[1]), _t(hp[2]), _t(hp[3]), _t(hp[4], torch.float64).to(dtype),
                     B.shape)
        bh = (c["pos1"], c["crd1"], c["pos2"], c["crd2"], host64(B.vals))
        ch = (hp[0], hp[1], hp[2], hp[3], host64(Cc.vals))
        ref, S = oracle.inner(bh, ch)
        assert_close(host64(spl.inner(B, Cc)), np.array([ref]), np.array([S]), RTOL[dtype],
                     "inner general CSF")
        assert_close(host64(spl.inner(Cc, B)), np.array([ref]), np.array([S]), RTOL[dtype],
                     "inner general CSF, swapped")
    # CSR: the three SpAdd3 operands share 30% of their rows
    c3 = configs.config3(scale=0.002, with_dense=False)
    shape = (c3["n"], c3["m"])
    mats = [_csr_dev(spl, c3[k], shape, dtype) for k in "BC"]
    hs = [(c3[k]["pos"].numpy(), c3[k]["crd"].numpy(), None, None, host64(m.vals))
          for k, m in zip("BC", mats)]
    ref, S = oracle.inner(hs[0], hs[1])
    assert_close(host64(spl.inner(mats[0], mats[1])), np.array([ref]), np.array([S]),
                 RTOL[dtype], "inner general CSR")
    # disjoint patterns give exactly 0; an empty operand too
    rs2 = np.random.RandomState(4)
    p, cc, v = tiny.csr(rs2, 50, 40, 0.2)
    A1 = spl.CSR(_t(p), _t(cc), _t(v, dtype), (50, 40))
    pe, ce = [0], []
    for i in range(50):
        row = sorted(set(int(x) for x in cc[p[i]:p[i + 1]] if x % 2 == 0))
        ce.extend(row)
        pe.append(len(ce))
    po, co = [0], []
    for i in range(50):
        row = sorted(set(int(x) for x in cc[p[i]:p[i + 1]] if x % 2 == 1))
        co.extend(row)
        po.append(len(co))
    E = spl.CSR(_t(pe), _t(ce), _t(np.ones(len(ce)), dtype), (50, 40))
    O = spl.CSR(_t(po), _t(co), _t(np.ones(len(co)), dtype), (50, 40))
    assert float(spl.inner(E, O).item()) == 0.0
    Z = spl.CSR(_t(np.zeros(51)), _t(np.zeros(0)), _t(np.zeros(0), dtype), (50, 40))
    assert float(spl.inner(Z, A1).item()) == 0.0 and float(spl.inner(A1, Z).item()) == 0.0


def _rows_csr(rows, ncols, rs, dtype):
    """CSR from a list of sorted column lists, uniform[-1, 1] values."""
    pos = np.zeros(len(rows) + 1, np.int64)
    pos[1:] = np.cumsum([len(r) for r in rows])
    crd = np.array([c for r in rows for c in r], np.int32)
    vals = rs.uniform(-1, 1, len(crd))
    return (pos.astype(np.int32), crd, vals)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_inner_general_staging_limits(dtype):
    """The co-iteration's LDS staging and its HBM-search fallback agree with the
    oracle: a range of 2048 units over more parents than the workgroup stages,
    a C segment longer than the staged coordinates, and a long C segment whose
    matching part is short enough to stage (clipped at both ends)."""
    spl = _spl()
    rs = np.random.RandomState(33)
    cases = []
    # one unit per parent: every 2048-unit range spans 2048 parents
    n, m = 6000, 300
    b_rows = [[int(rs.randint(m))] for _ in range(n)]
    c_rows = [sorted(rs.choice(m, size=rs.randint(0, 40), replace=False).tolist()) for _ in range(n)]
    for i in range(0, n, 3):  # make a third of them match
        if b_rows[i][0] not in c_rows[i]:
            c_rows[i] = sorted(c_rows[i] + b_rows[i])
    cases.append((b_rows, c_rows, m))
    # B: the first and the last column of a row; C: the full row of 10,000
    m = 10000
    b_rows = [[0, m - 1], [5, 7], [], [m - 2]]
    c_rows = [list(range(m)), list(range(0, m, 2)), list(range(m)), list(range(1, m, 3))]
    cases.append((b_rows, c_rows, m))
    # B: a middle window of a long row; C: the full row (the staged part is clipped)
    b_rows = [list(range(4000, 4100)), list(range(0, 3000, 7))]
    c_rows = [list(range(m)), list(range(m))]
    cases.append((b_rows, c_rows, m))
    for b_rows, c_rows, m in cases:
        bh, ch = _rows_csr(b_rows, m, rs, dtype), _rows_csr(c_rows, m, rs, dtype)
        n = len(b_rows)
        B = spl.CSR(_t(bh[0]), _t(bh[1]), _t(bh[2], torch.float64).to(dtype), (n, m))
        C = spl.CSR(_t(ch[0]), _t(ch[1]), _t(ch[2], torch.float64).to(dtype), (n, m))
        bh = (bh[0], bh[1], None, None, host64(B.vals))
        ch = (ch[0], ch[1], None, None, host64(C.vals))
        ref, S = oracle.inner(bh, ch)
        assert_close(host64(spl.inner(B, C)), np.array([ref]), np.array([S]), RTOL[dtype],
                     "inner general CSR staging")
        assert_close(host64(spl.inner(C, B)), np.array([ref]), np.array([S]), RTOL[dtype],
                     "inner general CSR staging, swapped")


# ------------------------------------------- (Dense, Dense, Compressed) -----

def _ddc(spl, c, dtype, vals_key="vals"):
    return spl.DDC(_t(c["pos2"]), _t(c["crd2"]), _t(c[vals_key], torch.float64).to(dtype),
                   (c["I"], c["J"], c["K"]))


def _tiny_ddc(seed, I=7, J=13, K=300, density=0.03, kind="float"):
    rs = np.random.RandomState(seed)
    p2, c2, v = tiny.ddc(rs, I, J, K, density, kind=kind)
    return dict(I=I, J=J, K=K, pos2=p2, crd2=c2, vals=v, vals2=rs.uniform(-1, 1, len(v)))


def _ddc_cases():
    # the patents-shaped workload scaled down (46 x 478 x 478, 2e5 values,
    # about 9 per fiber), a tiny one with many empty fibers, a single fiber,
    # and one with no values at all
    return [_numpy(configs.ddc(scale=0.002, R=32)), _tiny_ddc(1), _tiny_ddc(2, I=1, J=1),
            _tiny_ddc(3, I=3, J=4, density=0.0)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_ddc_spttv(dtype):
    spl = _spl()
    for c in _ddc_cases():
        B = _ddc(spl, c, dtype)
        cv = _t(np.linspace(-1, 1, c["K"]), torch.float64).to(dtype)
        ref, S = oracle.spttv_ddc(c["I"], c["J"], c["pos2"], c["crd2"], host64(B.vals),
                                  host64(cv))
        for sc in TTV_SCHEDULES:
            A = spl.spttv(B, cv, sched=spl.schedule(**sc))
            assert A.numel() == c["I"] * c["J"]
            assert_close(host64(A), ref, S, RTOL[dtype], f"ddc spttv {sc} I={c['I']}")


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_ddc_mttkrp(dtype):
    spl = _spl()
    rs = np.random.RandomState(11)
    for c in _ddc_cases():
        R = 32 if "C" in c else 5
        Cn = c.get("C", rs.normal(size=(c["J"], R)))
        Dn = c.get("D", rs.normal(size=(c["K"], R)))
        B = _ddc(spl, c, dtype)
        C = _t(Cn, torch.float64).to(torch.float32).to(dtype)
        D = _t(Dn, torch.float64).to(torch.float32).to(dtype)
        ref, S = oracle.mttkrp_ddc(c["I"], c["J"], c["pos2"], c["crd2"], host64(B.vals),
                                   host64(C), host64(D))
        for sc in MTTKRP_SCHEDULES + (MTTKRP_VEC4 if R % 4 == 0 else []):
            A = spl.mttkrp(B, C, D, sched=spl.schedule(**sc))
            assert_close(host64(A), ref, S, 1e-5, f"ddc mttkrp {dtype} {sc} I={c['I']}")
        # a caller workspace sized by the query (it holds the expanded level)
        ws = spl.workspace(N.OP_MTTKRP, B, R)
        A = spl.mttkrp(B, C, D, ws=ws)
        assert_close(host64(A), ref, S, 1e-5, "ddc mttkrp, caller workspace")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_ddc_inner_product(dtype):
    spl = _spl()
    for c in _ddc_cases()[:3]:
        I, J = c["I"], c["J"]
        B = _ddc(spl, c, dtype)
        bh = (None, None, c["pos2"], c["crd2"], host64(B.vals))
        # one pattern: aligned values
        B2 = _ddc(spl, c, dtype, "vals2")
        ref, S = oracle.inner3(I, J, bh, (None, None, c["pos2"], c["crd2"], host64(B2.vals)))
        assert_close(host64(spl.inner(B, B2)), np.array([ref]), np.array([S]), RTOL[dtype],
                     "ddc inner, one pattern")
        # another (Dense, Dense, Compressed) pattern, and the same one as CSF
        o = _tiny_ddc(40, I=I, J=J, K=c["K"], density=0.02 if c["K"] > 100 else 0.3)
        O = _ddc(spl, o, dtype)
        oh = (None, None, o["pos2"], o["crd2"], host64(O.vals))
        ref, S = oracle.inner3(I, J, bh, oh)
        assert_close(host64(spl.inner(B, O)), np.array([ref]), np.array([S]), RTOL[dtype],
                     "ddc inner, two patterns")
        q1, d1, q2, d2 = tiny.ddc_to_csf(o["pos2"], o["crd2"], I, J)
        Of = spl.CSF(_t(q1), _t(d1), _t(q2), _t(d2), O.vals, B.shape)
        for x, y, hx, hy in ((B, Of, bh, (q1, d1, q2, d2, host64(O.vals))),
                             (Of, B, (q1, d1, q2, d2, host64(O.vals)), bh)):
            ref, S = oracle.inner3(I, J, hx, hy)
            assert_close(host64(spl.inner(x, y)), np.array([ref]), np.array([S]), RTOL[dtype],
                         "ddc inner with CSF")


def test_ddc_errors():
    spl = _spl()
    import ctypes
    c = _tiny_ddc(5)
    B = _ddc(spl, c, torch.float64)
    ctx = spl.Context.get()
    s = B.struct()
    s.nfibers = c["I"] * c["J"] + 1
    assert ctx.lib.spl_validate(ctx.h, ctypes.byref(s), None) == N.ERR_SHAPE
    s = B.struct()
    s.level[2] = N.DENSE
    assert ctx.lib.spl_validate(ctx.h, ctypes.byref(s), None) == N.ERR_FORMAT
    spl.validate(B)  # well-formed: only the Compressed level is checked
    bad = spl.DDC(B.pos2, torch.flip(B.crd2, [0]).contiguous(), B.vals, B.shape)
    with pytest.raises(spl.SpleafError, match="INVALID"):
        spl.validate(bad)


def test_csf_leaves_deterministic():
    # fixed reduction orders everywhere (no floating-point atomics): a second
    # call gives the same bits
    spl = _spl()
    c = _numpy(configs.config4(scale=0.001, R=32))
    for dtype in (torch.float32, torch.bfloat16):
        B = _csf(spl, c, dtype)
        C = _t(c["C"], torch.float64).to(torch.float32).to(dtype)
        D = _t(c["D"], torch.float64).to(torch.float32).to(dtype)
        for sc in MTTKRP_SCHEDULES + MTTKRP_VEC4:
            a1 = spl.mttkrp(B, C, D, sched=spl.schedule(**sc)).clone()
            a2 = spl.mttkrp(B, C, D, sched=spl.schedule(**sc))
            assert torch.equal(a1, a2), (dtype, sc)
    B = _csf(spl, c, torch.float32)
    cv = _t(np.linspace(-1, 1, c["K"]), torch.float64).to(torch.float32)
    for sc in TTV_SCHEDULES:
        a1 = spl.spttv(B, cv, sched=spl.schedule(**sc)).clone()
        a2 = spl.spttv(B, cv, sched=spl.schedule(**sc))
        assert torch.equal(a1, a2), sc


def test_csf_tile_bounds_bit_exact():
    """The fiber-aligned non-zero split of a CSF tensor (the MTTKRP NNZ
    schedule's bounds) equals the oracle's bit for bit: empty slices,
    fibers longer than T, T = 1 and T past nnz."""
    spl = _spl()
    big = _numpy(configs.config4(scale=0.001, with_dense=False))
    for c, Ts in ((_tiny_csf(3), (1, 2, 3, 7, 16, 64, 1000)),
                  (big, (1000, 2048, 4099, 100000))):
        B = _csf(spl, c, torch.float32)
        nnz = len(c["crd2"])
        assert np.diff(c["pos2"]).max() > 3   # some fiber is longer than the smallest T
        for T in Ts + (nnz, nnz + 5):
            ts, tf = spl.csf_tile_bounds(B, T)
            rs_, rf, rp = oracle.csf_split(c["pos1"], c["pos2"], T)
            gf = tf.cpu().numpy()
            assert np.array_equal(ts.cpu().numpy(), rs_), T
            assert np.array_equal(gf, rf), T
            assert np.array_equal(c["pos2"][gf], rp), T


def test_csf_tile_bounds_errors():
    spl = _spl()
    c = _tiny_csf(4)
    B = _csf(spl, c, torch.float32)
    with pytest.raises(spl.SpleafError):
        spl.csf_tile_bounds(B, 0)
    rs = np.random.RandomState(2)
    pos2, crd2, v = tiny.ddc(rs, 3, 4, 20, 0.3)
    Bd = spl.DDC(_t(pos2), _t(crd2), _t(v, torch.float64).float(), (3, 4, 20))
    with pytest.raises(spl.SpleafError):
        spl.csf_tile_bounds(Bd, 8)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spttv_int64_positions_match_int32(dtype):
    spl = _spl()
    c = _numpy(configs.config4(scale=0.001, with_dense=False))
    B = _csf(spl, c, dtype)
    B64 = spl.CSF(B.pos1.to(torch.int64), B.crd1, B.pos2.to(torch.int64), B.crd2, B.vals,
                  B.shape)
    cv = _t(c["c"], torch.float64).to(dtype)
    ref, S = oracle.spttv(c["pos1"], c["pos2"], c["crd2"], host64(B.vals), host64(cv))
    for sc in (dict(kind="default"), dict(kind="merge", tile=8192, items_per_lane=4),
               dict(kind="merge", tile=3000, items_per_lane=8)):
        a32 = spl.spttv(B, cv, sched=spl.schedule(**sc))
        a64 = spl.spttv(B64, cv, sched=spl.schedule(**sc))
        assert torch.equal(a32, a64), sc
        assert_close(host64(a64), ref, S, RTOL[dtype], f"int64 spttv {sc}")
    with pytest.raises(spl.SpleafError, match="SPL_ERR_UNSUPPORTED"):
        spl.spttv(B64, cv, sched=spl.schedule(kind="row"))



@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_mttkrp_int64_positions_match_int32(dtype):
    # int64 pos1/pos2 (fiber starts staged relative to each chunk): the
    # same walk as with int32 positions, so identical bits
    spl = _spl()
    c = _numpy(configs.config4(scale=0.001, R=32))
    B = _csf(spl, c, dtype)
    B64 = spl.CSF(B.pos1.to(torch.int64), B.crd1, B.pos2.to(torch.int64), B.crd2, B.vals,
                  B.shape)
    C = _t(c["C"], torch.float64).to(torch.float32).to(dtype)
    D = _t(c["D"], torch.float64).to(torch.float32).to(dtype)
    ref, S = oracle.mttkrp(c["pos1"], c["crd1"], c["pos2"], c["crd2"], host64(B.vals),
                           host64(C), host64(D))
    scheds = [dict(kind="default"), dict(kind="merge", tile=512, col_tile=32, items_per_lane=4),
              dict(kind="merge", tile=4096, col_tile=32, items_per_lane=4),
              dict(kind="merge", tile=1, col_tile=64, items_per_lane=8),
              dict(kind="merge", tile=700, col_tile=32, items_per_lane=5)]
    if dtype == torch.bfloat16:
        scheds.append(dict(kind="merge", tile=700, col_tile=32, items_per_lane=4, variant=2))
        scheds.append(dict(kind="merge", tile=300, col_tile=32, items_per_lane=3))
    for sc in scheds:
        # by default FP32 takes 5 items with int32 positions and 4 with
        # int64: the int64 default walks as the int32 leaf with 4 items
        sc32 = dict(kind="merge", tile=512, col_tile=32, items_per_lane=4) \
            if sc["kind"] == "default" and dtype == torch.float32 else sc
        a32 = spl.mttkrp(B, C, D, sched=spl.schedule(**sc32))
        a64 = spl.mttkrp(B64, C, D, sched=spl.schedule(**sc))
        assert torch.equal(a32, a64), (dtype, sc)
        assert_close(host64(a64), ref, S, 1e-5, f"int64 mttkrp {dtype} {sc}")
    for bad in (dict(kind="nnz", tile=1000), dict(kind="row", tile=4),
                dict(kind="merge", variant=1)):
        with pytest.raises(spl.SpleafError, match="SPL_ERR_UNSUPPORTED"):
            spl.mttkrp(B64, C, D, sched=spl.schedule(**bad))
