"""Parity at the full benchmark sizes, on sampled outputs the oracle computes
one by one: the 2,000,000-row power-law matrix (SpMV, SpMM), the three
1,000,000-row matrices (SDDMM, SpAdd3) and the 1e8-nonzero CSF tensor
(SpTTV, SpMTTKRP, inner product).  Inputs are generated on the GPU and
copied to the host for the oracle; the schedules are the ones the benchmark
chooses among (its autotuner's candidates)."""
import json

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import assert_close, bf16_total_bound, host64, need_gpu
from workloads import configs

pytestmark = pytest.mark.gpu


def _spl():
    need_gpu()
    import paper_2207_13901_amd as spl
    from paper_2207_13901_amd import tuning
    return spl, tuning


def _sample_rows(pos, k=1500, seed=0):
    deg = np.diff(pos)
    rs = np.random.RandomState(seed)
    heavy = np.argsort(deg)[-60:]
    rows = np.unique(np.concatenate([rs.choice(len(deg), k, replace=False), heavy,
                                     [0, len(deg) - 1]]))
    return rows


@pytest.fixture(scope="module")
def c2():
    need_gpu()
    c = configs.config2(device="cuda")
    host = dict(pos=c["pos"].cpu().numpy(), crd=c["crd"].cpu().numpy())
    return c, host


def test_config2_spmv_sampled(c2):
    spl, tuning = _spl()
    c, h = c2
    n = c["n"]
    rows = _sample_rows(h["pos"])
    for dtype, rtol in ((torch.float32, 1e-5), (torch.float64, 1e-12)):
        B = spl.CSR(c["pos"], c["crd"], c["vals"].to(dtype), (n, n))
        x = c["x"].to(dtype)
        ref, S = oracle.spmv(h["pos"], h["crd"], host64(B.vals), host64(x), rows=rows)
        for cand in tuning.SPMV_CANDIDATES[4:]:  # skip the slowest row splits
            y = spl.spmv(B, x, sched=spl.schedule(**cand))
            assert_close(host64(y[torch.as_tensor(rows, device=y.device)]), ref, S, rtol,
                         f"spmv {dtype} {cand}")


def test_config2_coord_partition_windows_sampled(c2):
    # eight column blocks: the partition equals the oracle's on sampled rows,
    # and the eight windowed products add up to the SpMV
    spl, tuning = _spl()
    c, h = c2
    n = c["n"]
    rows = _sample_rows(h["pos"], k=300)
    bounds = np.linspace(0, n, 9).astype(np.int32)
    B = spl.CSR(c["pos"], c["crd"], c["vals"], (n, n))
    out = spl.coord_partition(B, torch.as_tensor(bounds, device=c["pos"].device))
    got = out[:, torch.as_tensor(rows, device=out.device)].cpu().numpy()
    for k, i in enumerate(rows):
        seg = h["crd"][h["pos"][i]:h["pos"][i + 1]]
        want = h["pos"][i] + np.searchsorted(seg, bounds, side="left")
        assert np.array_equal(got[:, k], want), i
    total = torch.zeros(n, dtype=torch.float64, device=out.device)
    for col in range(8):
        total += spl.spmv_window(B, out[col], out[col + 1], c["x"])
    ref, S = oracle.spmv(h["pos"], h["crd"], host64(B.vals), host64(c["x"]), rows=rows)
    assert_close(host64(total[torch.as_tensor(rows, device=total.device)]), ref, S, 1e-12,
                 "sum of column-block windows")


def test_config2_spmm_sampled(c2):
    spl, tuning = _spl()
    c, h = c2
    n = c["n"]
    rows = _sample_rows(h["pos"], k=400, seed=1)
    for dtype, rtol in ((torch.float32, 1e-5), (torch.bfloat16, 1e-5), (torch.float64, 1e-12)):
        B = spl.CSR(c["pos"], c["crd"], c["vals"].to(torch.float32).to(dtype), (n, n))
        D = c["B"].to(torch.float32).to(dtype)
        Dh = host64(D)
        ref, S = oracle.spmm(h["pos"], h["crd"], host64(B.vals), Dh, rows=rows)
        if dtype == torch.bfloat16:
            # (ii) total error against the oracle on the unrounded FP32 inputs
            ref32, S32 = oracle.spmm(h["pos"], h["crd"], host64(c["vals"].to(torch.float32)),
                                     host64(c["B"].to(torch.float32)), rows=rows)
        for cand in tuning.SPMM_CANDIDATES[1:]:
            A = spl.spmm(B, D, sched=spl.schedule(**cand))
            got = host64(A[torch.as_tensor(rows, device=A.device)])
            assert_close(got, ref, S, rtol, f"spmm {dtype} {cand}")
            if dtype == torch.bfloat16:
                assert_close(got, ref32, S32, bf16_total_bound(2), f"spmm bf16 total {cand}")
                print("spmm bf16 " + json.dumps(
                    {"schedule": cand, "vs_bf16_inputs": oracle.error_statement(got, ref, S),
                     "vs_fp32_inputs": oracle.error_statement(got, ref32, S32)}))
        del D


def test_config3_sddmm_and_spadd3():
    spl, _ = _spl()
    c = configs.config3(device="cuda")
    n = c["n"]
    Bm = c["B"]
    hpos, hcrd = Bm["pos"].cpu().numpy(), Bm["crd"].cpu().numpy()
    B = spl.CSR(Bm["pos"], Bm["crd"], Bm["vals"].to(torch.float32), (n, n))
    rows = _sample_rows(hpos, k=3000, seed=2)
    sub_pos = np.concatenate([[0], np.cumsum(np.diff(hpos)[rows])]).astype(np.int32)
    sel = np.concatenate([np.arange(hpos[r], hpos[r + 1]) for r in rows])
    C32 = c["Cd"].to(torch.float32)
    D32 = c["Dd"].to(torch.float32)
    # (ii) the oracle on the unrounded FP32 factors, for the BF16 forms
    ref32, S32 = oracle.sddmm(sub_pos, hcrd[sel], host64(B.vals)[sel],
                              host64(C32[torch.as_tensor(rows, device=C32.device)]), host64(D32))
    for fdt, variant in ((torch.float32, 0), (torch.bfloat16, 0), (torch.bfloat16, 1)):
        C = C32.to(fdt)
        D = D32.to(fdt)
        A = spl.sddmm(B, C, D, sched=spl.schedule(variant=variant))
        Ch = host64(C[torch.as_tensor(rows, device=C.device)])
        ref, S = oracle.sddmm(sub_pos, hcrd[sel], host64(B.vals)[sel], Ch, host64(D))
        got = host64(A)[sel]
        assert_close(got, ref, S, 1e-5, f"sddmm {fdt} variant {variant}")
        if fdt == torch.bfloat16:
            assert_close(got, ref32, S32, bf16_total_bound(2), f"sddmm bf16 total {variant}")
            print(f"sddmm bf16 variant {variant} " + json.dumps(
                {"vs_bf16_inputs": oracle.error_statement(got, ref, S),
                 "vs_fp32_inputs": oracle.error_statement(got, ref32, S32)}))
        del C, D
    ops = [spl.CSR(c[k]["pos"], c[k]["crd"], c[k]["vals"].to(torch.float32), (n, n))
           for k in "BCD"]
    A = spl.spadd3(*ops)
    host = [(c[k]["pos"].cpu().numpy(), c[k]["crd"].cpu().numpy(), host64(o.vals))
            for k, o in zip("BCD", ops)]
    rpos, rcrd, rvals, rS, rnnz = oracle.spadd3(*host)
    assert np.array_equal(A.pos.cpu().numpy(), rpos)
    assert np.array_equal(A.crd.cpu().numpy(), rcrd)
    assert_close(host64(A.vals), rvals, rS, 1e-5, "spadd3 full size")


def test_config4_csf_ops():
    spl, _ = _spl()
    c = configs.config4(device="cuda")
    I, J, K = c["I"], c["J"], c["K"]
    h = {k: c[k].cpu().numpy() for k in ("pos1", "crd1", "pos2", "crd2")}
    vals32 = c["vals"].to(torch.float32)
    B = spl.CSF(c["pos1"], c["crd1"], c["pos2"], c["crd2"], vals32, (I, J, K))
    cv = c["c"].to(torch.float32)
    # SpTTV over every fiber (one oracle pass)
    A = spl.spttv(B, cv)
    ref, S = oracle.spttv(h["pos1"], h["pos2"], h["crd2"], host64(vals32), host64(cv))
    assert_close(host64(A), ref, S, 1e-5, "spttv full size")
    # whole fibers per lane (schedule variant 2)
    A = spl.spttv(B, cv, sched=spl.schedule("merge", tile=8192, items_per_lane=8, variant=2))
    assert_close(host64(A), ref, S, 1e-5, "spttv full size, whole fibers per lane")
    del A, ref, S
    # the fiber-aligned non-zero split bounds on sampled tiles, each checked
    # by the oracle's preimage counts (the fiber holding position t*T, the
    # slice holding that fiber)
    for T in (2048, 65536):
        ts, tf = spl.csf_tile_bounds(B, T)
        ts, tf = ts.cpu().numpy(), tf.cpu().numpy()
        nt = len(tf) - 1
        assert nt == -(-int(h["crd2"].size) // T)
        assert (ts[-1], tf[-1]) == (I, h["crd1"].size)
        assert np.all(np.diff(tf) >= 0) and np.all(np.diff(ts) >= 0)
        for t in np.unique(np.random.RandomState(T).randint(1, nt, 12)):
            f = oracle.rows_finished_at(h["pos2"], int(t) * T)
            assert tf[t] == f, (T, t)
            assert ts[t] == oracle.rows_finished_at(h["pos1"], f), (T, t)
    # MTTKRP on sampled slices, FP32 and BF16
    rows = _sample_rows(h["pos1"], k=300, seed=3)
    C32 = c["C"].to(torch.float32)
    D32 = c["D"].to(torch.float32)
    ref32 = S32 = None
    for dt in (torch.float32, torch.bfloat16):
        Bt = B.with_vals(vals32.to(dt))
        C = C32.to(dt)
        D = D32.to(dt)
        M = spl.mttkrp(Bt, C, D)
        ref, S = oracle.mttkrp(h["pos1"], h["crd1"], h["pos2"], h["crd2"], host64(Bt.vals),
                               host64(C), host64(D), rows=rows)
        got = host64(M[torch.as_tensor(rows, device=M.device)])
        assert_close(got, ref, S, 1e-5, f"mttkrp {dt}")
        if dt == torch.float32:
            ref32, S32 = ref, S  # the FP32 inputs are the unrounded ones
        else:
            # (ii) three BF16-rounded factors per term: vals, C and D
            assert_close(got, ref32, S32, bf16_total_bound(3), "mttkrp bf16 total")
            print("mttkrp bf16 " + json.dumps(
                {"vs_bf16_inputs": oracle.error_statement(got, ref, S),
                 "vs_fp32_inputs": oracle.error_statement(got, ref32, S32)}))
    # inner product in FP64: uniform[0, 1] values, so no cancellation
    B64 = B.with_vals(c["vals"])
    C64 = B.with_vals(c["vals2"])
    a = spl.inner(B64, C64)
    ref, S = oracle.inner((h["pos1"], h["crd1"], h["pos2"], h["crd2"], c["vals"].cpu().numpy()),
                          (h["pos1"], h["crd1"], h["pos2"], h["crd2"], c["vals2"].cpu().numpy()))
    assert abs(float(a.item()) - ref) <= 1e-12 * S
    # the co-iteration path on the same coordinates held in other arrays
    Cg = spl.CSF(c["pos1"].clone(), c["crd1"].clone(), c["pos2"].clone(), c["crd2"].clone(),
                 c["vals2"], (I, J, K))
    ag = spl.inner(B64, Cg)
    assert abs(float(ag.item()) - ref) <= 1e-12 * S


def test_banded_weak_scaling_share_spmv_sampled():
    # one GPU's share of the paper's weak-scaling SpMV: 7e8 nonzeros, FP64
    spl, _ = _spl()
    c = configs.banded(device="cuda")
    n = c["n"]
    B = spl.CSR(c["pos"], c["crd"], c["vals"], (n, n))
    rs = np.random.RandomState(6)
    rows = np.unique(np.concatenate([rs.randint(0, n, 400), [0, 1, 16, 17, 18, n - 18, n - 17,
                                                              n - 2, n - 1]]))
    r = torch.as_tensor(rows, device="cuda")
    p0, p1 = c["pos"][r].long(), c["pos"][r + 1].long()
    cnt = (p1 - p0).cpu().numpy()
    idx = torch.cat([torch.arange(a, b, device="cuda") for a, b in zip(p0.tolist(), p1.tolist())])
    spos = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    ref, S = oracle.spmv(spos, c["crd"][idx].cpu().numpy(), c["vals"][idx].cpu().numpy(),
                         c["x"].cpu().numpy())
    for sc in (dict(kind="default"), dict(kind="row", lanes_per_row=32),
               dict(kind="nnz", tile=4096, items_per_lane=8)):
        y = spl.spmv(B, c["x"], sched=spl.schedule(**sc))
        assert_close(host64(y[r]), ref, S, 1e-12, f"banded spmv {sc}")


def test_spmv_int64_positions_past_2_31_sampled():
    # the banded matrix at 62,000,000 rows: 2,169,999,694 nonzeros (26 GB in
    # FP64 with int32 columns), so positions pass 2^31 and pos is int64
    spl, tuning = _spl()
    n = 62_000_000
    c = configs.banded(device="cuda", n=n, pos_dtype=torch.int64)
    nnz = int(c["crd"].numel())
    assert nnz > 2**31
    B = spl.CSR(c["pos"], c["crd"], c["vals"], (n, n))
    y = spl.spmv(B, c["x"])
    rs = np.random.RandomState(3)
    rows = np.unique(np.concatenate([rs.randint(0, n, 1500), [0, 1, n - 2, n - 1],
                                     np.arange(61_400_000, 61_400_050)]))
    pos = c["pos"].cpu().numpy()
    assert pos[rows[-1]] > 2**31
    lens = pos[rows + 1] - pos[rows]
    idx = np.concatenate([np.arange(pos[r], pos[r + 1]) for r in rows])
    it = torch.as_tensor(idx, device=c["crd"].device)
    crd_s = c["crd"][it].cpu().numpy()
    val_s = c["vals"][it].cpu().numpy()
    pos_s = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ref, S = oracle.spmv(pos_s, crd_s, val_s, c["x"].cpu().numpy())
    got = y[torch.as_tensor(rows, device=y.device)].cpu().numpy()
    assert_close(got, ref, S, 1e-12, "int64 positions, sampled rows")
    del y
    # SpMM with N = 8 on the same matrix (int64 positions, vector lanes): the
    # sampled rows' columns renumbered into a compact copy of the dense rows
    # they gather
    N = 8
    D = torch.empty(n, N, dtype=torch.float64, device="cuda")
    D.copy_(c["x"][:, None] * torch.arange(1, N + 1, dtype=torch.float64, device="cuda"))
    A = spl.spmm(B, D)
    ucols, inv = np.unique(crd_s, return_inverse=True)
    Dh = D[torch.as_tensor(ucols, device="cuda")].cpu().numpy()
    ref, S = oracle.spmm(pos_s, inv.astype(np.int32), val_s, Dh)
    got = A[torch.as_tensor(rows, device=A.device)].cpu().numpy()
    assert_close(got, ref, S, 1e-12, "SpMM with int64 positions, sampled rows")
    del A, D
    # SpTTV with int64 positions: the same arrays as the last level of a
    # (Dense, Dense, Compressed) tensor of shape (n, 1, n), whose fibers are
    # the matrix's rows
    T = spl.DDC(c["pos"], c["crd"], c["vals"], (n, 1, n))
    At = spl.spttv(T, c["x"])
    got = At[torch.as_tensor(rows, device=At.device)].cpu().numpy()
    ref, S = oracle.spmv(pos_s, crd_s, val_s, c["x"].cpu().numpy())
    assert_close(got, ref, S, 1e-12, "SpTTV with int64 positions, sampled fibers")
    del B, c, At, it, T
    torch.cuda.empty_cache()


def test_mttkrp_int64_positions_past_2_31_sampled():
    # a CSF tensor of 2,214,592,512 positions (int64 pos1 and pos2; 8.9 GB
    # each of coordinates and FP32 values): MTTKRP with R = 32 on sampled
    # slices, several of them past position 2^31
    spl, _ = _spl()
    c = configs.csf_int64(device="cuda")
    I, J, K = c["I"], c["J"], c["K"]
    assert c["crd2"].numel() > 2**31
    B = spl.CSF(c["pos1"], c["crd1"], c["pos2"], c["crd2"], c["vals"], (I, J, K))
    M = spl.mttkrp(B, c["C"], c["D"])
    rs = np.random.RandomState(9)
    rows = np.unique(np.concatenate([rs.randint(0, I, 30), [0, 1, I - 2, I - 1],
                                     np.arange(1_040_000, 1_040_008)]))
    p1 = c["pos1"].cpu().numpy()
    p2 = c["pos2"][torch.as_tensor(np.concatenate([p1[rows], p1[rows + 1]]),
                                   device="cuda")].cpu().numpy()
    assert p2[len(rows):].max() > 2**31
    # the sampled slices as a small CSF: their fibers and positions
    sp1, sc1, sp2, sc2, sv = [0], [], [0], [], []
    for r in rows:
        f0, f1 = int(p1[r]), int(p1[r + 1])
        fpos = c["pos2"][f0:f1 + 1].cpu().numpy()
        sc1.append(c["crd1"][f0:f1].cpu().numpy())
        sp2.extend((fpos[1:] - fpos[0] + sp2[-1]).tolist())
        sc2.append(c["crd2"][fpos[0]:fpos[-1]].cpu().numpy())
        sv.append(c["vals"][fpos[0]:fpos[-1]].double().cpu().numpy())
        sp1.append(sp1[-1] + f1 - f0)
    ref, S = oracle.mttkrp(np.array(sp1, np.int32), np.concatenate(sc1), np.array(sp2, np.int32),
                           np.concatenate(sc2), np.concatenate(sv), host64(c["C"]), host64(c["D"]))
    got = host64(M[torch.as_tensor(rows, device=M.device)])
    assert_close(got, ref, S, 1e-5, "MTTKRP with int64 positions, sampled slices")
    del B, M, c
    torch.cuda.empty_cache()
