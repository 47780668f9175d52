"""GPU parity of the schedule selector's kernels against the float64
reference, and the selector's gain over the library's fixed default."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from tests import tiny
from tests.gpu_util import dev, need_gpu
from workloads import configs, corpus

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DB = os.path.join(ROOT, "paper_2207_13901_amd", "data", "autotune_db.jsonl")


def _spl():
    need_gpu()
    import paper_2207_13901_amd as spl
    from paper_2207_13901_amd import learned
    return spl, learned


def test_features_match_reference():
    spl, learned = _spl()
    mats = []
    c1 = configs.config1()
    mats.append((c1["pos"].numpy(), c1["crd"].numpy(), 4096, 4096))
    c2 = configs.config2(scale=0.005, with_dense=False)
    mats.append((c2["pos"].numpy(), c2["crd"].numpy(), c2["n"], c2["n"]))
    rs = np.random.RandomState(1)
    p, c, _ = tiny.csr(rs, 500, 300, 0.02, empty_rows=set(range(0, 500, 7)))
    mats.append((p, c, 500, 300))
    for i in (2, 3):  # a banded and a block-diagonal corpus matrix, shrunk
        s, pos, crd, _ = corpus.generate(i, "cpu", max_nnz=2e5)
        mats.append((pos.numpy(), crd.numpy(), s["n"], s["n"]))
    for pos, crd, n, m in mats:
        B = spl.CSR(torch.as_tensor(pos).to(dev()), torch.as_tensor(crd).to(dev()),
                    torch.zeros(len(crd), dtype=torch.float32, device=dev()), (n, m))
        got = learned.features(B).cpu().numpy().astype(np.float64)
        ref = mlp.features(pos, crd, m)
        np.testing.assert_allclose(got, ref, rtol=2e-6, atol=1e-6)


def _net_setup(learned, K, B, seed):
    rs = np.random.RandomState(seed)
    net = learned.Network(K, "cuda", seed)
    P = rs.normal(scale=0.3, size=net.n)
    net.P = torch.as_tensor(P.astype(np.float32), device=dev())
    P = net.P.double().cpu().numpy()  # the exact FP32 parameters
    X = rs.normal(size=(B, 7)).astype(np.float32)
    T = rs.normal(size=(B, K)).astype(np.float32)
    norm = np.concatenate([rs.normal(size=7), rs.uniform(0.5, 2.0, 7)]).astype(np.float32)
    net.norm = torch.as_tensor(norm, device=dev())
    return net, P, X, T, norm


@pytest.mark.parametrize("K,B", [(12, 37), (6, 1600), (1, 3)])
def test_forward_backward_adam_match_reference(K, B):
    spl, learned = _spl()
    net, P, X, T, norm = _net_setup(learned, K, B, K + B)
    Xt, Tt = torch.as_tensor(X, device=dev()), torch.as_tensor(T, device=dev())
    Y = net.forward(Xt).double().cpu().numpy()
    Yr, _ = mlp.forward(P, K, X.astype(np.float64), norm.astype(np.float64))
    assert np.linalg.norm(Y - Yr) <= 1e-5 * np.linalg.norm(Yr)
    loss, g = net.grad(Xt, Tt)
    lr_, gr = mlp.loss_and_grad(P, K, X.astype(np.float64), T.astype(np.float64),
                                norm.astype(np.float64))
    g = g.double().cpu().numpy()
    assert abs(float(loss.item()) - lr_) <= 1e-5 * lr_
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)
    # two Adam steps against the reference
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    Pr = P.copy()
    gt = torch.as_tensor(gr.astype(np.float32), device=dev())
    for step in (1, 2):
        net.adam(gt, 1e-3)
        Pr, m, v = mlp.adam(Pr, m, v, gr.astype(np.float32).astype(np.float64), 1e-3,
                            0.9, 0.999, 1e-8, step)
    np.testing.assert_allclose(net.P.double().cpu().numpy(), Pr, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss():
    spl, learned = _spl()
    rs = np.random.RandomState(5)
    X = rs.normal(size=(256, 7))
    times = np.exp(rs.normal(size=(256, 4)) + X[:, :1])  # depends on a feature
    sel = learned.Selector.fit("spmv", X, times, epochs=400, lr=3e-3, log_every=50)
    losses = [l for _, l in sel.history]
    assert losses[-1] < 0.5 * losses[0]


@pytest.mark.skipif(not os.path.exists(DB), reason="autotune database not collected")
def test_learned_selector_beats_fixed_default_on_held_out():
    """What the trained network gains over the library without it: held-out
    regret against exhaustive autotuning, below the regret of the library's
    fixed default schedule (the merge split)."""
    spl, learned = _spl()
    for op in ("spmv", "spmm"):
        res, _ = learned.train_and_evaluate(DB, op, count=2000, held_out=400, epochs=2000)
        assert res["learned"]["mean"] >= 0.0
        assert res["learned"]["mean"] < res["library_default"]["mean"], (op, res)


# ------------------------------------------ selection entry points of the ABI

def _csr_corpus(spl, i, max_nnz=3e5):
    from workloads import corpus as cp
    s, pos, crd, vals = cp.generate(i, dev(), max_nnz)
    return spl.CSR(pos, crd, vals.to(torch.float32), (s["n"], s["n"]))


def test_native_autotune_picks_its_fastest_candidate():
    spl, learned = _spl()
    B = _csr_corpus(spl, 1)
    n = B.shape[0]
    x = torch.ones(n, dtype=torch.float32, device=dev())
    y = torch.empty(n, dtype=torch.float32, device=dev())
    best, times = spl.autotune("spmv", B, x, y)  # the library's 12 candidates
    assert len(times) == 12 and all(t > 0 for t in times)
    assert best == spl.schedule_dict(spl.schedule(**learned.SPMV_CANDIDATES[int(np.argmin(times))]))
    C = torch.ones(n, 32, dtype=torch.float32, device=dev())
    A = torch.empty(n, 32, dtype=torch.float32, device=dev())
    cands = [dict(kind="row", col_tile=32), dict(kind="merge", tile=512, col_tile=32),
             dict(kind="nnz", tile=1024, col_tile=16)]
    best, times = spl.autotune("spmm", B, C, A, candidates=cands, reps=2)
    assert len(times) == 3 and best == spl.schedule_dict(spl.schedule(**cands[int(np.argmin(times))]))
    with pytest.raises(spl.SpleafError, match="ARG"):
        spl.autotune("spmv", B, x, y, candidates=[dict(kind="learned")])
    with pytest.raises(spl.SpleafError, match="UNSUPPORTED"):
        spl.autotune(spl._native.OP_SDDMM, B, x, y)


def _load_committed(spl, learned, op, ctx):
    d = json.load(open(os.path.join(learned.DATA_DIR, f"selector_{op}.json")))
    norm = np.concatenate([np.asarray(d["mu"]), 1.0 / np.asarray(d["sd"])])
    spl.mlp_load(op, d["candidates"], d["params"], norm, ctx=ctx)
    return learned.Selector.from_json(d), d


@pytest.mark.skipif(not os.path.exists(DB), reason="autotune database not collected")
def test_context_selector_matches_python_selector_and_learned_kind():
    spl, learned = _spl()
    ctx = spl.Context(0)
    for op in ("spmv", "spmm"):
        sel, d = _load_committed(spl, learned, op, ctx)
        cands, P, nrm = spl.mlp_save(op, ctx=ctx)
        assert cands == [spl.schedule_dict(spl.schedule(**c)) for c in d["candidates"]]
        assert np.array_equal(P, np.asarray(d["params"], dtype=np.float32))
        for i in (0, 5, 10, 15):
            B = _csr_corpus(spl, i)
            assert spl.mlp_predict(op, B, ctx=ctx) == spl.schedule_dict(spl.schedule(**sel.choose(B)))
    # SPL_SCHED_LEARNED runs the context's choice: bit-identical results
    B = _csr_corpus(spl, 7)
    n = B.shape[0]
    x = torch.linspace(-1, 1, n, dtype=torch.float32, device=dev())
    y1 = spl.spmv(B, x, sched=spl.schedule("learned"), ctx=ctx)
    y2 = spl.spmv(B, x, sched=spl.schedule(**spl.mlp_predict("spmv", B, ctx=ctx)), ctx=ctx)
    assert torch.equal(y1, y2)
    C = torch.linspace(-1, 1, n * 32, dtype=torch.float32, device=dev()).reshape(n, 32)
    A1 = spl.spmm(B, C, sched=spl.schedule("learned"), ctx=ctx)
    A2 = spl.spmm(B, C, sched=spl.schedule(**spl.mlp_predict("spmm", B, ctx=ctx)), ctx=ctx)
    assert torch.equal(A1, A2)
    # the workspace query covers every candidate the selection may pick
    need = spl.workspace_query(spl._native.OP_SPMM, B, 32, spl.schedule("learned"), ctx=ctx)
    for c in spl.mlp_save("spmm", ctx=ctx)[0]:
        assert need >= spl.workspace_query(spl._native.OP_SPMM, B, 32, spl.schedule(**c), ctx=ctx)


def test_selection_kinds_results_and_errors():
    spl, learned = _spl()
    ctx = spl.Context(0)  # fresh: no selector installed
    c2 = configs.config2(scale=0.002, N=32)
    n = c2["n"]
    B = spl.CSR(c2["pos"].to(dev()), c2["crd"].to(dev()), c2["vals"].to(dev()), (n, n))
    x = c2["x"].to(dev())
    ref, S = oracle.spmv(c2["pos"].numpy(), c2["crd"].numpy(), c2["vals"].numpy(), c2["x"].numpy())
    y = spl.spmv(B, x, sched=spl.schedule("autotune"), ctx=ctx)
    assert np.all(np.abs(y.cpu().numpy() - ref) <= 1e-12 * S)
    Cd = c2["B"].to(dev())
    refm, Sm = oracle.spmm(c2["pos"].numpy(), c2["crd"].numpy(), c2["vals"].numpy(), c2["B"].numpy())
    A = spl.spmm(B, Cd, sched=spl.schedule("autotune"), ctx=ctx)
    assert np.all(np.abs(A.cpu().numpy() - refm) <= 1e-12 * Sm)
    with pytest.raises(spl.SpleafError, match="UNSUPPORTED"):
        spl.spmv(B, x, sched=spl.schedule("learned"), ctx=ctx)
    with pytest.raises(spl.SpleafError, match="UNSUPPORTED"):
        spl.mlp_predict("spmv", B, ctx=ctx)
    with pytest.raises(spl.SpleafError, match="UNSUPPORTED"):
        spl.mlp_save("spmm", ctx=ctx)


def test_context_train_step_matches_network_steps():
    spl, learned = _spl()
    ctx = spl.Context(0)
    K, Bn = 5, 96
    rs = np.random.RandomState(3)
    net = learned.Network(K, "cuda", seed=3)
    mu, sd = rs.normal(size=7), rs.uniform(0.5, 2.0, 7)
    net.norm = torch.as_tensor(np.concatenate([mu, 1.0 / sd]).astype(np.float32), device=dev())
    cands = [dict(kind="merge", tile=256 * (k + 1)) for k in range(K)]
    spl.mlp_load("spmv", cands, net.P.cpu().numpy(), net.norm.cpu().numpy(), ctx=ctx)
    X = torch.as_tensor(rs.normal(size=(Bn, 7)).astype(np.float32), device=dev())
    T = torch.as_tensor(rs.normal(size=(Bn, K)).astype(np.float32), device=dev())
    for _ in range(5):
        loss_ctx = spl.mlp_train_step("spmv", X, T, 1e-3, ctx=ctx)
        loss_net, g = net.grad(X, T)
        net.adam(g, 1e-3)
        assert torch.equal(loss_ctx, loss_net)
    _, P, _ = spl.mlp_save("spmv", ctx=ctx)
    assert np.array_equal(P, net.P.cpu().numpy())
