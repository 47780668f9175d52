"""Learned schedule selection for SpMV and SpMM.

The selector maps the seven sparsity features of a CSR matrix (computed on
the GPU by spl_features) to, for every candidate schedule, a prediction of
log2(time / best time), and picks the candidate with the smallest
prediction.  It is trained on timings that the exhaustive autotuner records
over a seeded corpus of synthetic matrices; training (forward, backward and
Adam) and inference run in the library's own kernels.  The exhaustive
autotuner stays the fallback and the yardstick: regret = t(chosen) / t(best) - 1
per matrix, measured against it on held-out matrices.

Command line (GPU):
  python -m paper_2207_13901_amd.learned collect --count 2000 --out DB.jsonl
  python -m paper_2207_13901_amd.learned train --db DB.jsonl --out DIR
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import CSR, Context, schedule, spmm, spmv, tuning

IN = 7

SPMV_CANDIDATES = tuning.SPMV_CANDIDATES
SPMM_CANDIDATES: List[Dict] = [
    dict(kind="row", col_tile=32),
    dict(kind="nnz", tile=1024, col_tile=32, items_per_lane=16),
    dict(kind="merge", tile=256, col_tile=32, items_per_lane=8),
    dict(kind="merge", tile=512, col_tile=32, items_per_lane=16),
    dict(kind="merge", tile=1024, col_tile=32, items_per_lane=32),
    dict(kind="merge", tile=2048, col_tile=32, items_per_lane=16),
]
SPMM_COLS = 32

# What SPL_SCHED_DEFAULT resolves to for these operands (merge split, SpMV:
# 8 items per lane and one 2048-item chunk per tile; SpMM with 32 columns:
# col_tile 32, 16 items per group, four 128-item chunks per tile).
LIBRARY_DEFAULT = {
    "spmv": dict(kind="merge", tile=2048, items_per_lane=8),
    "spmm": dict(kind="merge", tile=512, col_tile=32, items_per_lane=16),
}

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def candidates(op: str) -> List[Dict]:
    return SPMV_CANDIDATES if op == "spmv" else SPMM_CANDIDATES


def features(B: CSR, ctx: Optional[Context] = None) -> torch.Tensor:
    """Seven features (float32, on B's device) computed by spl_features."""
    dev = B.vals.device
    ctx = ctx or Context.get(dev.index)
    feat = torch.empty(IN, dtype=torch.float32, device=dev)
    s = B.struct()
    stream = torch.cuda.current_stream(dev).cuda_stream
    ctx.check(ctx.lib.spl_features(ctx.h, ctypes.byref(s), feat.data_ptr(), None, 0, stream),
              "spl_features")
    return feat


class Network:
    """Parameters and optimizer state of the selector network (on GPU)."""

    def __init__(self, K: int, device="cuda", seed: int = 0):
        self.K = K
        self.dev = torch.device(device)
        self.ctx = Context.get(self.dev.index)
        self.n = int(self.ctx.lib.spl_mlp_param_count(K))
        if self.n == 0:
            raise ValueError("K must be 1..256")
        rs = np.random.RandomState(seed)
        P = np.zeros(self.n, dtype=np.float32)
        # He initialization of the three weight matrices, zero biases
        o = 0
        for fan_in, fan_out in ((IN, 64), (64, 64), (64, K)):
            w = rs.normal(scale=math.sqrt(2.0 / fan_in), size=fan_out * fan_in)
            P[o:o + w.size] = w
            o += w.size + fan_out
        self.P = torch.as_tensor(P, device=self.dev)
        self.m = torch.zeros_like(self.P)
        self.v = torch.zeros_like(self.P)
        self.step = 0
        self.norm: Optional[torch.Tensor] = None

    def _stream(self):
        return torch.cuda.current_stream(self.dev).cuda_stream

    def forward(self, X: torch.Tensor, act: Optional[torch.Tensor] = None) -> torch.Tensor:
        B = X.shape[0]
        Y = torch.empty(B, self.K, dtype=torch.float32, device=self.dev)
        norm_ptr = self.norm.data_ptr() if self.norm is not None else None
        self.ctx.check(self.ctx.lib.spl_mlp_forward(
            self.ctx.h, self.K, self.P.data_ptr(), X.data_ptr(), norm_ptr, B, Y.data_ptr(),
            act.data_ptr() if act is not None else None, self._stream()), "spl_mlp_forward")
        return Y

    def grad(self, X: torch.Tensor, T: torch.Tensor):
        """(loss tensor, gradient tensor) of the mean squared error."""
        B = X.shape[0]
        act = torch.empty((128 + IN) * B, dtype=torch.float32, device=self.dev)
        Y = self.forward(X, act)
        g = torch.empty_like(self.P)
        loss = torch.empty(1, dtype=torch.float32, device=self.dev)
        ws = torch.empty((128 + self.K + 1) * B * 4, dtype=torch.uint8, device=self.dev)
        self.ctx.check(self.ctx.lib.spl_mlp_backward(
            self.ctx.h, self.K, self.P.data_ptr(), B, Y.data_ptr(), T.data_ptr(),
            act.data_ptr(), g.data_ptr(), loss.data_ptr(), ws.data_ptr(), ws.numel(),
            self._stream()), "spl_mlp_backward")
        return loss, g

    def adam(self, g: torch.Tensor, lr: float, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        self.ctx.check(self.ctx.lib.spl_adam_step(
            self.ctx.h, self.n, self.P.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
            g.data_ptr(), lr, b1, b2, eps, self.step, self._stream()), "spl_adam_step")


def targets(times: np.ndarray) -> np.ndarray:
    """log2 slowdown of every candidate against the fastest one."""
    best = times.min(axis=1, keepdims=True)
    return np.log2(times / best)


class Selector:
    """A trained network plus its candidate list and feature scaling."""

    def __init__(self, op: str, net: Network, mu: np.ndarray, sd: np.ndarray):
        self.op = op
        self.net = net
        self.mu, self.sd = mu, sd
        net.norm = torch.as_tensor(np.concatenate([mu, 1.0 / sd]).astype(np.float32),
                                   device=net.dev)

    @staticmethod
    def fit(op: str, X: np.ndarray, times: np.ndarray, epochs: int = 3000, lr: float = 3e-3,
            seed: int = 0, device="cuda", log_every: int = 0):
        K = times.shape[1]
        mu = X.mean(0)
        sd = X.std(0) + 1e-6
        net = Network(K, device, seed)
        sel = Selector(op, net, mu, sd)
        Xt = torch.as_tensor(X.astype(np.float32), device=net.dev)
        Tt = torch.as_tensor(targets(times).astype(np.float32), device=net.dev)
        history = []
        for e in range(epochs):
            loss, g = net.grad(Xt, Tt)
            net.adam(g, lr)
            if log_every and (e % log_every == 0 or e == epochs - 1):
                history.append((e, float(loss.item())))
        sel.history = history
        return sel

    def predict_scores(self, X: np.ndarray) -> np.ndarray:
        Xt = torch.as_tensor(np.asarray(X, dtype=np.float32).reshape(-1, IN), device=self.net.dev)
        return self.net.forward(Xt).cpu().numpy()

    def choose(self, B: CSR) -> Dict:
        """Schedule for matrix B: features and network on the GPU."""
        f = features(B).reshape(1, IN)
        Y = self.net.forward(f)
        k = int(torch.argmin(Y[0]).item())
        return candidates(self.op)[k]

    def to_json(self) -> dict:
        return dict(op=self.op, K=self.net.K, params=self.net.P.cpu().tolist(),
                    mu=self.mu.tolist(), sd=self.sd.tolist(), candidates=candidates(self.op))

    @staticmethod
    def from_json(d: dict, device="cuda") -> "Selector":
        net = Network(d["K"], device)
        net.P = torch.as_tensor(np.asarray(d["params"], dtype=np.float32), device=net.dev)
        return Selector(d["op"], net, np.asarray(d["mu"]), np.asarray(d["sd"]))


def regret(times: np.ndarray, choice: np.ndarray) -> dict:
    """Regret of a choice per matrix against the fastest candidate."""
    best = times.min(axis=1)
    r = times[np.arange(len(times)), choice] / best - 1.0
    return dict(mean=float(r.mean()), geomean=float(np.exp(np.mean(np.log1p(r))) - 1.0),
                p90=float(np.percentile(r, 90)), max=float(r.max()), n=int(len(r)))


def evaluate(sel: Selector, X: np.ndarray, times: np.ndarray, train_times: np.ndarray) -> dict:
    scores = sel.predict_scores(X)
    learned = regret(times, scores.argmin(1))
    K = times.shape[1]
    cands = candidates(sel.op)
    # the best single fixed candidate, chosen on the training set
    fixed = int(np.argmin([np.mean(train_times[:, k] / train_times.min(1)) for k in range(K)]))
    # the schedule the library resolves SPL_SCHED_DEFAULT to
    lib_default = LIBRARY_DEFAULT[sel.op]
    default = next(k for k, c in enumerate(cands) if c == lib_default)
    rule_kind = "row" if sel.op == "spmv" else "nnz"
    rule = min((k for k, c in enumerate(cands) if c["kind"] == rule_kind),
               key=lambda k: np.mean(train_times[:, k] / train_times.min(1)))
    return dict(
        learned=learned,
        best_fixed_on_train=dict(candidate=cands[fixed], **regret(times, np.full(len(times), fixed))),
        library_default=dict(candidate=cands[default], **regret(times, np.full(len(times), default))),
        paper_rule=dict(candidate=cands[rule], **regret(times, np.full(len(times), rule))),
        per_candidate={json.dumps(c, sort_keys=True): regret(times, np.full(len(times), k))["mean"]
                       for k, c in enumerate(cands)},
    )


# ----------------------------------------------------------------- collect

def collect(ids, out_path: str, device="cuda", reps: int = 5, max_nnz: float = 1e8,
            with_spmm: bool = True) -> None:
    """Append one JSON line per matrix: spec, features and the measured time
    of every SpMV (and SpMM) candidate.  Ids already in the file are skipped,
    so collection resumes after an interruption."""
    from workloads import corpus
    done = set()
    if os.path.exists(out_path):
        with open(out_path) as f:
            done = {json.loads(l)["id"] for l in f if l.strip()}
    dev = torch.device(device)
    t0 = time.time()
    last = t0
    with open(out_path, "a") as out:
        for count, i in enumerate(ids):
            if i in done:
                continue
            s, pos, crd, vals = corpus.generate(i, dev, max_nnz)
            n = s["n"]
            B = CSR(pos, crd, vals, (n, n))
            x = torch.ones(n, dtype=torch.float32, device=dev)
            y = torch.empty(n, dtype=torch.float32, device=dev)
            row = dict(s, feat=features(B).cpu().tolist())
            row["spmv_ms"] = [
                tuning.time_call(lambda sc=schedule(**c): spmv(B, x, y, sched=sc), reps=reps)
                for c in SPMV_CANDIDATES]
            if with_spmm:
                D = torch.ones(n, SPMM_COLS, dtype=torch.float32, device=dev)
                A = torch.empty(n, SPMM_COLS, dtype=torch.float32, device=dev)
                row["spmm_ms"] = [
                    tuning.time_call(lambda sc=schedule(**c): spmm(B, D, A, sched=sc), reps=reps)
                    for c in SPMM_CANDIDATES]
                del D, A
            out.write(json.dumps(row) + "\n")
            out.flush()
            del B, pos, crd, vals, x, y
            if time.time() - last > 30:
                last = time.time()
                print(f"[collect] {count + 1}/{len(ids)} matrices, {last - t0:.0f}s",
                      flush=True)


def load_db(path: str, op: str):
    rows = [json.loads(l) for l in open(path) if l.strip()]
    key = f"{op}_ms"
    rows = [r for r in rows if key in r]
    ids = np.array([r["id"] for r in rows])
    X = np.array([r["feat"] for r in rows], dtype=np.float64)
    T = np.array([r[key] for r in rows], dtype=np.float64)
    return ids, X, T, rows


def train_and_evaluate(db: str, op: str, count: int, held_out: int, epochs: int = 3000,
                       lr: float = 3e-3, device="cuda") -> dict:
    from workloads import corpus
    ids, X, T, _ = load_db(db, op)
    train_ids, test_ids = corpus.split(count, held_out)
    tr = np.isin(ids, train_ids)
    te = np.isin(ids, test_ids)
    sel = Selector.fit(op, X[tr], T[tr], epochs=epochs, lr=lr, device=device,
                       log_every=max(1, epochs // 10))
    res = evaluate(sel, X[te], T[te], T[tr])
    res["train_loss"] = sel.history
    res["train_matrices"] = int(tr.sum())
    res["held_out_matrices"] = int(te.sum())
    res["learned_on_train"] = regret(T[tr], sel.predict_scores(X[tr]).argmin(1))
    return res, sel


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--start", type=int, default=0)
    c.add_argument("--count", type=int, default=2000)
    c.add_argument("--out", required=True)
    c.add_argument("--max-nnz", type=float, default=1e8)
    c.add_argument("--no-spmm", action="store_true")
    t = sub.add_parser("train")
    t.add_argument("--db", required=True)
    t.add_argument("--count", type=int, default=2000)
    t.add_argument("--held-out", type=int, default=400)
    t.add_argument("--epochs", type=int, default=3000)
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if a.cmd == "collect":
        collect(range(a.start, a.start + a.count), a.out, max_nnz=a.max_nnz,
                with_spmm=not a.no_spmm)
    else:
        os.makedirs(a.out, exist_ok=True)
        report = {}
        for op in ("spmv", "spmm"):
            res, sel = train_and_evaluate(a.db, op, a.count, a.held_out, epochs=a.epochs)
            report[op] = res
            with open(os.path.join(a.out, f"selector_{op}.json"), "w") as f:
                json.dump(sel.to_json(), f)
            print(f"[train] {op}: learned {res['learned']} default {res['library_default']}",
                  flush=True)
        with open(os.path.join(a.out, "regret.json"), "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
