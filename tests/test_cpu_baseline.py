"""Host checks of the benchmark's CPU comparison (double-precision OpenMP
SpMV/SpMM loops) and of the error statement the benchmark reports."""
import numpy as np

import oracle
from workloads import configs


def test_openmp_baseline_matches_oracle():
    c = configs.config2(scale=0.002, N=8)
    pos, crd = c["pos"].numpy(), c["crd"].numpy()
    vals, x, D = c["vals"].numpy(), c["x"].numpy(), c["B"].numpy()
    base = oracle.CpuBaseline()
    assert base.threads() >= 1
    y = np.empty(len(pos) - 1)
    A = np.empty((len(pos) - 1, D.shape[1]))
    base.spmv(pos, crd, vals, x, y)
    base.spmm(pos, crd, vals, np.ascontiguousarray(D), A)
    ref, S = oracle.spmv(pos, crd, vals, x)
    assert np.all(np.abs(y - ref) <= 1e-12 * S)
    ref, S = oracle.spmm(pos, crd, vals, D)
    assert np.all(np.abs(A - ref) <= 1e-12 * S)


def test_error_statement_values():
    ref = np.array([1.0, -2.0, 0.0, 4.0])
    S = np.array([2.0, 2.0, 0.0, 8.0])
    got = np.array([1.5, -2.0, 0.0, 3.0])
    st = oracle.error_statement(got, ref, S)
    # |err| / S over S > 0: 0.25, 0, 0.125
    assert st["max_err_over_S"] == 0.25
    assert st["median_err_over_S"] == 0.125
    assert np.isclose(st["rel_l2"], np.sqrt(0.25 + 1.0) / np.sqrt(1 + 4 + 16))
    assert st["entries"] == 4
    assert oracle.error_statement(ref, ref, S)["rel_l2"] == 0.0
