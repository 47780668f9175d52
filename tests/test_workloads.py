"""The seeded workload generators keep the structure their recipes state
(CPU, small scale): exact totals, caps, distinct sorted coordinates, the
shared-row overlap of the SpAdd3 operands, the banded pattern, and
counter-based (prefix-stable) random streams."""
import numpy as np
import torch

from workloads import configs, gen


def _rows_distinct_sorted(pos, crd, m):
    for i in range(len(pos) - 1):
        r = crd[pos[i]:pos[i + 1]]
        assert np.all(np.diff(r) > 0), i
        assert r.size == 0 or (r[0] >= 0 and r[-1] < m), i


def test_counter_based_streams_are_prefix_stable():
    k = gen.key_for(2, 2)
    a = gen.values(k, 1000)
    b = gen.values(k, 37)
    assert torch.equal(a[:37], b)
    u = gen.uniform(k, torch.arange(1000, dtype=torch.int64))
    assert float(u.min()) >= 0.0 and float(u.max()) < 1.0
    assert abs(float(u.mean()) - 0.5) < 0.05


def test_powerlaw_matrix_exact_total_and_cap():
    c = configs.config2(scale=0.01, with_dense=False)
    pos, crd = c["pos"].numpy(), c["crd"].numpy()
    deg = np.diff(pos)
    assert pos[-1] == 16 * c["n"]
    assert deg.max() == c["cap"]
    assert deg.min() >= 1
    _rows_distinct_sorted(pos, crd, c["n"])


def test_spadd3_operands_share_thirty_percent_of_rows():
    c = configs.config3(scale=0.01, with_dense=False)
    n = c["n"]
    shared = c["shared"]
    assert abs(shared.mean() - 0.3) < 0.05
    mats = [(c[k]["pos"].numpy(), c[k]["crd"].numpy()) for k in "BCD"]
    for pos, crd in mats:
        _rows_distinct_sorted(pos, crd, n)
        assert abs(pos[-1] / n - 8.0) < 0.5
    (pb, cb), (pc, cc), (pd, cd) = mats
    for i in np.nonzero(shared)[0][:200]:
        rb = cb[pb[i]:pb[i + 1]]
        assert np.array_equal(rb, cc[pc[i]:pc[i + 1]]) and np.array_equal(rb, cd[pd[i]:pd[i + 1]])


def test_csf_tensor_exact_nonzeros_and_distinct_fibers():
    c = configs.config4(scale=0.001, with_dense=False)
    pos1, crd1 = c["pos1"].numpy(), c["crd1"].numpy()
    pos2, crd2 = c["pos2"].numpy(), c["crd2"].numpy()
    assert pos2[-1] == int(round(1e8 * 0.001))
    _rows_distinct_sorted(pos1, crd1, c["J"])
    _rows_distinct_sorted(pos2, crd2, c["K"])
    assert np.all(np.diff(pos2) >= 1)  # every fiber holds a value


def test_banded_pattern():
    n, w = 1000, 17
    c = configs.banded(n=n, half_width=w)
    pos, crd = c["pos"].numpy(), c["crd"].numpy()
    assert pos[-1] == n * (2 * w + 1) - w * (w + 1)
    for i in (0, 1, w, w + 1, 500, n - w - 1, n - 1):
        assert list(crd[pos[i]:pos[i + 1]]) == list(range(max(0, i - w), min(n - 1, i + w) + 1))
    assert c["vals"].dtype == torch.float64 and c["x"].numel() == n


def test_ddc_tensor_exact_nonzeros_and_layout():
    c = configs.ddc(scale=0.001, with_dense=False)
    I, J, K = c["I"], c["J"], c["K"]
    pos2, crd2 = c["pos2"].numpy(), c["crd2"].numpy()
    assert pos2.size == I * J + 1 and pos2[0] == 0
    assert pos2[-1] == int(round(1e8 * 0.001)) == crd2.size
    _rows_distinct_sorted(pos2, crd2, K)
    per_slice = pos2[np.arange(1, I + 1) * J] - pos2[np.arange(I) * J]
    assert per_slice.max() - per_slice.min() <= 1
