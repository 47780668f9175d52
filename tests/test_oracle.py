"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

The oracle's loops are checked against (a) dense numpy.einsum on the same
index-notation statements (an independent evaluator), (b) closed forms such as
identity and permutation matrices and unit vectors, (c) invariants such as
commutativity and linearity, and (d) the image/preimage definitions of
Sec. III-A evaluated by brute force over sets.  Small-integer values make
every sum exact, so those comparisons are bit-exact.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from tests import tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SEEDS = range(40)


def close(a, b, S, rtol=1e-15):
    """Normwise-per-entry comparison |a-b| <= rtol*S (+ exact when S == 0)."""
    a, b, S = np.asarray(a), np.asarray(b), np.asarray(S)
    assert a.shape == b.shape
    assert np.all(np.abs(a - b) <= rtol * S + 1e-300), np.max(np.abs(a - b) - rtol * S)


# ----------------------------------------------------------------- SpMV ----

@pytest.mark.parametrize("seed", SEEDS)
def test_spmv_matches_einsum(seed):
    rs = np.random.RandomState(seed)
    n, m = rs.randint(1, 30), rs.randint(1, 30)
    pos, crd, vals = tiny.csr(rs, n, m, rs.uniform(0, 1), empty_rows={0, n - 1})
    x = rs.uniform(-1, 1, m)
    a, S = oracle.spmv(pos, crd, vals, x)
    Bd, _ = brute.dense_csr(pos, crd, vals, (n, m))
    close(a, brute.spmv(Bd, x), S, 1e-14)
    np.testing.assert_allclose(S, brute.spmv(np.abs(Bd), np.abs(x)), rtol=1e-14)


@pytest.mark.parametrize("seed", range(10))
def test_spmv_integer_values_bit_exact(seed):
    rs = np.random.RandomState(100 + seed)
    pos, crd, vals = tiny.csr(rs, 25, 31, 0.4, empty_rows={3}, full_rows={7},
                              kind="int")
    x = rs.randint(-4, 5, 31).astype(np.float64)
    a, _ = oracle.spmv(pos, crd, vals, x)
    Bd, _ = brute.dense_csr(pos, crd, vals, (25, 31))
    assert np.array_equal(a, Bd @ x)


def test_spmv_identity_permutation_unit_vectors():
    rs = np.random.RandomState(7)
    n = 50
    x = rs.uniform(-1, 1, n)
    ident = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
             np.ones(n))
    assert np.array_equal(oracle.spmv(*ident, x)[0], x)
    perm = rs.permutation(n).astype(np.int32)
    P = (np.arange(n + 1, dtype=np.int32), perm, np.ones(n))
    assert np.array_equal(oracle.spmv(*P, x)[0], x[perm])
    pos, crd, vals = tiny.csr(rs, n, n, 0.2)
    Bd, _ = brute.dense_csr(pos, crd, vals, (n, n))
    for j in (0, 13, n - 1):
        e = np.zeros(n)
        e[j] = 1.0
        assert np.array_equal(oracle.spmv(pos, crd, vals, e)[0], Bd[:, j])
    ones = oracle.spmv(pos, crd, vals, np.ones(n))[0]
    np.testing.assert_allclose(ones, Bd.sum(1), rtol=1e-14, atol=1e-15)


def test_spmv_empty_and_row_subset():
    pos = np.zeros(5, dtype=np.int32)
    a, S = oracle.spmv(pos, np.zeros(0, np.int32), np.zeros(0), np.ones(3))
    assert np.array_equal(a, np.zeros(4)) and np.array_equal(S, np.zeros(4))
    rs = np.random.RandomState(3)
    pos, crd, vals = tiny.csr(rs, 20, 20, 0.3)
    x = rs.uniform(-1, 1, 20)
    full, _ = oracle.spmv(pos, crd, vals, x)
    rows = np.array([19, 0, 5, 5])
    sub, _ = oracle.spmv(pos, crd, vals, x, rows=rows)
    assert np.array_equal(sub, full[rows])


def test_spmv_linearity():
    rs = np.random.RandomState(11)
    pos, crd, vals = tiny.csr(rs, 40, 40, 0.3)
    x1, x2 = rs.uniform(-1, 1, 40), rs.uniform(-1, 1, 40)
    a1, S1 = oracle.spmv(pos, crd, vals, x1)
    a2, S2 = oracle.spmv(pos, crd, vals, x2)
    a12, _ = oracle.spmv(pos, crd, vals, 2.0 * x1 - 3.0 * x2)
    close(a12, 2 * a1 - 3 * a2, 2 * S1 + 3 * S2, 1e-14)


# ----------------------------------------------------------------- SpMM ----

@pytest.mark.parametrize("seed", range(20))
def test_spmm_matches_einsum_and_columns(seed):
    rs = np.random.RandomState(200 + seed)
    n, m, N = rs.randint(1, 25), rs.randint(1, 25), rs.randint(1, 9)
    pos, crd, vals = tiny.csr(rs, n, m, rs.uniform(0, 1), empty_rows={n // 2})
    C = rs.uniform(-1, 1, (m, N))
    A, S = oracle.spmm(pos, crd, vals, C)
    Bd, _ = brute.dense_csr(pos, crd, vals, (n, m))
    close(A, brute.spmm(Bd, C), S, 1e-14)
    for j in range(N):
        assert np.array_equal(A[:, j], oracle.spmv(pos, crd, vals, C[:, j])[0])


def test_spmm_identity_operand_gives_dense():
    rs = np.random.RandomState(5)
    pos, crd, vals = tiny.csr(rs, 12, 9, 0.5)
    A, _ = oracle.spmm(pos, crd, vals, np.eye(9))
    Bd, _ = brute.dense_csr(pos, crd, vals, (12, 9))
    assert np.array_equal(A, Bd)
    rows = np.array([11, 2])
    sub, _ = oracle.spmm(pos, crd, vals, np.eye(9), rows=rows)
    assert np.array_equal(sub, Bd[rows])


# --------------------------------------------------------------- SpAdd3 ----

def _dense_union(ops, shape):
    dens = [brute.dense_csr(*o, shape) for o in ops]
    return brute.spadd3(dens[0][0], dens[0][1], dens[1][0], dens[1][1],
                        dens[2][0], dens[2][1])


@pytest.mark.parametrize("seed", range(30))
def test_spadd3_matches_dense_union(seed):
    rs = np.random.RandomState(300 + seed)
    n, m = rs.randint(1, 20), rs.randint(1, 20)
    ops = [tiny.csr(rs, n, m, rs.uniform(0, 0.7), empty_rows={0}) for _ in range(3)]
    pos, crd, vals, S, nnz = oracle.spadd3(*ops)
    assert pos[-1] == nnz == len(crd)
    Vd, Md = _dense_union(ops, (n, m))
    assert nnz == Md.sum()
    for i in range(n):
        cols = crd[pos[i]:pos[i + 1]]
        assert np.array_equal(cols, np.nonzero(Md[i])[0])
        close(vals[pos[i]:pos[i + 1]], Vd[i, cols], S[pos[i]:pos[i + 1]], 1e-15)


def test_spadd3_invariants():
    rs = np.random.RandomState(9)
    n, m = 30, 25
    B, C, D = (tiny.csr(rs, n, m, 0.3) for _ in range(3))
    ref = oracle.spadd3(B, C, D)
    for perm in ((C, B, D), (D, C, B), (B, D, C)):
        got = oracle.spadd3(*perm)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        close(got[2], ref[2], ref[3], 1e-15)
    # B + C is C + B bit for bit in IEEE arithmetic
    assert np.array_equal(oracle.spadd3(C, B, D)[2], ref[2])
    empty = (np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    pos, crd, vals, _, _ = oracle.spadd3(B, empty, empty)
    assert np.array_equal(pos, B[0]) and np.array_equal(crd, B[1])
    assert np.array_equal(vals, B[2])
    pos3, crd3, vals3, _, _ = oracle.spadd3(B, B, B)
    assert np.array_equal(pos3, B[0]) and np.array_equal(crd3, B[1])
    np.testing.assert_allclose(vals3, 3 * B[2], rtol=1e-15)
    # cancellation keeps the coordinate (structural union)
    negB = (B[0], B[1], -B[2])
    pos0, crd0, vals0, _, _ = oracle.spadd3(B, negB, empty)
    assert np.array_equal(crd0, B[1]) and np.all(vals0 == 0.0)


# ---------------------------------------------------------------- SDDMM ----

@pytest.mark.parametrize("seed", range(20))
def test_sddmm_matches_einsum(seed):
    rs = np.random.RandomState(400 + seed)
    n, m, K = rs.randint(1, 20), rs.randint(1, 20), rs.randint(1, 12)
    pos, crd, vals = tiny.csr(rs, n, m, rs.uniform(0, 1))
    C, D = rs.uniform(-1, 1, (n, K)), rs.uniform(-1, 1, (m, K))
    A, S = oracle.sddmm(pos, crd, vals, C, D)
    Bd, Bm = brute.dense_csr(pos, crd, vals, (n, m))
    ref = brute.sddmm(Bd, C, D)
    rows = np.repeat(np.arange(n), np.diff(pos))
    close(A, ref[rows, crd], S, 1e-14)
    # full pattern: A = B o (C D^T) computed as a GEMM
    posf, crdf, valsf = tiny.csr(rs, n, m, 1.0)
    Af, Sf = oracle.sddmm(posf, crdf, valsf, C, D)
    Bdf, _ = brute.dense_csr(posf, crdf, valsf, (n, m))
    close(Af, (Bdf * (C @ D.T)).ravel(), Sf, 1e-14)


def test_sddmm_unit_factors():
    rs = np.random.RandomState(4)
    pos, crd, vals = tiny.csr(rs, 15, 17, 0.4)
    A, _ = oracle.sddmm(pos, crd, vals, np.ones((15, 1)), np.ones((17, 1)))
    assert np.array_equal(A, vals)


# ----------------------------------------------------------- CSF kernels ---

@pytest.mark.parametrize("seed", range(20))
def test_spttv_mttkrp_inner_match_einsum(seed):
    rs = np.random.RandomState(500 + seed)
    I, J, K, R = rs.randint(1, 8), rs.randint(1, 8), rs.randint(1, 8), rs.randint(1, 6)
    p1, c1, p2, c2, v = tiny.csf(rs, I, J, K, rs.uniform(0.05, 1), empty_slices={0})
    Td, Tm = brute.dense_csf(p1, c1, p2, c2, v, (I, J, K))
    c = rs.uniform(-1, 1, K)
    A, S = oracle.spttv(p1, p2, c2, v, c)
    ref = brute.spttv(Td, c)
    fib_i = np.repeat(np.arange(I), np.diff(p1))
    close(A, ref[fib_i, c1], S, 1e-14)
    Cf, Df = rs.uniform(-1, 1, (J, R)), rs.uniform(-1, 1, (K, R))
    M, SM = oracle.mttkrp(p1, c1, p2, c2, v, Cf, Df)
    close(M, brute.mttkrp(Td, Cf, Df), SM, 1e-14)
    v2 = rs.uniform(-1, 1, len(v))
    a, Sa = oracle.inner((p1, c1, p2, c2, v), (p1, c1, p2, c2, v2))
    close(np.array([a]), np.array([np.dot(v, v2)]), np.array([Sa]), 1e-14)
    # different patterns: the co-iteration keeps only shared coordinates
    q1, d1, q2, d2, w = tiny.csf(rs, I, J, K, rs.uniform(0.05, 1))
    Ud, _ = brute.dense_csf(q1, d1, q2, d2, w, (I, J, K))
    a2, Sa2 = oracle.inner((p1, c1, p2, c2, v), (q1, d1, q2, d2, w))
    close(np.array([a2]), np.array([brute.inner(Td, Ud)]), np.array([Sa2]), 1e-14)


def test_csf_closed_forms():
    rs = np.random.RandomState(8)
    I, J, K = 6, 7, 9
    p1, c1, p2, c2, v = tiny.csf(rs, I, J, K, 0.4)
    Td, _ = brute.dense_csf(p1, c1, p2, c2, v, (I, J, K))
    fib_i = np.repeat(np.arange(I), np.diff(p1))
    for k in (0, 4, K - 1):
        e = np.zeros(K)
        e[k] = 1.0
        A, _ = oracle.spttv(p1, p2, c2, v, e)
        assert np.array_equal(A, Td[fib_i, c1, k])
    M, _ = oracle.mttkrp(p1, c1, p2, c2, v, np.ones((J, 1)), np.ones((K, 1)))
    np.testing.assert_allclose(M[:, 0], Td.sum(axis=(1, 2)), rtol=1e-14, atol=1e-15)
    a, _ = oracle.inner((p1, c1, p2, c2, v), (p1, c1, p2, c2, v))
    assert a >= 0 and abs(a - np.sum(Td * Td)) <= 1e-14 * a
    # linearity of MTTKRP in a factor
    C1, C2, D = rs.uniform(-1, 1, (J, 3)), rs.uniform(-1, 1, (J, 3)), rs.uniform(-1, 1, (K, 3))
    M1, S1 = oracle.mttkrp(p1, c1, p2, c2, v, C1, D)
    M2, S2 = oracle.mttkrp(p1, c1, p2, c2, v, C2, D)
    M12, _ = oracle.mttkrp(p1, c1, p2, c2, v, C1 + C2, D)
    close(M12, M1 + M2, S1 + S2, 1e-14)


def test_inner_order2():
    rs = np.random.RandomState(12)
    B = tiny.csr(rs, 10, 12, 0.4)
    C = tiny.csr(rs, 10, 12, 0.4)
    Bd, _ = brute.dense_csr(*B, (10, 12))
    Cd, _ = brute.dense_csr(*C, (10, 12))
    a, S = oracle.inner((B[0], B[1], None, None, B[2]), (C[0], C[1], None, None, C[2]))
    close(np.array([a]), np.array([brute.inner(Bd, Cd)]), np.array([S]), 1e-14)


# ------------------------------------ value-range partition of a level ----

@pytest.mark.parametrize("seed", range(12))
def test_coord_partition_is_the_preimage_of_value_ranges(seed):
    rs = np.random.RandomState(1300 + seed)
    n, m = rs.randint(1, 30), rs.randint(1, 40)
    pos, crd, vals = tiny.csr(rs, n, m, rs.uniform(0.0, 0.8), empty_rows={0})
    ncolors = rs.randint(1, 6)
    inner = np.sort(rs.randint(-3, m + 4, ncolors - 1))
    bounds = np.concatenate([[rs.randint(-2, 1)], inner, [m + rs.randint(0, 3)]]).astype(np.int32)
    out = oracle.coord_partition(pos, crd, bounds)
    assert out.shape == (ncolors + 1, n)
    for i in range(n):
        for c in range(ncolors):
            want = {p for p in range(pos[i], pos[i + 1]) if bounds[c] <= crd[p] < bounds[c + 1]}
            assert set(range(out[c, i], out[c + 1, i])) == want, (i, c)
    # the colors cover every stored coordinate once
    assert np.array_equal(out[0], pos[:-1]) and np.array_equal(out[-1], pos[1:])


def test_coord_partition_windows_sum_to_spmv():
    rs = np.random.RandomState(77)
    n, m = 40, 64
    pos, crd, vals = tiny.csr(rs, n, m, 0.3, empty_rows={3, 39}, full_rows={5}, kind="int")
    x = rs.randint(-3, 4, m).astype(np.float64)
    bounds = np.array([0, 10, 10, 33, 50, 64], dtype=np.int32)  # one empty color
    out = oracle.coord_partition(pos, crd, bounds)
    total = np.zeros(n)
    Bd, _ = brute.dense_csr(pos, crd, vals, (n, m))
    for c in range(len(bounds) - 1):
        a, _ = oracle.spmv_window(out[c], out[c + 1], crd, vals, x)
        # the window of color c is B's column block [bounds[c], bounds[c+1])
        blk = np.zeros_like(Bd)
        blk[:, bounds[c]:bounds[c + 1]] = Bd[:, bounds[c]:bounds[c + 1]]
        assert np.array_equal(a, brute.spmv(blk, x))
        total += a
    y, _ = oracle.spmv(pos, crd, vals, x)
    assert np.array_equal(total, y)
    # one color over all columns is the whole row
    one = oracle.coord_partition(pos, crd, np.array([0, m], dtype=np.int32))
    a, _ = oracle.spmv_window(one[0], one[1], crd, vals, x)
    assert np.array_equal(a, y)


# ------------------------------------- (Dense, Dense, Compressed) tensors --

@pytest.mark.parametrize("seed", range(12))
def test_ddc_kernels_match_einsum(seed):
    rs = np.random.RandomState(900 + seed)
    I, J, K, R = rs.randint(1, 6), rs.randint(1, 6), rs.randint(1, 7), rs.randint(1, 5)
    p2, c2, v = tiny.ddc(rs, I, J, K, rs.uniform(0.05, 0.9))
    Td, _ = brute.dense_ddc(p2, c2, v, (I, J, K))
    c = rs.uniform(-1, 1, K)
    A, S = oracle.spttv_ddc(I, J, p2, c2, v, c)
    close(A, brute.spttv(Td, c).reshape(-1), S, 1e-14)
    Cf, Df = rs.uniform(-1, 1, (J, R)), rs.uniform(-1, 1, (K, R))
    M, SM = oracle.mttkrp_ddc(I, J, p2, c2, v, Cf, Df)
    close(M, brute.mttkrp(Td, Cf, Df), SM, 1e-14)
    rows = np.array([I - 1, 0], dtype=np.int64)
    Mr, _ = oracle.mttkrp_ddc(I, J, p2, c2, v, Cf, Df, rows=rows)
    assert np.array_equal(Mr, M[rows])
    # inner products: DDC with DDC, DDC with CSF (both orders), CSF with CSF
    q2, d2, w = tiny.ddc(rs, I, J, K, rs.uniform(0.05, 0.9))
    Ud, _ = brute.dense_ddc(q2, d2, w, (I, J, K))
    ref = brute.inner(Td, Ud)
    a, Sa = oracle.inner3(I, J, (None, None, p2, c2, v), (None, None, q2, d2, w))
    close(np.array([a]), np.array([ref]), np.array([Sa]), 1e-14)
    e1, f1, e2, f2 = tiny.ddc_to_csf(q2, d2, I, J)
    a, Sa = oracle.inner3(I, J, (None, None, p2, c2, v), (e1, f1, e2, f2, w))
    close(np.array([a]), np.array([ref]), np.array([Sa]), 1e-14)
    a, Sa = oracle.inner3(I, J, (e1, f1, e2, f2, w), (None, None, p2, c2, v))
    close(np.array([a]), np.array([ref]), np.array([Sa]), 1e-14)
    b1, g1, b2, g2 = tiny.ddc_to_csf(p2, c2, I, J)
    a, Sa = oracle.inner3(I, J, (b1, g1, b2, g2, v), (e1, f1, e2, f2, w))
    close(np.array([a]), np.array([ref]), np.array([Sa]), 1e-14)


def test_ddc_reduces_to_csr_and_csf():
    rs = np.random.RandomState(31)
    I, J, K = 4, 5, 9
    p2, c2, v = tiny.ddc(rs, I, J, K, 0.35, kind="int")
    # integer values: every sum is exact, so the results match bit for bit
    c = rs.randint(-3, 4, K).astype(np.float64)
    A, _ = oracle.spttv_ddc(I, J, p2, c2, v, c)
    # as a CSR matrix of I*J rows (the Dense levels fused), SpTTV is SpMV
    y, _ = oracle.spmv(p2, c2, v, c)
    assert np.array_equal(A, y)
    # as CSF with the empty fibers dropped: the CSF oracle on the fibers kept
    q1, d1, q2, d2 = tiny.ddc_to_csf(p2, c2, I, J)
    Af, _ = oracle.spttv(q1, q2, d2, v, c)
    fib = np.repeat(np.arange(I), np.diff(q1)) * J + d1
    assert np.array_equal(A[fib], Af)
    empty = np.setdiff1d(np.arange(I * J), fib)
    assert np.all(A[empty] == 0.0)
    Cf, Df = rs.randint(-2, 3, (J, 3)).astype(float), rs.randint(-2, 3, (K, 3)).astype(float)
    M, _ = oracle.mttkrp_ddc(I, J, p2, c2, v, Cf, Df)
    Mf, _ = oracle.mttkrp(q1, d1, q2, d2, v, Cf, Df)
    assert np.array_equal(M, Mf)


# ------------------------------------------------------- partition math ----

def image(pos, src_rows):
    """Sec. III-A: every destination named by a colored source gets the color."""
    out = set()
    for i in src_rows:
        out |= set(range(pos[i], pos[i + 1]))
    return out


def preimage(pos, dst_positions):
    """Sec. III-A: every source naming a colored destination gets the color."""
    return {i for i in range(len(pos) - 1)
            if set(range(pos[i], pos[i + 1])) & set(dst_positions)}


def test_golden_image_fig6a():
    g = json.load(open(os.path.join(GOLDEN, "image_fig6a.json")))
    pos = g["pos_half_open"]
    for i, s in enumerate(g["source_sets"]):
        assert list(range(pos[i], pos[i + 1])) == s
    for color, rows in g["source_colors"].items():
        assert sorted(image(pos, rows)) == g["expected_image"][color]
    tr, tp = oracle.row_split(np.array(pos, np.int32), 1)
    assert list(range(tp[0], tp[1])) == g["expected_image"]["red"]


def test_golden_preimage_fig5b():
    g = json.load(open(os.path.join(GOLDEN, "preimage_fig5b.json")))
    pos = np.array(g["pos_half_open"], np.int32)
    nnz = int(pos[-1])
    T = -(-nnz // g["pieces"])
    tr, tp = oracle.nnz_split(pos, T)
    ranges = [[int(tp[t]), int(tp[t + 1])] for t in range(len(tp) - 1)]
    assert ranges == g["expected_position_ranges"]
    for t, (p0, p1) in enumerate(ranges):
        assert sorted(preimage(pos, range(p0, p1))) == g["expected_preimage_rows"][t]


def _check_split(pos, tr, tp, kind, size):
    n = len(pos) - 1
    nnz = int(pos[-1])
    nt = len(tr) - 1
    assert tr[0] == 0 and tp[0] == 0 and tr[-1] == n and tp[-1] == nnz
    assert np.all(np.diff(tr) >= 0) and np.all(np.diff(tp) >= 0)
    finished = set()
    for t in range(nt):
        # positions of tile t are disjoint from the others and cover [0, nnz)
        p0, p1 = int(tp[t]), int(tp[t + 1])
        rows = set(range(tr[t], tr[t + 1]))
        finished |= rows
        # every row finished in tile t ends inside (p0, p1], or at p0 == 0
        for i in rows:
            end = int(pos[i + 1])
            assert (p0 < end <= p1) or (end <= p0 and (t == 0 or end == p0) and end <= p1)
        # rows named by positions of the tile (preimage) lie in
        # [tr[t], tr[t+1]]: finished here, or continued to a later tile
        pre = preimage(pos, range(p0, p1))
        assert pre <= set(range(tr[t], tr[t + 1] + 1))
        if kind == "nnz":
            assert p0 == min(t * size, nnz)
        if kind == "merge":
            assert tr[t] + tp[t] == min(t * size, n + nnz)
        if kind == "row":
            assert tr[t] == min(t * size, n)
            assert sorted(image(pos, rows)) == list(range(p0, p1))
    assert finished == set(range(n))


@pytest.mark.parametrize("seed", range(25))
def test_splits_against_set_definitions(seed):
    rs = np.random.RandomState(600 + seed)
    n = rs.randint(1, 40)
    empty = set(rs.choice(n, size=rs.randint(0, n), replace=False).tolist())
    pos, crd, vals = tiny.csr(rs, n, 30, rs.uniform(0, 0.6), empty_rows=empty)
    for T in (1, 2, 3, 7, 64):
        _check_split(pos, *oracle.nnz_split(pos, T), "nnz", T)
        _check_split(pos, *oracle.merge_split(pos, T), "merge", T)
        _check_split(pos, *oracle.row_split(pos, T), "row", T)


@pytest.mark.parametrize("seed", range(10))
def test_pieces_reassemble_whole_spmv(seed):
    """P pieces of a split, each summing only its own positions, plus the
    carried partial rows, give the whole product (Sec. II-D: the non-zero
    algorithm reduces boundary rows into the output)."""
    rs = np.random.RandomState(700 + seed)
    n = rs.randint(1, 50)
    pos, crd, vals = tiny.csr(rs, n, 20, rs.uniform(0, 0.8),
                              empty_rows=set(range(0, n, 5)), kind="int")
    x = rs.randint(-4, 5, 20).astype(np.float64)
    whole, _ = oracle.spmv(pos, crd, vals, x)
    prod = vals * x[crd]
    for split, size in ((oracle.nnz_split, 4), (oracle.merge_split, 5),
                        (oracle.row_split, 3)):
        tr, tp = split(pos, size)
        y = np.full(n, np.nan)
        carries = {}
        for t in range(len(tr) - 1):
            p0, p1 = tp[t], tp[t + 1]
            for i in range(tr[t], tr[t + 1]):      # rows finished in tile t
                lo, hi = max(pos[i], p0), pos[i + 1]
                y[i] = prod[lo:hi].sum()
            r = tr[t + 1]                           # row still open at p1
            if r < n and p1 > max(pos[r], p0):
                carries[r] = carries.get(r, 0.0) + prod[max(pos[r], p0):p1].sum()
        for r, v in carries.items():
            y[r] += v
        assert np.array_equal(y, whole)


def _owner(pos):
    """owner[q] = the parent entry whose segment [pos[e], pos[e+1]) holds
    child q: the expansion of a Compressed level, written independently of
    the counting the split functions do."""
    owner = np.full(int(pos[-1]), -1, np.int64)
    for e in range(len(pos) - 1):
        owner[int(pos[e]):int(pos[e + 1])] = e
    return owner


@pytest.mark.parametrize("seed", range(12))
def test_csf_split_against_set_definitions(seed):
    """The fused (i,j,k) non-zero partition of a CSF tensor (Sec. II-B
    fusion, then blocks of T positions), snapped to fibers and carried to
    slices (Sec. III-A image and preimage, Table I), checked against the
    set definitions by brute force: the boundary of block t is the first
    position of the fiber that holds position t*T, and its slice is the
    slice that holds that fiber; the tiles' positions partition [0, nnz)
    into whole fibers; the fibers and slices named by a tile's positions
    (preimages) lie in its own range."""
    rs = np.random.RandomState(900 + seed)
    I, J, K = int(rs.randint(1, 12)), int(rs.randint(1, 7)), int(rs.randint(1, 40))
    empty = set(rs.choice(I, size=rs.randint(0, I), replace=False).tolist())
    p1, c1, p2, c2, v = tiny.csf(rs, I, J, K, rs.uniform(0.05, 0.9), empty_slices=empty)
    F, nnz = int(p1[-1]), int(p2[-1])
    fib_of = _owner(p2)     # position -> fiber
    sl_of = _owner(p1)      # fiber -> slice
    for T in sorted({1, 2, 3, 5, 17, max(nnz, 1), nnz + 7}):
        ts, tf, tp = oracle.csf_split(p1, p2, T)
        nt = len(tf) - 1
        assert nt == max(1, -(-nnz // T))
        assert (ts[0], tf[0], tp[0]) == (0, 0, 0)
        assert (ts[-1], tf[-1], tp[-1]) == (I, F, nnz)
        assert np.all(np.diff(tp) >= 0) and np.all(np.diff(tf) >= 0) and np.all(np.diff(ts) >= 0)
        for t in range(1, nt):
            f = int(fib_of[t * T])
            assert tf[t] == f
            assert tp[t] == int(np.flatnonzero(fib_of == f)[0])
            assert ts[t] == int(sl_of[f])
        tile_of = np.full(nnz, -1)
        for t in range(nt):
            tile_of[tp[t]:tp[t + 1]] = t
            fibs = set(fib_of[tp[t]:tp[t + 1]].tolist())
            assert fibs <= set(range(tf[t], tf[t + 1]))
            slices = set(sl_of[f] for f in fibs)
            assert slices <= set(range(ts[t], ts[t + 1] + 1))
        assert np.all(tile_of >= 0)                     # every position covered once
        for f in range(F):                              # fiber aligned
            assert len(set(tile_of[p2[f]:p2[f + 1]].tolist())) <= 1


# ---- transposition and CSC (the CSR of the transpose read by columns)

@pytest.mark.parametrize("seed", range(5))
def test_transpose_matches_dense_transpose_and_is_an_involution(seed):
    rs = np.random.RandomState(seed)
    n, m = 9 + seed, 13 - seed
    pos, crd, vals = tiny.csr(rs, n, m, 0.3, empty_rows={2}, full_rows={4})
    tpos, tcrd, tvals = oracle.transpose(pos, crd, vals, (n, m))
    Bd, Bm = brute.dense_csr(pos, crd, vals, (n, m))
    Td, Tm = brute.dense_csr(tpos, tcrd, tvals, (m, n))
    assert np.array_equal(Td, Bd.T) and np.array_equal(Tm, Bm.T)
    for c in range(m):  # rows of B^T strictly increasing
        assert np.all(np.diff(tcrd[tpos[c]:tpos[c + 1]]) > 0)
    p2, c2, v2 = oracle.transpose(tpos, tcrd, tvals, (m, n))
    assert np.array_equal(p2, pos) and np.array_equal(c2, crd) and np.array_equal(v2, vals)


def test_transpose_edge_cases():
    # no entries; one column; one row
    tpos, tcrd, tvals = oracle.transpose(np.zeros(4, np.int32), np.zeros(0, np.int32),
                                         np.zeros(0), (3, 5))
    assert np.array_equal(tpos, np.zeros(6, np.int32)) and tcrd.size == 0
    pos = np.array([0, 1, 1, 2], np.int32)
    tpos, tcrd, tvals = oracle.transpose(pos, np.array([0, 0], np.int32), np.array([2., 3.]),
                                         (3, 1))
    assert list(tpos) == [0, 2] and list(tcrd) == [0, 2] and list(tvals) == [2., 3.]
    tpos, tcrd, _ = oracle.transpose(np.array([0, 3], np.int32), np.array([1, 4, 6], np.int32),
                                     np.ones(3), (1, 7))
    assert list(tpos) == [0, 0, 1, 1, 1, 2, 2, 3] and list(tcrd) == [0, 0, 0]


@pytest.mark.parametrize("seed", range(4))
def test_csc_spmv_matches_einsum_and_the_transposed_csr(seed):
    rs = np.random.RandomState(10 + seed)
    n, m = 11, 8  # A is n x m, stored by columns: the CSR of the m x n A^T
    kind = "int" if seed % 2 else "float"
    cpos, crd, vals = tiny.csr(rs, m, n, 0.35, empty_rows={3}, kind=kind)
    x = rs.randint(-4, 5, m).astype(np.float64) if kind == "int" else rs.uniform(-1, 1, m)
    y, S = oracle.csc_spmv(cpos, crd, vals, x, n)
    At, _ = brute.dense_csr(cpos, crd, vals, (m, n))
    want = np.einsum("ij,j->i", At.T, x)
    if kind == "int":
        assert np.array_equal(y, want)
    else:
        assert np.allclose(y, want, rtol=0, atol=1e-14)
    rpos, rcrd, rvals = oracle.transpose(cpos, crd, vals, (m, n))
    y2, S2 = oracle.spmv(rpos, rcrd, rvals, x)
    assert np.allclose(y, y2, rtol=0, atol=1e-15 * max(1, S.max())) and np.allclose(S, S2)
