"""Pins of the general index-notation oracle (oracle/tin.py) against what
fixes it independently: numpy.einsum on the densified operands (index notation
is einsum; a sum of terms is the sum of the terms' einsums), the plain-loop C
oracle of the seven fixed statements, exact small-integer results, and the
structural pattern rules (intersection within a product, union across a sum,
a term with no sparse operand on the column index stores every column)."""
import numpy as np
import pytest

import oracle
from oracle import brute
from oracle import tin as T
from tests import tiny


def _csr(rs, n, m, d, kind="float"):
    pos, crd, vals = tiny.csr(rs, n, m, d, empty_rows={1}, kind=kind)
    return pos, crd, vals, T.Sparse.csr(pos, crd, vals, (n, m))


def test_parse():
    lhs, terms = T.parse("A(i,j) = B(i,j) * c(j) - C(i, j)*d(j) + E(i,j)")
    assert lhs == ("A", ["i", "j"])
    assert [s for s, _ in terms] == [1, -1, 1]
    assert terms[1][1] == [("C", ["i", "j"]), ("d", ["j"])]
    lhs, terms = T.parse("a = -B(i,j,k)*C(i,j,k)")
    assert lhs == ("a", []) and terms[0][0] == -1
    with pytest.raises(ValueError):
        T.parse("A(i) = B(i,j) $ c(j)")


@pytest.mark.parametrize("seed", range(6))
def test_products_match_einsum(seed):
    rs = np.random.RandomState(seed)
    n, m, K = 7, 6, 5
    bp, bc, bv, B = _csr(rs, n, m, 0.4)
    cp, cc, cv, C = _csr(rs, n, m, 0.5)
    Bd, _ = brute.dense_csr(bp, bc, bv, (n, m))
    Cd, _ = brute.dense_csr(cp, cc, cv, (n, m))
    x = rs.uniform(-1, 1, m)
    Dm = rs.uniform(-1, 1, (m, K))
    Ck = rs.uniform(-1, 1, (n, K))
    cases = [
        ("a(i) = B(i,j) * x(j)", "ij,j->i", [Bd, x], dict(B=B, x=x)),
        ("A(i,k) = B(i,j) * D(j,k)", "ij,jk->ik", [Bd, Dm], dict(B=B, D=Dm)),
        ("A(i,j) = B(i,j) * C(i,j)", "ij,ij->ij", [Bd, Cd], dict(B=B, C=C)),
        ("a = B(i,j) * C(i,j)", "ij,ij->", [Bd, Cd], dict(B=B, C=C)),
        ("A(i,j) = B(i,j) * G(i,k) * D(j,k)", "ij,ik,jk->ij", [Bd, Ck, Dm], dict(B=B, G=Ck, D=Dm)),
    ]
    for stmt, spec, dense, ops in cases:
        got, S = T.evaluate(stmt, ops)
        want = np.einsum(spec, *dense)
        assert np.allclose(got, want, rtol=0, atol=1e-14 * max(1.0, np.max(np.abs(S)))), stmt
        assert np.all(S >= np.abs(got) - 1e-15)


def test_three_index_statements_match_einsum():
    rs = np.random.RandomState(3)
    I, J, K, R = 5, 4, 6, 3
    p1, c1, p2, c2, v = tiny.csf(rs, I, J, K, 0.35, empty_slices={2})
    B = T.Sparse.csf(p1, c1, p2, c2, v, (I, J, K))
    Bd, _ = brute.dense_csf(p1, c1, p2, c2, v, (I, J, K))
    c, d = rs.uniform(-1, 1, J), rs.uniform(-1, 1, K)
    Cm, Dm = rs.uniform(-1, 1, (J, R)), rs.uniform(-1, 1, (K, R))
    got, _ = T.evaluate("a(i) = B(i,j,k) * c(j) * d(k)", dict(B=B, c=c, d=d))
    assert np.allclose(got, np.einsum("ijk,j,k->i", Bd, c, d), rtol=0, atol=1e-13)
    got, _ = T.evaluate("A(i,l) = B(i,j,k) * C(j,l) * D(k,l)", dict(B=B, C=Cm, D=Dm))
    assert np.allclose(got, np.einsum("ijk,jl,kl->il", Bd, Cm, Dm), rtol=0, atol=1e-13)
    # the (Dense, Dense, Compressed) form of the same values
    q2, k2, w = tiny.ddc(rs, I, J, K, 0.3)
    Dd = T.Sparse.ddc(q2, k2, w, (I, J, K))
    Dde, _ = brute.dense_ddc(q2, k2, w, (I, J, K))
    got, _ = T.evaluate("A(i,j) = B(i,j,k) * d(k)", dict(B=Dd, d=d))
    assert np.allclose(got, np.einsum("ijk,k->ij", Dde, d), rtol=0, atol=1e-13)


def test_sums_match_einsum_of_terms_and_keep_the_union():
    rs = np.random.RandomState(4)
    n, m = 8, 7
    bp, bc, bv, B = _csr(rs, n, m, 0.35)
    cp, cc, cv, C = _csr(rs, n, m, 0.35)
    Bd, Bm = brute.dense_csr(bp, bc, bv, (n, m))
    Cd, Cm = brute.dense_csr(cp, cc, cv, (n, m))
    x, y = rs.uniform(-1, 1, m), rs.uniform(-1, 1, m)
    stmt = "A(i,j) = B(i,j) * x(j) - C(i,j) * y(j)"
    got, _ = T.evaluate(stmt, dict(B=B, C=C, x=x, y=y))
    assert np.allclose(got, Bd * x - Cd * y, rtol=0, atol=1e-14)
    pos, crd = T.pattern(stmt, dict(B=B, C=C, x=x, y=y), (n, m))
    mask = np.zeros((n, m), bool)
    for i in range(n):
        mask[i, crd[pos[i]:pos[i + 1]]] = True
    assert np.array_equal(mask, Bm | Cm)
    assert all(np.all(np.diff(crd[pos[i]:pos[i + 1]]) > 0) for i in range(n))
    # a product keeps the intersection
    pos, crd = T.pattern("A(i,j) = B(i,j) * C(i,j)", dict(B=B, C=C), (n, m))
    mask[:] = False
    for i in range(n):
        mask[i, crd[pos[i]:pos[i + 1]]] = True
    assert np.array_equal(mask, Bm & Cm)
    # a term with a dense operand on j stores every column
    E = rs.uniform(-1, 1, (n, m))
    pos, crd = T.pattern("A(i,j) = B(i,j) + E(i,j)", dict(B=B, E=E), (n, m))
    assert np.array_equal(np.diff(pos), np.full(n, m))


def test_fixed_statements_match_the_c_oracle():
    rs = np.random.RandomState(5)
    n, m, N = 9, 8, 3
    bp, bc, bv, B = _csr(rs, n, m, 0.4)
    x = rs.uniform(-1, 1, m)
    Dm = rs.uniform(-1, 1, (m, N))
    got, S = T.evaluate("a(i) = B(i,j) * c(j)", dict(B=B, c=x))
    ref, rS = oracle.spmv(bp, bc, bv, x)
    assert np.allclose(got, ref, rtol=0, atol=1e-15) and np.allclose(S, rS)
    got, S = T.evaluate("A(i,j) = B(i,k) * C(k,j)", dict(B=B, C=Dm))
    ref, rS = oracle.spmm(bp, bc, bv, Dm)
    assert np.allclose(got, ref, rtol=0, atol=1e-15) and np.allclose(S, rS)
    # SpAdd3: the union pattern and B, C, D sums
    cp, cc, cv, C = _csr(rs, n, m, 0.3)
    dp, dc, dv, D = _csr(rs, n, m, 0.3)
    stmt = "A(i,j) = B(i,j) + C(i,j) + D(i,j)"
    rpos, rcrd, rvals, rS, _ = oracle.spadd3((bp, bc, bv), (cp, cc, cv), (dp, dc, dv))
    pos, crd = T.pattern(stmt, dict(B=B, C=C, D=D), (n, m))
    assert np.array_equal(pos, rpos) and np.array_equal(crd, rcrd)
    vals, S = T.evaluate(stmt, dict(B=B, C=C, D=D))
    got = np.array([vals[i, j] for i in range(n) for j in crd[pos[i]:pos[i + 1]]])
    assert np.allclose(got, rvals, rtol=0, atol=1e-15)
    # SpTTV's pattern-preserving output: B's fibers
    p1, c1, p2, c2, v = tiny.csf(rs, 5, 6, 7, 0.3, empty_slices={0})
    Bt = T.Sparse.csf(p1, c1, p2, c2, v, (5, 6, 7))
    cvec = rs.uniform(-1, 1, 7)
    pos, crd = T.pattern("A(i,j) = B(i,j,k) * c(k)", dict(B=Bt, c=cvec), (5, 6))
    assert np.array_equal(pos, p1) and np.array_equal(crd, c1)
    vals, _ = T.evaluate("A(i,j) = B(i,j,k) * c(k)", dict(B=Bt, c=cvec))
    ref, _ = oracle.spttv(p1, p2, c2, v, cvec)
    got = np.array([vals[i, j] for i in range(5) for j in c1[p1[i]:p1[i + 1]]])
    assert np.allclose(got, ref, rtol=0, atol=1e-15)


def test_integer_values_exact_and_cancellation_kept():
    rs = np.random.RandomState(6)
    n, m = 6, 9
    bp, bc, bv, B = _csr(rs, n, m, 0.5, kind="int")
    Bd, Bm = brute.dense_csr(bp, bc, bv, (n, m))
    x = rs.randint(-4, 5, m).astype(np.float64)
    got, _ = T.evaluate("a(i) = B(i,j) * x(j) * x(j)", dict(B=B, x=x))
    assert np.array_equal(got, Bd @ (x * x))
    stmt = "A(i,j) = B(i,j) - B2(i,j)"
    ops = dict(B=B, B2=B)
    pos, crd = T.pattern(stmt, ops, (n, m))
    assert np.array_equal(pos, bp) and np.array_equal(crd, bc)
    vals, S = T.evaluate(stmt, ops)
    assert not vals.any() and np.array_equal(S, 2 * np.abs(Bd))


def test_rows_restricts_the_first_index():
    rs = np.random.RandomState(7)
    _, _, _, B = _csr(rs, 10, 5, 0.5)
    x = rs.uniform(-1, 1, 5)
    full, S = T.evaluate("a(i) = B(i,j) * x(j)", dict(B=B, x=x))
    part, Sp = T.evaluate("a(i) = B(i,j) * x(j)", dict(B=B, x=x), rows=[7, 2, 9])
    assert np.array_equal(part, full[[7, 2, 9]]) and np.array_equal(Sp, S[[7, 2, 9]])
