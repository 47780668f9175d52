"""Tiny seeded sparse operands for oracle pins (numpy RandomState)."""
import numpy as np


def csr(rs, n, m, density, empty_rows=(), full_rows=(), kind="float"):
    pos = [0]
    crd = []
    for i in range(n):
        if i in empty_rows:
            cols = []
        elif i in full_rows:
            cols = list(range(m))
        else:
            cols = sorted(np.nonzero(rs.rand(m) < density)[0].tolist())
        crd.extend(cols)
        pos.append(len(crd))
    nnz = len(crd)
    if kind == "int":
        vals = rs.randint(-4, 5, size=nnz).astype(np.float64)
    else:
        vals = rs.uniform(-1, 1, size=nnz)
    return (np.array(pos, dtype=np.int32), np.array(crd, dtype=np.int32),
            vals)


def csf(rs, I, J, K, density, kind="float", empty_slices=()):
    pos1, crd1, pos2, crd2 = [0], [], [0], []
    for i in range(I):
        if i not in empty_slices:
            for j in range(J):
                ks = sorted(np.nonzero(rs.rand(K) < density)[0].tolist())
                if ks:
                    crd1.append(j)
                    crd2.extend(ks)
                    pos2.append(len(crd2))
        pos1.append(len(crd1))
    nnz = len(crd2)
    if kind == "int":
        vals = rs.randint(-4, 5, size=nnz).astype(np.float64)
    else:
        vals = rs.uniform(-1, 1, size=nnz)
    a = lambda v: np.array(v, dtype=np.int32)  # noqa: E731
    return a(pos1), a(crd1), a(pos2), a(crd2), vals


def ddc(rs, I, J, K, density, kind="float"):
    """(Dense, Dense, Compressed) tensor: pos2 over all I*J fibers (some
    empty), crd2, vals."""
    pos2, crd2 = [0], []
    for _ in range(I * J):
        ks = sorted(np.nonzero(rs.rand(K) < density)[0].tolist())
        crd2.extend(ks)
        pos2.append(len(crd2))
    nnz = len(crd2)
    if kind == "int":
        vals = rs.randint(-4, 5, size=nnz).astype(np.float64)
    else:
        vals = rs.uniform(-1, 1, size=nnz)
    a = lambda v: np.array(v, dtype=np.int32)  # noqa: E731
    return a(pos2), a(crd2), vals


def ddc_to_csf(pos2, crd2, I, J):
    """The same tensor with its empty fibers dropped and the middle level
    compressed: (pos1, crd1, pos2, crd2)."""
    pos1, crd1, q2 = [0], [], [0]
    for i in range(I):
        for j in range(J):
            f = i * J + j
            if pos2[f + 1] > pos2[f]:
                crd1.append(j)
                q2.append(int(pos2[f + 1]))
        pos1.append(len(crd1))
    a = lambda v: np.array(v, dtype=np.int32)  # noqa: E731
    return a(pos1), a(crd1), a(q2), np.asarray(crd2, dtype=np.int32)
