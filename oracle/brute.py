"""Dense brute-force evaluation by numpy.einsum (test infrastructure).

Tensor index notation (paper, Sec. II-A) is exactly what einsum evaluates:
every index letter is a loop and a letter missing from the output is summed.
Densifying a tiny sparse operand and calling einsum with the statement's index
letters therefore gives the value of each of the seven statements of
Sec. VI-A independently of the coordinate-tree loops in ``oracle.c``.  Output
patterns are the structural masks: the stored coordinates of the sparse
operand(s), not the numerically nonzero entries.
"""
from __future__ import annotations

import numpy as np


def dense_csr(pos, crd, vals, shape):
    """Densify a CSR matrix; also return the structural mask."""
    A = np.zeros(shape, dtype=np.float64)
    M = np.zeros(shape, dtype=bool)
    for i in range(shape[0]):
        for p in range(pos[i], pos[i + 1]):
            A[i, crd[p]] += float(vals[p])
            M[i, crd[p]] = True
    return A, M


def dense_csf(pos1, crd1, pos2, crd2, vals, shape):
    """Densify a CSF (Dense, Compressed, Compressed) 3-tensor and its mask."""
    T = np.zeros(shape, dtype=np.float64)
    M = np.zeros(shape, dtype=bool)
    for i in range(shape[0]):
        for f in range(pos1[i], pos1[i + 1]):
            j = crd1[f]
            for p in range(pos2[f], pos2[f + 1]):
                T[i, j, crd2[p]] += float(vals[p])
                M[i, j, crd2[p]] = True
    return T, M


def dense_ddc(pos2, crd2, vals, shape):
    """Densify a (Dense, Dense, Compressed) 3-tensor (fiber f = i*J + j) and
    its mask."""
    T = np.zeros(shape, dtype=np.float64)
    M = np.zeros(shape, dtype=bool)
    I, J, _ = shape
    for i in range(I):
        for j in range(J):
            f = i * J + j
            for p in range(pos2[f], pos2[f + 1]):
                T[i, j, crd2[p]] += float(vals[p])
                M[i, j, crd2[p]] = True
    return T, M


def spmv(Bd, c):
    return np.einsum("ij,j->i", Bd, c)


def spmm(Bd, C):
    return np.einsum("ik,kj->ij", Bd, C)


def sddmm(Bd, C, D):
    # A(i,j) = B(i,j) C(i,k) D(j,k)
    return np.einsum("ij,ik,jk->ij", Bd, C, D)


def spttv(Bd, c):
    return np.einsum("ijk,k->ij", Bd, c)


def mttkrp(Bd, C, D):
    return np.einsum("ijk,jl,kl->il", Bd, C, D)


def inner(Bd, Cd):
    return float(np.einsum("ijk,ijk->", Bd, Cd)) if Bd.ndim == 3 else \
        float(np.einsum("ij,ij->", Bd, Cd))


def spadd3(Bd, Bm, Cd, Cm, Dd, Dm):
    """Values of B+C+D and the union of the three structural masks."""
    return Bd + Cd + Dd, Bm | Cm | Dm
