"""Statements and seeded operands for the index-notation leaf generator's
tests: the host tests compile the generated source of each, the GPU tests
run it against the general oracle (oracle/tin.py)."""
import numpy as np
import torch

from tests import tiny

# (statement, output kind, operand recipe); output kinds: "dense", "csr",
# "scalar".  Recipes name each operand's format: csr, csf, ddc (sparse),
# vec / mat (dense) with their index extents taken from the statement.
CASES = [
    # outside the seven fixed statements
    ("A(i,j) = B(i,j) * C(i,j)", "csr", dict(B="csr", C="csr")),
    ("A(i,j) = B(i,j) * C(i,j)", "dense", dict(B="csr", C="csr")),
    ("a(i) = B(i,j,k) * c(j) * d(k)", "dense", dict(B="csf", c="vec", d="vec")),
    ("A(i,j) = B(i,j) + C(i,j)", "csr", dict(B="csr", C="csr")),
    ("A(i,j) = B(i,j) - C(i,j)", "csr", dict(B="csr", C="csr")),
    ("a = B(i,j) * C(i,j)", "scalar", dict(B="csr", C="csr")),
    ("A(i,j) = B(i,j) * c(j) + C(i,j) * d(j)", "csr", dict(B="csr", C="csr", c="vec", d="vec")),
    ("A(i,j) = B(i,j) + E(i,j)", "csr", dict(B="csr", E="mat")),
    ("A(i,j) = B(i,j,k) * c(k)", "dense", dict(B="ddc", c="vec")),
    ("a(i) = B(i,j,k) * C(i,j,k)", "dense", dict(B="csf", C="csf")),
    # the fixed statements through the generator
    ("a(i) = B(i,j) * c(j)", "dense", dict(B="csr", c="vec")),
    ("A(i,k) = B(i,j) * C(j,k)", "dense", dict(B="csr", C="mat")),
    ("A(i,j) = B(i,j) + C(i,j) + D(i,j)", "csr", dict(B="csr", C="csr", D="csr")),
    ("A(i,j) = B(i,j) * C(i,k) * D(j,k)", "csr", dict(B="csr", C="mat", D="mat")),
    ("A(i,j) = B(i,j,k) * c(k)", "csr", dict(B="csf", c="vec")),
    ("A(i,l) = B(i,j,k) * C(j,l) * D(k,l)", "dense", dict(B="csf", C="mat", D="mat")),
    ("a = B(i,j,k) * C(i,j,k)", "scalar", dict(B="csf", C="csf")),
]

# index extents: i spans several 256-thread workgroups with a ragged tail
EXTENTS = dict(i=600, j=40, k=30, l=6)
SMALL = dict(i=37, j=9, k=7, l=5)  # for the slow scalar oracle


def _parse(stmt):
    from oracle import tin as T
    return T.parse(stmt)


def make(stmt, recipe, dtype, seed, kind="float", extents=EXTENTS, device="cpu"):
    """Operands for `stmt`: {name: spl object or torch tensor} for the library
    and {name: oracle object or numpy array} for the oracle."""
    import paper_2207_13901_amd as spl
    from oracle import tin as T
    lhs, terms = _parse(stmt)
    rs = np.random.RandomState(seed)
    lib, ref = {}, {}
    dev = torch.device(device)

    def t32(a):
        return torch.as_tensor(np.asarray(a, dtype=np.int32), device=dev)

    def vals_of(v):
        v = torch.as_tensor(np.asarray(v, dtype=np.float64)).to(dtype)
        return v.to(dev), v.double().numpy()

    for _, factors in terms:
        for name, vs in factors:
            if name in lib:
                continue
            shape = tuple(extents[v] for v in vs)
            fmt = recipe[name]
            if fmt == "csr":
                pos, crd, v = tiny.csr(rs, shape[0], shape[1], 0.3, empty_rows={1, 7},
                                       full_rows={3}, kind=kind)
                tv, hv = vals_of(v)
                lib[name] = spl.CSR(t32(pos), t32(crd), tv, shape)
                ref[name] = T.Sparse.csr(pos, crd, hv, shape)
            elif fmt == "csf":
                p1, c1, p2, c2, v = tiny.csf(rs, *shape, 0.2, kind=kind, empty_slices={2})
                tv, hv = vals_of(v)
                lib[name] = spl.CSF(t32(p1), t32(c1), t32(p2), t32(c2), tv, shape)
                ref[name] = T.Sparse.csf(p1, c1, p2, c2, hv, shape)
            elif fmt == "ddc":
                p2, c2, v = tiny.ddc(rs, *shape, 0.2, kind=kind)
                tv, hv = vals_of(v)
                lib[name] = spl.DDC(t32(p2), t32(c2), tv, shape)
                ref[name] = T.Sparse.ddc(p2, c2, hv, shape)
            else:
                a = (rs.randint(-4, 5, shape) if kind == "int" else rs.uniform(-1, 1, shape))
                tv, hv = vals_of(a)
                lib[name], ref[name] = tv, hv
    out_shape = tuple(extents[v] for v in lhs[1])
    return lib, ref, out_shape
