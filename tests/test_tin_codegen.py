"""Host checks of the index-notation front-end and leaf generator: the
generated HIP source of every test statement compiles for gfx950, and
statements outside the generator's form are refused with the documented
status (no GPU: spl_tin_source takes no context)."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import tempfile

import pytest
import torch

from tests.tin_cases import CASES, SMALL, make

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _out(spl, kind, shape, dtype):
    if kind == "csr":
        e = torch.empty(0, dtype=torch.int32)
        return spl.CSR(torch.empty(shape[0] + 1, dtype=torch.int32), e,
                       torch.empty(0, dtype=dtype), shape)
    if kind == "scalar":
        return torch.empty(1, dtype=torch.float64)
    return torch.empty(shape, dtype=dtype)


def _source(stmt, kind, recipe, dtype):
    import paper_2207_13901_amd as spl
    lib, _, shape = make(stmt, recipe, dtype, seed=0, extents=SMALL)
    return spl.tin_source(stmt, _out(spl, kind, shape, dtype), **lib)


def _compile(src):
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "leaf.hip")
        with open(path, "w") as f:
            f.write("#include <hip/hip_runtime.h>\n" + src)
        r = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O3",
                            "--cuda-device-only", "-c", path, "-o", os.path.join(d, "leaf.o")],
                           capture_output=True, text=True)
        return r.returncode, r.stderr


def test_generated_sources_compile():
    srcs = [(stmt, _source(stmt, kind, recipe, dt)) for stmt, kind, recipe in CASES
            for dt in (torch.float64, torch.float32)]
    with cf.ThreadPoolExecutor(8) as ex:
        results = list(ex.map(lambda s: _compile(s[1]), srcs))
    for (stmt, src), (rc, err) in zip(srcs, results):
        assert rc == 0, f"{stmt}:\n{err}\n{src}"


def test_csr_output_has_count_and_fill_kernels():
    src = _source("A(i,j) = B(i,j) + C(i,j)", "csr", dict(B="csr", C="csr"), torch.float64)
    assert "tin_count" in src and "tin_fill" in src and "tin_eval" not in src
    # union: the merge runs until both lists are exhausted
    assert "while (q0_1 < e0_1 || q1_1 < e1_1)" in src
    src = _source("A(i,j) = B(i,j) * C(i,j)", "csr", dict(B="csr", C="csr"), torch.float64)
    assert "while (q0_1 < e0_1 && q1_1 < e1_1)" in src


@pytest.mark.parametrize("stmt,operands_of,recipe,match", [
    # a thread per output row: a statement that scatters across rows
    ("a(j) = B(i,j) * c(i)", None, dict(B="csr", c="vec"), "SPL_ERR_UNSUPPORTED"),
    ("A(i,j) = B(i,j) + c(i)", None, dict(B="csr", c="vec"), "SPL_ERR_UNSUPPORTED"),
    ("a(i) = B(i,i)", "a(i) = B(i,j)", dict(B="csr"), "SPL_ERR_UNSUPPORTED"),
    ("A(i,j) = B(i,j) ** C(i,j)", "A(i,j) = B(i,j) * C(i,j)", dict(B="csr", C="csr"),
     "SPL_ERR_ARG"),
    ("A(i,j) = B(i,j) * Q(i,j)", "A(i,j) = B(i,j)", dict(B="csr"), "SPL_ERR_ARG"),
])
def test_refusals(stmt, operands_of, recipe, match):
    import paper_2207_13901_amd as spl
    lib, _, _ = make(operands_of or stmt, recipe, torch.float64, seed=1, extents=SMALL)
    lhs = stmt.split("=")[0]
    names = lhs[lhs.index("(") + 1:lhs.index(")")].split(",")
    out = torch.empty(tuple(SMALL[v.strip()] for v in names), dtype=torch.float64)
    with pytest.raises(spl.SpleafError, match=match):
        spl.tin_source(stmt, out, **lib)


def test_shape_and_dtype_errors():
    import paper_2207_13901_amd as spl
    lib, _, _ = make("a(i) = B(i,j) * c(j)", dict(B="csr", c="vec"), torch.float64, seed=2,
                     extents=SMALL)
    out = torch.empty(SMALL["i"], dtype=torch.float64)
    with pytest.raises(spl.SpleafError, match="SPL_ERR_SHAPE"):
        spl.tin_source("a(i) = B(i,j) * c(j)", out, B=lib["B"],
                       c=torch.empty(SMALL["j"] + 1, dtype=torch.float64))
    with pytest.raises(spl.SpleafError, match="SPL_ERR_DTYPE"):
        spl.tin_source("a(i) = B(i,j) * c(j)", out, B=lib["B"],
                       c=torch.empty(SMALL["j"], dtype=torch.float32))
    with pytest.raises(spl.SpleafError, match="SPL_ERR_SHAPE"):  # scalar out of two entries
        spl.tin_source("a = B(i,j) * B2(i,j)", torch.empty(2, dtype=torch.float64), B=lib["B"],
                       B2=lib["B"])
