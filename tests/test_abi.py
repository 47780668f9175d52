"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/*.h declares, and its pure host logic (index-notation
parsing, status names, argument errors) behaves as documented."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(spl_\w+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2207_13901_amd import _native
    return _native.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_2207_13901_amd import _native
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
        assert name in _native.SIGNATURES, f"{name} missing from the binding"


def test_op_tin_round_trip(lib):
    import paper_2207_13901_amd as spl
    for op in range(7):
        tin = spl.op_tin(op)
        assert spl.op_parse(tin) == op
    assert spl.op_parse(" y ( r ) = M ( r , s ) * v ( s ) ") == 0
    assert spl.op_parse("X(p,q)=Y(p,q)+Z(p,q)+W(p,q)") == 2
    assert spl.op_parse("s()=B(i,j,k)*C(i,j,k)") == 6
    assert spl.op_parse("A(i,j)=B(i,j)*C(i,k)*D(j,k)") == 3
    for bad in ("a(i)=B(j,i)*c(j)", "A(i,j)=B(i,j)*C(i,k)*D(k,j)", "A(i,j)=B(i,j)+C(i,j)",
                "a(i)=B(i,j)*c(j)*d(j)", "a(i)=B(i,j)-c(j)", ""):
        with pytest.raises(spl.SpleafError):
            spl.op_parse(bad)


def test_status_strings_and_null_args(lib):
    assert lib.spl_status_string(0) == b"SPL_OK"
    assert lib.spl_status_string(6) == b"SPL_ERR_WORKSPACE"
    assert lib.spl_context_create(0, None) == 1
    assert lib.spl_context_destroy(None) == 0
    assert lib.spl_spmv(None, None, None, None, None, None, 0, None) == 1
    assert lib.spl_last_error(None) == b""
    out = ctypes.c_int32()
    assert lib.spl_op_parse(None, ctypes.byref(out)) == 1
