"""Helpers shared by the GPU parity tests."""
import numpy as np
import pytest
import torch

RTOL = {torch.float64: 1e-12, torch.float32: 1e-5, torch.bfloat16: 1e-5}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev():
    return torch.device("cuda", 0)


def host64(t):
    """Exact float64 host copy of a device tensor (f64/f32/bf16)."""
    return t.detach().to("cpu").to(torch.float64).numpy()


def assert_close(got, ref, S, rtol, what=""):
    """|got - ref| <= rtol * S entrywise (S = sum of |terms|, exact when S == 0)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    err = np.abs(got - ref)
    bad = err > rtol * S
    if bad.any():
        k = np.argmax(err - rtol * S)
        raise AssertionError(
            f"{what}: {int(bad.sum())} entries beyond rtol {rtol}: worst index "
            f"{np.unravel_index(k, got.shape)} got {got.flat[k]!r} ref {ref.flat[k]!r} "
            f"S {S.flat[k]!r}")
    return float(np.max(err / np.where(S > 0, S, 1.0))) if err.size else 0.0


# Unit roundoff of BF16: 8 significand bits, round to nearest even.
BF16_U = 2.0 ** -8


def bf16_total_bound(k, rtol=1e-5):
    """Bound on |got - ref| / S when `got` sums products of k BF16-rounded
    factors (the rest exact) to within rtol, and ref, S come from the oracle
    on the unrounded inputs: rounding moves each term t by at most
    ((1 + u)^k - 1)|t|, and the accumulation error rtol is relative to the
    rounded terms' sum of magnitudes, at most (1 + u)^k S."""
    g = (1.0 + BF16_U) ** k
    return (g - 1.0) + rtol * g
