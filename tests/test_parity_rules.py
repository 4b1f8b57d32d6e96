"""CPU checks of the parity rules themselves (tests/parity.py): the BF16
bound rests on round-to-nearest bfloat16 having unit roundoff 2^-8, and it
must cover the error of a BF16 correlation with FP32 accumulation."""
import numpy as np
import pytest

from tests import parity

torch = pytest.importorskip("torch")


def test_bf16_unit_roundoff_is_2_to_minus_8():
    """Round-to-nearest bfloat16 (torch's CPU conversion) keeps 8 significant
    bits: the relative rounding error reaches just under 2^-8, so a bound built
    on 2^-9 would be half the worst case."""
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(1.0, 2.0, 1 << 20), rng.standard_normal(1 << 20) * 1e3]).astype(np.float32)
    xb = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    rel = np.abs(xb.astype(np.float64) - x) / np.abs(x.astype(np.float64))
    assert rel.max() <= parity.U_BF16
    assert rel.max() > 0.99 * parity.U_BF16


@pytest.mark.parametrize("N,r,m", [(16, 4, 9), (48, 10, 9), (128, 32, 9)])
def test_bf16_bound_covers_a_simulated_bf16_correlation(N, r, m):
    """Correlation of bf16-rounded non-negative data accumulated in FP32 stays
    within the bound, and the bound is at least the rounding term 2^-7."""
    rng = np.random.default_rng(N + r)
    T = rng.random((m, N, N)).astype(np.float32)
    S = rng.random((m, N + 2 * r, N + 2 * r)).astype(np.float32)
    Tb = torch.from_numpy(T).to(torch.bfloat16).to(torch.float32).numpy()
    Sb = torch.from_numpy(S).to(torch.bfloat16).to(torch.float32).numpy()
    tol = parity.bf16_tol(N, r, m)
    assert tol >= 2 * parity.U_BF16
    E1 = float(np.sum(T.astype(np.float64) ** 2))
    worst = 0.0
    for dy, dx in ((0, 0), (r, r), (2 * r, 0), (0, 2 * r)):
        W = S[:, dy:dy + N, dx:dx + N].astype(np.float64)
        Wb = Sb[:, dy:dy + N, dx:dx + N]
        C = float(np.sum(T.astype(np.float64) * W))
        Cb = float(np.sum((Tb * Wb).astype(np.float32), dtype=np.float32))
        E2 = float(np.sum(W * W))
        worst = max(worst, 2 * abs(Cb - C) / (E1 + E2))
    assert worst <= tol, (worst, tol)
