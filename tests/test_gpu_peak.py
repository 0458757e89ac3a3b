"""The matrix-core rate kernel behind the measured FP64 peak (volpot_peak_mfma): its products
are checked against the values the header states, so the flops it is credited with are done."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _expected(iters):
    # thread sum: iters * 8 chains * sum over its output rows i = 4 r + l // 16 (r < 4), column
    # j = l % 16, of sum_c A[i][c] B[c][j]; lane 16 c + m holds A[m][c] and B[c][m]
    A = np.array([[1.0 + (16 * c + m) / 1024.0 for c in range(4)] for m in range(16)])
    B = np.array([[1.0 - (16 * c + m) / 1024.0 for m in range(16)] for c in range(4)])
    D = A @ B
    per_lane = np.array([sum(D[4 * r + l // 16, l % 16] for r in range(4)) for l in range(64)])
    return iters * 8 * per_lane


@pytest.mark.parametrize("blocks,iters", [(1, 1), (3, 7), (64, 100)])
def test_peak_kernel_products(device, blocks, iters):
    import torch

    from paper_2501_17967_amd.volpot import peak_mfma

    out = torch.zeros(256 * blocks, dtype=torch.float64, device=device)
    flops = peak_mfma(blocks, iters, out)
    torch.cuda.synchronize()
    assert flops == blocks * 4 * iters * 8 * 2048
    got = out.cpu().numpy().reshape(blocks * 4, 64)
    exp = _expected(iters)
    assert np.max(np.abs(got - exp[None, :])) <= 1e-13 * np.max(np.abs(exp))
