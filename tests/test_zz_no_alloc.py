"""GPU test of volpot_strip_apply_noalloc, the strip apply whose work vectors live in the
library's static per-device array: its output must equal volpot_strip_apply's on the same plan,
bit for bit (same kernels, same arithmetic), on two calls in a row, the second on a smaller strip
(so that the array keeps the first call's contents when the second one runs)."""
import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu


def _annulus(n_panel, n_gl, R):
    s, _ = np.polynomial.legendre.leggauss(n_gl)
    h = np.pi / n_panel
    th = (2 * h * np.arange(n_panel))[:, None] + h * (s[None, :] + 1)
    return np.stack([R * np.cos(th), R * np.sin(th)], axis=2)


def test_noalloc_strip_apply_equals_the_allocating_apply(device):
    import torch

    from paper_2501_17967_amd import StripPlan

    f_np = lambda p: np.sin(3 * p[:, 0]) * np.exp(p[:, 1]) + 0.5
    big = (gen.star_curve(n_panels=56, order=16, scale=1.0).nodes.reshape(56, 16, 2),
           gen.star_curve(n_panels=56, order=16, scale=0.93).nodes.reshape(56, 16, 2), 24, 16)
    small = (_annulus(12, 16, 0.9), _annulus(12, 16, 0.75), 16, 10)
    for name, (g, gt, q, n_r) in (("56 x 24 x 16 star strip", big), ("12 x 16 x 10 annulus (smaller)", small)):
        print("no-alloc strip case: %s" % name, flush=True)
        sp = StripPlan(g, gt, q, n_r)
        f = torch.from_numpy(f_np(sp.nodes.reshape(-1, 2))).to(device)
        ref = sp.apply(f)
        out = torch.full_like(ref, float("nan"))
        sp.apply(f, out=out, noalloc=True)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), out.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
        sp.close()


def test_noalloc_rejects_a_strip_beyond_the_static_array(device):
    from paper_2501_17967_amd import StripPlan, volpot

    # (4 n + 4) m > 131072 doubles: 1,200 panels at n_r = 32 (m = 30)
    g, gt = _annulus(1200, 4, 0.9), _annulus(1200, 4, 0.89)
    import torch

    sp = StripPlan(g, gt, 4, 32)
    f = torch.zeros(sp.shape, dtype=torch.float64, device=device)
    out = torch.empty_like(f)
    with pytest.raises(volpot.VolpotError) as e:
        sp.apply(f, out=out, noalloc=True)
    assert e.value.code == volpot.ERR_ARG
    sp.close()
