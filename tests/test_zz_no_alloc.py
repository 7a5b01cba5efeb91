"""The allocation-free L1 objective (lf_l1_loss_noalloc) through the C ABI:
the same loss and gradient as lf_l1_loss, bit for bit, and within the
oracle's tolerance (Sec. 3.4, Eq. training-objectives, data term), on two
calls in a row, the second with a smaller input that reuses the shared
device scratch.  Requires an MI355X."""
import numpy as np
import pytest

from oracle import losses as OL
from tests.gpu_common import dev

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    t = np.exp(rng.normal(0, 1.5, n)).astype(np.float32)
    p = (t * np.exp(rng.normal(0, 0.2, n))).astype(np.float32)
    p[: n // 9] = t[: n // 9]  # exact ties: sign(0) = 0
    return p, t


def test_noalloc_l1_equals_the_allocating_entry_point():
    import torch
    import paper_2608_29269_amd as lf
    tr = lf.Tracer()
    for n, seed in ((3 * 1024 * 1024 + 37, 1), (1000, 2), (0, 3)):
        p, t = _inputs(n, seed)
        pd, td = dev(p), dev(t)
        loss_a, grad_a = tr.l1_loss(pd, td)
        loss_b = torch.full((), -1.0, device="cuda")
        grad_b = torch.full_like(pd, -7.0)
        tr.l1_loss_noalloc(pd, td, loss_b, grad_b)
        tr.sync()
        assert float(loss_b) == float(loss_a), (n, float(loss_b), float(loss_a))
        assert torch.equal(grad_b.view(torch.int32), grad_a.view(torch.int32)), n
        ref, gref = OL.l1_loss(p, t)
        assert abs(float(loss_b) - ref) <= 1e-6 * abs(ref) + 1e-7, (n, float(loss_b), ref)
        g = grad_b.cpu().numpy().astype(np.float64)
        assert np.array_equal(np.sign(g), np.sign(gref))
        assert np.all(np.abs(g - gref) <= 2.0 ** -24 * np.abs(gref)), n
    # loss only
    p, t = _inputs(257, 4)
    loss_c = torch.zeros((), device="cuda")
    tr.l1_loss_noalloc(dev(p), dev(t), loss_c, None)
    assert abs(float(loss_c) - OL.l1_loss(p, t)[0]) <= 1e-6 * OL.l1_loss(p, t)[0]
    with pytest.raises(lf.LFError):
        tr.l1_loss_noalloc(dev(p), dev(t), None)
