"""The allocation-free loss/gradient entry point (axp_mlp_loss_grad_noalloc)
against the allocating one (axp_mlp_loss_grad) through the C ABI.

Both run the same kernels in the same order over the same inputs (the
weight gradient is a fixed-order sum of per-chunk partials), so loss and
gradient agree bit for bit.  Two calls in a row, the second with fewer
samples, show that the static scratch left by a larger call does not leak
into a smaller one; a call beyond the scratch's capacity is refused before
any launch.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


def _samples(n, seed):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.rand((n, 16), generator=g, dtype=torch.float32) * 2 - 1
    y = torch.randn((n,), generator=g, dtype=torch.float32) * 0.1
    w = torch.rand((n,), generator=g, dtype=torch.float32) + 0.5
    return X.cuda(), y.cuda(), w.cuda()


@pytest.mark.parametrize("n_hidden,n_layers,sizes", [(64, 2, (9000, 1234)), (32, 4, (20000, 700)),
                                                     (64, 4, (15497, 15000))])
def test_noalloc_matches_allocating_entry_point(axp, n_hidden, n_layers, sizes):
    import torch
    net = axp.Mlp(n_hidden=n_hidden, n_layers=n_layers, seed=7, device=0)
    npar = net.n_params()
    for call, n in enumerate(sizes):
        print(f"[gpu] no-alloc loss/grad, H={n_hidden} L={n_layers}, call {call}, n={n}", flush=True)
        X, y, w = _samples(n, seed=100 + call)
        loss_out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        grad_out = torch.full((npar,), float("nan"), dtype=torch.float32, device="cuda")
        net.loss_grad_noalloc(X, y, w, loss_out, grad_out)
        torch.cuda.synchronize()
        lo, go = loss_out.cpu().numpy(), grad_out.cpu().numpy()
        ref_loss, ref_grad = net.loss_grad(X, y, w, want_grad=True)
        assert lo[0] == ref_loss
        assert lo[1] == pytest.approx(float(w.double().sum()), rel=1e-12)
        assert np.array_equal(go, ref_grad)
        assert np.isfinite(go).all() and np.abs(go).max() > 0
    # the network's own gradient is the allocating call's, untouched by the variant
    assert net.info()["adam_steps"] == 0
    net.close()


def test_noalloc_refuses_sizes_beyond_the_static_scratch(axp):
    import torch
    net = axp.Mlp(n_hidden=64, n_layers=4, seed=1, device=0)
    X, y, w = _samples(15498, seed=3)          # one sample above the limit at H = 64, L = 4
    loss_out = torch.zeros((2,), dtype=torch.float64, device="cuda")
    grad_out = torch.zeros((net.n_params(),), dtype=torch.float32, device="cuda")
    with pytest.raises(axp.AxpError) as e:
        net.loss_grad_noalloc(X, y, w, loss_out, grad_out)
    assert e.value.code == -1 and "static scratch" in str(e.value)      # AXP_E_ARG
    torch.cuda.synchronize()
    assert float(loss_out.abs().sum()) == 0.0 and float(grad_out.abs().sum()) == 0.0
    # the network stays usable: a call within the limit still agrees
    X, y, w = X[:4000].contiguous(), y[:4000].contiguous(), w[:4000].contiguous()
    net.loss_grad_noalloc(X, y, w, loss_out, grad_out)
    torch.cuda.synchronize()
    ref_loss, ref_grad = net.loss_grad(X, y, w, want_grad=True)
    assert loss_out[0].item() == ref_loss and np.array_equal(grad_out.cpu().numpy(), ref_grad)
    net.close()
