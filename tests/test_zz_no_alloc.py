"""fr_mlp_grad_static (the allocation-free MLP gradient, static device scratch) against
fr_mlp_grad (context workspace) through the C ABI: equal gradients and losses on two
calls in a row, the second with a smaller batch, and its argument errors."""
import numpy as np
import pytest

from paper_2408_16509_amd import frmi, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx():
    ctx = frmi.Context(inputs.hex_box((2, 2, 2)), system=0, order=2)
    rng = np.random.default_rng(5)
    ctx.mlp_set_weights(inputs.mlp_glorot(43), rng.normal(size=16), 0.5 + rng.uniform(size=16))
    return ctx


def test_static_gradient_equals_workspace_gradient():
    assert torch.cuda.is_available()
    ctx = _ctx()
    rng = np.random.default_rng(11)
    g_out = torch.full((5313,), float("nan"), dtype=torch.float32, device="cuda")
    l_out = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    for n in (frmi.FR_MLP_STATIC_MAX_BATCH, 777, 1):
        x = torch.tensor(rng.normal(size=(n, 16)), dtype=torch.float32, device="cuda")
        y = torch.tensor(rng.normal(size=n), dtype=torch.float32, device="cuda")
        g_ref, l_ref = ctx.mlp_grad(x, y)
        ctx.mlp_grad_static(x, y, g_out, l_out)
        torch.cuda.synchronize()
        # the same kernels with a fixed reduction order: identical bits
        assert torch.equal(g_out, g_ref), n
        assert torch.equal(l_out, l_ref), n
        assert torch.isfinite(g_out).all()
    ctx.close()


def test_static_gradient_argument_errors():
    ctx = _ctx()
    x = torch.zeros((frmi.FR_MLP_STATIC_MAX_BATCH + 1, 16), dtype=torch.float32, device="cuda")
    y = torch.zeros(frmi.FR_MLP_STATIC_MAX_BATCH + 1, dtype=torch.float32, device="cuda")
    g = torch.empty(5313, dtype=torch.float32, device="cuda")
    l = torch.empty(1, dtype=torch.float32, device="cuda")
    with pytest.raises(frmi.FrError) as ei:
        ctx.mlp_grad_static(x, y, g, l)
    assert ei.value.status == frmi.FR_ERR_ARG
    with pytest.raises(frmi.FrError) as ei:
        ctx.mlp_grad_static(x[:0], y[:0], g, l)
    assert ei.value.status == frmi.FR_ERR_ARG
    ctx.close()
    fresh = frmi.Context(inputs.hex_box((2, 2, 2)), system=0, order=2)
    with pytest.raises(frmi.FrError) as ei:
        fresh.mlp_grad_static(x[:4], y[:4], g, l)
    assert ei.value.status == frmi.FR_ERR_STATE
    fresh.close()
