"""GPU: surrogate-network kernels (BF16 MFMA forward and backward, Adam)
against the FP64 reference with BF16 rounding at the same points.

Bars: the two sides round the same values to BF16, but a value computed in
FP32 on the device and in FP64 on the host can land on different sides of a
BF16 rounding boundary (probability ~1e-5 per value, error 2^-8 relative
when it happens).  The 3-256-256-256-10 network at batch 512 holds about
1.3e5 BF16 activations per layer, so a few such flips per layer are
expected, each moving the relative L2 of a tensor by about
2^-8 / sqrt(1.3e5) ~ 1e-5; measured over three seeds: outputs <= 7.4e-5,
gradients <= 3.2e-4 (a bias row).  Tensors are therefore held to relative
L2 2e-4 (outputs) and 1e-3 (gradients), the loss to 1e-4; a 1 %-scale
mistake (a transposed stride, a dropped bias row sum) fails them tenfold.
The small networks have no flips at these seeds and agree to ~3e-8.
"""
import sys

import numpy as np
import pytest
import torch

import paper_1705_01801_amd as lbw
from oracle import mlp as ref

pytestmark = pytest.mark.gpu

WIDTHS = [3, 256, 256, 256, 10]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def setup(seed, B, widths=WIDTHS):
    rng = np.random.default_rng(seed)
    p = ref.init_params(widths, rng) + rng.normal(scale=0.02, size=sum(
        widths[l] * widths[l + 1] + widths[l + 1] for l in range(len(widths) - 1)))
    p = p.astype(np.float32).astype(np.float64)
    x = rng.uniform(-1, 1, size=(B, widths[0])).astype(np.float32).astype(np.float64)
    t = rng.normal(size=(B, widths[-1])).astype(np.float32).astype(np.float64)
    w = (rng.uniform(size=(B, widths[-1])) > 0.1).astype(np.float64)
    net = lbw.MLP(widths, max_batch=max(B, 64))
    net.set_params(p)
    return net, p, x, t, w


@pytest.mark.parametrize("widths,B", [(WIDTHS, 512), ([3, 40, 17, 10], 37), ([5, 33, 1], 1)])
def test_forward_matches_reference(widths, B):
    net, p, x, _, _ = setup(3, B, widths)
    say("mlp forward", widths, B)
    y = net.forward(x).cpu().numpy()
    yr, _ = ref.forward(p, widths, x)
    assert rel(y, yr) <= 2e-4
    assert np.array_equal(net.get_params(), p.astype(np.float32))


@pytest.mark.parametrize("widths,B", [(WIDTHS, 512), ([3, 40, 17, 10], 37)])
def test_gradients_match_reference(widths, B):
    net, p, x, t, w = setup(4, B, widths)
    say("mlp gradients", widths, B)
    loss, grad = net.loss_grad(x, t, w, want_grad=True)
    lr_, gr = ref.loss_grad(p, widths, x, t, w)
    assert abs(loss.item() / lr_ - 1) <= 1e-4
    g = grad.cpu().numpy()
    off = 0
    for l in range(len(widths) - 1):
        nW = widths[l] * widths[l + 1]
        nb = widths[l + 1]
        assert rel(g[off: off + nW], gr[off: off + nW]) <= 1e-3, ("W", l)
        off += nW
        assert rel(g[off: off + nb], gr[off: off + nb]) <= 1e-3, ("b", l)
        off += nb


def test_adam_step_matches_reference():
    net, p, x, t, w = setup(5, 128)
    _, grad = net.loss_grad(x, t, w, want_grad=True)
    g = grad.cpu().numpy().astype(np.float64)
    net.adam_step(lr=1e-3)
    p1 = net.get_params().astype(np.float64)
    pr, _, _ = ref.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, 1e-3, 0.9, 0.999, 1e-8)
    assert np.abs(p1 - pr).max() <= 1e-6


def test_training_reduces_loss():
    rng = np.random.default_rng(6)
    widths = [3, 64, 64, 4]
    net = lbw.MLP(widths, max_batch=256)
    net.set_params(ref.init_params(widths, rng))
    x = rng.uniform(-1, 1, size=(256, 3))
    t = np.stack([np.sin(2 * x[:, 0]) * x[:, 1], x[:, 2] ** 2, np.cos(x.sum(1)), x[:, 0] * x[:, 2]], axis=1)
    l0 = net.loss_grad(x, t)[0].item()
    for _ in range(600):
        net.loss_grad(x, t)
        net.adam_step(lr=3e-3)
    l1 = net.loss_grad(x, t)[0].item()
    say("mlp training loss", l0, "->", l1)
    assert l1 < l0 / 50


def test_mlp_errors():
    with pytest.raises(lbw.LbwError):
        lbw.MLP([3, 0, 2], max_batch=4)
    net = lbw.MLP([3, 8, 2], max_batch=4)
    with pytest.raises(lbw.LbwError):
        net.adam_step()
    x = torch.zeros((5, 3), dtype=torch.float32, device="cuda")
    y = torch.zeros((5, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(lbw.LbwError):  # batch above max_batch
        lbw.check(lbw.lib().lbw_mlp_forward(net.handle, x.data_ptr(), 5, y.data_ptr()))
    assert net.forward(np.zeros((5, 3), np.float32)).shape == (5, 2)  # the binding splits large batches


@pytest.mark.parametrize("widths,B,steps", [(WIDTHS, 512, 25), ([3, 40, 17, 10], 37, 7)])
def test_graph_training_matches_step_by_step(widths, B, steps):
    """lbw_mlp_train (one captured step replayed, schedule on the device)
    against the same steps issued one call at a time with the rate computed
    on the host: the same arithmetic, so the parameters agree to float
    rounding of the schedule."""
    import math
    netA, p, x, t, w = setup(7, B, widths)
    netB, _, _, _, _ = setup(7, B, widths)
    dev = torch.device("cuda", torch.cuda.current_device())
    xt = torch.as_tensor(x.astype(np.float32), device=dev)
    tt = torch.as_tensor(t.astype(np.float32), device=dev)
    wt = torch.as_tensor(w.astype(np.float32), device=dev)
    wsum = float(w.sum())
    say("mlp graph training", widths, B, steps)
    lossA = netA.train(xt, tt, wt, steps=steps, lr=3e-3, lr_floor=1e-5, weight_sum=wsum)
    for s in range(steps):
        lossB = netB.loss_grad(xt, tt, wt, weight_sum=wsum)[0].item()
        netB.adam_step(lr=3e-3 * 0.5 * (1.0 + math.cos(math.pi * (s / steps))) + 1e-5)
    pa, pb = netA.get_params(), netB.get_params()
    assert np.abs(pa - pb).max() <= 1e-5 * np.abs(pb).max(), np.abs(pa - pb).max()
    assert abs(lossA - lossB) <= 1e-5 * abs(lossB)
    # training moved the parameters and continues from the same Adam state
    assert np.abs(pa - p.astype(np.float32)).max() > 1e-4
    netA.train(xt, tt, wt, steps=3, lr=1e-3, weight_sum=wsum)
    for s in range(3):
        netB.loss_grad(xt, tt, wt, weight_sum=wsum)
        netB.adam_step(lr=1e-3 * 0.5 * (1.0 + math.cos(math.pi * (s / 3))) + 1e-5)
    assert np.abs(netA.get_params() - netB.get_params()).max() <= 1e-5 * np.abs(pb).max()
    with pytest.raises(lbw.LbwError):
        netA.train(xt, tt, wt, steps=0)
