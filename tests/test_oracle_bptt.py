"""Pins of the BPTT oracle (oracle/bptt.py) against things other than itself:

  * smooth mode: the adjoint equals central finite differences of the loss (float64)
    for every weight on the masks, reset term included;
  * spiking mode: the adjoint equals PyTorch autograd (CPU, float64) of the same forward
    with a custom surrogate-gradient spike function and a detached reset;
  * the forward's membrane trajectory under constant input equals its closed form
    V_t = w (1 - beta^(t+1)) / (1 - beta) up to the first spike, which falls at the
    closed-form step, and reset by subtraction takes theta off the next step;
  * the loss equals torch's cross entropy of the maximum readout;
  * the float32 forward takes the same decisions as the float64 one on a small case
    and agrees within float32 rounding.
"""
import math

import numpy as np
import pytest

from oracle import bptt


def _instance(seed=0, B=3, T=40, C=12, H=32, O=4, p_in=0.3, p_rec=0.2, gain=2.0):
    rng = np.random.default_rng(seed)
    x = (rng.random((B, T, C)) < 0.3).astype(np.float64)
    m_in = rng.random((C, H)) < p_in
    m_rec = rng.random((H, H)) < p_rec
    np.fill_diagonal(m_rec, False)
    fan = C * p_in + H * p_rec
    w_in = gain * rng.standard_normal((C, H)) / math.sqrt(fan) * m_in
    w_rec = gain * rng.standard_normal((H, H)) / math.sqrt(fan) * m_rec
    w_out = rng.standard_normal((H, O)) / math.sqrt(H)
    y = rng.integers(0, O, size=B)
    return x, w_in, w_rec, w_out, y, m_in, m_rec


BETA = math.exp(-1.0 / 20.0)


def _loss(x, w_in, w_rec, w_out, y, smooth):
    return bptt.forward(x, w_in, w_rec, w_out, y, BETA, BETA, smooth=smooth)["loss"]


def test_smooth_adjoint_equals_finite_differences():
    x, w_in, w_rec, w_out, y, m_in, m_rec = _instance()
    fw = bptt.forward(x, w_in, w_rec, w_out, y, BETA, BETA, smooth=True)
    s = fw["s"]
    assert 0.05 < s.mean() < 0.95          # operating point where the sigmoid is not flat
    g_in, g_rec, g_out = bptt.backward(fw, x, w_in, w_rec, w_out, y, BETA, BETA, smooth=True)
    h = 1e-7   # truncation error falls as h^2 (checked down to 1e-7); rounding ~ 1e-9
    mats = {"in": (w_in, g_in, m_in), "rec": (w_rec, g_rec, m_rec),
            "out": (w_out, g_out, np.ones_like(w_out, bool))}
    for name, (w, g, mask) in mats.items():
        idx = np.argwhere(mask)
        worst = 0.0
        for (a, b) in idx:
            wp, wm = w.copy(), w.copy()
            wp[a, b] += h
            wm[a, b] -= h
            args_p = {"in": (wp, w_rec, w_out), "rec": (w_in, wp, w_out), "out": (w_in, w_rec, wp)}[name]
            args_m = {"in": (wm, w_rec, w_out), "rec": (w_in, wm, w_out), "out": (w_in, w_rec, wm)}[name]
            fd = (_loss(x, *args_p, y, True) - _loss(x, *args_m, y, True)) / (2 * h)
            worst = max(worst, abs(fd - g[a, b]))
        scale = np.abs(g[mask]).max()
        assert worst <= 1e-6 * scale + 1e-8, (name, worst, scale)


def test_spiking_adjoint_equals_torch_autograd_with_surrogate():
    torch = pytest.importorskip("torch")
    x, w_in, w_rec, w_out, y, m_in, m_rec = _instance(seed=1, T=60, gain=3.0)
    fw = bptt.forward(x, w_in, w_rec, w_out, y, BETA, BETA, smooth=False)
    assert fw["s"].sum() > 20
    g_in, g_rec, g_out = bptt.backward(fw, x, w_in, w_rec, w_out, y, BETA, BETA, smooth=False)

    class Spike(torch.autograd.Function):
        @staticmethod
        def forward(ctx, z):
            ctx.save_for_backward(z)
            return (z >= 0).to(z.dtype)

        @staticmethod
        def backward(ctx, g):
            (z,) = ctx.saved_tensors
            return g / (1.0 + 25.0 * z.abs()) ** 2

    X = torch.tensor(x)
    Wi = torch.tensor(w_in, requires_grad=True)
    Wr = torch.tensor(w_rec, requires_grad=True)
    Wo = torch.tensor(w_out, requires_grad=True)
    B, T, _ = x.shape
    v = torch.zeros(B, w_in.shape[1], dtype=torch.float64)
    s = torch.zeros_like(v)
    u = torch.zeros(B, w_out.shape[1], dtype=torch.float64)
    us = []
    for t in range(T):
        v = BETA * v + X[:, t] @ Wi + s @ Wr - 1.0 * s.detach()
        s = Spike.apply(v - 1.0)
        u = BETA * u + s @ Wo
        us.append(u)
    m = torch.stack(us).max(dim=0).values
    loss = torch.nn.functional.cross_entropy(m, torch.tensor(y))
    loss.backward()
    assert abs(loss.item() - fw["loss"]) < 1e-12
    for g, W, mask in ((g_in, Wi, m_in), (g_rec, Wr, m_rec), (g_out, Wo, None)):
        ref = W.grad.numpy()
        if mask is not None:
            ref = ref * mask
            g = g * mask
        assert np.abs(ref).max() > 0
        assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max()


def test_forward_closed_form_constant_input():
    T, w, theta = 80, 0.07, 1.0
    x = np.ones((1, T, 1))
    w_in = np.full((1, 1), w)
    w_rec = np.zeros((1, 1))
    w_out = np.ones((1, 1))
    fw = bptt.forward(x, w_in, w_rec, w_out, np.zeros(1, np.int64), BETA, BETA)
    v = fw["v"][:, 0, 0]
    closed = w * (1 - BETA ** (np.arange(T) + 1)) / (1 - BETA)
    first = int(np.argmax(closed >= theta))
    assert closed[first] >= theta and first > 0
    assert np.allclose(v[: first + 1], closed[: first + 1], rtol=1e-12, atol=0)
    assert fw["s"][:, 0, 0].nonzero()[0][0] == first
    # reset by subtraction: the step after the spike loses theta
    assert abs(v[first + 1] - (BETA * v[first] + w - theta)) < 1e-12


def test_loss_is_cross_entropy_of_max_readout():
    torch = pytest.importorskip("torch")
    x, w_in, w_rec, w_out, y, _, _ = _instance(seed=2, gain=3.0)
    fw = bptt.forward(x, w_in, w_rec, w_out, y, BETA, BETA)
    m = fw["u"].max(axis=0)
    assert np.array_equal(m, fw["m"])
    assert np.array_equal(fw["tmax"], fw["u"].argmax(axis=0))
    ce = torch.nn.functional.cross_entropy(torch.tensor(m), torch.tensor(y)).item()
    assert abs(ce - fw["loss"]) < 1e-12


def test_float32_forward_tracks_float64():
    x, w_in, w_rec, w_out, y, _, _ = _instance(seed=3, gain=3.0)
    f64 = bptt.forward(x, w_in, w_rec, w_out, y, BETA, BETA)
    f32 = bptt.forward(x, w_in, w_rec, w_out, y, BETA, BETA, dtype=np.float32)
    assert f32["v"].dtype == np.float32
    assert np.array_equal(f32["s"], f64["s"].astype(np.float32))
    assert np.all(np.abs(f32["v"] - f64["v"]) <= 1e-5 * (np.abs(f64["v"]) + 1.0))
    assert abs(f32["loss"] - f64["loss"]) < 1e-5
