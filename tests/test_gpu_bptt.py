"""GPU parity of the surrogate-gradient BPTT form (forward + hand-written adjoint,
through the C ABI and the torch.autograd.Function) against the oracle:

  * forward: the oracle's float32 forward sums every current in the kernel's order, so
    spikes, membrane checkpoints, readout maxima and their steps must be bit-identical;
    the loss (float32 on the GPU, float64 in the oracle) within 1e-5 relative;
  * backward: the oracle's float64 adjoint on the same trajectory; every gradient entry
    within 1e-4 relative, with an absolute floor of 1e-6 of the largest entry of its
    matrix, for the spiking mode and the smooth mode (whose oracle adjoint is pinned to
    finite differences), on ragged checkpoint segments and a batch below one wavefront;
  * autograd: loss.backward() through the Function equals the plan's backward, scaled
    by the incoming gradient;
  * the full recurrent workload (64 x 250 steps, 700 inputs, 1,024 hidden, 20 readouts).
"""
import math

import numpy as np
import pytest

from oracle import bptt as ob
from paper_1912_07423_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-4    # elementwise relative bar of the gradients
FLOOR = 1e-6   # absolute floor, as a fraction of the matrix's largest entry


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    return gpu_available


def _run(d, checkpoint, smooth=False, g_scale=None, eager=False):
    import torch
    from paper_1912_07423_amd.bptt import RecurrentLIF
    B, T, C = d["x"].shape
    H, O = d["w_out"].shape
    plan = RecurrentLIF(d["mask_in"], d["mask_rec"], O, B, T, checkpoint=checkpoint,
                        dt_ms=d["dt_ms"], smooth=smooth, eager=eager)
    v_in, v_rec = plan.csr_values(d["w_in"], d["w_rec"])
    dev = plan.device
    x = torch.tensor(d["x"], device=dev)
    w_in = torch.tensor(v_in, device=dev, requires_grad=True)
    w_rec = torch.tensor(v_rec, device=dev, requires_grad=True)
    w_out = torch.tensor(d["w_out"], device=dev, requires_grad=True)
    y = torch.tensor(d["labels"].astype(np.int32), device=dev)
    loss = plan.loss(x, w_in, w_rec, w_out, y)
    (loss * g_scale if g_scale is not None else loss).backward()
    torch.cuda.synchronize()
    return plan, loss.item(), (w_in.grad.cpu().numpy(), w_rec.grad.cpu().numpy(),
                               w_out.grad.cpu().numpy())


def _compare(d, checkpoint, smooth=False):
    B, T, C = d["x"].shape
    beta = math.exp(-d["dt_ms"] / 20.0)
    plan, loss, (g_in, g_rec, g_out) = _run(d, checkpoint, smooth)
    # dense float32 weights exactly as the GPU holds them
    w_in = np.zeros_like(d["w_in"], np.float32)
    w_rec = np.zeros_like(d["w_rec"], np.float32)
    w_in[d["mask_in"]] = d["w_in"][d["mask_in"]]
    w_rec[d["mask_rec"]] = d["w_rec"][d["mask_rec"]]
    fw = ob.forward(d["x"], w_in, w_rec, d["w_out"], d["labels"], np.float32(beta), np.float32(beta),
                    smooth=smooth, dtype=np.float32)
    s, vck, m, tm = plan.trace()
    assert np.array_equal(s.view(np.uint32), fw["s"].view(np.uint32)), "spikes differ"
    ck = [min(t, T - 1) for t in range(checkpoint - 1, T + checkpoint - 1, checkpoint)]
    assert np.array_equal(vck.view(np.uint32), fw["v"][ck].view(np.uint32)), "checkpoints differ"
    assert np.array_equal(m.view(np.uint32), fw["m"].view(np.uint32))
    assert np.array_equal(tm, fw["tmax"])
    assert abs(loss - fw["loss"]) <= 1e-5 * abs(fw["loss"])
    r_in, r_rec, r_out = ob.backward(fw, d["x"], w_in, w_rec, d["w_out"], d["labels"],
                                     float(np.float32(beta)), float(np.float32(beta)), smooth=smooth)
    got_in, got_rec = plan.dense(g_in, g_rec)
    for name, got, ref, mask in (("in", got_in, r_in, d["mask_in"]), ("rec", got_rec, r_rec, d["mask_rec"]),
                                 ("out", g_out, r_out, None)):
        if mask is not None:
            ref = ref * mask
        scale = np.abs(ref).max()
        if scale == 0:            # e.g. recurrent weights of a one-step sequence
            assert not np.any(got), name
            continue
        # elementwise: |got - ref| <= 1e-4 |ref| + a floor of 1e-6 of the matrix's largest
        # entry (float32 sums of up to B T terms cancel in the smallest entries)
        err = np.abs(got - ref)
        bound = RTOL * np.abs(ref) + FLOOR * scale
        worst = np.unravel_index(np.argmax(err / bound), err.shape)
        rel = err / np.maximum(np.abs(ref), FLOOR * scale)
        print(f"[bptt] d{name}: max elementwise |err| / (|ref| or the floor) = {rel.max():.2e}, "
              f"max |err| / max |ref| = {err.max() / scale:.2e}", flush=True)
        assert np.all(err <= bound), (name, worst, got[worst], ref[worst])
    return plan, fw


def _small(seed=5, B=8, T=60, C=20, H=48, O=5):
    return W.bptt_inputs(batch=B, steps=T, n_in=C, n_hidden=H, n_out=O, p_in=0.4, p_rec=0.3,
                         rate_lo=100.0, rate_hi=400.0, seed=seed)


@pytest.mark.parametrize("checkpoint", [7, 25, 1])
def test_spiking_mode_matches_oracle(checkpoint):
    d = _small()
    plan, fw = _compare(d, checkpoint)
    assert fw["s"].sum() > 50


def test_smooth_mode_matches_oracle():
    _compare(_small(seed=6), 10, smooth=True)


def test_inputs_other_than_0_and_1():
    """Inputs that are not all 0 or 1 (some spikes scaled by 0.5 or 3) take the value
    gathers instead of the batch masks, with the oracle's results."""
    d = _small(seed=10)
    rng = np.random.default_rng(10)
    d["x"] = (d["x"] * rng.choice(np.array([0.5, 1.0, 3.0], np.float32), size=d["x"].shape)).astype(np.float32)
    assert np.any((d["x"] != 0) & (d["x"] != 1))
    _compare(d, 10)


def test_recurrent_rows_wider_than_the_ell_form():
    """In-degrees above 256 (300 hidden neurons, p_rec = 0.95) leave the hidden steps on
    the CSR form of the recurrent sums; the results are the oracle's all the same."""
    d = W.bptt_inputs(batch=8, steps=30, n_in=20, n_hidden=300, n_out=5, p_in=0.4, p_rec=0.95,
                      rate_lo=100.0, rate_hi=400.0, seed=11)
    assert d["mask_rec"].sum(axis=0).max() > 256
    plan, fw = _compare(d, 10)
    assert fw["s"].sum() > 50


def test_batch_below_one_wavefront_and_single_step():
    _compare(_small(seed=7, B=3, T=1), 4)
    _compare(_small(seed=8, B=64, T=33, H=70), 32)


def test_autograd_scales_with_incoming_gradient():
    d = _small(seed=9)
    _, _, g1 = _run(d, 10)
    _, _, g3 = _run(d, 10, g_scale=3.0)
    for a, b in zip(g1, g3):
        # the incoming 3 enters at dL/dmax, so the roundings differ from 3 x (gradient):
        # elementwise 1e-5 relative with the floor of the oracle comparison
        ref = 3.0 * a
        assert np.all(np.abs(b - ref) <= 1e-5 * np.abs(ref) + FLOOR * np.abs(ref).max())


@pytest.mark.parametrize("smooth", [False, True])
def test_graph_replays_equal_eager_launches(smooth):
    """The passes' bodies replayed from their HIP graphs give bit-identical losses and
    gradients to the same kernels launched one by one, on every replay, with other
    eager work (weight updates, a second plan, host reads) between the replays."""
    import torch
    from paper_1912_07423_amd.bptt import RecurrentLIF
    d = _small(seed=12)
    B, T, C = d["x"].shape
    H, O = d["w_out"].shape
    plans = {e: RecurrentLIF(d["mask_in"], d["mask_rec"], O, B, T, checkpoint=9, dt_ms=d["dt_ms"],
                             smooth=smooth, eager=e) for e in (True, False)}
    v_in, v_rec = plans[True].csr_values(d["w_in"], d["w_rec"])
    dev = plans[True].device
    x = torch.tensor(d["x"], device=dev)
    y = torch.tensor(d["labels"].astype(np.int32), device=dev)
    w0 = [torch.tensor(v_in, device=dev), torch.tensor(v_rec, device=dev), torch.tensor(d["w_out"], device=dev)]
    for rep in range(4):
        out = {}
        for e, plan in plans.items():
            ws = [w.clone().requires_grad_(True) for w in w0]
            loss = plan.loss(x, *ws, y)
            loss.backward()
            torch.cuda.synchronize()
            out[e] = [loss.detach().cpu().numpy()] + [w.grad.cpu().numpy() for w in ws]
        for a, b in zip(out[True], out[False]):
            assert np.array_equal(np.asarray(a).view(np.uint32), np.asarray(b).view(np.uint32)), f"replay {rep}"
        # eager work between replays: a small weight change, read back on the host
        w0 = [w + 1e-3 * torch.sin(w * (rep + 1)) for w in w0]
        assert np.isfinite(w0[0].cpu().numpy()).all()


def test_full_recurrent_workload():
    d = W.bptt_inputs()
    print("[bptt] full size: B=64 T=250 C=700 H=1024 O=20", flush=True)
    _compare(d, 25)
