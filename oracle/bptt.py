"""Surrogate-gradient backpropagation through time of a recurrent LIF network: the
forward pass and its hand-derived adjoint, written out from the definitions.

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU library.

Model (dimensionless, one step per dt).  Sec. I notes that backpropagation through
spikes needs a continuous stand-in for the spike; here it is a fast-sigmoid
surrogate:
    I_t  = W_in^T x_t + W_rec^T s_{t-1}
    V_t  = beta V_{t-1} + I_t - theta s_{t-1}          (reset by subtraction)
    s_t  = H(V_t - theta)                              spiking mode (H(0) = 1)
         = 1/2 + 1/2 a / (1 + |a|),  a = slope (V_t - theta)   smooth mode
    U_t  = beta_out U_{t-1} + W_out^T s_t              (leaky readout)
    L    = mean_b CE(max_t U_t[b], y_b)
with V_{-1} = s_{-1} = U_{-1} = 0.  The adjoint, for t = T-1 .. 0 with
lamU_T = lamV_T = 0:
    lamU_t = dL/dU_t + beta_out lamU_{t+1}
    dL/ds_t = W_out lamU_t + W_rec lamV_{t+1} - theta lamV_{t+1} [not if detach_reset]
    lamV_t = beta lamV_{t+1} + sigma'(V_t - theta) dL/ds_t
    dW_rec[i, j] = sum_{t,b} s_{t-1}[b, i] lamV_t[b, j]
    dW_in[c, j]  = sum_{t,b} x_t[b, c] lamV_t[b, j]
    dW_out[i, o] = sum_{t,b} s_t[b, i] lamU_t[b, o]
where dL/dU_t is non-zero only at the first time step that attains each maximum, and
sigma'(z) = 1 / (1 + slope |z|)^2 (spiking mode: the fast-sigmoid surrogate; the reset
term is detached) or 1/2 slope / (1 + slope |z|)^2 (smooth mode: the exact derivative
of s, reset term included, so that finite differences check every term).

Summation order of the forward currents: per target, sources in ascending index,
input projection first, then the recurrent one, accumulated one term at a time in the
requested dtype.  With float32 this is the GPU kernel's order, so both sides take
every spike decision and every argmax over time on identical values; the adjoint is
then compared within a tolerance.  Dense matrices carry exact zeros off the
connectivity masks (adding a zero term does not change a sum).
"""
import numpy as np


def _spike(z, slope, smooth, dt):
    if smooth:
        a = dt(slope) * z
        return dt(0.5) + dt(0.5) * (a / (dt(1.0) + np.abs(a)))
    return (z >= 0).astype(dt)


def _surrogate(z, slope, smooth):
    d = 1.0 + slope * np.abs(z)
    g = 1.0 / (d * d)
    return 0.5 * slope * g if smooth else g


def forward(x, w_in, w_rec, w_out, labels, beta, beta_out, theta=1.0, slope=25.0,
            smooth=False, dtype=np.float64):
    """x [B, T, C] (0/1), w_in [C, H], w_rec [H, H], w_out [H, O] dense with zeros off
    the masks; labels [B].  Returns the trajectories and the loss (float64)."""
    dt = np.dtype(dtype).type
    x = np.asarray(x, dtype)
    w_in, w_rec, w_out = (np.asarray(a, dtype) for a in (w_in, w_rec, w_out))
    B, T, C = x.shape
    H, O = w_out.shape
    b_, bo_, th_ = dt(beta), dt(beta_out), dt(theta)
    v = np.zeros((T, B, H), dtype)
    s = np.zeros((T, B, H), dtype)
    u = np.zeros((T, B, O), dtype)
    v_prev = np.zeros((B, H), dtype)
    s_prev = np.zeros((B, H), dtype)
    u_prev = np.zeros((B, O), dtype)
    for t in range(T):
        cur = np.zeros((B, H), dtype)
        # terms whose presynaptic value is zero for the whole batch are skipped: they
        # would add exact zeros
        for c in np.nonzero(x[:, t, :].any(axis=0))[0]:   # input projection, ascending
            cur = cur + x[:, t, c, None] * w_in[None, c, :]
        for i in np.nonzero(s_prev.any(axis=0))[0]:       # recurrent, ascending source
            cur = cur + s_prev[:, i, None] * w_rec[None, i, :]
        vt = b_ * v_prev
        vt = vt + cur
        vt = vt - th_ * s_prev
        st = _spike(vt - th_, slope, smooth, dt)
        ro = np.zeros((B, O), dtype)
        for i in np.nonzero(st.any(axis=0))[0]:           # readout, ascending source
            ro = ro + st[:, i, None] * w_out[None, i, :]
        ut = bo_ * u_prev
        ut = ut + ro
        v[t], s[t], u[t] = vt, st, ut
        v_prev, s_prev, u_prev = vt, st, ut
    # maximum over time and the first step that attains it
    m = u[0].copy()
    tmax = np.zeros((B, O), np.int64)
    for t in range(1, T):
        better = u[t] > m
        m = np.where(better, u[t], m)
        tmax = np.where(better, t, tmax)
    m64 = m.astype(np.float64)
    mx = m64.max(axis=1, keepdims=True)
    lse = mx[:, 0] + np.log(np.exp(m64 - mx).sum(axis=1))
    loss = float(np.mean(lse - m64[np.arange(B), labels]))
    return {"v": v, "s": s, "u": u, "m": m, "tmax": tmax, "loss": loss}


def backward(fw, x, w_in, w_rec, w_out, labels, beta, beta_out, theta=1.0, slope=25.0,
             smooth=False, detach_reset=None):
    """The adjoint of `forward` in float64 on the forward's trajectories.  Returns
    dense gradients (d_w_in, d_w_rec, d_w_out); callers read them on the masks."""
    if detach_reset is None:
        detach_reset = not smooth
    x = np.asarray(x, np.float64)
    w_rec = np.asarray(w_rec, np.float64)
    w_out = np.asarray(w_out, np.float64)
    v = fw["v"].astype(np.float64)
    s = fw["s"].astype(np.float64)
    T, B, H = v.shape
    O = w_out.shape[1]
    m = fw["m"].astype(np.float64)
    p = np.exp(m - m.max(axis=1, keepdims=True))
    p /= p.sum(axis=1, keepdims=True)
    dm = p.copy()
    dm[np.arange(B), labels] -= 1.0
    dm /= B
    lam_u = np.zeros((T, B, O))
    nxt = np.zeros((B, O))
    for t in range(T - 1, -1, -1):
        g = np.where(fw["tmax"] == t, dm, 0.0)
        nxt = g + beta_out * nxt
        lam_u[t] = nxt
    lam_v = np.zeros((T, B, H))
    nxt_v = np.zeros((B, H))
    for t in range(T - 1, -1, -1):
        ds = lam_u[t] @ w_out.T + nxt_v @ w_rec.T
        if not detach_reset:
            ds = ds - theta * nxt_v
        nxt_v = beta * nxt_v + _surrogate(v[t] - theta, slope, smooth) * ds
        lam_v[t] = nxt_v
    # sums over (t, b) as matrix products of the [T*B, .] trajectories
    s_prev = np.concatenate([np.zeros((1, B, H)), s[:-1]], axis=0)
    lv = lam_v.reshape(T * B, H)
    d_w_rec = s_prev.reshape(T * B, H).T @ lv
    d_w_in = x.transpose(1, 0, 2).reshape(T * B, -1).T @ lv
    d_w_out = s.reshape(T * B, H).T @ lam_u.reshape(T * B, O)
    return d_w_in, d_w_rec, d_w_out
