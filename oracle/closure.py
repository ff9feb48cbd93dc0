"""Learned tail closure: reference definitions (FP64, test infrastructure).

The plain method sums each mode's history over its whole window of M_n lags
(section 3.1).  The closure keeps only the newest M'_n = ceil(c M_n) lags
(c = 1/4) of modes with M'_n >= 18 and replaces the discarded tail

    tail^X_n = sum_{j = M'_n}^{M_n - 1} w^X_{n,j} H^X_n(lag j),   X in {T, N},

by a small network per history kind.  None of this is in the paper: parity
of the closure's accuracy is unpinned by it (the plain full-window method
is the reference), while the network arithmetic below is pinned by finite
differences and by the identities in ``tests/test_oracle_closure.py``.

Network input (33 reals): T_cut / 100 with T_cut = c_s |k_n| M'_n dt, then
the 16 oldest kept history values a_k = H^X_n(lag M'_n - 16 + k),
k = 0..15, as (Re, Im) pairs divided by their RMS r = sqrt(mean |a_k|^2).
Output (2 reals) y, a correction to the constant extrapolation of the
oldest kept value a_15 over the discarded lags:

    tail = D^X_n a_15 + (y_0 + i y_1) r / (c_s |k_n|),
    D^X_n = sum_{j = M'_n}^{M_n - 1} w^X_{n,j}.

With y = 0 the closure is exact for a history that stays constant beyond
the kept window.  Hidden layers
2 x 64 with the erf form of GELU.  Parameters (6466 reals, this order):
W1[33][64], b1[64], W2[64][64], b2[64], W3[64][2], b3[2], with
h1 = gelu(x W1 + b1), h2 = gelu(h1 W2 + b2), y = h2 W3 + b3.
Inference on the GPU uses bfloat16 weights and layer inputs with float32
accumulation; ``forward(..., bf16=True)`` reproduces those roundings.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_IN, N_HID, N_OUT = 33, 64, 2
N_AMP = 16
MIN_KEPT = N_AMP + 2        # M' >= 18: the 16 inputs are lags >= 2 (ring entries)
T_SCALE = 100.0
SHAPES = ((N_IN, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_OUT), (N_OUT,))
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def unpack(p):
    """Split a flat parameter vector into (W1, b1, W2, b2, W3, b3)."""
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts])


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = math.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, size=s))
        else:
            parts.append(np.zeros(s))
    return pack(parts)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(p, x, bf16_inputs=False):
    """y for inputs x (n, 33).  With ``bf16_inputs`` the three weight
    matrices and the three layer inputs are rounded to bfloat16 first."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    r = bf16 if bf16_inputs else (lambda a: a)
    z1 = r(x) @ r(W1) + b1
    h1 = gelu(z1)
    z2 = r(h1) @ r(W2) + b2
    h2 = gelu(z2)
    return r(h2) @ r(W3) + b3


def loss_and_grad(p, x, t):
    """Mean squared error L = mean over samples of sum_o (y_o - t_o)^2 and
    its gradient with respect to the flat parameters (analytic backward)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    z1 = x @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    y = h2 @ W3 + b3
    d = y - t
    L = float(np.sum(d * d) / n)
    dy = 2.0 * d / n
    gW3 = h2.T @ dy
    gb3 = dy.sum(0)
    dz2 = (dy @ W3.T) * gelu_grad(z2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    return L, pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_steps(p, m, v, t, x, y, batch, steps, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """``steps`` Adam updates; minibatch k is rows [k*batch, (k+1)*batch)
    of (x, y) taken cyclically from the first row after the previous call's
    last (the caller passes t = updates so far).  Returns (p, m, v, t, losses)."""
    p, m, v = (np.array(a, dtype=np.float64) for a in (p, m, v))
    n = x.shape[0]
    losses = []
    for _ in range(steps):
        start = (t * batch) % n
        idx = (start + np.arange(batch)) % n
        L, g = loss_and_grad(p, x[idx], y[idx])
        losses.append(L)
        t += 1
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p = p - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v, t, np.array(losses)


# ----------------------------------------------------------------- windows
def kept_lags(M, cut=0.25):
    """M'_n = ceil(cut M_n) where M'_n >= 18 and M'_n < M_n, else M_n (the
    mode keeps its whole window)."""
    M = np.asarray(M, dtype=np.int64)
    Mk = np.ceil(cut * M - 1e-9).astype(np.int64)
    use = (Mk >= MIN_KEPT) & (Mk < M)
    return np.where(use, Mk, M), use


def features(H_lags, Mk, Tcut):
    """Network input and scale r for one mode and kind.

    ``H_lags[j]`` is the history value at lag j (index 0 unused); returns
    (x (33,), r) with r = 0 (and x = 0) when the 16 values are all zero."""
    a = np.array([H_lags[Mk - N_AMP + k] for k in range(N_AMP)], dtype=np.complex128)
    r = math.sqrt(float(np.mean(np.abs(a) ** 2)))
    x = np.zeros(N_IN)
    x[0] = Tcut / T_SCALE
    if r > 0:
        x[1::2] = a.real / r
        x[2::2] = a.imag / r
    return x, r


def discarded_weight(w_mode, Mk, M):
    """D = sum of the weights of the discarded lags Mk .. M-1 (``w_mode[j]``
    is the weight of lag j)."""
    return float(np.sum(np.asarray(w_mode, dtype=np.float64)[Mk:M]))


def oldest_kept(x, r):
    """a_15, the oldest kept history value, from the network input."""
    return (x[..., 31] + 1j * x[..., 32]) * r


def tail_from_output(y, r, cs_k, D, a_old):
    """tail = D a_15 + (y_0 + i y_1) r / (c_s |k_n|)."""
    return D * a_old + (y[..., 0] + 1j * y[..., 1]) * r / cs_k


def target_from_tail(tail, r, cs_k, D, a_old):
    """The output a perfect network would give: (tail - D a_15) c_s |k_n| / r."""
    z = (tail - D * a_old) * cs_k / r
    return np.stack([z.real, z.imag], axis=-1)
