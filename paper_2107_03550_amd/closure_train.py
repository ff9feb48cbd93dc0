"""Training workflow of the learned tail closure (through the C ABI only).

    pairs = collect_pairs(plans, dt, steps, every)   # plain runs -> (X, Y) per kind
    nets = train_networks(pairs, steps=..., batch=..., lr=...)
    plan.set_closure(nets[0], nets[1], cut)

Pairs come from plain (full-window) FP32 runs: every ``every`` steps each
plan's history gives, for every mode the cut would close, the network input
and the exact tail scaled as the network's output (sbiem_closure_sample).
"""

from __future__ import annotations

import numpy as np

from ._lib import CLOSURE_PARAMS, ClosureTrainer


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases (float32, parameter order of the ABI)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = ((33, 64), (64,), (64, 64), (64,), (64, 2), (2,))
    parts = []
    for s in shapes:
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == CLOSURE_PARAMS
    return p


def collect_pairs(plans, dt, steps, every, cut=0.25, batch=None):
    """Run ``plans`` (plain FP32, state and dt set; a Batch may drive them)
    for ``steps`` steps, sampling every ``every`` steps.  Returns
    [(X_shear, Y_shear), (X_normal, Y_normal)] as float32 arrays."""
    xs = [[], []]
    ys = [[], []]
    done = 0
    while done < steps:
        k = min(every, steps - done)
        if batch is not None:
            batch.run(k)
        else:
            for p in plans:
                p.run(dt, k)
        done += k
        for p in plans:
            X, Y, R = p.closure_sample(cut)
            for kind in (0, 1):
                use = R[kind] > 0
                xs[kind].append(X[kind][use])
                ys[kind].append(Y[kind][use])
    return [(np.concatenate(xs[k]), np.concatenate(ys[k])) for k in (0, 1)]


def train_networks(pairs, steps=3000, batch=1024, lr=2e-3, seed=0, lr_final=2e-4):
    """One network per kind, Adam with a step size decaying geometrically from
    ``lr`` to ``lr_final``; the pairs are shuffled once (seeded).  Returns
    (params_shear, params_normal, losses_shear, losses_normal)."""
    out, losses = [], []
    rng = np.random.Generator(np.random.PCG64(seed))
    for kind, (X, Y) in enumerate(pairs):
        order = rng.permutation(len(X))
        X, Y = X[order], Y[order]
        tr = ClosureTrainer(init_params(seed + kind))
        chunk = 100
        ls = []
        for k0 in range(0, steps, chunk):
            frac = k0 / max(1, steps)
            ls.append(tr.train(X, Y, batch, min(chunk, steps - k0), lr * (lr_final / lr) ** frac))
        out.append(tr.params.copy())
        losses.append(np.concatenate(ls))
    return out[0], out[1], losses[0], losses[1]
