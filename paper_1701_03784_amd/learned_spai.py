"""Training of the learned-SPAI network on the device (axp_mlp_* kernels).

Training data are the pattern pairs of meshes whose plain SPAI the library
computes (axp_spai_pairs); the loss is the weighted mean squared error of
the predicted Jacobi-scaled entries.  PyTorch only holds the device buffers.
"""

from __future__ import annotations

import time

import numpy as np

from .axpic import Mlp, make_ctx


def training_pairs(meshes, spai_level=3, max_pairs_per_mesh=None, seed=0, log=None):
    """Features and targets of the plain SPAI of every mesh (synth.Mesh-like)."""
    rng = np.random.default_rng(seed)
    Xs, ys = [], []
    for i, m in enumerate(meshes):
        t0 = time.perf_counter()
        c = make_ctx(m, spai_level=spai_level, dt=1e-30)
        X, y, _ = c.spai_pairs()
        c.close()
        if max_pairs_per_mesh is not None and len(y) > max_pairs_per_mesh:
            sel = rng.choice(len(y), max_pairs_per_mesh, replace=False)
            X, y = X[sel], y[sel]
        Xs.append(X)
        ys.append(y)
        if log:
            log(f"training mesh {i}: {m.n_tris} faces, {len(y)} pairs ({time.perf_counter() - t0:.1f} s)")
    return np.concatenate(Xs), np.concatenate(ys)


def train(net: Mlp, X, y, epochs=20, batch=8192, lr=2e-3, lr_final=2e-4, seed=0, log=None):
    """Adam on shuffled minibatches (one shuffle, then sequential batches).
    Returns the mean training loss of every epoch."""
    import torch
    n = len(y)
    perm = np.random.default_rng(seed).permutation(n)
    Xd = torch.from_numpy(np.ascontiguousarray(X[perm], dtype=np.float32)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y[perm], dtype=np.float32)).cuda()
    wd = torch.ones(n, dtype=torch.float32, device="cuda")
    hist = []
    steps = epochs * ((n + batch - 1) // batch)
    k = 0
    for ep in range(epochs):
        tot = 0.0
        for b0 in range(0, n, batch):
            b1 = min(n, b0 + batch)
            loss = net.loss_grad(Xd[b0:b1], yd[b0:b1], wd[b0:b1])
            tot += loss * (b1 - b0)
            a = k / max(1, steps - 1)
            net.adam_step(lr * (1 - a) + lr_final * a)
            k += 1
        hist.append(tot / n)
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.3e}")
    return hist
