"""Training data and training loop of the learned warm start.

The data are the solver's own results: a cold-started rollout records, for
every world and step, the features of the step (state, previous impulses by
slot, generalized forces of the step) and the converged impulses by slot.
The network is trained on the device by the library's matrix-core forward,
backward and Adam kernels; PyTorch only holds the buffers and draws the
minibatch permutation.
"""
from __future__ import annotations

import numpy as np
import torch

from . import kamx


def collect(model, steps, device="cuda:0"):
    """Run ``steps`` steps of ``model`` (in its current warm-start mode) and
    return features X [steps * n_worlds, n_features] and targets
    Y [steps * n_worlds, n_slots] as device tensors."""
    nf, ns = model.feature_dims()
    n = model.n_worlds
    X = torch.empty((steps * n, nf), dtype=torch.float32, device=device)
    Y = torch.empty((steps * n, ns), dtype=torch.float32, device=device)
    for s in range(steps):
        model.features(out=X[s * n:(s + 1) * n])
        model.step(1)
        model.impulse_slots(out=Y[s * n:(s + 1) * n])
    torch.cuda.synchronize()
    return X, Y


def normalization(X, Y):
    """Per-column mean and standard deviation of inputs and targets.  An
    input's spread is floored at 1e-3 of its root-mean-square value, so
    nearly constant columns (quaternion components of bodies that hardly
    turn) are not scaled up to their rounding noise."""
    mu, sd = X.mean(dim=0), X.std(dim=0)
    rms = torch.sqrt(mu * mu + sd * sd)
    sd = torch.sqrt(sd * sd + (1e-3 * rms) ** 2 + 1e-12)
    return mu, sd, Y.mean(dim=0), Y.std(dim=0)


def train(net, X, Y, epochs=20, batch=4096, lr=1e-3, lr_final=1e-5, seed=0, log=None):
    """Adam over shuffled minibatches with a cosine learning-rate decay from
    ``lr`` to ``lr_final``.  Returns the mean loss of every epoch."""
    g = torch.Generator(device=X.device)
    g.manual_seed(int(seed))
    n = X.shape[0]
    nb = n // batch
    total = max(epochs * nb, 1)
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    acc = torch.zeros(1, dtype=torch.float32, device=X.device)
    history = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=X.device)
        acc.zero_()
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * k / total))
            net.train_step(X.index_select(0, idx), Y.index_select(0, idx), rate, loss=loss)
            acc += loss
            k += 1
        history.append(float(acc.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {history[-1]:.4e}")
    return history


def validation_loss(net, X, Y, batch=4096):
    """Mean squared error of the standardised outputs (no update)."""
    n = X.shape[0]
    se, cnt = 0.0, 0
    sd = net.out_std
    for b in range(0, n - batch + 1, batch):
        y = net.forward(X[b:b + batch])
        t = Y[b:b + batch]
        se += float((((y - t) / sd) ** 2).sum().item())
        cnt += t.numel()
    return se / max(cnt, 1)


def fit(model_factory, train_steps, epochs=60, batch=4096, lr=1e-3, seed=0, n_hidden=256, log=None, capacity=None):
    """Collect a cold rollout from ``model_factory()`` and train a network
    on it (batch capacity: ``capacity`` worlds, at least ``batch``).
    Returns (net, info)."""
    m = model_factory()
    X, Y = collect(m, train_steps)
    nf, ns = m.feature_dims()
    m.close()
    mu_x, sd_x, mu_y, sd_y = normalization(X, Y)
    net = kamx.MLP(nf, ns, n_hidden=n_hidden, max_batch=max(batch, capacity or 0), seed=seed)
    net.set_normalization(mu_x, sd_x, mu_y, sd_y + 1e-6)
    net.out_mean, net.out_std = mu_y, sd_y + 1e-6
    # hold out the last tenth of the rollout
    n_val = max(X.shape[0] // 10 // batch, 1) * batch
    hist = train(net, X[:-n_val], Y[:-n_val], epochs=epochs, batch=batch, lr=lr, seed=seed, log=log)
    val = validation_loss(net, X[-n_val:], Y[-n_val:], batch=batch)
    return net, dict(samples=int(X.shape[0] - n_val), held_out=int(n_val), train_loss=hist, val_loss=val)
