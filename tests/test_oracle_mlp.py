"""Pins of the FP64 warm-start network reference (oracle/mlp.py): bfloat16
rounding against hand-worked bit patterns and torch's independent
conversion, GELU against its closed form and torch's erf implementation,
gradients against central finite differences, Adam against its closed form
under a constant gradient."""
import math

import numpy as np
import pytest

from oracle import mlp as M


def test_bf16_round_bit_patterns():
    one = 1.0
    assert M.bf16_round(one) == 1.0
    # exactly half an ulp (2^-8) above 1: tie, mantissa of 1 is even
    assert M.bf16_round(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8: tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert M.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    # just above the tie rounds up
    assert M.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert M.bf16_round(-(1.0 + 2.0 ** -8 + 2.0 ** -20)) == -(1.0 + 2.0 ** -7)
    assert M.bf16_round(0.0) == 0.0
    assert np.isinf(M.bf16_round(3.4028234663852886e38))  # FP32 max rounds past the bf16 max
    assert np.isnan(M.bf16_round(np.nan))


def test_bf16_round_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 5000), rng.normal(0, 1e4, 5000)])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def test_gelu_closed_form_and_torch():
    torch = pytest.importorskip("torch")
    assert M.gelu(np.array([0.0]))[0] == 0.0
    # gelu(1) = Phi(1) = 0.5 (1 + erf(1/sqrt 2))
    assert abs(M.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    z = np.linspace(-8, 8, 1601)
    ref = torch.nn.functional.gelu(torch.tensor(z, dtype=torch.float64), approximate="none").numpy()
    assert np.abs(M.gelu(z) - ref).max() < 1e-15
    assert abs(M.gelu(np.array([30.0]))[0] - 30.0) < 1e-12 and abs(M.gelu(np.array([-30.0]))[0]) < 1e-12
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.abs(M.gelu_grad(z) - fd).max() < 1e-8


def tiny_net(rng, n_in=5, n_hidden=8, n_out=3, bf16_weights=False):
    fp, op = M.pad64(n_in), M.pad64(n_out)
    W1 = np.zeros((n_hidden, fp))
    W1[:, :n_in] = rng.normal(0, 0.6, (n_hidden, n_in))
    W3 = np.zeros((op, n_hidden))
    W3[:n_out] = rng.normal(0, 0.5, (n_out, n_hidden))
    b3 = np.zeros(op)
    b3[:n_out] = rng.normal(0, 0.1, n_out)
    net = M.MLP(n_in, n_hidden, n_out, W1, rng.normal(0, 0.1, n_hidden), rng.normal(0, 0.4, (n_hidden, n_hidden)),
                rng.normal(0, 0.1, n_hidden), W3, b3,
                mu_in=np.r_[rng.normal(0, 1, n_in), np.zeros(fp - n_in)],
                s_in=np.r_[rng.uniform(0.5, 2, n_in), np.ones(fp - n_in)],
                mu_out=np.r_[rng.normal(0, 1, n_out), np.zeros(op - n_out)],
                sigma_out=np.r_[rng.uniform(0.5, 2, n_out), np.ones(op - n_out)])
    if bf16_weights:
        for p in (net.W1, net.W2, net.W3):
            p[...] = M.bf16_round(p)
    return net


@pytest.mark.parametrize("bf16_weights", [False, True])
def test_gradients_against_finite_differences(bf16_weights):
    rng = np.random.default_rng(1)
    net = tiny_net(rng, bf16_weights=bf16_weights)
    x = rng.normal(0, 1, (7, net.n_in))
    t = rng.normal(0, 1, (7, net.n_out))
    loss, grads = M.loss_and_grads(net, x, t, bf16=False)
    h = 1e-6
    for p, g in zip(net.params(), grads):
        flat = p.reshape(-1)
        gflat = g.reshape(-1)
        # active entries only (padding columns of W1 see x^ = 0; padded outputs are masked)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = M.loss_and_grads(net, x, t, bf16=False)
            flat[i] = old - h
            lm, _ = M.loss_and_grads(net, x, t, bf16=False)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[i]) <= 1e-6 * max(abs(fd), 1e-3), (p.shape, i, fd, gflat[i])


def test_output_destandardisation_and_padding_mask():
    rng = np.random.default_rng(2)
    net = tiny_net(rng)
    x = rng.normal(0, 1, (4, net.n_in))
    y, c = M.forward(net, x, bf16=False)
    assert y.shape == (4, net.n_out)
    assert np.allclose(y, net.mu_out[:3] + net.sigma_out[:3] * c["yn"][:, :3], rtol=0, atol=1e-14)
    # padded inputs carry zero after normalisation whatever mu_in holds there
    net.mu_in[net.n_in:] = 5.0
    assert np.all(M.normalise_input(net, x)[:, net.n_in:] == 0.0)
    # targets equal to the prediction give zero loss and zero gradients
    loss, grads = M.loss_and_grads(net, x, y, bf16=False)
    assert loss < 1e-28 and max(np.abs(g).max() for g in grads) < 1e-14


def test_adam_closed_form_under_constant_gradient():
    """With a constant gradient g the bias-corrected moments equal g and g^2
    at every step, so each update is lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    net = tiny_net(rng)
    before = [p.copy() for p in net.params()]
    g = [rng.normal(0, 1, p.shape) for p in net.params()]
    lr = 1e-3
    for k in range(1, 6):
        M.adam_step(net, g, lr)
        for p0, p, gg in zip(before, net.params(), g):
            expect = p0 - k * lr * gg / (np.abs(gg) + M.ADAM_EPS)
            assert np.abs(p - expect).max() < 1e-12


def test_bf16_emulated_gradients_stay_near_exact():
    """Rounding the operands to bfloat16 perturbs gradients by about the
    bfloat16 unit (2^-8 relative); a wrong rounding point or a dropped term
    would not stay this close."""
    rng = np.random.default_rng(4)
    net = tiny_net(rng, n_in=40, n_hidden=32, n_out=16)
    x = rng.normal(0, 1, (64, net.n_in))
    t = rng.normal(0, 1, (64, net.n_out))
    _, g64 = M.loss_and_grads(net, x, t, bf16=False)
    _, g16 = M.loss_and_grads(net, x, t, bf16=True)
    for a, b in zip(g64, g16):
        assert np.abs(a - b).max() <= 0.03 * np.abs(a).max()


def test_training_reduces_loss_on_a_linear_map():
    rng = np.random.default_rng(5)
    net = tiny_net(rng, n_in=6, n_hidden=16, n_out=4)
    A = rng.normal(0, 1, (4, 6))
    x = rng.normal(0, 1, (128, 6))
    t = net.mu_out[:4] + x @ A.T
    first = None
    for _ in range(300):
        loss, grads = M.loss_and_grads(net, x, t, bf16=False)
        first = loss if first is None else first
        M.adam_step(net, grads, 1e-2)
    assert loss < 0.05 * first
    assert not math.isnan(loss)
