"""Pins of the learned indicator's FP64 oracle (CPU).  BF16 rounding, the
loss and Adam are checked against library routines; gradients against
central finite differences; features against hand-computed values."""
import numpy as np
import pytest
import torch

import synth
from oracle import OracleMesh
from oracle import mlp


def data(n=300, seed=3):
    X = synth.uniform_pm1(seed, n * 16).reshape(n, 16) * 2.0
    y = (np.floor((synth.uniform01(seed + 1, n)) * 3) - 1).astype(np.int8)
    return X, y


def test_bf16_rounding_matches_library_conversion():
    x = np.concatenate([synth.uniform_pm1(11, 5000) * 10.0 ** np.linspace(-5, 5, 5000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_loss_matches_library_cross_entropy():
    X, y = data()
    w = mlp.init_weights(5)
    cw = np.array([2.0, 0.5, 3.0])
    loss, _ = mlp.loss_and_grad(w, X, y, cw, emulate=False)
    z3 = torch.tensor(mlp.forward(w, X, emulate=False)["z3"])
    ref = torch.nn.functional.cross_entropy(z3, torch.tensor(y.astype(np.int64) + 1), weight=torch.tensor(cw))
    assert loss == pytest.approx(float(ref), rel=1e-12)


def test_gradient_matches_central_differences():
    X, y = data(120, 7)
    w = mlp.init_weights(9)
    cw = np.array([1.5, 1.0, 2.5])
    _, g = mlp.loss_and_grad(w, X, y, cw, emulate=False)
    rng = np.random.default_rng(0)
    idx = rng.choice(len(w), 200, replace=False)
    h = 1e-6
    fd = np.zeros(len(idx))
    for j, i in enumerate(idx):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd[j] = (mlp.loss_and_grad(wp, X, y, cw, emulate=False)[0] - mlp.loss_and_grad(wm, X, y, cw, emulate=False)[0]) / (2 * h)
    err = np.linalg.norm(fd - g[idx]) / np.linalg.norm(g[idx])
    assert err <= 1e-6, err


def test_emulated_gradient_close_to_exact():
    """BF16 operand rounding perturbs the gradient by ~2^-8 relative, no more."""
    X, y = data(200, 8)
    w = mlp.init_weights(10)
    cw = np.ones(3)
    _, ge = mlp.loss_and_grad(w, X, y, cw, emulate=True)
    _, gx = mlp.loss_and_grad(w, X, y, cw, emulate=False)
    assert np.linalg.norm(ge - gx) / np.linalg.norm(gx) < 3e-2


def test_adam_matches_library():
    w0 = mlp.init_weights(2)
    g = synth.uniform_pm1(4, len(w0))
    m = np.zeros_like(w0)
    v = np.zeros_like(w0)
    w, m, v = mlp.adam_step(w0, g, m, v, 1)
    w, m, v = mlp.adam_step(w, 0.5 * g, m, v, 2)
    p = torch.nn.Parameter(torch.tensor(w0))
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for gg in (g, 0.5 * g):
        opt.zero_grad()
        p.grad = torch.tensor(gg)
        opt.step()
    assert np.allclose(w, p.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_training_reduces_loss():
    X, y = data(400, 12)
    y = np.where(X[:, 0] > 0.5, 1, np.where(X[:, 0] < -0.5, -1, 0)).astype(np.int8)
    w = mlp.init_weights(3)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    l0 = mlp.loss_and_grad(w, X, y, np.ones(3))[0]
    for t in range(1, 301):
        _, g = mlp.loss_and_grad(w, X, y, np.ones(3))
        w, m, v = mlp.adam_step(w, g, m, v, t, lr=1e-2)
    l1 = mlp.loss_and_grad(w, X, y, np.ones(3))[0]
    assert l1 < 0.3 * l0


def test_features_hand_computed():
    """A density ramp rho = 1 + a x inside one block: r0 = a dx / rho_min over
    the block's cells (central difference of a linear profile); p uniform
    gives r1 = 0; neighbour slots copy the neighbours' values."""
    m = OracleMesh(3, (3, 1, 1), 8, 2, 1.0 / 3)
    xc = m.forest.cell_centres(8, 1.0 / 3)
    a = 0.3
    rho = 1.0 + a * xc[:, 0]
    U = synth.conserved_from_primitive(rho, [0 * rho] * 3, 1.0 + 0 * rho, 1.4)
    m.interior()[...] = np.moveaxis(U, 0, 1)
    m.ghost_fill()
    r = m.raw_features()
    dx = 1.0 / 24
    # middle block (away from the periodic seam): max at the smallest density
    rho_min = 1.0 + a * xc[1, 0].min()
    assert r[1, 0] == pytest.approx(a * dx / rho_min, rel=1e-12)
    assert r[1, 1] == 0.0
    F = mlp.features(m.forest, r, lmax=2, ndim=3)
    assert F[1, 0] == pytest.approx(np.log1p(r[1, 0]), rel=1e-15)
    assert F[1, 3] == pytest.approx(np.log1p(r[0, 0]), rel=1e-15)   # -x neighbour
    assert F[1, 5] == pytest.approx(np.log1p(r[2, 0]), rel=1e-15)   # +x neighbour
    assert np.all(F[:, 15] == 0)
