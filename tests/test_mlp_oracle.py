"""Pins of the surrogate network's FP64 CPU oracle (no GPU): its backward pass
against central finite differences of its own loss, and its BF16 rounding
against torch's float -> bfloat16 conversion."""
import numpy as np
import torch

from oracle import mlp


def test_param_layout_count():
    assert mlp.NPARAMS == 64 * 2 + 64 + 2 * (64 * 64 + 64) + 16 * 64 + 16


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, mlp.NPARAMS)
    inp = rng.uniform(-1, 1, (8, 2))
    tgt = rng.normal(0, 1, (8, 16))
    loss, g, _ = mlp.loss_grad_f64(p, inp, tgt)
    idx = np.concatenate([rng.choice(mlp.NPARAMS, 300, replace=False), np.arange(128, 192), [mlp.NPARAMS - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAMS)
        e[i] = h
        fd = (mlp.loss_grad_f64(p + e, inp, tgt)[0] - mlp.loss_grad_f64(p - e, inp, tgt)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    # exact ties (low 16 bits 0x8000) with even and odd upper halves: round half to even
    hi = rng.integers(0x0080, 0x7F00, 2000).astype(np.uint32)
    ties = ((hi << 16) | 0x8000).view(np.float32).astype(np.float64)
    a = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 5000), rng.uniform(-1e4, 1e4, 5000),
                        ties, -ties])
    want = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(a), want)


def test_bf16_gradient_close_to_f64():
    rng = np.random.default_rng(2)
    p = rng.normal(0, 0.2, mlp.NPARAMS)
    inp = rng.uniform(-1, 1, (64, 2))
    tgt = rng.normal(0, 1, (64, 16))
    _, g64, _ = mlp.loss_grad_f64(p, inp, tgt)
    _, g16, _ = mlp.loss_grad_bf16(p, inp, tgt)
    assert np.linalg.norm(g16 - g64) < 2e-2 * np.linalg.norm(g64)
