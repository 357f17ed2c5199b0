"""Pins of the surrogate network's FP64 CPU oracle (no GPU): its backward pass
against central finite differences of its own loss, its BF16 rounding against
torch's float -> bfloat16 conversion, the split-BF16 operands of its device
form against the plain FP64 network, and its optimiser (Adam, cosine
learning-rate schedule) against closed-form trajectories and torch.optim."""
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


def test_split_pair_carries_16_bits():
    """hi + lo of the split BF16 pair is within 2^-17 relative of the value,
    hi is the BF16 rounding of the value and lo that of the remainder."""
    rng = np.random.default_rng(3)
    a = np.concatenate([rng.normal(0, 1, 5000), np.tanh(rng.normal(0, 2, 5000)), rng.normal(0, 1e-3, 2000)])
    hi, lo = mlp.split(a)
    assert np.array_equal(hi, mlp.bf16(a))
    assert np.all(np.abs(hi + lo - a) <= 2.0 ** -17 * np.abs(a))
    assert np.array_equal(lo, mlp.bf16(a - hi))


def test_device_forward_close_to_f64():
    """The kernels' split-BF16 products carry ~16 bits: outputs within 4e-5 of
    the plain FP64 network's scale; one BF16 half left out is ~100x worse."""
    rng = np.random.default_rng(4)
    p = rng.normal(0, 0.3, mlp.NPARAMS)
    inp = rng.uniform(-1, 1, (256, 2))
    y64 = mlp.loss_grad_f64(p, inp, np.zeros((256, 16)))[2]
    yd = mlp.forward_device(p, inp)
    assert np.max(np.abs(yd - y64)) <= 4e-5 * np.max(np.abs(y64))


def test_device_gradient_close_to_f64():
    rng = np.random.default_rng(2)
    p = rng.normal(0, 0.2, mlp.NPARAMS)
    inp = rng.uniform(-1, 1, (64, 2))
    tgt = rng.normal(0, 1, (64, 16))
    _, g64, _ = mlp.loss_grad_f64(p, inp, tgt)
    _, gd, _ = mlp.loss_grad_device(p, inp, tgt)
    assert np.linalg.norm(gd - g64) < 2e-2 * np.linalg.norm(g64)


# ---- optimiser pins: closed forms of Adam and the cosine schedule, and the
# independent implementations in torch.optim (same published definitions) ----

def test_adam_first_step_closed_form():
    """Step 1 from zero moments: m_hat = g and v_hat = g^2 exactly, so every
    parameter moves by lr g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    p = rng.normal(size=500)
    g = rng.normal(size=500) * 10.0 ** rng.uniform(-9, 2, 500)
    z = np.zeros(500)
    p1, m1, v1 = mlp.adam_step(p, z, z, g, 3e-3, 1)
    want = p - 3e-3 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p1, want, rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g, rtol=1e-15, atol=0) and np.allclose(v1, 1e-3 * g * g, rtol=1e-14, atol=0)


def test_adam_constant_gradient_trajectory():
    """A constant gradient keeps m_hat = g and v_hat = g^2 at every step, so
    after T steps p = p0 - sum_t lr_t g / (|g| + eps)."""
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=64)
    g = rng.normal(size=64)
    p, m, v = p0.copy(), np.zeros(64), np.zeros(64)
    lrs = [mlp.cosine_lr(t, 1e-2, 1e-4, 40) for t in range(60)]
    for t, lr in enumerate(lrs):
        p, m, v = mlp.adam_step(p, m, v, g, lr, t + 1)
    want = p0 - sum(lrs) * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(p - want)) <= 1e-12 * np.max(np.abs(p0 - want))


def test_adam_zero_gradient_is_a_no_op():
    p = np.random.default_rng(7).normal(size=100)
    z = np.zeros(100)
    q, m, v = p, z, z
    for t in range(1, 6):
        q, m, v = mlp.adam_step(q, m, v, z, 1e-2, t)
    assert np.array_equal(q, p) and not m.any() and not v.any()


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(8)
    p0 = rng.normal(size=300)
    grads = [rng.normal(size=300) * rng.uniform(0.01, 3.0) for _ in range(25)]
    lrs = [mlp.cosine_lr(t, 5e-3, 5e-5, 25) for t in range(25)]
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=lrs[0], betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0, np.zeros(300), np.zeros(300)
    for t, (g, lr) in enumerate(zip(grads, lrs)):
        for grp in opt.param_groups:
            grp["lr"] = lr
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = mlp.adam_step(p, m, v, g, lr, t + 1)
    assert np.max(np.abs(p - w.detach().numpy())) <= 1e-13 * np.max(np.abs(p - p0))


def test_cosine_schedule_end_points_and_torch():
    lr0, lrf, T = 3e-3, 3e-5, 1000
    assert mlp.cosine_lr(0, lr0, lrf, T) == lr0
    assert mlp.cosine_lr(T, lr0, lrf, T) == lrf and mlp.cosine_lr(5 * T, lr0, lrf, T) == lrf
    assert abs(mlp.cosine_lr(T // 2, lr0, lrf, T) - 0.5 * (lr0 + lrf)) < 1e-18
    seq = np.array([mlp.cosine_lr(t, lr0, lrf, T) for t in range(T + 1)])
    assert np.all(np.diff(seq) < 0)
    # torch's closed form of CosineAnnealingLR with eta_min = lr_final, T_max = total
    w = torch.zeros(1, requires_grad=True)
    sch = torch.optim.lr_scheduler.CosineAnnealingLR(torch.optim.SGD([w], lr=lr0), T_max=T, eta_min=lrf)
    for t in (0, 1, 7, 250, 500, 999, 1000):
        sch.last_epoch = t
        assert abs(sch._get_closed_form_lr()[0] - mlp.cosine_lr(t, lr0, lrf, T)) <= 1e-15


def test_train_applies_schedule_per_global_step():
    """train() from global step t0 equals the same steps taken one by one with
    adam_step at cosine_lr(t0 + i), the gradient taken at the current parameters."""
    rng = np.random.default_rng(9)
    p0 = rng.normal(0, 0.3, mlp.NPARAMS)
    batches = [(rng.uniform(-1, 1, (16, 2)), rng.normal(0, 1, (16, 16))) for _ in range(3)]
    p, m, v, losses = mlp.train(p0, batches, 1e-2, 1e-3, 10, grad=mlp.loss_grad_f64, t0=4)
    q, mq, vq = p0.copy(), np.zeros(mlp.NPARAMS), np.zeros(mlp.NPARAMS)
    for i, (inp, tgt) in enumerate(batches):
        loss, g, _ = mlp.loss_grad_f64(q, inp, tgt)
        assert loss == losses[i]
        q, mq, vq = mlp.adam_step(q, mq, vq, g, mlp.cosine_lr(4 + i, 1e-2, 1e-3, 10), 5 + i)
    assert np.array_equal(p, q) and np.array_equal(m, mq) and np.array_equal(v, vq)
