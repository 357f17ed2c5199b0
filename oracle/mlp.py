"""FP64 CPU oracle of the PDF surrogate network (test infrastructure only).

Network: (u, v) -> 64 -> 64 -> 64 -> 16, tanh hidden activations, linear
output, mean-squared-error loss over a batch.  Flat parameter layout (shared
with the library's checkpoints): W1[64][2], b1[64], W2[64][64], b2[64],
W3[64][64], b3[64], W4[16][64], b4[16].

Training (the library's optimiser; the surrogate is a growth path of this
project, so these follow their published definitions, not the paper):
  * ``adam_step``: one Adam update, Kingma & Ba, "Adam: a method for
    stochastic optimization" (ICLR 2015), algorithm 1, with bias-corrected
    first and second moments;
  * ``cosine_lr``: cosine annealing of the learning rate without restarts
    (Loshchilov & Hutter, "SGDR", ICLR 2017, eq. 5 with one period), indexed
    by the 0-based global step and held at its final value after the period;
  * ``train``: steps of (gradient of the step's batch at the current
    parameters, then ``adam_step`` at ``cosine_lr`` of that step).

Two evaluations:
  * ``loss_grad_f64``: plain FP64 forward/backward (pinned against central
    finite differences of its own loss in the tests);
  * ``loss_grad_device``: FP64 arithmetic on the operands the library's
    kernels consume, so that GPU outputs and gradients can be compared with
    it: the first layer (two inputs) in full precision; layers 2-4 as
    products of split BF16 operands (value = hi + lo, both BF16; products
    hi*hi + lo*hi + hi*lo); the backward pass on BF16-rounded signals,
    weights and layer inputs (hi halves), the first layer's weight gradient
    in full precision.
Written from the chain rule, independently of the HIP code.
"""
import math

import numpy as np

H, O = 64, 16
SHAPES = [("W1", (H, 2)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
          ("W4", (O, H)), ("b4", (O,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def _identity(a):
    return np.asarray(a, np.float64)


def split(a):
    """The BF16 pair (hi, lo) that carries a on the matrix cores: hi = bf16(a),
    lo = bf16(a - hi), so hi + lo holds about 16 significant bits of a."""
    a = np.asarray(a, np.float64)
    hi = bf16(a)
    return hi, bf16(a - hi)


def _plain_product(a, W):
    return a @ W.T


def _split_product(a, W):
    """sum_k a[b][k] W[n][k] from the BF16 halves of both operands:
    a_hi W_hi + a_lo W_hi + a_hi W_lo (the lo x lo term is not formed)."""
    ah, al = split(a)
    Wh, Wl = split(W)
    return ah @ Wh.T + al @ Wh.T + ah @ Wl.T


def _hi(a):
    return bf16(a)


def _loss_grad(p, inp, tgt, device):
    """device=False: plain FP64.  device=True: the operands of the library's
    kernels -- layer 1 in full precision on the given inputs, layers 2-4 as
    split-BF16 products; back-propagated signals and the weights and layer
    inputs they meet rounded to BF16 (hi halves)."""
    prod = _split_product if device else _plain_product
    rnd = bf16 if device else _identity
    hi = _hi if device else _identity
    P = unpack(p)
    W = {k: P[k] for k in P if k.startswith("W")}
    x = np.asarray(inp, np.float64)               # [B][2]
    z1 = x @ W["W1"].T + P["b1"]
    h1 = np.tanh(z1)
    h2 = np.tanh(prod(h1, W["W2"]) + P["b2"])
    h3 = np.tanh(prod(h2, W["W3"]) + P["b3"])
    y = prod(h3, W["W4"]) + P["b4"]
    a1, a2, a3 = hi(h1), hi(h2), hi(h3)
    B = inp.shape[0]
    d = y - tgt
    loss = np.mean(d * d)
    dy = 2.0 * d / (B * O)
    g = {}
    dyr = rnd(dy)
    g["W4"] = dyr.T @ a3
    g["b4"] = dy.sum(0)
    dh = dyr @ hi(W["W4"])
    dz = dh * (1.0 - h3 * h3)
    dzr = rnd(dz)
    g["W3"] = dzr.T @ a2
    g["b3"] = dz.sum(0)
    dh = dzr @ hi(W["W3"])
    dz = dh * (1.0 - h2 * h2)
    dzr = rnd(dz)
    g["W2"] = dzr.T @ a1
    g["b2"] = dz.sum(0)
    dh = dzr @ hi(W["W2"])
    dz = dh * (1.0 - h1 * h1)
    g["W1"] = dz.T @ x
    g["b1"] = dz.sum(0)
    return loss, pack(g), y


def loss_grad_f64(p, inp, tgt):
    """(loss, flat gradient, outputs) in plain FP64."""
    return _loss_grad(p, inp, np.asarray(tgt, np.float64), False)


def loss_grad_device(p, inp, tgt):
    """(loss, flat gradient, outputs) in FP64 on the operands the kernels use."""
    return _loss_grad(p, inp, np.asarray(tgt, np.float64), True)


def forward_device(p, inp):
    """Network outputs [B][16] on the kernels' operands (the inference path)."""
    return _loss_grad(p, inp, np.zeros((len(inp), O)), True)[2]


# ---- optimiser -------------------------------------------------------------------------

ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def cosine_lr(t, lr0, lr_final, total):
    """Learning rate of 0-based step t: lr_final + (lr0 - lr_final)(1 + cos(pi t/total))/2
    for t <= total, lr_final after."""
    frac = min(1.0, t / float(total))
    return lr_final + 0.5 * (lr0 - lr_final) * (1.0 + math.cos(math.pi * frac))


def adam_step(p, m, v, g, lr, t, b1=ADAM_B1, b2=ADAM_B2, eps=ADAM_EPS):
    """Adam update number t (>= 1) of parameters p with moments m, v and
    gradient g; returns the new (p, m, v)."""
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    p = np.asarray(p, np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v


def train(p0, batches, lr0, lr_final, total, grad=loss_grad_device, t0=0, m0=None, v0=None):
    """Run len(batches) steps from parameters p0 (global steps t0, t0+1, ...):
    each step takes the gradient of its batch (inp, tgt) at the current
    parameters, then one Adam update at cosine_lr of that step.  Returns
    (p, m, v, losses)."""
    p = np.asarray(p0, np.float64).copy()
    m = np.zeros_like(p) if m0 is None else np.asarray(m0, np.float64).copy()
    v = np.zeros_like(p) if v0 is None else np.asarray(v0, np.float64).copy()
    losses = []
    for i, (inp, tgt) in enumerate(batches):
        t = t0 + i
        loss, g, _ = grad(p, inp, tgt)
        losses.append(loss)
        p, m, v = adam_step(p, m, v, g, cosine_lr(t, lr0, lr_final, total), t + 1)
    return p, m, v, np.array(losses)
