"""FP64 CPU oracle of the PDF surrogate network (test infrastructure only).

Network: (u, v) -> 64 -> 64 -> 64 -> 16, tanh hidden activations, linear
output, mean-squared-error loss over a batch.  Flat parameter layout (shared
with the library's checkpoints): W1[64][2], b1[64], W2[64][64], b2[64],
W3[64][64], b3[64], W4[16][64], b4[16].

Two evaluations:
  * ``loss_grad_f64``: plain FP64 forward/backward (pinned against central
    finite differences of its own loss in the tests);
  * ``loss_grad_bf16``: FP64 arithmetic on the BF16-rounded operands that the
    matrix-core kernels consume (weights, layer inputs, back-propagated
    signals), so that GPU gradients can be compared with it.
Written from the chain rule, independently of the HIP code.
"""
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


def _loss_grad(p, inp, tgt, rnd):
    P = unpack(p)
    x = rnd(inp)                                   # [B][2]
    W = {k: (rnd(P[k]) if k.startswith("W") else P[k]) for k in P}
    z1 = x @ W["W1"].T + P["b1"]
    h1 = np.tanh(z1)
    a1 = rnd(h1)
    h2 = np.tanh(a1 @ W["W2"].T + P["b2"])
    a2 = rnd(h2)
    h3 = np.tanh(a2 @ W["W3"].T + P["b3"])
    a3 = rnd(h3)
    y = a3 @ W["W4"].T + P["b4"]
    B = inp.shape[0]
    d = y - tgt
    loss = np.mean(d * d)
    dy = 2.0 * d / (B * O)
    g = {}
    dyr = rnd(dy)
    g["W4"] = dyr.T @ a3
    g["b4"] = dy.sum(0)
    dh = dyr @ W["W4"]
    dz = dh * (1.0 - h3 * h3)
    dzr = rnd(dz)
    g["W3"] = dzr.T @ a2
    g["b3"] = dz.sum(0)
    dh = dzr @ W["W3"]
    dz = dh * (1.0 - h2 * h2)
    dzr = rnd(dz)
    g["W2"] = dzr.T @ a1
    g["b2"] = dz.sum(0)
    dh = dzr @ W["W2"]
    dz = dh * (1.0 - h1 * h1)
    dzr = rnd(dz)
    g["W1"] = dzr.T @ x
    g["b1"] = dz.sum(0)
    return loss, pack(g), y


def loss_grad_f64(p, inp, tgt):
    """(loss, flat gradient, outputs) in plain FP64."""
    return _loss_grad(p, np.asarray(inp, np.float64), np.asarray(tgt, np.float64), _identity)


def loss_grad_bf16(p, inp, tgt):
    """(loss, flat gradient, outputs) in FP64 on BF16-rounded matrix operands."""
    return _loss_grad(p, np.asarray(inp, np.float64), np.asarray(tgt, np.float64), bf16)


def forward_bf16(p, inp):
    """Network outputs [B][16] on BF16-rounded operands (inference path)."""
    return _loss_grad(p, np.asarray(inp, np.float64), np.zeros((len(inp), O)), bf16)[2]
