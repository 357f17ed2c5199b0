"""Parity criteria between the HIP path and the FP64 oracle.

Stated tolerances: FP64 values within 1e-12 relative; FP32-arithmetic values
within 1e-5 relative wherever |xf| > 1e-8; indices and knot values bit-exact.

A literal relative bound cannot hold where the interpolant cancels to near
zero (both sides correct, rounding of O(M) terms left in an O(0) result), so
each bound carries the arithmetic's own floor: c * eps * S, where S is the
oracle's error scale of that value (largest stencil magnitude, propagated
through any extrapolation formula) and, in FP64, (1 + L) covers the rounding
of the cell parameter u (log of a ratio times 1/Delta: L = largest 1/Delta of
the grid).  The literal pass fraction is always reported next to it.

Values outside the arithmetic's range: an extrapolated value beyond the FP64
range is the same infinity on both sides; an oracle value at or beyond the
top of the FP32 range is, in FP32 arithmetic, the infinity of its sign
(round-to-nearest overflow), which is what the FP32 variant must return.
"""
import numpy as np

EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps
F32_MAX = float(np.finfo(np.float32).max)


def grid_L(grid):
    inv = []
    for xk, qk in zip(grid.xknots, grid.q2knots):
        inv.append(np.max(1.0 / np.diff(np.log(xk))))
        inv.append(np.max(1.0 / np.diff(np.log(qk))))
    return float(np.max(inv[0::2]) + np.max(inv[1::2]))


def check_f64(gpu, ora, scale, L, rtol=1e-12, c=4.0):
    """Returns (ok mask, literal-pass fraction, max eq.(1) difference)."""
    gpu = np.asarray(gpu, np.float64)
    both_nan = np.isnan(gpu) & np.isnan(ora)
    same_inf = np.isinf(ora) & (gpu == ora)  # an extrapolation beyond the FP64 range, on both sides
    with np.errstate(invalid="ignore"):  # inf - inf where both overflowed: taken by same_inf
        diff = np.abs(gpu - ora)
    ok = both_nan | same_inf | (diff <= rtol * np.abs(ora) + c * EPS64 * scale * (1.0 + L))
    finite = np.isfinite(ora)
    lit = both_nan | same_inf | (diff <= rtol * np.abs(ora))
    r = diff[finite] / (np.abs(ora[finite]) + 1e-16)
    return ok, float(lit.mean()), float(r.max()) if r.size else 0.0


def check_f32(gpu, ora, scale, rtol=1e-5, floor=1e-8, c=4.0):
    gpu = np.asarray(gpu, np.float64)
    both_nan = np.isnan(gpu) & np.isnan(ora)
    with np.errstate(invalid="ignore"):  # inf - inf beyond the FP32 range: taken by `over` below
        diff = np.abs(gpu - ora)
    small = np.abs(ora) <= floor
    # a value at or beyond the top of the FP32 range is the infinity of its sign in
    # FP32 arithmetic (round-to-nearest overflow), which no relative bound expresses
    over = (np.abs(ora) >= F32_MAX * (1.0 - rtol)) & np.isinf(gpu) & (np.sign(gpu) == np.sign(ora))
    ok = both_nan | small | over | (diff <= rtol * np.abs(ora) + c * EPS32 * scale)
    lit = both_nan | small | over | (diff <= rtol * np.abs(ora))
    finite = np.isfinite(ora) & ~small & ~over
    r = diff[finite] / (np.abs(ora[finite]) + 1e-16)
    return ok, float(lit.mean()), float(r.max()) if r.size else 0.0


def describe_failures(ok, gpu, ora, x, q2, pids, limit=5):
    bad = np.argwhere(~ok)
    lines = []
    for i, j in bad[:limit]:
        lines.append("point %d (x=%r, q2=%r) pid %r: gpu=%r oracle=%r" % (i, x[i], q2[i], pids[j], gpu[i, j], ora[i, j]))
    return "%d mismatches; first: \n" % len(bad) + "\n".join(lines)
