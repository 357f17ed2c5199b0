"""Pins of the FK-contraction oracle: closed forms (one-hot tables pick single
PDF values, an all-ones table gives exact row sums), linearity, and plain
loops on tiny inputs."""
import math

import numpy as np

from oracle import fk


def test_one_hot_table_selects_values():
    rng = np.random.default_rng(0)
    pdf = rng.normal(size=(5, 37))
    ks = [0, 3, 36, 17]
    table = np.zeros((len(ks), 37))
    for d, k in enumerate(ks):
        table[d, k] = 1.0
    assert np.array_equal(fk.contract(pdf, table), pdf[:, ks])


def test_ones_table_gives_row_sums():
    rng = np.random.default_rng(1)
    pdf = rng.integers(-1000, 1000, size=(4, 50)).astype(np.float64)   # exact in FP64
    out = fk.contract(pdf, np.ones((3, 50)))
    for r in range(4):
        assert np.all(out[r] == math.fsum(pdf[r]))


def test_loops_and_linearity():
    rng = np.random.default_rng(2)
    pdf = rng.normal(size=(3, 11))
    t1, t2 = rng.normal(size=(4, 11)), rng.normal(size=(4, 11))
    a = fk.contract(pdf, t1)
    assert np.allclose(a, fk.contract_loops(pdf, t1), rtol=1e-14, atol=1e-14)
    assert np.allclose(fk.contract(pdf, 2.0 * t1 - t2), 2.0 * a - fk.contract(pdf, t2), rtol=1e-13, atol=1e-13)
    assert np.all(fk.abs_scale(pdf, t1) >= np.abs(a))
