"""tests/golden/tiny_grid.json (written by tests/golden/make_golden.py from
oracle/ only): the oracle must reproduce it bit for bit (any change to the
oracle's arithmetic shows here and must be justified), and the HIP path must
match it within the parity tolerance."""
import json
import os

import numpy as np
import pytest

import oracle
from tolerance import check_f32, check_f64

HERE = os.path.dirname(os.path.abspath(__file__))


def load():
    with open(os.path.join(HERE, "golden", "tiny_grid.json")) as f:
        d = json.load(f)
    g = oracle.Grid([np.array(a) for a in d["xknots"]], [np.array(a) for a in d["q2knots"]],
                    [np.array(v) for v in d["values"]], d["pids"])
    f64 = lambda a: np.array([float(v) for v in a])  # noqa: E731
    return (d, g, f64(d["x"]), f64(d["q2"]), np.array([[float(v) for v in r] for r in d["xf"]]),
            np.array([[float(v) for v in r] for r in d["xf_scale"]]), f64(d["alphas"]))


def grid_L(g):
    return float(max(np.max(1.0 / np.diff(np.log(t))) for t in g.xknots)
                 + max(np.max(1.0 / np.diff(np.log(t))) for t in g.q2knots))


def test_oracle_reproduces_golden():
    d, g, x, q2, xf, sc, al = load()
    o, s = oracle.xfxq2(g, d["pids"], x, q2, with_scale=True)
    assert np.array_equal(o.view(np.uint64), xf.view(np.uint64))
    assert np.array_equal(s.view(np.uint64), sc.view(np.uint64))
    a = oracle.alphas_q2(np.array(d["alphas_q2knots"]), np.array(d["alphas_values"]), q2)
    assert np.array_equal(a.view(np.uint64), al.view(np.uint64))


def test_golden_covers_every_region():
    d, g, x, q2, xf, sc, al = load()
    k, ix, iq, reg = oracle.locate(g, x, q2)
    assert {0, 1, 2, 3, 4, 5, 8} <= set(np.unique(reg).tolist())   # inside, low x, low/high Q^2, corners, invalid
    assert np.any(q2 == g.q2knots[1][0]) and np.any(k == 1) and np.any(k == 0)


@pytest.mark.gpu
def test_gpu_matches_golden():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2009_06635_amd import pdfmi
    d, g, x, q2, xf, sc, al = load()
    m = pdfmi.load_grid(g.xknots, g.q2knots, g.vals, d["pids"])
    try:
        pdfmi.load_alphas(np.array(d["alphas_q2knots"]), np.array(d["alphas_values"]))
        xd = torch.from_numpy(x).to("cuda:0")
        qd = torch.from_numpy(q2).to("cuda:0")
        o64, a = pdfmi.xfxq2_alphas(m, d["pids"], xd, qd)
        o32 = pdfmi.xfxq2_f32(m, d["pids"], xd, qd)
        assert check_f64(o64.cpu().numpy(), xf, sc, grid_L(g))[0].all()
        assert check_f32(o32.cpu().numpy(), xf, sc)[0].all()
        a = a.cpu().numpy()
        fin = ~np.isnan(al)
        assert np.array_equal(np.isnan(a), np.isnan(al))
        assert np.max(np.abs(a[fin] - al[fin]) / np.abs(al[fin])) < 1e-13
    finally:
        pdfmi.unload(m)
