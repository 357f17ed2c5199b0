"""The C ABI from a plain C program (tests/capi_demo.c, built with the
library): a grid, an alpha_s table and query points are handed over in a
file; the program loads them with pdf_load_grid / pdf_load_alphas, evaluates
pdf_xfxq2 and pdf_alphas_q2 on the null stream and writes the results back,
which must match the oracle; it also trains a surrogate a few steps through
the training-options struct and evaluates it for every stored flavour and a
flavour subset, whose columns must be those of the full call."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2009_06635_amd import synth
from tolerance import check_f64, describe_failures, grid_L

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "capi_demo")


def write_input(path, g, qk, av, x, q2):
    K, P = len(g.xknots), len(g.pids)
    shape = np.array([[len(xk), len(qq)] for xk, qq in zip(g.xknots, g.q2knots)], np.int32).ravel()
    knots = np.concatenate([np.concatenate([xk, qq]) for xk, qq in zip(g.xknots, g.q2knots)]).astype(np.float64)
    values = np.concatenate([np.asarray(v, np.float64).ravel() for v in g.values])
    with open(path, "wb") as f:
        f.write(np.array([K, P], np.int32).tobytes())
        f.write(shape.tobytes())
        f.write(np.asarray(g.pids, np.int32).tobytes())
        f.write(np.array([len(knots)], np.int64).tobytes())
        f.write(knots.tobytes())
        f.write(np.array([len(values)], np.int64).tobytes())
        f.write(values.tobytes())
        f.write(np.array([len(qk)], np.int32).tobytes())
        f.write(np.asarray(qk, np.float64).tobytes())
        f.write(np.asarray(av, np.float64).tobytes())
        f.write(np.array([len(x)], np.int64).tobytes())
        f.write(np.asarray(x, np.float64).tobytes())
        f.write(np.asarray(q2, np.float64).tobytes())


def test_plain_c_program(tmp_path):
    assert os.path.exists(EXE), "tests/capi_demo is built with the library (paper_2009_06635_amd/build.py)"
    g = synth.config2_grid()
    qk, av = synth.config2_alphas()
    x, q2 = synth.config2_queries(n=5000, seed=60, out_fraction=0.05)
    x = np.concatenate([x, [0.0, np.nan]])
    q2 = np.concatenate([q2, [10.0, 10.0]])
    inp, outp = tmp_path / "in.bin", tmp_path / "out.bin"
    write_input(inp, g, qk, av, x, q2)
    res = subprocess.run([EXE, str(inp), str(outp)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    n, P = len(x), len(g.pids)
    buf = outp.read_bytes()
    raw = np.frombuffer(buf, np.float64, n * P + n + 1)
    xf = raw[:n * P].reshape(n, P)
    al = raw[n * P:n * P + n]
    nerr = raw[n * P + n:].view(np.int64)[0]
    f32 = np.frombuffer(buf, np.float32, offset=8 * (n * P + n + 1))
    sur = f32[:n * P].reshape(n, P)
    sub = f32[n * P:n * P + 3 * n].reshape(n, 3)
    loss = f32[n * P + 3 * n:]
    assert len(loss) == 5 and np.all(np.isfinite(loss)) and np.all(loss > 0)
    # the surrogate's flavour subset {21, last stored, -1} is those columns of the all-flavour call
    for j, pid in enumerate([21, g.pids[-1], -1]):
        assert np.array_equal(sub[:, j], sur[:, g.pids.index(pid)], equal_nan=True), pid
    ora, scale = oracle.xfxq2(oracle.Grid(g.xknots, g.q2knots, g.values, g.pids), g.pids, x, q2, with_scale=True)
    ok = check_f64(xf, ora, scale, grid_L(g))[0]
    assert ok.all(), describe_failures(ok, xf, ora, x, q2, g.pids)
    oa = oracle.alphas_q2(qk, av, q2)
    fin = ~np.isnan(oa)
    assert np.array_equal(np.isnan(al), np.isnan(oa))
    assert np.max(np.abs(al[fin] - oa[fin]) / np.abs(oa[fin])) < 1e-13
    assert nerr == 2  # the two invalid x (alpha_s sees valid Q^2 there)
