"""Queries from several host threads, each on its own stream, against one
loaded member: every thread's outputs must be bit-identical to the same
calls made from one thread, and each thread's error message stays its own.
"""
import threading

import numpy as np
import pytest

from paper_2009_06635_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2009_06635_amd import pdfmi  # noqa: E402

DEV = "cuda:0"
NTHREADS = 4


@pytest.fixture(scope="module")
def setup():
    g = synth.config2_grid()
    m = pdfmi.load_synth(g)
    pdfmi.load_alphas(*synth.config2_alphas())
    inputs = []
    for t in range(NTHREADS):
        x, q2 = synth.config2_queries(n=200_000 + 977 * t, seed=700 + t, out_fraction=0.05)
        inputs.append((torch.from_numpy(x).to(DEV), torch.from_numpy(q2).to(DEV)))
    # reference: the same calls from this thread, one after the other
    ref = []
    for xd, qd in inputs:
        o64, a = pdfmi.xfxq2_alphas(m, g.pids, xd, qd)
        o32 = pdfmi.xfxq2_f32(m, g.pids[::2], xd, qd)
        ref.append((o64.cpu(), a.cpu(), o32.cpu()))
    yield g, m, inputs, ref
    pdfmi.unload(m)


def test_threads_on_their_own_streams_match_serial(setup):
    g, m, inputs, ref = setup
    results = [None] * NTHREADS
    errors = []

    def work(t):
        try:
            s = torch.cuda.Stream()
            xd, qd = inputs[t]
            with torch.cuda.stream(s):
                o64 = torch.empty((xd.shape[0], len(g.pids)), dtype=torch.float64, device=DEV)
                a = torch.empty(xd.shape[0], dtype=torch.float64, device=DEV)
                o32 = torch.empty((xd.shape[0], len(g.pids[::2])), dtype=torch.float32, device=DEV)
                for _ in range(5):
                    pdfmi.xfxq2_alphas(m, g.pids, xd, qd, out=o64, alphas_out=a, stream=s)
                    pdfmi.xfxq2_f32(m, g.pids[::2], xd, qd, out=o32, stream=s)
            s.synchronize()
            results[t] = (o64.cpu(), a.cpu(), o32.cpu())
        except Exception as exc:  # reported by the main thread
            errors.append(repr(exc))

    threads = [threading.Thread(target=work, args=(t,)) for t in range(NTHREADS)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert not errors, errors
    for t in range(NTHREADS):
        for got, want in zip(results[t], ref[t]):
            assert torch.equal(got, want), t


def test_error_messages_are_per_thread(setup):
    g, m, inputs, _ = setup
    xd, qd = inputs[0]
    seen = {}
    ready = threading.Barrier(2)

    def bad():
        with pytest.raises(pdfmi.PdfError):
            pdfmi.xfxq2(m, [7], xd, qd)  # invalid flavour id
        seen["bad"] = pdfmi.last_error()
        ready.wait()

    def good():
        ready.wait()
        seen["good"] = pdfmi.last_error()

    threads = [threading.Thread(target=bad), threading.Thread(target=good)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
    assert "flavour" in seen["bad"]
    assert "flavour" not in seen["good"]
