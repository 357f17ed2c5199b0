"""A member loaded from an LHAPDF6 file gives bit-identical results to the
same arrays passed to pdf_load_grid, and the .info alpha_s table likewise."""
import numpy as np
import pytest

from paper_2009_06635_amd import synth
import lhapdf_files as lf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2009_06635_amd import pdfmi  # noqa: E402

DEV = "cuda:0"


def test_lhapdf_member_and_alphas(tmp_path):
    g = synth.config2_grid()
    p = tmp_path / "set_0000.dat"
    lf.write_member(p, [lf.q_of(q) for q in g.q2knots], g.xknots, g.values, g.pids)
    xk, qk, vs, pids = pdfmi.read_lhapdf(p)
    ma = pdfmi.load_lhapdf(p)
    mb = pdfmi.load_grid(xk, qk, vs, pids)
    try:
        x, q2 = synth.config2_queries(n=200_000, seed=77)
        xd = torch.from_numpy(x).to(DEV)
        qd = torch.from_numpy(q2).to(DEV)
        a = pdfmi.xfxq2(ma, g.pids, xd, qd).cpu().numpy()
        b = pdfmi.xfxq2(mb, g.pids, xd, qd).cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    finally:
        pdfmi.unload(ma)
        pdfmi.unload(mb)
    aq2, aa = synth.config2_alphas()
    info = tmp_path / "set.info"
    info.write_text(lf.info_text(lf.q_of(aq2), aa))
    rq2, ra = pdfmi.read_lhapdf_alphas(info)
    q = torch.from_numpy(np.exp(np.random.default_rng(3).uniform(-1.0, 25.0, 50_000))).to(DEV)
    pdfmi.load_lhapdf_alphas(info)
    r1 = pdfmi.alphas_q2(q).cpu().numpy()
    pdfmi.load_alphas(rq2, ra)
    r2 = pdfmi.alphas_q2(q).cpu().numpy()
    assert np.array_equal(r1.view(np.uint64), r2.view(np.uint64))
