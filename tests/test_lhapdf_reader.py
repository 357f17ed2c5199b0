"""LHAPDF6 file reader (host only): lhagrid1 member files and .info alpha_s
lists, written by tests/lhapdf_files.py, read back exactly through the C ABI;
layout variants and malformed files."""
import os
import tempfile

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from paper_2009_06635_amd import synth
import lhapdf_files as lf

pdfmi = pytest.importorskip("paper_2009_06635_amd.pdfmi")


def write(tmp_path, g, name="m_0000.dat", **kw):
    p = tmp_path / name
    lf.write_member(p, [lf.q_of(q) for q in g.q2knots], g.xknots, g.values, g.pids, **kw)
    return p


def check_same(g, got):
    xk, qk, vs, pids = got
    assert pids == [int(p) for p in g.pids]
    assert len(xk) == g.K
    for k in range(g.K):
        assert np.array_equal(xk[k], g.xknots[k])
        assert np.array_equal(qk[k], lf.read_back_q2(lf.q_of(g.q2knots[k])))
        assert np.array_equal(vs[k], g.values[k])


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_round_trip(tmp_path, which):
    g = synth.config1_grid() if which == "c1" else synth.config2_grid()
    got = pdfmi.read_lhapdf(write(tmp_path, g))
    check_same(g, got)
    assert pdfmi.validate_grid(*got) == pdfmi.PDF_OK


def test_layout_variants(tmp_path):
    rng = np.random.default_rng(4)
    g = synth.tiny_grid(rng, K=2, nx=5, nq=[4, 6], npid=3, pids=[0, 1, -1])
    hdr = ("PdfType: central", "Format: lhagrid1", "FromMCReplica: 0", "  ")
    for kw in (dict(eol="\r\n"), dict(sep="  \t "), dict(header=hdr)):
        p = write(tmp_path, g, **kw)
        with open(p, "a") as f:
            f.write("\n\n")
        check_same(g, pdfmi.read_lhapdf(p))


def corrupt(tmp_path, g, fn):
    text = lf.member_text([lf.q_of(q) for q in g.q2knots], g.xknots, g.values, g.pids)
    p = tmp_path / "bad.dat"
    p.write_text(fn(text))
    return p


@pytest.mark.parametrize("case", ["no_sep", "short_row", "missing_rows", "pid_mismatch", "format", "not_number",
                                  "no_blocks", "unterminated"])
def test_malformed(tmp_path, case):
    rng = np.random.default_rng(5)
    g = synth.tiny_grid(rng, K=2, nx=4, nq=[4, 5], npid=2)
    lines_of = lambda t: t.split("\n")
    def drop_value(t):
        L = lines_of(t)
        L[5] = " ".join(L[5].split()[:-1])
        return "\n".join(L)
    def drop_row(t):
        L = lines_of(t)
        del L[6]
        return "\n".join(L)
    def pid_change(t):
        L = lines_of(t)
        i = [j for j, l in enumerate(L) if l == "---"][1] + 3   # flavour line of sub-grid 1
        L[i] = "21 3"
        return "\n".join(L)
    fns = {
        "no_sep": lambda t: t.replace("---\n", "", 1),
        "short_row": drop_value,
        "missing_rows": drop_row,
        "pid_mismatch": pid_change,
        "format": lambda t: t.replace("lhagrid1", "lhagrid2"),
        "not_number": lambda t: t.replace("e-01", "e-0x", 1) if "e-01" in t else t.replace("e+00", "e+0x", 1),
        "no_blocks": lambda t: "PdfType: central\nFormat: lhagrid1\n---\n",
        "unterminated": lambda t: t[: t.rstrip("\n").rfind("\n")],
    }
    with pytest.raises(pdfmi.PdfError) as e:
        pdfmi.read_lhapdf(corrupt(tmp_path, g, fns[case]))
    assert e.value.code == pdfmi.PDF_ERR_GRID


def test_missing_file(tmp_path):
    with pytest.raises(pdfmi.PdfError) as e:
        pdfmi.read_lhapdf(tmp_path / "nope.dat")
    assert e.value.code == pdfmi.PDF_ERR_ARG


def test_alphas_info(tmp_path):
    q2, a = synth.config2_alphas()
    q = lf.q_of(q2)
    p = tmp_path / "set.info"
    p.write_text(lf.info_text(q, a))
    rq2, ra = pdfmi.read_lhapdf_alphas(p)
    assert np.array_equal(rq2, lf.read_back_q2(q))
    assert np.array_equal(ra, a)
    assert pdfmi.validate_alphas(rq2, ra) == pdfmi.PDF_OK
    p.write_text(lf.info_text(q, a[:-1]))
    with pytest.raises(pdfmi.PdfError):
        pdfmi.read_lhapdf_alphas(p)
    p.write_text("AlphaS_Vals: [0.1, 0.2]\n")
    with pytest.raises(pdfmi.PdfError):
        pdfmi.read_lhapdf_alphas(p)


@settings(max_examples=40, deadline=None, derandomize=True)
@given(st.integers(1, 3), st.integers(2, 8), st.lists(st.integers(2, 6), min_size=3, max_size=3), st.integers(1, 13),
       st.lists(st.floats(allow_nan=False, allow_infinity=False), min_size=1, max_size=40),
       st.sampled_from(["\n", "\r\n"]), st.sampled_from([" ", "\t", "  \t "]), st.integers(0, 2**31 - 1))
def test_drawn_members_read_back_exactly(K, nx, nqs, npid, special, eol, sep, seed):
    """Drawn grid shapes and flavour counts, values of any finite magnitude
    and sign (subnormals, the largest doubles, signed zeros) planted among
    random ones, and drawn line ends and separators: read back bit for bit."""
    rng = np.random.default_rng(seed)
    g = synth.tiny_grid(rng, K=K, nx=nx, nq=nqs[:K], npid=npid)
    vals = [v.copy() for v in g.values]
    for s in special:
        k = int(rng.integers(0, K))
        vals[k][tuple(int(rng.integers(0, d)) for d in vals[k].shape)] = s
    g = g.with_values(vals)
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "m_0000.dat")
        lf.write_member(p, [lf.q_of(q) for q in g.q2knots], g.xknots, g.values, g.pids, eol=eol, sep=sep)
        check_same(g, pdfmi.read_lhapdf(p))
