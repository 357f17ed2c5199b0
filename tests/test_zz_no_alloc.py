"""pdf_fk_contract_noalloc (partial sums in the library's fixed device scratch
array, no allocation) against pdf_fk_contract (partial sums in a workspace the
library allocates), through the C ABI: bit-identical outputs on two calls in a
row, the second smaller than the first, a call needing no partial sums, and a
size whose partial sums exceed the scratch (rejected before anything is
queued, output untouched)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2009_06635_amd import pdfmi  # noqa: E402

DEV = "cuda:0"
LIB = pdfmi.library()
P = ctypes.c_void_p


def call(fn, pdf, table, out):
    nrep, K = pdf.shape
    ndat = table.shape[0]
    rc = fn(P(pdf.data_ptr()), P(table.data_ptr()), ctypes.c_int32(nrep), ctypes.c_int32(ndat),
            ctypes.c_int64(K), P(out.data_ptr()), P(0))
    return rc


def both(nrep, ndat, K, seed):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    pdf = torch.randn((nrep, K), dtype=torch.float64, device=DEV, generator=g)
    table = torch.randn((ndat, K), dtype=torch.float64, device=DEV, generator=g)
    want = torch.full((nrep, ndat), float("nan"), dtype=torch.float64, device=DEV)
    got = torch.full((nrep, ndat), float("nan"), dtype=torch.float64, device=DEV)
    assert call(LIB.pdf_fk_contract, pdf, table, want) == pdfmi.PDF_OK, pdfmi.last_error()
    torch.cuda.synchronize()
    assert call(LIB.pdf_fk_contract_noalloc, pdf, table, got) == pdfmi.PDF_OK, pdfmi.last_error()
    torch.cuda.synchronize()
    return want, got


def test_noalloc_matches_allocating_call_twice():
    # first call: K = 31395 (a 2415-point x grid times 13 flavours) splits into many slices
    print("noalloc call 1: nrep 100, ndat 256, K 31395", flush=True)
    want, got = both(100, 256, 31395, 1)
    assert torch.equal(want.view(torch.int64), got.view(torch.int64))
    assert not torch.isnan(got).any()
    # second call, smaller: the scratch still holds the first call's partial sums
    print("noalloc call 2: nrep 40, ndat 200, K 5000", flush=True)
    want, got = both(40, 200, 5000, 2)
    assert torch.equal(want.view(torch.int64), got.view(torch.int64))
    assert not torch.isnan(got).any()


def test_noalloc_single_slice_and_empty():
    print("noalloc: single slice 3 x 5 x 7", flush=True)
    want, got = both(3, 5, 7, 3)
    assert torch.equal(want.view(torch.int64), got.view(torch.int64))
    e = torch.empty((0, 10), dtype=torch.float64, device=DEV)
    t = torch.ones((4, 10), dtype=torch.float64, device=DEV)
    o = torch.empty((0, 4), dtype=torch.float64, device=DEV)
    assert call(LIB.pdf_fk_contract_noalloc, e, t, o) == pdfmi.PDF_OK


def test_noalloc_rejects_partials_beyond_scratch():
    # 640 x 12800 outputs in 8 x 100 tiles of 80 x 128: more than one K slice of 65.5 MB of partial sums
    nrep, ndat, K = 640, 12800, 1024
    print("noalloc: oversize %d x %d x %d must be rejected" % (nrep, ndat, K), flush=True)
    pdf = torch.ones((nrep, K), dtype=torch.float64, device=DEV)
    table = torch.ones((ndat, K), dtype=torch.float64, device=DEV)
    out = torch.full((nrep, ndat), 7.0, dtype=torch.float64, device=DEV)
    rc = call(LIB.pdf_fk_contract_noalloc, pdf, table, out)
    torch.cuda.synchronize()
    assert rc == pdfmi.PDF_ERR_ARG
    assert "scratch" in pdfmi.last_error()
    assert bool((out == 7.0).all())
