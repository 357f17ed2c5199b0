"""FK-style contraction on the FP64 matrix cores vs the FP64 oracle: ragged
tile edges in every dimension, K not a multiple of the K step, determinism,
and the multi-member pipeline (batched evaluation of many members on one x
grid at one Q^2, then the contraction)."""
import numpy as np
import pytest

import oracle
from oracle import fk as ofk
from paper_2009_06635_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_2009_06635_amd import pdfmi  # noqa: E402

DEV = "cuda:0"
EPS = np.finfo(np.float64).eps


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(DEV)


def check(pdf, table, out):
    want = ofk.contract(pdf, table)
    K = pdf.shape[1]
    tol = 2.0 * max(K, 1) * EPS * ofk.abs_scale(pdf, table)
    assert np.all(np.abs(out - want) <= tol), np.max(np.abs(out - want) / np.maximum(tol, 1e-300))


@pytest.mark.parametrize("nrep,ndat,K", [(1, 1, 1), (1, 1, 0), (3, 5, 7), (63, 64, 31), (64, 65, 32), (65, 63, 33),
                                         (130, 100, 1000), (400, 257, 3 * 13 * 11), (70, 70, 20000),
                                         (5, 300, 31395)])
def test_contract_matches_oracle(nrep, ndat, K):
    rng = np.random.default_rng(nrep * 1000 + ndat + K)
    pdf = rng.normal(size=(nrep, K))
    table = rng.normal(size=(ndat, K)) * (rng.uniform(size=(ndat, K)) < 0.3)   # sparse-ish like FK tables
    out = pdfmi.fk_contract(dev(pdf), dev(table)).cpu().numpy()
    check(pdf, table, out)


@pytest.mark.parametrize("nrep", [400, 1000])
def test_contract_full_size_sampled(nrep):
    """The benchmarked shape (a 2415-point x grid times 13 flavours against a
    1024-row table), in the launch configuration the library picks for it
    (80-row member tiles at 400 members, 64-row at 1000; K split into slices):
    sampled member rows against the oracle, every table row."""
    ndat, K = 1024, 2415 * 13
    print("fk full size: nrep %d ndat %d K %d" % (nrep, ndat, K), flush=True)
    g = torch.Generator(device=DEV)
    g.manual_seed(nrep)
    pdf = torch.randn((nrep, K), dtype=torch.float64, device=DEV, generator=g)
    table = torch.randn((ndat, K), dtype=torch.float64, device=DEV, generator=g)
    out = pdfmi.fk_contract(pdf, table).cpu().numpy()
    rows = np.unique(np.concatenate([[0, 15, 16, 63, 64, 79, 80, nrep - 1],
                                     np.random.default_rng(nrep).integers(0, nrep, 8)]))
    check(pdf[rows].cpu().numpy(), table.cpu().numpy(), out[rows])


def test_contract_deterministic_and_empty():
    rng = np.random.default_rng(7)
    p, t = dev(rng.normal(size=(77, 4000))), dev(rng.normal(size=(90, 4000)))
    a = pdfmi.fk_contract(p, t).cpu().numpy()
    b = pdfmi.fk_contract(p, t).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    e = torch.empty((0, 10), dtype=torch.float64, device=DEV)
    assert pdfmi.fk_contract(e, t[:, :10].contiguous()).shape == (0, 90)


def test_members_on_x_grid_then_contract():
    """The paper's multi-member layout: N members x (x grid of nx points) x 13
    flavours at one Q^2, then a synthetic FK table."""
    members = synth.config3_members(n_members=21)
    g0 = members[0]
    nx, pids = 150, synth.PIDS_13
    x = np.exp(np.linspace(np.log(2e-6), np.log(0.9), nx))
    q2 = np.full(nx, 1.65 ** 2 * 1.01)
    ids = [pdfmi.load_synth(g) for g in members]
    try:
        xd, qd = dev(x), dev(q2)
        F = torch.empty((len(ids), nx, len(pids)), dtype=torch.float64, device=DEV)
        reqs = [(m, pids, xd, qd, F[r]) for r, m in enumerate(ids)]
        pdfmi.xfxq2_batched(reqs, out_f64=True)
        rng = np.random.default_rng(3)
        table = rng.normal(size=(200, nx * len(pids)))
        T = pdfmi.fk_contract(F.reshape(len(ids), -1), dev(table)).cpu().numpy()
        Fo = np.stack([oracle.xfxq2(oracle.Grid(g.xknots, g.q2knots, g.values, g.pids), pids, x, q2)
                       for g in members]).reshape(len(ids), -1)
        want = ofk.contract(Fo, table)
        scale = ofk.abs_scale(Fo, table)
        assert np.all(np.abs(T - want) <= 1e-11 * scale + 1e-300)
    finally:
        for m in ids:
            pdfmi.unload(m)
