"""FP64 CPU oracle of the FastKernel-style contraction (test infrastructure
only; nothing in the library imports it).

Section 4.3 of the paper: theory predictions are convolutions of FK tables
with PDFs evaluated on an x grid, computed for many members at once.  For a
table fk[d][k] over k = (x point, flavour) and member values pdf[r][k]:
    T[r][d] = sum_k pdf[r][k] * fk[d][k]
The definition is written out here as an FP64 matrix product, and as plain
loops for tiny cases (the pins check one against the other and both against
closed forms).
"""
import numpy as np


def contract(pdf, fk):
    """T = pdf @ fk^T in FP64 ([nrep][K] x [ndat][K] -> [nrep][ndat])."""
    pdf = np.asarray(pdf, np.float64).reshape(len(pdf), -1)
    fk = np.asarray(fk, np.float64).reshape(len(fk), -1)
    return pdf @ fk.T


def contract_loops(pdf, fk):
    """The same sum as plain loops (small inputs only)."""
    pdf = np.asarray(pdf, np.float64).reshape(len(pdf), -1)
    fk = np.asarray(fk, np.float64).reshape(len(fk), -1)
    out = np.zeros((len(pdf), len(fk)))
    for r in range(len(pdf)):
        for d in range(len(fk)):
            s = 0.0
            for k in range(pdf.shape[1]):
                s += pdf[r, k] * fk[d, k]
            out[r, d] = s
    return out


def abs_scale(pdf, fk):
    """sum_k |pdf[r][k] fk[d][k]| (the scale of the rounding error of any
    summation order)."""
    return contract(np.abs(pdf), np.abs(fk))
