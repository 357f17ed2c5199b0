"""Writers of LHAPDF6-layout text files for the reader tests: a member file
in the lhagrid1 layout (header, '---', per sub-grid x knots / Q knots /
flavour ids / nx*nq value lines with the Q index fastest, '---') and a
.info file with the alpha_s knot lists.  Numbers are written with 17
significant digits, so they read back exactly."""
import numpy as np


def fmt(v):
    return "%.17e" % float(v)


def member_text(qknots, xknots, values, pids, header=("PdfType: central", "Format: lhagrid1"),
                eol="\n", sep=" "):
    lines = list(header) + ["---"]
    for xk, qk, v in zip(xknots, qknots, values):
        lines.append(sep.join(fmt(a) for a in xk))
        lines.append(sep.join(fmt(a) for a in qk))
        lines.append(sep.join(str(int(p)) for p in pids))
        for ix in range(len(xk)):
            for iq in range(len(qk)):
                lines.append(sep.join(fmt(a) for a in v[ix, iq]))
        lines.append("---")
    return eol.join(lines) + eol


def write_member(path, qknots, xknots, values, pids, **kw):
    with open(path, "w", newline="") as f:
        f.write(member_text(qknots, xknots, values, pids, **kw))


def info_text(qs, alphas, per_line=6):
    def flow(vals):
        items = [fmt(v) for v in vals]
        rows = [", ".join(items[i:i + per_line]) for i in range(0, len(items), per_line)]
        return "[" + ",\n    ".join(rows) + "]"
    return ("SetDesc: synthetic set for reader tests\n"
            "NumMembers: 1\n"
            "AlphaS_Type: ipol\n"
            "AlphaS_Qs: " + flow(qs) + "\n"
            "AlphaS_Vals: " + flow(alphas) + "\n"
            "Flavors: [-5, -4, -3, -2, -1, 1, 2, 3, 4, 5, 21]\n")


def q_of(q2):
    """Q knots whose squares are the given Q^2 knots where possible (the
    tests compare with the squares of the written Q values)."""
    return np.sqrt(np.asarray(q2, np.float64))


def read_back_q2(q):
    """Q^2 of Q knots as written in the text (17 digits) and squared in FP64."""
    return np.array([float(fmt(v)) for v in q]) ** 2
