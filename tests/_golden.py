"""Readers for the small text fixtures under tests/golden (values printed in
the paper, each line carrying its citation)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_values():
    out = {}
    with open(os.path.join(GOLDEN, "paper_values.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


def table1():
    """{N: [L2 at nu = 0, 0.1, 0.2, 0.25, 0.3]} from the paper's Table."""
    rows = np.loadtxt(os.path.join(GOLDEN, "table1_l2_jx.txt"), comments="#")
    return {int(r[0]): list(r[1:]) for r in rows}


TABLE1_NUS = (0.0, 0.1, 0.2, 0.25, 0.3)
