"""Readers for the hand-written fixtures under tests/golden/."""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line.split()


def d3q19_ordering():
    """(c[19,3] int, w[19] Fraction, opp[19] int) of the canonical ordering."""
    c, w, opp = [], [], []
    for r in _rows("d3q19_ordering.txt"):
        c.append([int(v) for v in r[1:4]])
        w.append(Fraction(int(r[4]), int(r[5])))
        opp.append(int(r[6]))
    return np.array(c, dtype=np.int64), w, np.array(opp, dtype=np.int64)


def idx_4cube():
    """(solid cells, {node_id: 18 neighbour ids}) of the hand-worked 4^3 example."""
    solid, nodes = [], {}
    for r in _rows("idx_4cube.txt"):
        if r[0] == "solid":
            solid = [int(v) for v in r[1:]]
        elif r[0] == "node":
            nodes[int(r[1])] = [int(v) for v in r[2:]]
    return solid, nodes


def table8():
    """{scheme: (full_pdfs, full_bytes, ind_pdfs, ind_idx, ind_bytes)} of Table 8."""
    out = {}
    for r in _rows("table8_bytes.txt"):
        out[r[0]] = tuple(int(v) for v in r[1:])
    return out
