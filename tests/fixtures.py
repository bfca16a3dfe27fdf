"""Parser for the paper-derived graph fixtures under tests/golden/."""
import os

import numpy as np

from paper_2601_17707_amd.synth import from_edges

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_graphs(name):
    """{graph name: (Graph, {expect key: int})} from a fixture file."""
    out = {}
    cur = None
    with open(os.path.join(GOLDEN, name)) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "graph":
                cur = dict(name=tok[1], n_u=int(tok[2]), n_v=int(tok[3]), edges=[], expect={})
            elif tok[0] == "expect":
                cur["expect"][tok[1]] = int(tok[2])
            elif tok[0] == "edge":
                cur["edges"].append((int(tok[1]), int(tok[2]), 1 if tok[3] == "+" else -1))
            elif tok[0] == "end":
                e = np.array(cur["edges"], np.int64).reshape(-1, 3)
                g = from_edges(cur["n_u"], cur["n_v"], e[:, 0], e[:, 1], e[:, 2], dict(name=cur["name"]))
                out[cur["name"]] = (g, cur["expect"])
                cur = None
            else:
                raise ValueError(f"bad fixture line: {raw!r}")
    return out


def load_table8():
    total = None
    classes = []
    with open(os.path.join(GOLDEN, "table8_identity.txt")) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "expect":
                total = int(tok[2])
            elif tok[0] == "class":
                classes.append((tok[1], int(tok[2]), tok[3]))
    return total, classes
