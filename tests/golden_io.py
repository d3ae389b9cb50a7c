"""Reader for the small hand-worked text fixtures under tests/golden/."""
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str) -> dict:
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


def csr(d: dict, prefix: str):
    rows, cols = (int(x) for x in d[prefix + ".shape"])
    return synth.CSR(rows, cols,
                     np.array([int(x) for x in d[prefix + ".row_ptr"]], dtype=np.int64),
                     np.array([int(x) for x in d.get(prefix + ".col", [])], dtype=np.int32),
                     np.array([float(x) for x in d.get(prefix + ".val", [])], dtype=np.float64))
