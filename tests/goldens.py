"""Reader for the small text fixtures under tests/golden/."""

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_fixture(name):
    out = {"A": [], "T": [], "pivot": []}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            if key in ("A", "T"):
                out[key].append([float(v) for v in vals])
            elif key == "pivot":
                out["pivot"].append(tuple(int(v) for v in vals))
            elif key in ("m", "n", "pivots"):
                out[key] = int(vals[0])
            elif key == "status":
                out[key] = vals[0]
            elif key == "objective":
                out[key] = float(vals[0])
            else:
                out[key] = np.array([float(v) for v in vals])
    out["A"] = np.array(out["A"])
    out["T"] = np.array(out["T"])
    return out
