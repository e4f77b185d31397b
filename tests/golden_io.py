"""Reader for the hand-worked text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(":")
            rows = [[float(t) for t in part.split()] for part in rest.split(";")]
            arr = np.array(rows, dtype=np.float64)
            if arr.size == 1:
                out[key.strip()] = float(arr.reshape(-1)[0])
            else:
                out[key.strip()] = arr[0] if len(rows) == 1 else arr
    return out
