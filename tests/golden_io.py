"""Reader for the small text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str) -> dict:
    rows, out, mode = [], {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line == "matrix":
                mode = "matrix"
                continue
            head = line.split()[0]
            if head in ("mr", "val", "loc", "col_ind", "col_nnz", "col_ptr"):
                mode = None
                out[head] = [float(x) for x in line.split()[1:]]
                continue
            if mode == "matrix":
                rows.append([float(x) for x in line.split()])
    out["matrix"] = np.array(rows, dtype=np.float32)
    out["mr"] = int(out["mr"][0])
    return out
