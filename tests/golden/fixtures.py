"""Readers of the text fixtures in this folder."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def pathfinder_fig3():
    """{"kepler": 6x6, "maxwell": 4x4} matrices of the paper's Figure 3."""
    out, name, rows, n = {}, None, [], 0
    with open(os.path.join(HERE, "pathfinder_fig3.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0].isalpha():
                name, n, rows = parts[0], int(parts[1]), []
                continue
            rows.append([float(x) for x in parts])
            if len(rows) == n:
                out[name] = np.array(rows)
    return out
