"""Reader for the hand-worked fixtures in this folder (no arithmetic of the method)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def hand_examples():
    out = []
    with open(os.path.join(HERE, "hand_examples.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, shape, data, expect = [s.strip() for s in line.split("|")]
            N, F, T = (int(x) for x in shape.split())
            v = np.array([int(b, 16) for b in data.split()], dtype=np.uint8).reshape(T, F, N)
            vals = np.array([[int(c) for c in e.split(",")] for e in expect.split()], dtype=np.int64)
            out.append((name, v, vals.reshape(F, N * (N + 1) // 2, 2)))
    return out
