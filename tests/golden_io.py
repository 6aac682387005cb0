"""Reader for the hand-derived golden examples under tests/golden/."""
from __future__ import annotations

import glob
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_files():
    return sorted(glob.glob(os.path.join(GOLDEN_DIR, "*.txt")))


def load(path: str) -> dict:
    lines = []
    with open(path) as f:
        for raw in f:
            s = raw.split("#", 1)[0].strip()
            if s:
                lines.append(s.split())
    out = {"name": os.path.basename(path)}
    i = 0
    while i < len(lines):
        key = lines[i][0]
        if key in ("input", "output"):
            r, c = int(lines[i][1]), int(lines[i][2])
            rows = [[int(v) for v in lines[i + 1 + j]] for j in range(r)]
            arr = np.array(rows, dtype=np.int64).reshape(r, c)
            assert arr.min() >= 0 and arr.max() <= 255
            out[key] = arr.astype(np.uint8)
            i += 1 + r
        elif key == "changed":
            out[key] = [int(v) for v in lines[i][1:]]
            i += 1
        else:
            out[key] = int(lines[i][1])
            i += 1
    return out
