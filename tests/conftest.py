import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def load_fixture(name):
    """Parse a hand-derived golden case (format in tests/golden/README.txt)."""
    import numpy as np

    dtype, pts, deaths, vdeaths = None, [], None, None
    mode = None
    with open(os.path.join(GOLDEN, name)) as f:
        for raw in f:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "dtype":
                dtype = {"int8": np.int8, "int16": np.int16}[tok[1]]
            elif tok[0] == "points":
                mode = "points"
            elif tok[0] in ("deaths", "vertex_deaths"):
                vals = [0xFFFFFFFF if t == "inf" else int(t) for t in tok[1:]]
                if tok[0] == "deaths":
                    deaths = np.array(vals, dtype=np.uint32)
                else:
                    vdeaths = np.array(vals, dtype=np.uint32)
                mode = None
            elif mode == "points":
                pts.append([int(t) for t in tok])
    return np.array(pts, dtype=dtype), deaths, vdeaths


def golden_cases():
    return sorted(f for f in os.listdir(GOLDEN) if f.endswith(".txt") and f != "README.txt")
