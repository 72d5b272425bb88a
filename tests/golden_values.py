"""Reader of the fixtures in tests/golden/: `key = value` lines, `#` comments
(each file states where in the paper its values are printed)."""

import os

_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str) -> dict:
    out = {}
    with open(os.path.join(_DIR, name + ".txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (s.strip() for s in line.split("=", 1))
                out[k] = float(v)
    return out
