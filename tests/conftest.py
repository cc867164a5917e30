import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def load_golden(name):
    """Parse a tests/golden fixture: (edges, [(tri, pattern)], complete)."""
    edges, tris, complete = [], [], False
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("edge "):
                edges.append([int(v) for v in line.split()[1:]])
            elif line.startswith("triangle "):
                lhs, rhs = line[len("triangle "):].split(":")
                tris.append((tuple(int(x) - 1 for x in lhs.split()), int(rhs)))
            elif line == "complete":
                complete = True
    return edges, tris, complete


_EXPECTED = None


def expected_counts(sha256):
    """The oracle's stored exact counts for an input (tests/golden/
    expected_counts.json, written by tests/golden/make_expected_counts.py
    from the CPU oracle alone), keyed by the input's SHA-256; None if absent."""
    global _EXPECTED
    if _EXPECTED is None:
        import json
        with open(os.path.join(ROOT, "tests", "golden", "expected_counts.json")) as fh:
            _EXPECTED = json.load(fh)
    return _EXPECTED.get(sha256)


def int64_digest(a):
    """SHA-256 of an int64 array's little-endian bytes (as the stored t digests)."""
    import hashlib
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()
