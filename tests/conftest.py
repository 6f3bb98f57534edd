import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_golden(name):
    """Parse a tests/golden/hand_example_*.txt fixture."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", name)
    lines = [l.strip() for l in open(path) if l.strip() and not l.startswith("#")]
    d = {"edges": []}
    it = iter(lines)
    for l in it:
        k, _, rest = l.partition(" ")
        if k == "edges":
            for _ in range(d["m"]):
                a, b, c = next(it).split()
                d["edges"].append((int(a), int(b), int(c)))
        elif k in ("n", "m", "total", "count"):
            d[k] = int(rest)
        elif k == "mask":
            d["mask"] = np.array([int(x) for x in rest.split()], np.uint8)
        elif k == "rounds":
            d["rounds"] = [dict((kv.split("=")[0], int(kv.split("=")[1]))
                                for kv in r.split(",")) for r in rest.split()]
    e = np.array(d["edges"], dtype=np.int64).reshape(-1, 3)
    d["u"], d["v"], d["w"] = (e[:, 0].astype(np.int32), e[:, 1].astype(np.int32),
                              e[:, 2].astype(np.uint32))
    return d


@pytest.fixture(scope="session")
def golden():
    return load_golden
