"""Helpers shared by the GPU tests: move seeded inputs to cuda:0 and call the
library through its binding (which calls the C ABI)."""
import hashlib
import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HASHES = os.path.join(ROOT, "tests", "golden", "fullsize_hashes.json")


def to_dev(*arrays):
    import torch
    dev = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev) for a in arrays]


def gpu_msf(u, v, w, n, **kw):
    import paper_2302_12199_amd as msf
    tu, tv, tw = to_dev(np.asarray(u, np.int32), np.asarray(v, np.int32),
                        np.asarray(w, np.uint32))
    mask, total, stats = msf.compute(tu, tv, tw, n, **kw)
    return mask.cpu().numpy(), total, stats


def sha(mask):
    return hashlib.sha256(np.ascontiguousarray(mask, np.uint8).tobytes()).hexdigest()


def golden_hashes():
    return json.load(open(HASHES))


def banner(msg):
    print(f"\n[gpu-test] {msg}", flush=True)
