"""Writes tests/golden/fullsize_hashes.json: for every named full-size workload,
the SHA-256 of the oracle's MSF mask (uint8 per edge), its total weight and
edge count.  Calls only graphgen (inputs) and oracle (Kruskal); run on a CPU:

    python tests/golden/make_fullsize_hashes.py [workload ...]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_hashes.json")


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names or list(graphgen.WORKLOADS):
        t = time.time()
        u, v, w, n = graphgen.workload(name)
        mask, total, count = oracle.kruskal(u, v, w, n)
        data[name] = {"n": int(n), "m": int(len(u)),
                      "input_sha256": hashlib.sha256(u.tobytes() + v.tobytes() + w.tobytes()).hexdigest(),
                      "mask_sha256": hashlib.sha256(mask.tobytes()).hexdigest(),
                      "total": int(total), "msf_edges": int(count)}
        print(name, data[name], f"{time.time() - t:.1f}s", flush=True)
        del u, v, w, mask
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
