"""Writes the oracle results of the benchmark workloads (synth/workloads.py) that the GPU
tests compare against:

    c2_n1024.json     every frame of the n=1024 batch (512 frames)
    c3_n4096.json     12 frames of the n=4096 batch, integral and fractional, spread over
                      the batch (its oracle decodes take minutes each: dense Cholesky per
                      Newton step)
    c4_irr8192.json   frames of the irregular n=8192 batch

    python tests/golden/make_configs.py [c2|c3|c4 ...] [--jobs 8]

Calls only the oracle and the seeded input generators. Each record holds the decoded word
(hex of the packed bits), the flag, the objective gamma^T u and the oracle's counts."""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

# frames per workload: all of c2; for c3 and c4 the first frames, the ones whose hard
# decisions violate the most checks (the hardest), and positions spread over the batch
FRAMES = {
    "c2": list(range(512)),
    "c3": [0, 1, 2, 3, 26, 53, 67, 127, 160, 190, 222, 255],
    "c4": [0, 1, 32, 64, 102, 127],
}
FILES = {"c2": "c2_n1024.json", "c3": "c3_n4096.json", "c4": "c4_irr8192.json"}

_cache = {}


def _workload(name):
    if name not in _cache:
        from synth.workloads import WORKLOADS
        _cache[name] = WORKLOADS[name]()
    return _cache[name]


def run(job):
    name, f = job
    import oracle
    code, G = _workload(name)
    g = G[f].astype(np.float64)
    t = time.time()
    r = oracle.decode(code, g)
    return name, f, {"xhat_hex": np.packbits(r.xhat).tobytes().hex(), "flag": int(r.flag),
                     "objective": float(r.objective), "malp_iters": int(r.malp_iters),
                     "ipm_iters": int(r.ipm_iters), "p_max": int(r.p_max),
                     "oracle_s": round(time.time() - t, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["c2", "c3", "c4"])
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    import oracle
    oracle.build(force=False)
    for name in args.which:
        out = {"workload": name, "frames": {}}
        jobs = [(name, f) for f in FRAMES[name]]
        with ProcessPoolExecutor(args.jobs) as ex:
            for nm, f, rec in ex.map(run, jobs):
                out["frames"][str(f)] = rec
                print(nm, f, rec["flag"], rec["malp_iters"], f"{rec['oracle_s']:.0f} s", flush=True)
        with open(os.path.join(HERE, FILES[name]), "w") as fh:
            json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
