"""Writes large_codes.json: oracle results for a few frames of the n=4096 (3,6) and n=8192
irregular workloads, whose oracle decodes take minutes each (dense Cholesky per Newton step).

    python tests/golden/make_large.py [--jobs 6]

Calls only the oracle and the seeded input generators."""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

# (name, code, channel, frames): the channel recipes of the two workloads
CASES = [
    ("n4096_awgn_1.75dB", ("regular", 4096), ("awgn", 1.75, 256, 3), [0, 1, 2, 3]),
    ("n8192_irregular_bsc_0.04", ("irregular", 8192), ("bsc", 0.04, 128, 4), [0, 1]),
]


def gamma_of(channel, code_n, frame):
    from synth.channel import batch_awgn, batch_bsc
    if channel[0] == "awgn":
        _, ebn0, nf, stream = channel
        return batch_awgn(code_n, 0.5, ebn0, nf, stream=stream)[frame]
    _, p, nf, stream = channel
    return batch_bsc(code_n, p, nf, stream=stream)[frame]


def code_of(spec):
    from synth.codes import irregular_code, regular_code
    return regular_code(spec[1]) if spec[0] == "regular" else irregular_code(spec[1])


def run(job):
    name, spec, channel, f = job
    import oracle
    code = code_of(spec)
    g = gamma_of(channel, code.n, f)
    t = time.time()
    r = oracle.decode(code, g)
    return name, f, {"xhat_hex": np.packbits(r.xhat).tobytes().hex(), "flag": int(r.flag),
                     "objective": float(r.objective), "malp_iters": int(r.malp_iters),
                     "ipm_iters": int(r.ipm_iters), "oracle_s": time.time() - t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    args = ap.parse_args()
    jobs = [(name, spec, ch, f) for name, spec, ch, frames in CASES for f in frames]
    out = {name: {"code": list(spec), "channel": list(ch), "frames": {}} for name, spec, ch, _ in CASES}
    with ProcessPoolExecutor(args.jobs) as ex:
        for name, f, rec in ex.map(run, jobs):
            out[name]["frames"][str(f)] = rec
            print(name, f, rec["flag"], rec["malp_iters"], f"{rec['oracle_s']:.0f} s", flush=True)
    with open(os.path.join(HERE, "large_codes.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
