"""Launch-shape autotuning: picks the threads per frame (BLOCK) of the decode kernel for a code
by timing a sample batch with each candidate, and remembers the choice per code shape.

The hot path is latency-bound; one wave per frame avoids barriers between the levels of the
triangular solves, wider blocks shorten the column passes of long codes. Which wins depends on
the code size and on whether the frame's working set fits in LDS, so it is measured."""
from __future__ import annotations

import json
import os

_CACHE: dict = {}


def _key(code, precision):
    return f"m{code.m}_n{code.n}_p{precision}"


def tune_block(ctx, code, gamma, candidates=(64, 128, 256), cache_file=None):
    """gamma: CUDA tensor [frames, n], a representative sample. Sets ctx's BLOCK option to the
    fastest candidate and returns {"block": b, "ms": {b: time}}."""
    import torch
    prec = int(ctx.get_option("PRECISION"))
    key = _key(code, prec)
    if cache_file and os.path.exists(cache_file) and not _CACHE:
        with open(cache_file) as fh:
            _CACHE.update(json.load(fh))
    if key in _CACHE:
        ctx.set_option("BLOCK", _CACHE[key]["block"])
        return _CACHE[key]
    old = ctx.get_option("BLOCK")
    stream = torch.cuda.current_stream(gamma.device)
    out = ctx.batch_outputs(code, gamma.shape[0], gamma.device, want_stats=False)
    times = {}
    for b in candidates:
        ctx.set_option("BLOCK", b)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.decode_batch(code, gamma, out=out, want_stats=False, stream=stream)
        e1.record(stream)
        e1.synchronize()
        times[b] = e0.elapsed_time(e1)
    best = min(times, key=times.get)
    ctx.set_option("BLOCK", best if best else old)
    rec = {"block": best, "ms": times}
    _CACHE[key] = rec
    if cache_file:
        with open(cache_file, "w") as fh:
            json.dump(_CACHE, fh, indent=1)
    return rec
