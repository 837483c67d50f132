"""Serving: frames of different codes and lengths submitted one at a time to lpdec_server
(continuous batching over four streams, admission by HBM footprint and slot count) give the
same result as the same frame decoded alone, and the oracle's result."""
import numpy as np
import pytest

from synth.channel import awgn_llr, frame_seed
from synth.codes import irregular_code, regular_code
from tests.gpu_util import cuda, host, make_ctx, obj_close

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("budget_mb,slots", [(512, 256), (8, 6)])
def test_mixed_lengths_match_alone(orc, budget_mb, slots):
    """The second case admits only a handful of frames at a time (8 MB of workspace, 6
    slots), so later requests wait for earlier ones to retire."""
    import torch
    from paper_0902_0657_amd import Code
    ctx = make_ctx()
    codes = [regular_code(96), regular_code(256), irregular_code(256), regular_code(1024)]
    Cs = [Code.from_synth(ctx, c) for c in codes]
    rng = np.random.Generator(np.random.PCG64(11))
    reqs = []
    srv = ctx.server(hbm_budget_bytes=budget_mb << 20, max_slots=slots)
    try:
        for k in range(40):
            ci = int(rng.integers(0, len(codes)))
            ebn0 = float(rng.uniform(1.5, 3.0))
            g = awgn_llr(codes[ci].n, ebn0, 0.5, frame_seed(123, ci, k))
            reqs.append((srv.submit(Cs[ci], g), ci, g))
        srv.drain()
        got = [srv.poll(t, codes[ci].n) for t, ci, _ in reqs]
    finally:
        srv.close()
    for (t, ci, g), r in zip(reqs, got):
        assert r is not None, t
        xh, fl, ob, lat = r
        assert lat > 0.0
        out = ctx.decode_batch(Cs[ci], cuda(g[None, :], torch.float64))
        torch.cuda.synchronize()
        assert fl == int(host(out["flag"])[0]) and np.array_equal(xh, host(out["xhat"])[0])
        assert ob == float(host(out["obj"])[0])          # same kernel, same frame: bit-identical
        if codes[ci].n <= 256:
            o = orc.decode(codes[ci], g)
            assert fl == o.flag and np.array_equal(xh, o.xhat) and obj_close(ob, o.objective, g)
    ctx.close()
