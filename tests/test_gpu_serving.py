"""Serving: frames of different codes and lengths submitted one at a time to lpdec_server
(continuous batching over streams, or persistent per-code kernels; admission by HBM footprint
and slot count) give the same result as the same frame decoded alone, and the oracle's
result."""
import numpy as np
import pytest

from synth.channel import awgn_llr, frame_seed
from synth.codes import irregular_code, regular_code
from tests.gpu_util import cuda, host, make_ctx, obj_close

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("budget_mb,slots", [(512, 256), (8, 6)])
def test_mixed_lengths_match_alone(orc, budget_mb, slots, mode):
    """The second case admits only a handful of frames at a time (8 MB of workspace, 6
    slots), so later requests wait for earlier ones to retire; in the persistent mode the
    four codes' engines then share the 8 MB."""
    import torch
    from paper_0902_0657_amd import Code
    ctx = make_ctx(SERVER_MODE=mode)
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


def test_persistent_engine_leaves_when_idle_and_returns():
    """Persistent mode: requests that arrive after the engine's kernel has left on its idle
    timeout (about 5 ms) start it again; a server closed while its kernel is resident stops it."""
    import time
    import torch
    from paper_0902_0657_amd import Code
    ctx = make_ctx(SERVER_MODE=1)
    code = regular_code(256)
    C = Code.from_synth(ctx, code)
    gs = [awgn_llr(code.n, 2.0, 0.5, frame_seed(321, 0, k)) for k in range(15)]
    got = []
    srv = ctx.server(hbm_budget_bytes=256 << 20, max_slots=64)
    try:
        for part in (gs[:5], gs[5:10]):
            tk = [srv.submit(C, g) for g in part]
            srv.drain()
            got += [srv.poll(t, code.n) for t in tk]
            time.sleep(0.1)
        tk = [srv.submit(C, g) for g in gs[10:]]
        srv.drain()
        got += [srv.poll(t, code.n) for t in tk]
        srv.submit(C, gs[0])   # still queued or running when the server closes
    finally:
        srv.close()
    out = ctx.decode_batch(C, cuda(np.stack(gs), torch.float64))
    torch.cuda.synchronize()
    xh, fl, ob = host(out["xhat"]), host(out["flag"]), host(out["obj"])
    for k, r in enumerate(got):
        assert r is not None, k
        assert r[1] == int(fl[k]) and np.array_equal(r[0], xh[k]) and r[2] == float(ob[k])
    ctx.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_large_codes_in_the_mix_match_alone(mode):
    """The serving mix's large codes, (3,6) n=4096 and the irregular n=8192 code, beside n=256
    and n=1024 (Eb/N0 2.5-3.5 dB, so that every frame finishes in seconds): each result is
    bit-identical to the same frame decoded alone. The 1 GiB budget admits only a few
    workgroups for the large codes (their dense-fallback matrices take 34 and 134 MB per
    workgroup), so their requests queue for each other."""
    import torch
    from paper_0902_0657_amd import Code
    ctx = make_ctx(SERVER_MODE=mode)
    codes = [regular_code(256), regular_code(1024), regular_code(4096), irregular_code(8192)]
    Cs = [Code.from_synth(ctx, c) for c in codes]
    rng = np.random.Generator(np.random.PCG64(12))
    reqs = []
    srv = ctx.server(hbm_budget_bytes=1 << 30, max_slots=64)
    try:
        for k in range(24):
            ci = k % len(codes)
            g = awgn_llr(codes[ci].n, float(rng.uniform(2.5, 3.5)), 0.5, frame_seed(124, ci, k))
            reqs.append((srv.submit(Cs[ci], g), ci, g))
        print(f"[serving mode {mode}] 24 requests submitted", flush=True)
        srv.drain()
        got = [srv.poll(t, codes[ci].n) for t, ci, _ in reqs]
    finally:
        srv.close()
    for (t, ci, g), r in zip(reqs, got):
        assert r is not None, t
        xh, fl, ob, lat = r
        out = ctx.decode_batch(Cs[ci], cuda(g[None, :], torch.float64))
        torch.cuda.synchronize()
        assert fl == int(host(out["flag"])[0]) and np.array_equal(xh, host(out["xhat"])[0]), (t, ci)
        assert ob == float(host(out["obj"])[0])
    ctx.close()
