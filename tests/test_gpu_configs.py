"""GPU parity on the benchmark workloads at their full launch sizes (synth/workloads.py),
against oracle results stored by tests/golden/make_configs.py (which calls only the oracle):

    n=1024 (3,6), 512 frames in one launch: every frame, FP64 and FP32 PCG vectors
    n=4096 (3,6), 256 frames in one launch: 12 stored frames spread over the batch
    irregular n=8192, 128 frames in one launch: the stored frames

Decoded word and flag bit-exact, objective within 1e-6 relative to the IPM's gap scale. Every
frame of every launch is also checked against properties that hold at any size: no numerical
failure, at most one cut per check (p <= m), u within the fundamental polytope up to the
violation threshold at which MALP stops, a flag-1 frame's decisions satisfy every check and are
the rounding of its LP solution."""
import json
import os
import sys

import numpy as np
import pytest

from synth import workloads
from tests import refs
from tests.gpu_util import cuda, host, make_ctx, obj_close

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FILES = {"c2": "c2_n1024.json", "c3": "c3_n4096.json", "c4": "c4_irr8192.json"}


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.close()


def _golden(name):
    return json.load(open(os.path.join(GOLDEN, FILES[name])))["frames"]


def _launch(ctx, name, precision=-1):
    import torch
    from paper_0902_0657_amd import Code
    code, G = workloads.WORKLOADS[name]()
    C = Code.from_synth(ctx, code)
    dt = torch.float32 if G.dtype == np.float32 else torch.float64
    print(f"[{name}] launch of {G.shape[0]} frames, n={code.n}, precision {precision}", flush=True)
    ctx.set_option("PRECISION", precision)
    try:
        out = ctx.decode_batch(C, cuda(G, dt), want_u=True)
        torch.cuda.synchronize()
    finally:
        ctx.set_option("PRECISION", -1)
    return code, G.astype(np.float64), out


def _invariants(code, out):
    st, fl, xh, u = host(out["stats"]), host(out["flag"]), host(out["xhat"]), host(out["u"])
    assert np.all(fl >= 0), [(f, int(fl[f])) for f in np.nonzero(fl < 0)[0]]
    assert np.all(st[:, 3] <= code.m)
    H = code.dense()
    for f in range(fl.shape[0]):
        assert refs.max_parity_violation(code, u[f]) < 1e-4 + 1e-6, f   # MALP's TAU_VIOL
        if fl[f] == 1:
            assert not ((H @ xh[f]) % 2).any(), f
            assert np.array_equal(xh[f], (u[f] > 0.5).astype(np.uint8)), f


def _against_golden(code, G, out, gold):
    xh, fl, ob = host(out["xhat"]), host(out["flag"]), host(out["obj"])
    bad = []
    for k, rec in gold.items():
        f = int(k)
        want = np.unpackbits(np.frombuffer(bytes.fromhex(rec["xhat_hex"]), np.uint8))[:code.n]
        if fl[f] != rec["flag"]:
            bad.append((f, "flag", int(fl[f]), rec["flag"]))
        elif not obj_close(ob[f], rec["objective"], G[f]):
            bad.append((f, "objective", float(ob[f]), rec["objective"]))
        elif not np.array_equal(xh[f], want):
            bad.append((f, "decisions", np.nonzero(xh[f] != want)[0][:8].tolist()))
    return bad


@pytest.mark.parametrize("precision", [1, 0])
def test_c2_n1024_all_frames(ctx, precision):
    """All 512 frames of the n=1024 launch against the oracle, strictly: no frame may differ
    in a decision, flat optimal face or not."""
    code, G, out = _launch(ctx, "c2", precision)
    _invariants(code, out)
    gold = _golden("c2")
    assert len(gold) == G.shape[0]
    bad = _against_golden(code, G, out, gold)
    assert not bad, (len(bad), bad[:10])
    fl = host(out["flag"])
    print(f"[c2] precision {precision}: {int((fl == 1).sum())} integral, {int((fl == 0).sum())} fractional, "
          f"0 mismatches", flush=True)


def test_c3_n4096_full_launch(ctx):
    code, G, out = _launch(ctx, "c3")
    _invariants(code, out)
    gold = _golden("c3")
    assert {r["flag"] for r in gold.values()} >= {0, 1}   # integral and fractional frames
    bad = _against_golden(code, G, out, gold)
    assert not bad, bad


def test_c4_irregular_n8192_full_launch(ctx):
    """Every frame of this batch decodes integral (BSC p=0.04 is below the code's LP threshold);
    the stored frames include the ones whose hard decisions violate the most checks."""
    code, G, out = _launch(ctx, "c4")
    _invariants(code, out)
    bad = _against_golden(code, G, out, _golden("c4"))
    assert not bad, bad
