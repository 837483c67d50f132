"""GPU ALP decoding (Algorithm 1) against the oracle's: decoded word and flag bit-exact,
objective within 1e-6 of the IPM's gap scale, and the same number of LPs and cuts in the
largest LP (the cut lists follow the same decisions of Algorithm 2)."""
import numpy as np
import pytest

from synth.channel import batch_awgn, batch_bsc
from synth.codes import irregular_code, regular_code
from tests.gpu_util import make_ctx, obj_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.close()


def _check(ctx, orc, code, G, capacity_ok=False):
    """capacity_ok: a frame may instead end with LPDEC_FLAG_ALP_CAPACITY (-6), when some
    variable lies in more than 16 of its cuts (possible with the degree-8 variables of the
    irregular code); such frames are counted and returned."""
    from paper_0902_0657_amd import Code, stats_table
    C = Code.from_synth(ctx, code)
    print(f"[alp] n={code.n}: {G.shape[0]} frames", flush=True)
    out = ctx.alp_decode_batch(C, G)
    st = stats_table(out["stats"])
    bad, cap = [], []
    for f in range(G.shape[0]):
        r = orc.alp_decode(code, G[f])
        if capacity_ok and out["flag"][f] == -6:
            cnt = np.bincount(r.cuts[:, 0], minlength=code.m)
            deg = np.zeros(code.n, int)
            for j in range(code.m):
                deg[code.row(j)] += cnt[j]
            assert deg.max() > 16, f   # the oracle's cut list overflows the encoding as well
            cap.append(f)
            continue
        if not (out["flag"][f] == r.flag and np.array_equal(out["xhat"][f], r.xhat)
                and obj_close(out["obj"][f], r.objective, G[f])):
            bad.append((f, int(out["flag"][f]), r.flag, float(out["obj"][f]), r.objective))
        elif not (st["malp_iters"][f] == r.malp_iters and st["p_max"][f] == r.p_max):
            bad.append((f, "counts", int(st["malp_iters"][f]), r.malp_iters, int(st["p_max"][f]), r.p_max))
    assert not bad, bad[:5]
    return out, st, cap


def test_alp_regular_n96(ctx, orc):
    code = regular_code(96)
    G = np.concatenate([batch_awgn(code.n, 0.5, s, 16, stream=141, snr_index=i) for i, s in enumerate((1.0, 1.5, 2.5))])
    out, st, _ = _check(ctx, orc, code, G)
    assert (out["flag"] == 0).sum() >= 3


def test_alp_regular_n256_and_irregular_bsc(ctx, orc):
    _check(ctx, orc, regular_code(256), batch_awgn(256, 0.5, 1.5, 24, stream=142))
    code = irregular_code(256)
    out, st, cap = _check(ctx, orc, code, batch_bsc(code.n, 0.06, 16, stream=143), capacity_ok=True)
    print(f"[alp] irregular n=256: {len(cap)} of 16 frames beyond the 16-cut column capacity", flush=True)
    assert len(cap) < 16


def test_alp_larger_lps_than_malp(ctx, orc):
    """Sec. III-D: ALP keeps every cut, so its largest LP is at least MALP-A's last one, while
    both reach the same LP optimum."""
    import torch
    from paper_0902_0657_amd import Code, stats_table
    from tests.gpu_util import cuda, host
    code = regular_code(256)
    C = Code.from_synth(ctx, code)
    G = batch_awgn(code.n, 0.5, 1.5, 32, stream=144)
    a = ctx.alp_decode_batch(C, G)
    m = ctx.decode_batch(C, cuda(G, torch.float64))
    torch.cuda.synchronize()
    sa, sm = stats_table(a["stats"]), stats_table(m["stats"])
    assert np.array_equal(a["flag"], host(m["flag"])) and np.array_equal(a["xhat"], host(m["xhat"]))
    assert np.all(sa["p_max"] >= sm["p_max"])
