"""GPU parity of the whole decoder against the oracle: decoded word and certificate flag
bit-exact on every frame, LP objective within 1e-6 relative to the IPM's gap scale, per-iteration cut
sets identical. A frame where the two disagree on integrality fails the test."""
import json
import os

import numpy as np
import pytest

from synth.channel import awgn_llr, batch_awgn, batch_bsc, frame_seed
from synth.codes import from_dense, irregular_code, regular_code
from tests.gpu_util import cuda, host, make_ctx, obj_close

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.close()


def _code(ctx, code):
    from paper_0902_0657_amd import Code
    return Code.from_synth(ctx, code)


def _compare(orc, code, G, out, oracle_frames=None, opts=None):
    """Every listed frame equal to the oracle: flag and decoded word bit-exact, objective within
    1e-6 relative to the IPM's gap scale."""
    xh, fl, ob = host(out["xhat"]), host(out["flag"]), host(out["obj"])
    frames = range(G.shape[0]) if oracle_frames is None else oracle_frames
    bad = []
    for f in frames:
        r = orc.decode(code, G[f], opts)
        if not (fl[f] == r.flag and obj_close(ob[f], r.objective, G[f])):
            bad.append((f, int(fl[f]), r.flag, float(ob[f]), r.objective))
        elif not np.array_equal(xh[f], r.xhat):
            bad.append((f, "decisions", np.nonzero(xh[f] != r.xhat)[0][:8].tolist()))
    assert not bad, bad[:5]


@pytest.mark.parametrize("precision", [1, 0])
def test_config1_n96_all_frames(ctx, orc, precision):
    """Plain configuration: (3,6) n=96, AWGN 2.0 dB, 200 frames."""
    import torch
    code = regular_code(96)
    C = _code(ctx, code)
    G = batch_awgn(code.n, 0.5, 2.0, 200, stream=1)
    ctx.set_option("PRECISION", precision)
    try:
        out = ctx.decode_batch(C, cuda(G, torch.float64))
        torch.cuda.synchronize()
    finally:
        ctx.set_option("PRECISION", -1)
    _compare(orc, code, G, out)


def test_single_frame_plain_form(ctx, orc):
    """lpdec_decode: one frame per launch, host pointers, FP64."""
    code = regular_code(96)
    C = _code(ctx, code)
    G = batch_awgn(code.n, 0.5, 2.0, 12, stream=1)
    for f in range(G.shape[0]):
        xh, flag, obj, st, u = ctx.decode(C, G[f])
        r = orc.decode(code, G[f])
        assert np.array_equal(xh, r.xhat) and flag == r.flag and obj_close(obj, r.objective, G[f])
        assert st["malp_iters"] == r.malp_iters


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n,snrs", [(96, [1.0, 1.5, 2.5]), (256, [1.5, 2.0])])
def test_fp32_llr_batches(ctx, orc, n, snrs, precision):
    """FP32 LLRs; PCG vectors in FP32 (with FP64 refinement) or FP64."""
    import torch
    code = regular_code(n)
    C = _code(ctx, code)
    G = np.concatenate([batch_awgn(code.n, 0.5, s, 40, stream=2, snr_index=i) for i, s in enumerate(snrs)])
    G = G.astype(np.float32)
    ctx.set_option("PRECISION", precision)
    try:
        out = ctx.decode_batch(C, cuda(G, torch.float32))
        torch.cuda.synchronize()
    finally:
        ctx.set_option("PRECISION", -1)
    _compare(orc, code, G.astype(np.float64), out)


@pytest.mark.parametrize("mode", [0, 1])
def test_cut_traces_match(ctx, orc, mode):
    import torch
    code = regular_code(96)
    C = _code(ctx, code)
    G = batch_awgn(code.n, 0.5, 1.5, 24, stream=3)
    ctx.set_option("MALP_MODE", mode)
    try:
        out = ctx.decode_batch_trace(C, cuda(G, torch.float64), trace_cap=60)
    finally:
        ctx.set_option("MALP_MODE", 0)
    tr, st = host(out["trace"]).view(np.uint32), host(out["stats"])
    opts = orc.OracleOpts(malp_mode=mode)
    for f in range(G.shape[0]):
        r = orc.decode(code, G[f], opts, trace=True)
        assert st[f, 0] == r.malp_iters
        k = min(r.malp_iters, 60)
        assert np.array_equal(tr[f, :k], r.trace_mask[:k]), f
    _compare(orc, code, G, out, opts=opts)


def test_irregular_bsc(ctx, orc):
    import torch
    code = irregular_code(256)
    C = _code(ctx, code)
    G = batch_bsc(code.n, 0.06, 48, stream=4)
    out = ctx.decode_batch(C, cuda(G, torch.float64))
    torch.cuda.synchronize()
    _compare(orc, code, G, out)


def test_hamming_pseudocodeword(ctx, orc):
    """The (7,4,3) pseudocodeword of the remark after Corollary 5."""
    import torch
    g = json.load(open(os.path.join(GOLDEN, "hamming743.json")))
    code = from_dense(np.array(g["H"]))
    C = _code(ctx, code)
    G = np.array([g["gamma"]])
    out = ctx.decode_batch(C, cuda(G, torch.float64), want_u=True)
    torch.cuda.synchronize()
    assert host(out["flag"])[0] == 0
    assert np.abs(host(out["u"])[0] - np.array(g["pseudocodeword"])).max() < 1e-6


def test_edge_cases(ctx, orc):
    """A codeword as hard decision solves no LP; NaN in one frame fails only that frame;
    an empty batch is a no-op."""
    import torch
    code = regular_code(96)
    C = _code(ctx, code)
    G = batch_awgn(code.n, 0.5, 2.0, 6, stream=5)
    G[0] = np.abs(G[0]) + 0.1            # hard decision = all-zero codeword
    G[3, 5] = np.nan
    out = ctx.decode_batch(C, cuda(G, torch.float64))
    torch.cuda.synchronize()
    fl, st, xh = host(out["flag"]), host(out["stats"]), host(out["xhat"])
    assert fl[0] == 1 and st[0, 0] == 0 and not xh[0].any()
    assert fl[3] < 0
    for f in (1, 2, 4, 5):
        r = orc.decode(code, G[f])
        assert fl[f] == r.flag and np.array_equal(xh[f], r.xhat)
    empty = ctx.decode_batch(C, cuda(np.zeros((0, code.n)), torch.float64))
    torch.cuda.synchronize()
    assert empty["flag"].numel() == 0


@pytest.mark.parametrize("opt,val", [("MTS_REUSE", 2), ("MTS_REUSE", 4), ("WARM_START", 1), ("PRECOND", 2),
                                     ("PRECOND", 3), ("PRECOND", 4), ("PRECOND", 0),
                                     ("PRECOND", 5)])
def test_preconditioner_reuse_and_warm_start(ctx, orc, opt, val):
    """The preconditioning set kept over several IPM iterations of an LP (MTS_REUSE), each
    Newton solve started from the previous direction (WARM_START), or the preconditioner
    from Algorithm 8 (PRECOND 2): the decode still equals the oracle's; reuse runs fewer
    triangular-set searches."""
    import torch
    from paper_0902_0657_amd import stats_table
    code = regular_code(256)
    C = _code(ctx, code)
    G = batch_awgn(code.n, 0.5, 1.5, 24, stream=12)
    default = ctx.get_option(opt)
    outs = {}
    for v in (default, val):
        ctx.set_option(opt, v)
        try:
            outs[v] = ctx.decode_batch(C, cuda(G, torch.float64))
            torch.cuda.synchronize()
        finally:
            ctx.set_option(opt, default)
    _compare(orc, code, G, outs[val])
    if opt == "MTS_REUSE":
        s1, sr = stats_table(host(outs[default]["stats"])), stats_table(host(outs[val]["stats"]))
        assert sr["mts_rounds"].sum() < s1["mts_rounds"].sum()


def test_malp_cycle_frame(ctx, orc):
    """The n=256 frame whose LLR gamma_164 is about -3e-6: without the box clamp of Theorem 2a
    the cut sets alternate with period 2 up to the MALP cap. Both sides must reach the LP
    optimum with flag 1, in both MALP modes."""
    import torch
    from synth.channel import awgn_llr, frame_seed
    code = regular_code(256)
    C = _code(ctx, code)
    G = awgn_llr(code.n, 1.6537604712821115, 0.5, frame_seed(91, 0, 145))[None, :]
    for mode in (0, 1):
        ctx.set_option("MALP_MODE", mode)
        try:
            out = ctx.decode_batch(C, cuda(G, torch.float64))
            torch.cuda.synchronize()
        finally:
            ctx.set_option("MALP_MODE", 0)
        assert host(out["flag"])[0] == 1
        _compare(orc, code, G, out, opts=orc.OracleOpts(malp_mode=mode))



def test_malp_cut_cycle_frame(ctx, orc):
    """The n=1024 frame at 1.99 dB whose LP optimum is flat along one cut at the IPM's
    accuracy: MALP-A's cut sets alternate between two LPs that differ in the cut of check 96.
    Both sides end the decode at the first recurrence (LPDEC_FLAG_CUT_CYCLE) with the costlier
    LP's solution; MALP-B decodes it normally. The frame came from a serving run, where it ended
    at the MALP cap before the recurrence test existed."""
    import torch
    from synth.channel import awgn_llr, frame_seed
    code = regular_code(1024)
    C = _code(ctx, code)
    G = awgn_llr(code.n, 1.9857919617105901, 0.5, frame_seed(84, 1, 578))[None, :]
    for mode, flag in ((0, -7), (1, 0)):
        ctx.set_option("MALP_MODE", mode)
        try:
            out = ctx.decode_batch(C, cuda(G, torch.float64))
            torch.cuda.synchronize()
        finally:
            ctx.set_option("MALP_MODE", 0)
        assert host(out["flag"])[0] == flag
        _compare(orc, code, G, out, opts=orc.OracleOpts(malp_mode=mode))

def _sweep_oracle(args):
    import oracle as O
    n, mode, f = args
    from synth.channel import uniform_snr_awgn
    _, gamma = uniform_snr_awgn(n, 1.5, 3.0, 92, f)
    r = O.decode(regular_code(n), gamma, O.OracleOpts(malp_mode=mode))
    return r.xhat, r.flag, r.objective


@pytest.mark.parametrize("mode", [0, 1])
def test_uniform_snr_sweep_n256(ctx, orc, mode):
    """2000 frames of the n=256 code, Eb/N0 uniform in [1.5, 3] dB, in one launch (a resident
    set of workgroups taking frames in turn): no negative flag, and every frame equal to the
    oracle, strictly."""
    import multiprocessing as mp
    import torch
    from synth.channel import uniform_snr_awgn
    n, F = 256, 2000
    code = regular_code(n)
    C = _code(ctx, code)
    G = np.stack([uniform_snr_awgn(n, 1.5, 3.0, 92, f)[1] for f in range(F)])
    ctx.set_option("MALP_MODE", mode)
    try:
        out = ctx.decode_batch(C, cuda(G, torch.float64))
        torch.cuda.synchronize()
    finally:
        ctx.set_option("MALP_MODE", 0)
    xh, fl, ob = host(out["xhat"]), host(out["flag"]), host(out["obj"])
    assert np.all(fl >= 0), [(f, int(fl[f])) for f in np.nonzero(fl < 0)[0]][:10]
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        ref = pool.map(_sweep_oracle, [(n, mode, f) for f in range(F)], chunksize=16)
    bad = [f for f in range(F) if not (fl[f] == ref[f][1] and np.array_equal(xh[f], ref[f][0])
                                        and obj_close(ob[f], ref[f][2], G[f]))]
    assert not bad, bad[:10]


@pytest.mark.parametrize("block", [64, 256])
def test_dense_fallback_path(ctx, orc, block):
    """With a PCG budget of 2 iterations every Newton solve misses its goal, so every LP after
    its first Newton step runs on the dense Cholesky fallback: that path alone must decode
    like the oracle. n=256 gives LPs of up to ~128 rows (several 32-row tiles and a ragged
    last one); one wave per frame, and four waves sharing the trailing tile updates."""
    import torch
    code = regular_code(256)
    C = _code(ctx, code)
    G = batch_awgn(code.n, 0.5, 1.5, 24, stream=9)
    ctx.set_option("PCG_MAXIT", 2)
    ctx.set_option("REF_MAX", 0)
    ctx.set_option("BLOCK", block)
    try:
        out = ctx.decode_batch(C, cuda(G, torch.float64))
        torch.cuda.synchronize()
    finally:
        ctx.set_option("PCG_MAXIT", 0)
        ctx.set_option("REF_MAX", 3)
        ctx.set_option("BLOCK", 0)
    st = host(out["stats"])
    from paper_0902_0657_amd import stats_table
    s = stats_table(st)
    assert np.all(s["direct_solves"][s["malp_iters"] > 0] > 0)
    _compare(orc, code, G, out)


def test_autotune_block(ctx, orc, tmp_path):
    """The launch-shape tuner times each candidate, keeps the fastest in the context and in its
    cache file, and the tuned context still decodes like the oracle."""
    import torch
    from paper_0902_0657_amd import autotune
    code = regular_code(96)
    C = _code(ctx, code)
    G = batch_awgn(code.n, 0.5, 2.0, 16, stream=21)
    g = cuda(G, torch.float64)
    cache = str(tmp_path / "tune.json")
    autotune._CACHE.clear()
    try:
        rec = autotune.tune_block(ctx, C, g, candidates=(64, 128), cache_file=cache)
        assert rec["block"] in (64, 128) and set(rec["ms"]) == {64, 128}
        assert int(ctx.get_option("BLOCK")) == rec["block"]
        assert os.path.exists(cache)
        out = ctx.decode_batch(C, g)
        torch.cuda.synchronize()
        _compare(orc, code, G, out)
    finally:
        ctx.set_option("BLOCK", 0)
        autotune._CACHE.clear()


@pytest.mark.parametrize("order", [0, 1])
def test_claimed_frames_and_dispatch_order_do_not_change_results(order):
    """A batch larger than the device holds at once (300 frames at 256 threads, one workgroup
    per compute unit) runs as one resident set of workgroups that take the frames in turn, in
    index order or, with DISPATCH_ORDER 1, by descending syndrome weight: each output, the LP
    point u and the iteration counts must still belong to their own frame. The same frames
    decoded in batches of 100 (one workgroup per frame) give identical results."""
    import torch
    from paper_0902_0657_amd import Code
    ctx = make_ctx(DISPATCH_ORDER=order, BLOCK=256)
    code = regular_code(96)
    C = Code.from_synth(ctx, code)
    G = np.concatenate([batch_awgn(code.n, 0.5, s, 150, stream=404, snr_index=i)
                        for i, s in enumerate((1.5, 3.0))])
    big = ctx.decode_batch(C, cuda(G, torch.float64), want_u=True)
    parts = [ctx.decode_batch(C, cuda(G[k:k + 100], torch.float64), want_u=True) for k in range(0, 300, 100)]
    torch.cuda.synchronize()
    for key in ("xhat", "flag", "obj", "u"):
        a = host(big[key])
        b = np.concatenate([host(p[key]) for p in parts])
        assert np.array_equal(a, b), key
    sa = host(big["stats"])
    sb = np.concatenate([host(p["stats"]) for p in parts])
    assert np.array_equal(sa[:, :10], sb[:, :10])   # the counts; the clock ticks vary
    ctx.close()
