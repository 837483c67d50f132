"""GPU parity of the individual hot-path steps against the oracle, on shared inputs.

Integer work is compared bit for bit (Algorithm 2 cut sets, Algorithm 7 pairing and level
schedule); floating-point steps against the FP64 oracle / exact linear algebra with the
tolerances stated per test."""
import numpy as np
import pytest

from synth.channel import awgn_llr, frame_seed
from synth.codes import regular_code, irregular_code
from tests.gpu_util import cuda, host, make_ctx, obj_close, snapshot_d2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx()
    yield c
    c.close()


def _code(ctx, code):
    from paper_0902_0657_amd import Code
    return Code.from_synth(ctx, code)


def _u_points(rng, nf, n):
    U = []
    for f in range(nf):
        kind = f % 4
        if kind == 0:
            U.append(rng.random(n))
        elif kind == 1:
            U.append(rng.integers(0, 5, n) / 4.0)            # ties and exact halves
        elif kind == 2:
            U.append(rng.integers(0, 2, n).astype(float))    # integral points
        else:
            U.append(np.clip(0.5 + rng.normal(0, 1e-3, n), 0, 1))
    return np.stack(U)


@pytest.mark.parametrize("n", [96, 1024])
def test_cut_search_bit_exact(ctx, orc, n):
    import torch
    code = regular_code(n)
    C = _code(ctx, code)
    rng = np.random.Generator(np.random.PCG64(100 + n))
    U = _u_points(rng, 8, n)
    vm, viol, lhs = ctx.cut_search_batch(C, cuda(U, torch.float64))
    vm, viol, lhs = host(vm).view(np.uint32), host(viol), host(lhs)
    for f in range(U.shape[0]):
        for j in range(code.m):
            v, V, l = orc.find_cut(U[f, code.row(j)], tau_viol=1e-4)
            assert vm[f, j] == V and bool(viol[f, j]) == v and lhs[f, j] == l, (f, j)


def _weights(rng, nf, q, kind):
    if kind == "ties":
        return rng.integers(0, 4, (nf, q)).astype(np.float32)
    if kind == "spread":
        return (10.0 ** rng.uniform(-8, 8, (nf, q))).astype(np.float32)
    return rng.random((nf, q)).astype(np.float32)


@pytest.mark.parametrize("n,kind", [(96, "uniform"), (96, "ties"), (96, "spread"), (1024, "uniform"),
                                    (1024, "ties"), (1024, "spread"), (4096, "spread")])
def test_mts_pairing_and_levels_bit_exact(ctx, orc, n, kind):
    import torch
    code = regular_code(n)
    C = _code(ctx, code)
    rng = np.random.Generator(np.random.PCG64(7 + n))
    nf = 6
    hascut = (rng.random((nf, code.m)) < rng.uniform(0.5, 1.0, (nf, 1))).astype(np.uint8)
    hascut[0] = 1                                   # every check carries a cut
    W = _weights(rng, nf, code.n + code.m, kind)
    pair, lb, lf, rounds = ctx.mts_batch(C, cuda(hascut, torch.uint8), cuda(W, torch.float32))
    pair, lb, lf, rounds = host(pair), host(lb), host(lf), host(rounds)
    for f in range(nf):
        po, order = orc.mts(code, hascut[f], W[f])
        lbo, lfo = orc.mts_levels(code, hascut[f], po, order)
        assert np.array_equal(pair[f], po), f
        assert np.array_equal(lb[f], lbo) and np.array_equal(lf[f], lfo), f
        assert 1 <= rounds[f] <= max(1, int(hascut[f].sum()))


def test_mts_irregular_bit_exact(ctx, orc):
    import torch
    code = irregular_code(8192)
    C = _code(ctx, code)
    rng = np.random.Generator(np.random.PCG64(77))
    hascut = (rng.random((2, code.m)) < 0.8).astype(np.uint8)
    W = _weights(rng, 2, code.n + code.m, "spread")
    pair, lb, lf, _ = ctx.mts_batch(C, cuda(hascut, torch.uint8), cuda(W, torch.float32))
    for f in range(2):
        po, order = orc.mts(code, hascut[f], W[f])
        lbo, lfo = orc.mts_levels(code, hascut[f], po, order)
        assert np.array_equal(host(pair)[f], po)
        assert np.array_equal(host(lb)[f], lbo) and np.array_equal(host(lf)[f], lfo)


@pytest.mark.parametrize("expand", [0, 1])
@pytest.mark.parametrize("n,kind", [(96, "uniform"), (96, "ties"), (96, "spread"), (1024, "uniform"),
                                    (1024, "ties"), (1024, "spread"), (4096, "spread")])
def test_mts_rowwise_pairing_and_levels_bit_exact(ctx, orc, n, kind, expand):
    """Algorithm 8 with diagonal (PRECOND 2) or triangular (PRECOND 3) expansion: the matched
    column of every row and both level schedules equal the oracle's."""
    import torch
    code = regular_code(n)
    C = _code(ctx, code)
    rng = np.random.Generator(np.random.PCG64(11 + n))
    nf = 6
    hascut = (rng.random((nf, code.m)) < rng.uniform(0.5, 1.0, (nf, 1))).astype(np.uint8)
    hascut[0] = 1
    W = _weights(rng, nf, code.n + code.m, kind)
    ctx.set_option("PRECOND", 2 + expand)
    try:
        pair, lb, lf, rounds = ctx.mts_batch(C, cuda(hascut, torch.uint8), cuda(W, torch.float32))
    finally:
        ctx.set_option("PRECOND", 1)
    pair, lb, lf = host(pair), host(lb), host(lf)
    for f in range(nf):
        po, _ = orc.mts_row(code, hascut[f], W[f], expand=expand)
        lbo, lfo = orc.mts_levels_any(code, hascut[f], po)
        assert np.array_equal(pair[f], po), f
        assert np.array_equal(lb[f], lbo) and np.array_equal(lf[f], lfo), f


@pytest.mark.parametrize("n,kind", [(96, "uniform"), (96, "ties"), (96, "spread"), (1024, "uniform"),
                                    (1024, "ties"), (1024, "spread"), (4096, "spread")])
def test_mts_incremental_pairing_and_levels_bit_exact(ctx, orc, n, kind):
    """Algorithm 6 with the Triangulation Step of Algorithm 5 (PRECOND 5): the chosen set, the
    row each column is matched with and both level schedules equal the oracle's."""
    import torch
    code = regular_code(n)
    C = _code(ctx, code)
    rng = np.random.Generator(np.random.PCG64(13 + n))
    nf = 6 if n < 4096 else 2
    hascut = (rng.random((nf, code.m)) < rng.uniform(0.5, 1.0, (nf, 1))).astype(np.uint8)
    hascut[0] = 1
    W = _weights(rng, nf, code.n + code.m, kind)
    ctx.set_option("PRECOND", 5)
    try:
        pair, lb, lf, calls = ctx.mts_batch(C, cuda(hascut, torch.uint8), cuda(W, torch.float32))
    finally:
        ctx.set_option("PRECOND", 1)
    pair, lb, lf, calls = host(pair), host(lb), host(lf), host(calls)
    for f in range(nf):
        po, order, _ = orc.mts_inc(code, hascut[f], W[f])
        lbo, lfo = orc.mts_levels_any(code, hascut[f], po)
        assert np.array_equal(pair[f], po), f
        assert np.array_equal(lb[f], lbo) and np.array_equal(lf[f], lfo), f
        assert calls[f] >= 1


def _lp_case(orc, code, seed, snr=1.5):
    gamma = awgn_llr(code.n, snr, 1 - code.m / code.n, frame_seed(seed, 0, 0))
    res = orc.decode(code, gamma, trace=True)
    if res.malp_iters == 0:
        return None
    return gamma, res.trace_mask[-1]


def _dense_Q(orc, code, gamma, masks, d2):
    A, b, c = orc.lp_dense(code, gamma, masks)
    rows = np.nonzero(masks)[0]
    d2q = np.concatenate([d2[:code.n], d2[code.n + rows]])
    return (A * d2q) @ A.T, rows


@pytest.mark.parametrize("precision", [0, 1])
def test_normal_matvec(ctx, orc, precision):
    import torch
    code = regular_code(256)
    C = _code(ctx, code)
    rng = np.random.Generator(np.random.PCG64(31))
    cases = [c for c in (_lp_case(orc, code, 300 + s) for s in range(10)) if c is not None][:4]
    G = np.stack([c[0] for c in cases])
    M = np.stack([c[1] for c in cases]).astype(np.uint32)
    D2 = 10.0 ** rng.uniform(-3, 3, (len(cases), code.n + code.m))
    Hh = rng.standard_normal((len(cases), code.m))
    l = host(ctx.normal_matvec_batch(C, cuda(M.view(np.int32), torch.int32), cuda(G, torch.float64),
                                     cuda(D2, torch.float64), cuda(Hh, torch.float64), precision))
    for f in range(len(cases)):
        Q, rows = _dense_Q(orc, code, G[f], M[f], D2[f])
        ref = Q @ Hh[f, rows]
        scale = np.abs(Q) @ np.abs(Hh[f, rows])
        tol = 1e-13 if precision else 2e-6
        assert np.all(np.abs(l[f, rows] - ref) <= tol * scale + 1e-300)
        off = np.setdiff1d(np.arange(code.m), rows)
        assert np.all(l[f, off] == 0)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("ipm_iter", [2, 8, 14, 40])
def test_newton_solve(ctx, orc, precision, ipm_iter):
    """PCG + refinement on realistic D^2 snapshots (the oracle's iterates after 2, 8 and 14
    interior-point iterations, kappa up to ~1e11): the reported FP64 residual
    ||w - Q y|| / ||w|| is the true one, it is small, and y matches the Cholesky solution to
    the accuracy that residual allows (kappa-scaled)."""
    import torch
    code = regular_code(256)
    C = _code(ctx, code)
    rng = np.random.Generator(np.random.PCG64(41))
    cases = [c for c in (_lp_case(orc, code, 400 + s) for s in range(12)) if c is not None][:4]
    G = np.stack([c[0] for c in cases])
    M = np.stack([c[1] for c in cases]).astype(np.uint32)
    D2 = np.stack([snapshot_d2(orc, code, G[f], M[f], ipm_iter) for f in range(len(cases))])
    W = rng.standard_normal((len(cases), code.m)) * (M != 0)
    y, its, res = ctx.newton_solve_batch(C, cuda(M.view(np.int32), torch.int32), cuda(G, torch.float64),
                                         cuda(D2, torch.float64), cuda(W, torch.float64), precision)
    y, its, res = host(y), host(its), host(res)
    for f in range(len(cases)):
        Q, rows = _dense_Q(orc, code, G[f], M[f], D2[f])
        r = W[f, rows] - Q @ y[f, rows]
        nw = np.linalg.norm(W[f, rows])
        rel = np.linalg.norm(r) / nw
        # the library's FP64 residual and this one differ by their rounding, which grows
        # with |Q| |y| (large near the end of the interior-point method)
        floor = 1e-14 * np.linalg.norm(np.abs(Q) @ np.abs(y[f, rows])) / nw
        assert abs(rel - res[f]) <= 1e-3 * rel + floor
        # refinement (switching to FP64 when FP32 stalls) reaches 1e-8 up to kappa 1e9, and a
        # residual within 10 kappa eps up to kappa 1e12 (measured: 1.5e-7 at kappa 2.5e11, in
        # both precisions). Past that (the last iterations reach kappa ~ 1e18) CG stalls in FP64
        # too; a round that would increase the residual is undone, so the result is never
        # worse than dy = 0.
        kappa = np.linalg.cond(Q)
        if kappa < 1e9:
            assert rel <= 1e-8, (f, rel, kappa)
        elif kappa < 1e12:
            assert rel <= 1e-15 * kappa, (f, rel, kappa)
        else:
            assert res[f] <= 1.0, (f, res[f], kappa)   # in the library's own FP64 arithmetic
        if kappa < 1e12:
            yref = orc.normal_solve(code, G[f], M[f], D2[f], W[f])
            err = np.linalg.norm(y[f] - yref) / np.linalg.norm(yref)
            assert err <= max(1e-9, 10 * kappa * max(rel, 1e-16)), (f, err, kappa, rel)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n", [96, 256])
def test_ipm_matches_oracle(ctx, orc, precision, n):
    """Every LP of oracle MALP-A decodes (the cut sets of their traces) solved by the library's
    interior-point method alone: status 0, objective within R1, the solution within 1e-4."""
    import torch
    code = regular_code(n)
    C = _code(ctx, code)
    G, M = [], []
    for s in range(30):
        g = awgn_llr(code.n, 1.5, 0.5, frame_seed(500 + s, 0, 0))
        res = orc.decode(code, g, trace=True)
        for k in range(res.malp_iters):
            G.append(g)
            M.append(res.trace_mask[k])
        if len(G) >= 24:
            break
    G, M = np.stack(G), np.stack(M).astype(np.uint32)
    x, y, z, its, status = ctx.ipm_batch(C, cuda(M.view(np.int32), torch.int32), cuda(G, torch.float64), precision)
    x, status = host(x), host(status)
    for f in range(len(G)):
        assert status[f] == 0
        rc, xo, yo, zo, ito = orc.ipm(code, G[f], M[f])
        u_g = np.where(G[f] >= 0, x[f, :code.n], 1 - x[f, :code.n])
        u_o = np.where(G[f] >= 0, xo[:code.n], 1 - xo[:code.n])
        assert obj_close(G[f] @ u_g, G[f] @ u_o, G[f])
        assert np.abs(u_g - u_o).max() < 1e-4
