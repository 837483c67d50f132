"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code: brute force over odd subsets and
codewords, the full LP relaxation solved by HiGHS, closed forms (Wagner's rule for a single
parity check, Lemma 1), the paper's worked pseudocodeword, theorem invariants, and the
block Newton system of Sec. IV-B.
"""
import itertools
import json
import os

import numpy as np
import pytest

from synth.channel import awgn_llr, batch_awgn, bsc_llr, frame_seed, uniform_snr_awgn
from synth.codes import from_dense, irregular_code, regular_code
from tests import refs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Algorithm 2 + Theorem 1
def test_alg2_matches_bruteforce_and_theorem1(orc):
    rng = np.random.Generator(np.random.PCG64(11))
    cases = []
    for d in range(2, 9):
        for _ in range(300):
            cases.append(rng.random(d))
        for _ in range(50):  # values on the grid {0, 1/4, 1/2, 3/4, 1}: ties and exact halves
            cases.append(rng.integers(0, 5, size=d) / 4.0)
        for _ in range(30):
            cases.append(rng.integers(0, 2, size=d).astype(float))
    for u in cases:
        d = len(u)
        lhs_all = {}
        for V in refs.odd_subsets(d):
            Vs = set(V)
            lhs_all[V] = sum((1 - u[k]) if k in Vs else u[k] for k in range(d))
        viol = [V for V, v in lhs_all.items() if v < 1 - 1e-6]
        strict = [V for V, v in lhs_all.items() if v < 1]
        assert len(strict) <= 1                         # Theorem 1
        got, vmask, lhs = orc.find_cut(u)
        Vgot = tuple(k for k in range(d) if (vmask >> k) & 1)
        assert len(Vgot) % 2 == 1
        assert abs(lhs - lhs_all[Vgot]) < 1e-12
        assert lhs == pytest.approx(min(lhs_all.values()), abs=1e-12)   # V minimises the LHS
        assert got == bool(viol)
        if viol:
            assert Vgot == viol[0]


# ---------------------------------------------------------------- augmented form (Sec. IV-B)
def _x_space(code, gamma, masks):
    """Sign transform written from its definition: x_i = u_i if gamma_i >= 0 else 1 - u_i,
    one slack per cut row; rows in ascending check order."""
    rows = [j for j in range(code.m) if masks[j]]
    p, n = len(rows), code.n
    A = np.zeros((p, n + p))
    b = np.zeros(p)
    for r, j in enumerate(rows):
        a, bb = refs.cut_row_u(code, j, int(masks[j]))
        for i in range(n):
            if gamma[i] < 0 and a[i] != 0:
                bb -= a[i]
                a[i] = -a[i]
        A[r, :n] = a
        A[r, n + r] = 1.0
        b[r] = bb
    c = np.concatenate([np.abs(gamma), np.zeros(p)])
    return A, b, c


def _random_masks(code, rng, frac=0.6):
    masks = np.zeros(code.m, dtype=np.uint32)
    for j in range(code.m):
        if rng.random() < frac:
            d = len(code.row(j))
            V = rng.choice(d, size=rng.choice(np.arange(1, d + 1, 2)), replace=False)
            masks[j] = sum(1 << int(k) for k in V)
    return masks


def test_sign_transform_exact(orc):
    rng = np.random.Generator(np.random.PCG64(5))
    code = regular_code(60)
    for _ in range(20):
        gamma = rng.standard_normal(code.n)
        masks = _random_masks(code, rng)
        A, b, c = orc.lp_dense(code, gamma, masks)
        A2, b2, c2 = _x_space(code, gamma, masks)
        assert np.array_equal(A, A2) and np.array_equal(b, b2) and np.array_equal(c, c2)
        # dyadic u: the u-space slack of every cut equals b - A_std x exactly
        u = rng.integers(0, 9, size=code.n) / 8.0
        x = np.where(gamma >= 0, u, 1 - u)
        rows = [j for j in range(code.m) if masks[j]]
        for r, j in enumerate(rows):
            a, bb = refs.cut_row_u(code, j, int(masks[j]))
            assert bb - a @ u == b[r] - A[r, :code.n] @ x


# ---------------------------------------------------------------- IPM on one LP (Sec. IV-B)
def test_ipm_matches_highs_and_kkt(orc):
    code = regular_code(96)
    checked = 0
    for f in range(12):
        gamma = awgn_llr(code.n, 1.5, 0.5, frame_seed(21, 0, f))
        res = orc.decode(code, gamma, trace=True)
        for k in range(res.malp_iters):
            masks = res.trace_mask[k]
            rc, x, y, z, its = orc.ipm(code, gamma, masks)
            assert rc == 0 and its < 100
            A, b, c = _x_space(code, gamma, masks)
            assert np.all(x > 0) and np.all(z > 0)
            assert np.linalg.norm(A @ x - b) / (1 + np.linalg.norm(b)) < 1e-8
            assert np.linalg.norm(A.T @ y + z - c) / (1 + np.linalg.norm(c)) < 1e-8
            assert x @ z / (1 + abs(c @ x)) < 1e-8
            u = np.where(gamma >= 0, x[:code.n], 1 - x[:code.n])
            fun, _ = refs.cutset_lp(code, gamma, masks)
            assert gamma @ u == pytest.approx(fun, rel=1e-6, abs=1e-6)
            # the decoder's u^k is the LP solution put back on the box (Theorem 2a)
            assert gamma @ np.clip(u, 0.0, 1.0) == pytest.approx(res.trace_obj[k], abs=1e-12)
            checked += 1
    assert checked > 20


def test_newton_block_system(orc):
    """(dx, dy, dz) solve the 3x3 block Newton system of Sec. IV-B."""
    rng = np.random.Generator(np.random.PCG64(9))
    code = regular_code(60)
    for _ in range(10):
        gamma = rng.standard_normal(code.n)
        masks = _random_masks(code, rng)
        A, b, c = _x_space(code, gamma, masks)
        p, q = A.shape
        x = rng.uniform(0.1, 2, q)
        z = rng.uniform(0.1, 2, q)
        y = rng.standard_normal(p)
        mu = 0.37
        dx, dy, dz = orc.newton(code, gamma, masks, x, y, z, mu)
        rb, rc, re = b - A @ x, c - A.T @ y - z, mu - x * z
        assert np.allclose(A @ dx, rb, atol=1e-9)
        assert np.allclose(A.T @ dy + dz, rc, atol=1e-9)
        assert np.allclose(z * dx + x * dz, re, atol=1e-9)


# ---------------------------------------------------------------- whole decoder
def _frames(code, snrs, per, stream):
    out = []
    for si, s in enumerate(snrs):
        for f in range(per):
            out.append(awgn_llr(code.n, s, 1 - code.m / code.n, frame_seed(stream, si, f)))
    return out


@pytest.mark.parametrize("mode", [0, 1])
def test_malp_equals_full_lp_decoding(orc, mode):
    """Theorem 2c: MALP reaches the LP-decoding optimum over the fundamental polytope."""
    code = regular_code(96)
    opts = orc.OracleOpts(malp_mode=mode)
    for gamma in _frames(code, [1.0, 1.5, 2.5], 8, 31):
        res = orc.decode(code, gamma, opts)
        assert res.status == 0
        fun, ustar = refs.feldman_lp(code, gamma)
        assert res.objective == pytest.approx(fun, rel=1e-6, abs=1e-6)
        assert np.abs(res.u - ustar).max() < 1e-5


def test_malp_irregular_bsc_equals_full_lp(orc):
    """The irregular ensemble and the BSC with the small continuous perturbation."""
    code = irregular_code(256)
    for f in range(10):
        gamma = bsc_llr(code.n, 0.08, frame_seed(41, 0, f))
        res = orc.decode(code, gamma)
        fun, _ = refs.feldman_lp(code, gamma)
        assert res.objective == pytest.approx(fun, rel=1e-6, abs=1e-6)


def test_integral_output_is_ml_codeword(orc):
    """ML certificate (Sec. II-B): an integral LP output is the ML codeword; the LP optimum
    never exceeds the ML cost."""
    n_int = 0
    for n in (24, 28):
        code = regular_code(n, no4=False)
        H = code.dense()
        for gamma in _frames(code, [0.5, 1.0, 2.0, 3.0], 10, 51):
            res = orc.decode(code, gamma)
            u_ml, c_ml, _, _ = refs.ml_decode(H, gamma)
            assert res.objective <= c_ml + 1e-6
            if res.flag == 1:
                n_int += 1
                assert np.array_equal(res.xhat, u_ml)
                assert res.objective == pytest.approx(c_ml, abs=1e-6)
    assert n_int > 20


def test_single_parity_check_wagner(orc):
    """m = 1 (Lemma 1: the check polytope is the codeword polytope): LP = ML = Wagner's rule."""
    rng = np.random.Generator(np.random.PCG64(3))
    for d in (3, 6, 7, 8):
        code = from_dense(np.ones((1, d), dtype=np.uint8))
        for _ in range(40):
            gamma = rng.standard_normal(d) * 2 + 0.3
            hard = (gamma < 0).astype(np.uint8)
            want = hard.copy()
            if hard.sum() % 2:
                k = int(np.argmin(np.abs(gamma)))
                want[k] ^= 1
            res = orc.decode(code, gamma)
            assert res.flag == 1
            assert np.array_equal(res.xhat, want)


def test_hard_decision_codeword_solves_no_lp(orc):
    code = regular_code(96)
    rng = np.random.Generator(np.random.PCG64(8))
    B = refs.gf2_nullspace(code.dense())
    for _ in range(10):
        cw = (rng.integers(0, 2, B.shape[0]) @ B) % 2
        gamma = rng.uniform(0.5, 3, code.n) * np.where(cw == 1, -1.0, 1.0)
        res = orc.decode(code, gamma)
        assert res.malp_iters == 0 and res.flag == 1
        assert np.array_equal(res.xhat, cw.astype(np.uint8))


def test_high_snr_all_zero(orc):
    code = regular_code(240)
    for gamma in _frames(code, [6.0], 10, 61):
        res = orc.decode(code, gamma)
        assert res.flag == 1 and not res.xhat.any()


def test_theorem_invariants(orc):
    """Theorem 2a (box), 2b (strictly increasing cost), 2c (at most n LPs), Theorem 3 /
    Corollary 3 (at most one cut per check, p <= m), Corollary 5 (at most m fractional
    entries), the counting bound of Corollary 4 in its proved form (the LP solution differs
    from the hard decision in at most as many places as there are tight parity inequalities,
    hence at most m), and Theorem 4 (the flipped set of an integral output has no stopping set)."""
    code = regular_code(96)
    n_frac = n_int = 0
    for gamma in _frames(code, [1.0, 1.5, 2.0], 20, 71):
        res = orc.decode(code, gamma, trace=True)
        assert res.status == 0
        assert res.u.min() > -1e-5 and res.u.max() < 1 + 1e-5   # IPM accuracy
        assert res.malp_iters <= code.n
        assert np.all(np.diff(res.trace_obj) > -1e-7)
        if res.malp_iters:
            assert res.trace_p.max() <= code.m
        hard = (gamma < 0).astype(float)
        nfr = int(np.sum(np.minimum(res.u, 1 - res.u) > 1e-4))
        assert nfr <= code.m
        moved = int(np.sum(np.abs(res.u - hard) > 1e-4))
        assert moved <= (res.p_final if res.malp_iters else 0) <= code.m
        if res.flag == 1:
            n_int += 1
            flipped = res.xhat != hard.astype(np.uint8)
            assert refs.peel(code, flipped)
        else:
            n_frac += 1
    assert n_int > 10 and n_frac > 3


def test_peeling_helper_matches_bruteforce():
    code = regular_code(24, no4=False)
    rng = np.random.Generator(np.random.PCG64(2))
    for _ in range(200):
        S = rng.random(code.n) < rng.uniform(0.1, 0.5)
        assert refs.peel(code, S) == (not refs.has_stopping_set(code, S))


def test_hamming743_pseudocodeword(orc):
    """The (7,4,3) pseudocodeword printed after Corollary 5: exactly m = 3 fractional entries,
    reached by LP decoding for a cost vector inside its normal cone."""
    g = json.load(open(os.path.join(GOLDEN, "hamming743.json")))
    code = from_dense(np.array(g["H"]))
    f = np.array(g["pseudocodeword"])
    for mode in (0, 1):
        res = orc.decode(code, np.array(g["gamma"]), orc.OracleOpts(malp_mode=mode))
        assert res.flag == 0
        assert np.abs(res.u - f).max() < 1e-6
        assert int(np.sum(np.abs(res.u - 0.5) < 1e-6)) == code.m == 3


# ---------------------------------------------------------------- Algorithm 7 + levels
def mts_scan(code, hascut, w):
    """Algorithm 7 by exhaustive scan: every step takes the degree-1 column of largest
    (float32 weight, -index) and eliminates its row. O(p q)."""
    n, m = code.n, code.m
    rows_of = {i: [] for i in range(n)}
    for j in range(m):
        if hascut[j]:
            for i in code.row(j):
                rows_of[int(i)].append(j)
    for j in range(m):
        if hascut[j]:
            rows_of[n + j] = [j]
    alive = {j for j in range(m) if hascut[j]}
    chosen = set()
    pair = np.full(m, -1, dtype=np.int32)
    order = []
    while alive:
        best, bkey, brow = None, None, None
        for c, rs in rows_of.items():
            if c in chosen:
                continue
            live = [r for r in rs if r in alive]
            if len(live) == 1:
                key = (np.float32(w[c]), -c)
                if bkey is None or key > bkey:
                    best, bkey, brow = c, key, live[0]
        pair[brow] = best
        order.append(brow)
        alive.discard(brow)
        chosen.add(best)
    return pair, np.array(order, dtype=np.int32)


def _weights(rng, q, kind):
    if kind == "ties":
        return rng.integers(0, 4, q).astype(np.float32)
    if kind == "spread":
        return (10.0 ** rng.uniform(-8, 8, q)).astype(np.float32)
    return rng.random(q).astype(np.float32)


@pytest.mark.parametrize("kind", ["uniform", "ties", "spread"])
def test_mts_heap_equals_scan_and_is_triangular(orc, kind):
    rng = np.random.Generator(np.random.PCG64(17))
    for n in (48, 96, 150):
        code = regular_code(n) if n >= 60 else regular_code(n, no4=False)
        for _ in range(6):
            hascut = (rng.random(code.m) < 0.8).astype(np.uint8)
            w = _weights(rng, code.n + code.m, kind)
            pair, order = orc.mts(code, hascut, w)
            p2, o2 = mts_scan(code, hascut, w)
            assert np.array_equal(pair, p2) and np.array_equal(order, o2)
            p = int(hascut.sum())
            assert len(order) == p and len(set(order.tolist())) == p
            # A_M with rows in elimination order and columns in the same order is upper
            # triangular with a nonzero diagonal (Algorithm 7)
            H = code.dense()
            cols = [int(pair[j]) for j in order]
            for k, j in enumerate(order):
                for l, c in enumerate(cols):
                    nz = (c >= code.n and c - code.n == j) or (c < code.n and H[j, c])
                    if l == k:
                        assert nz
                    elif l < k:
                        assert not nz


def test_mts_levels_are_longest_chains(orc):
    rng = np.random.Generator(np.random.PCG64(23))
    code = regular_code(120)
    n = code.n
    for _ in range(8):
        hascut = (rng.random(code.m) < 0.75).astype(np.uint8)
        w = _weights(rng, code.n + code.m, "spread")
        pair, order = orc.mts(code, hascut, w)
        lb, lf = orc.mts_levels(code, hascut, pair, order)
        pairrow = {int(pair[j]): j for j in range(code.m) if pair[j] >= 0}
        rows_of = {i: [j for j in range(code.m) if hascut[j] and i in code.row(j)] for i in range(n)}

        def deps_b(j):
            return [pairrow[int(i)] for i in code.row(j) if int(i) != pair[j] and int(i) in pairrow]

        def deps_f(j):
            c = int(pair[j])
            return [] if c >= n else [r for r in rows_of[c] if r != j]

        memo = {}

        def depth(j, deps, tag):
            if (tag, j) not in memo:
                d = deps(j)
                memo[(tag, j)] = 0 if not d else 1 + max(depth(k, deps, tag) for k in d)
            return memo[(tag, j)]

        for j in range(code.m):
            if hascut[j]:
                assert lb[j] == depth(j, deps_b, "b")
                assert lf[j] == depth(j, deps_f, "f")
            else:
                assert lb[j] == -1 and lf[j] == -1


# ---------------------------------------------------------------- PCG (Algorithm 4)
def _lp_instance(orc, code, seed):
    gamma = awgn_llr(code.n, 1.5, 0.5, frame_seed(seed, 0, 0))
    res = orc.decode(code, gamma, trace=True)
    masks = res.trace_mask[-1] if res.malp_iters else _random_masks(code, np.random.Generator(np.random.PCG64(seed)))
    return gamma, masks


def test_pcg_fp64_equals_cholesky(orc):
    rng = np.random.Generator(np.random.PCG64(4))
    code = regular_code(200)
    for s in range(4):
        gamma, masks = _lp_instance(orc, code, 80 + s)
        d2 = rng.uniform(0.1, 10, code.n + code.m)
        w = rng.standard_normal(code.m) * (masks != 0)
        y_ref = orc.normal_solve(code, gamma, masks, d2, w)
        for precond in (True, False):
            y, it, res = orc.pcg(code, gamma, masks, d2, w, tol=1e-12, maxit=2000, precond=precond)
            assert res[-1] <= 1e-12
            assert np.abs(y - y_ref).max() <= 1e-9 * max(1, np.abs(y_ref).max())


def test_pcg_exact_preconditioner_one_iteration(orc):
    """When D^2 vanishes off the preconditioning set, M = Q and PCG stops after one step."""
    rng = np.random.Generator(np.random.PCG64(6))
    code = regular_code(120)
    hits = 0
    for s in range(10):
        gamma, masks = _lp_instance(orc, code, 90 + s)
        hascut = (masks != 0).astype(np.uint8)
        w0 = rng.random(code.n + code.m).astype(np.float32)
        pair, _ = orc.mts(code, hascut, w0)
        inM = np.zeros(code.n + code.m, dtype=bool)
        inM[pair[pair >= 0]] = True
        d2 = np.where(inM, rng.uniform(0.5, 2, code.n + code.m), 0.0)
        pair2, _ = orc.mts(code, hascut, d2.astype(np.float32))
        if not np.array_equal(np.sort(pair2[pair2 >= 0]), np.sort(pair[pair >= 0])):
            continue
        hits += 1
        w = rng.standard_normal(code.m) * hascut
        y, it, res = orc.pcg(code, gamma, masks, d2, w, tol=1e-10, maxit=50)
        assert it == 1 and res[-1] < 1e-10
    assert hits >= 3


def test_stalled_ipm_floor_rule(orc):
    """Reading of the termination test: on degenerate LPs the plain normal equations stall near
    a relative gap of 1e-8 in FP64. Frames of the n=1024 batch (Eb/N0 1.5 dB, FP32 LLRs) whose
    last LP stalls there hit the iteration cap without the floor rule; with it they end at the
    LP-decoding optimum, checked against HiGHS on the full relaxation (Theorem 2c)."""
    code = regular_code(1024)
    G = batch_awgn(code.n, 0.5, 1.5, 54, stream=2024, snr_index=0).astype(np.float32)
    for f in (8, 53):
        gamma = G[f].astype(np.float64)
        stuck = orc.decode(code, gamma, orc.OracleOpts(eps_stall=0.0))
        assert stuck.flag == -1                       # the 1e-8 target alone is not reachable
        res = orc.decode(code, gamma)
        assert res.status == 0 and res.flag in (0, 1)
        fun, _ = refs.feldman_lp(code, gamma)
        scale = 1.0 + abs(fun - gamma[gamma < 0].sum())
        assert abs(res.objective - fun) <= 1e-7 * scale


# ---------------------------------------------------------------- Algorithm 8 + levels
def mts_row_dense(code, hascut, w):
    """Algorithm 8 on an explicit 0/1 residual matrix (rows = checks with a cut, columns = the
    n standard columns and the m slacks), zeroing columns as the algorithm states: the
    lowest-indexed row of degree 1 is matched with its column; with no such row the nonzero
    column of smallest (float32 weight, index) is zeroed; unmatched rows get their slack."""
    n, m = code.n, code.m
    H = code.dense()
    A = np.zeros((m, n + m), dtype=np.int8)
    for j in range(m):
        if hascut[j]:
            A[j, :n] = H[j]
            A[j, n + j] = 1
    pair = np.full(m, -1, dtype=np.int32)
    order = []
    while A.any():
        rows1 = np.nonzero(A.sum(axis=1) == 1)[0]
        if len(rows1):
            j = int(rows1[0])
            i = int(np.nonzero(A[j])[0][0])
            pair[j] = i
            order.append(j)
        else:
            i = min((np.float32(w[c]), int(c)) for c in np.nonzero(A.any(axis=0))[0])[1]
        A[:, i] = 0
    for j in range(m):
        if hascut[j] and pair[j] < 0:
            pair[j] = n + j
            order.append(j)
    return pair, np.array(order, dtype=np.int32)


@pytest.mark.parametrize("kind", ["uniform", "ties", "spread"])
def test_mts_row_equals_dense_and_is_lower_triangular(orc, kind):
    rng = np.random.Generator(np.random.PCG64(29))
    for n in (48, 96, 150):
        code = regular_code(n) if n >= 60 else regular_code(n, no4=False)
        H = code.dense()
        for _ in range(5):
            hascut = (rng.random(code.m) < 0.8).astype(np.uint8)
            w = _weights(rng, code.n + code.m, kind)
            pair, order = orc.mts_row(code, hascut, w)
            p2, o2 = mts_row_dense(code, hascut, w)
            assert np.array_equal(pair, p2) and np.array_equal(order, o2)
            p = int(hascut.sum())
            assert len(order) == p and len(set(order.tolist())) == p
            cols = [int(pair[j]) for j in order]
            assert len(set(cols)) == p
            # rows and columns in matching order: lower triangular with a nonzero diagonal
            for k, j in enumerate(order):
                for l, c in enumerate(cols):
                    nz = (c >= code.n and c - code.n == j) or (c < code.n and H[j, c])
                    if l == k:
                        assert nz
                    elif l > k:
                        assert not nz


def test_mts_row_single_check_keeps_heaviest_column(orc):
    """One check with a cut: no row has degree 1 until every column but one is gone, and the
    lightest go first, so the row is matched with its heaviest column (slack included)."""
    code = from_dense(np.array([[1, 1, 1, 1, 1, 0], [0, 1, 1, 1, 0, 1]], dtype=np.int8))
    rng = np.random.Generator(np.random.PCG64(31))
    for _ in range(20):
        w = rng.random(code.n + code.m).astype(np.float32)
        pair, order = orc.mts_row(code, np.array([1, 0], dtype=np.uint8), w)
        cand = list(code.row(0)) + [code.n + 0]
        assert pair[0] == max(cand, key=lambda c: (w[c], -c)) and pair[1] == -1
        assert order.tolist() == [0]


def test_levels_any_equals_ordered_levels_and_longest_chains(orc):
    """The order-free level computation agrees with the elimination-order one on Algorithm 7
    sets, and equals the longest dependency chains on Algorithm 8 sets."""
    rng = np.random.Generator(np.random.PCG64(37))
    code = regular_code(120)
    n = code.n
    for _ in range(6):
        hascut = (rng.random(code.m) < 0.75).astype(np.uint8)
        w = _weights(rng, code.n + code.m, "spread")
        pair, order = orc.mts(code, hascut, w)
        lb, lf = orc.mts_levels(code, hascut, pair, order)
        lb2, lf2 = orc.mts_levels_any(code, hascut, pair)
        assert np.array_equal(lb, lb2) and np.array_equal(lf, lf2)
        pair, order = orc.mts_row(code, hascut, w)
        lb, lf = orc.mts_levels_any(code, hascut, pair)
        pairrow = {int(pair[j]): j for j in range(code.m) if pair[j] >= 0}
        rows_of = {i: [j for j in range(code.m) if hascut[j] and i in code.row(j)] for i in range(n)}
        # longest chains by repeated relaxation (Bellman-Ford on the dependency graph)
        db = {j: [pairrow[int(i)] for i in code.row(j) if int(i) != pair[j] and int(i) in pairrow]
              for j in range(code.m) if hascut[j]}
        df = {j: ([] if pair[j] >= n else [r for r in rows_of[int(pair[j])] if r != j])
              for j in range(code.m) if hascut[j]}
        for deps, lev in ((db, lb), (df, lf)):
            L = {j: 0 for j in deps}
            for _ in range(len(deps) + 1):
                L = {j: (1 + max(L[k] for k in d)) if d else 0 for j, d in deps.items()}
            for j in deps:
                assert lev[j] == L[j]


def triangulation_step(code, hascut, pair):
    """Algorithm 5 on the preconditioning columns: repeatedly take a row with exactly one
    remaining column of the set and remove that column. Succeeds (returns True) iff A_M can
    be brought into triangular form by row and column permutations."""
    n = code.n
    H = code.dense()
    rows = [j for j in range(code.m) if hascut[j]]
    cols = {int(pair[j]) for j in rows}

    def nz(j, c):
        return (c >= n and c - n == j) or (c < n and H[j, c] != 0)
    left_rows, left_cols = set(rows), set(cols)
    while left_rows:
        pick = None
        for j in sorted(left_rows):
            cs = [c for c in left_cols if nz(j, c)]
            if len(cs) == 1:
                pick = (j, cs[0])
                break
        if pick is None:
            return False
        left_rows.discard(pick[0])
        left_cols.discard(pick[1])
    return True


def mts_row_tri_dense(code, hascut, w):
    """Algorithm 8 with triangular expansion on explicit matrices: the row-wise phase of
    mts_row_dense without its diagonal expansion, then the column-wise greedy search (largest
    (weight, -index) degree-1 column) on A-bar, the columns with no entry in a matched row."""
    n, m = code.n, code.m
    H = code.dense()
    A = np.zeros((m, n + m), dtype=np.int8)
    for j in range(m):
        if hascut[j]:
            A[j, :n] = H[j]
            A[j, n + j] = 1
    full = A.copy()
    pair = np.full(m, -1, dtype=np.int32)
    order = []
    while A.any():
        rows1 = np.nonzero(A.sum(axis=1) == 1)[0]
        if len(rows1):
            j = int(rows1[0])
            i = int(np.nonzero(A[j])[0][0])
            pair[j] = i
            order.append(j)
        else:
            i = min((np.float32(w[c]), int(c)) for c in np.nonzero(A.any(axis=0))[0])[1]
        A[:, i] = 0
    unmatched = [j for j in range(m) if hascut[j] and pair[j] < 0]
    matched = [j for j in range(m) if pair[j] >= 0]
    B = full.copy()
    B[matched, :] = 0
    bar = [c for c in range(n + m) if full[:, c].any() and not full[matched, c].any()]
    B = B[:, bar]
    live = set(unmatched)
    while live:
        best = None
        for k, c in enumerate(bar):
            rs = [j for j in live if B[j, k]]
            if len(rs) == 1 and (best is None or (np.float32(w[c]), -c) > best[0]):
                best = ((np.float32(w[c]), -c), c, rs[0])
        _, c, j = best
        pair[j] = c
        order.append(j)
        live.discard(j)
        B[j, :] = 0
    return pair, np.array(order, dtype=np.int32)


@pytest.mark.parametrize("kind", ["uniform", "ties", "spread"])
def test_mts_row_triangular_expansion_equals_dense_and_triangulates(orc, kind):
    rng = np.random.Generator(np.random.PCG64(41))
    for n in (48, 96):
        code = regular_code(n) if n >= 60 else regular_code(n, no4=False)
        for _ in range(5):
            hascut = (rng.random(code.m) < 0.8).astype(np.uint8)
            w = _weights(rng, code.n + code.m, kind)
            pair, order = orc.mts_row(code, hascut, w, expand=1)
            p2, o2 = mts_row_tri_dense(code, hascut, w)
            assert np.array_equal(pair, p2) and np.array_equal(order, o2)
            p = int(hascut.sum())
            assert len(order) == p and len({int(pair[j]) for j in order}) == p
            assert triangulation_step(code, hascut, pair)
            # the row-wise phase is the same for both expansions: rows that the diagonal
            # expansion did not give their slack keep their column
            pd, od = orc.mts_row(code, hascut, w, expand=0)
            for j in od:
                if pd[j] != code.n + j:
                    assert pair[j] == pd[j]


def test_triangulation_step_rejects_a_cycle(orc):
    """Algorithm 5 itself: the 2 x 2 all-ones block (a 4-cycle) cannot be triangularised."""
    code = from_dense(np.array([[1, 1, 0], [1, 1, 1]], dtype=np.int8))
    assert not triangulation_step(code, np.array([1, 1], np.uint8), np.array([0, 1], np.int32))
    assert triangulation_step(code, np.array([1, 1], np.uint8), np.array([0, 2], np.int32))


# ---------------------------------------------------------------- Theorem 2a/2b in the MALP loop
# A frame of the n=256 (3,6) code whose LLR gamma_164 is about -3e-6: the IPM leaves u_164 about
# 1.6e-4 below 0 (its cost is too small for the gap test to pin it), which, without the box
# clamp of Theorem 2a, makes Algorithm 2 report a violated cut at a left-hand side of 0.99984 and
# MALP-A replace a cut that still binds; the cut sets then alternate with period 2.
CYCLE_FRAME = dict(n=256, ebn0=1.6537604712821115, seed=frame_seed(91, 0, 145))


def test_malp_cycle_frame_reaches_lp_optimum(orc):
    code = regular_code(CYCLE_FRAME["n"])
    gamma = awgn_llr(code.n, CYCLE_FRAME["ebn0"], 0.5, CYCLE_FRAME["seed"])
    fun, ustar = refs.feldman_lp(code, gamma)
    scale = 1.0 + abs(fun - gamma[gamma < 0].sum())
    for mode in (0, 1):
        res = orc.decode(code, gamma, orc.OracleOpts(malp_mode=mode), trace=True)
        assert res.flag == 1, (mode, res.flag)
        assert abs(res.objective - fun) <= 1e-6 * scale
        assert np.array_equal(res.xhat, (ustar > 0.5).astype(np.uint8))
        assert np.all(np.diff(res.trace_obj) > 0)          # Theorem 2b
    # the planted mistake: no clamp. The recurrence test ends the cycle when LP 2 repeats
    # LP 0; the cost check (Theorem 2b) alone ends it at its first decrease; without either
    # the decode runs into the MALP cap
    bad = orc.decode(code, gamma, orc.OracleOpts(box_clamp=0), trace=True)
    assert bad.flag == -7 and bad.malp_iters <= 4
    bad = orc.decode(code, gamma, orc.OracleOpts(box_clamp=0, cycle_stop=0), trace=True)
    assert bad.flag == -5 and bad.malp_iters <= 4
    assert bad.trace_obj[-1] < bad.trace_obj[-2]
    worse = orc.decode(code, gamma, orc.OracleOpts(box_clamp=0, tau_cost=1.0, cycle_stop=0, malp_max=50))
    assert worse.flag == -3



# A frame of the n=1024 (3,6) code at 1.99 dB whose MALP-A cut sets alternate between two LPs
# that differ only in the cut of check 96 (odd sets 4 and 8). LP-A's optimum is unique but
# flat along cut B: HiGHS finds LP-A points whose cost exceeds the optimum by 1e-9 and that
# violate B by 6.9e-5, so the IPM's point (cost within its gap test) violates B by 2e-4, and
# LP-B's point in turn violates A. Theorem 2 assumes unique optima; at the IPM's accuracy that
# fails here, and both sides end the decode at the first recurrence of a cut set.
FLAT_FRAME = dict(n=1024, ebn0=1.9857919617105901, seed=frame_seed(84, 1, 578))


def test_malp_cut_cycle_ends_at_first_recurrence(orc):
    code = regular_code(FLAT_FRAME["n"])
    gamma = awgn_llr(code.n, FLAT_FRAME["ebn0"], 0.5, FLAT_FRAME["seed"])
    fun, ustar = refs.feldman_lp(code, gamma)
    scale = 1.0 + abs(fun - gamma[gamma < 0].sum())
    res = orc.decode(code, gamma, orc.OracleOpts(), trace=True)
    M = res.trace_mask
    assert res.flag == -7 and res.malp_iters < 25
    # the last LP solved is the one of two LPs back; the two LPs differ in one check's cut
    assert np.array_equal(M[-1], M[-3]) and np.count_nonzero(M[-1] != M[-2]) == 1
    # the output is the costlier LP's solution, optimal within the IPM's gap test
    assert res.objective >= res.trace_obj[-2]
    assert abs(res.objective - fun) <= 1e-6 * scale
    fa, _ = refs.cutset_lp(code, gamma, M[-1])
    fb, _ = refs.cutset_lp(code, gamma, M[-2])
    assert abs(fa - fun) <= 1e-12 * scale and fun - 1e-6 * scale < fb < fun
    # the decisions are those of the LP-decoding optimum; the point itself violates the other
    # LP's cut by more than tau_viol
    assert np.array_equal(res.xhat, (ustar > 0.5).astype(np.uint8))
    assert 1e-4 < refs.max_parity_violation(code, res.u) < 1e-3
    # MALP-B takes another path on this frame and ends normally (fractional output)
    resb = orc.decode(code, gamma, orc.OracleOpts(malp_mode=1))
    assert resb.flag == 0 and abs(resb.objective - fun) <= 1e-6 * scale
    # the planted mistake: without the recurrence test the two LPs alternate up to the cap
    bad = orc.decode(code, gamma, orc.OracleOpts(cycle_stop=0, malp_max=30), trace=True)
    assert bad.flag == -3
    assert all(np.array_equal(bad.trace_mask[k], bad.trace_mask[k - 2]) for k in range(20, 30))

def _sweep_frame(args):
    import oracle as O
    n, mode, f = args
    code = regular_code(n)
    e, gamma = uniform_snr_awgn(n, 1.5, 3.0, 92, f)
    r = O.decode(code, gamma, O.OracleOpts(malp_mode=mode), trace=True)
    gneg = gamma[gamma < 0].sum()
    costs = np.concatenate([[gneg], r.trace_obj])
    rel = np.diff(costs) / (1.0 + np.abs(costs[:-1] - gneg))
    return f, e, r.flag, float(rel.min()) if rel.size else np.inf, float(r.u.min()), float(r.u.max())


@pytest.mark.parametrize("n,mode,frames", [(256, 0, 2000), (256, 1, 2000), (1024, 0, 500)])
def test_malp_sweep_no_failures(orc, n, mode, frames):
    """No negative flag over a sweep of frames with Eb/N0 uniform in [1.5, 3] dB; every
    decode's LP costs increase (Theorem 2b, within the IPM's relative accuracy) and its
    output lies in the box (Theorem 2a)."""
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(_sweep_frame, [(n, mode, f) for f in range(frames)], chunksize=8)
    bad = [(f, e, fl) for f, e, fl, _, _, _ in res if fl < 0]
    assert not bad, bad[:10]
    assert min(r[3] for r in res) > -1e-8
    assert min(r[4] for r in res) >= 0.0 and max(r[5] for r in res) <= 1.0
    assert sum(r[2] == 0 for r in res) > frames // 50       # the sweep reaches fractional frames


# ---------------------------------------------------------------- Algorithm 5 + Algorithm 6
def _lp_pattern(code, hascut):
    """Nonzero pattern of the LP's A as a code: rows = checks with a cut, columns = the n
    standard columns and the slack column n+j of every such check (zero columns elsewhere)."""
    H = code.dense()
    rows = np.nonzero(hascut)[0]
    A = np.zeros((len(rows), code.n + code.m), dtype=np.uint8)
    for r, j in enumerate(rows):
        A[r, :code.n] = H[j]
        A[r, code.n + j] = 1
    return A


def _triangulable(A, S):
    """Algorithm 5 read from the paper on an explicit matrix: s times, some row with exactly one
    remaining column of S gives up that column (row and column zeroed); failure when no such
    row exists."""
    sub = A[:, S].astype(bool).copy()
    for _ in range(len(S)):
        deg = sub.sum(axis=1)
        r = np.nonzero(deg == 1)[0]
        if r.size == 0:
            return False
        i = int(np.nonzero(sub[r[0]])[0][0])
        sub[:, i] = False
        sub[r[0], :] = False
    return True


def _check_lower_triangular(code, hascut, inS, pair, order):
    """A_S in matching order: the columns of S in the k-th matched row are matched at or
    before position k, and the diagonal entries are nonzero."""
    A = _lp_pattern(code, hascut)
    rowpos = {int(j): r for r, j in enumerate(np.nonzero(hascut)[0])}
    pos = {int(pair[j]): k for k, j in enumerate(order)}
    assert len(pos) == len(order)
    for k, j in enumerate(order):
        a = A[rowpos[int(j)]]
        assert a[pair[j]]
        for c in np.nonzero(a)[0]:
            if inS[c]:
                assert pos[int(c)] <= k


def test_triangulation_step_is_peeling_and_triangulates(orc):
    """Algorithm 5 succeeds exactly when the column set holds no stopping set of the LP's
    extended Tanner graph (brute force), agrees with the explicit-matrix reading, and its
    pairing puts A_S in lower-triangular form."""
    from synth.codes import from_dense
    rng = np.random.Generator(np.random.PCG64(61))
    ok = fail = 0
    for n in (12, 16):
        code = regular_code(n, no4=False)
        for _ in range(60):
            hascut = (rng.random(code.m) < 0.8).astype(np.uint8)
            if not hascut.any():
                continue
            A = _lp_pattern(code, hascut)
            present = [c for c in range(code.n + code.m) if c < code.n or hascut[c - code.n]]
            S = sorted(rng.choice(present, size=int(rng.integers(1, min(9, len(present)) + 1)), replace=False).tolist())
            inS = np.zeros(code.n + code.m, np.uint8)
            inS[S] = 1
            k, pair, order = orc.triangulate(code, hascut, inS)
            succ = k == len(S)
            ext = from_dense(A)
            assert succ == _triangulable(A, S) == (not refs.has_stopping_set(ext, inS))
            if succ:
                ok += 1
                assert sorted(int(pair[j]) for j in order) == S
                _check_lower_triangular(code, hascut, inS, pair, order)
            else:
                fail += 1
    assert ok > 20 and fail > 20


def _mts_inc_dense(code, hascut, w):
    """Algorithm 6 read from the paper: columns by weight descending (index ascending on ties),
    each added while the set still passes the Triangulation Step, until p are chosen."""
    A = _lp_pattern(code, hascut)
    p = int(hascut.sum())
    cols = [c for c in range(code.n + code.m) if c < code.n or hascut[c - code.n]]
    cols.sort(key=lambda c: (-np.float32(w[c]), c))
    M = []
    for c in cols:
        if len(M) == p:
            break
        if _triangulable(A, M + [c]):
            M.append(c)
    return sorted(M)


@pytest.mark.parametrize("kind", ["uniform", "ties", "spread"])
def test_mts_inc_equals_dense_replay(orc, kind):
    rng = np.random.Generator(np.random.PCG64(62))
    for n in (48, 96):
        code = regular_code(n) if n >= 60 else regular_code(n, no4=False)
        for _ in range(4):
            hascut = (rng.random(code.m) < 0.8).astype(np.uint8)
            w = _weights(rng, code.n + code.m, kind)
            pair, order, calls = orc.mts_inc(code, hascut, w)
            p = int(hascut.sum())
            assert len(order) == p
            assert sorted(int(pair[j]) for j in order) == _mts_inc_dense(code, hascut, w)
            inS = np.zeros(code.n + code.m, np.uint8)
            inS[[int(pair[j]) for j in order]] = 1
            _check_lower_triangular(code, hascut, inS, pair, order)
            assert calls >= p


def test_mts_inc_closed_forms(orc):
    """Slack columns heavier than every standard column: M is the slack set (A_M = I). One
    check: M is its heaviest column."""
    code = regular_code(96)
    rng = np.random.Generator(np.random.PCG64(63))
    hascut = (rng.random(code.m) < 0.7).astype(np.uint8)
    w = np.concatenate([rng.random(code.n), 2.0 + rng.random(code.m)]).astype(np.float32)
    pair, order, _ = orc.mts_inc(code, hascut, w)
    assert all(pair[j] == code.n + j for j in np.nonzero(hascut)[0])
    one = np.zeros(code.m, np.uint8)
    one[5] = 1
    w = rng.random(code.n + code.m).astype(np.float32)
    pair, order, _ = orc.mts_inc(code, one, w)
    cand = list(code.row(5)) + [code.n + 5]
    assert pair[5] == max(cand, key=lambda c: (np.float32(w[c]), -c))


# ---------------------------------------------------------------- ALP decoding (Algorithm 1)
@pytest.mark.parametrize("snr", [1.0, 1.5, 2.5])
def test_alp_equals_lp_decoding_and_malp(orc, snr):
    """Theorem 2c for ALP: its last LP solution is the LP-decoding optimum, the same as MALP-A's
    and HiGHS' over every odd-set inequality. Theorem 1: an iteration adds at most one cut per
    check (the new cuts of each LP have distinct checks). Theorem 2b: costs increase. Every cut
    kept is satisfied at the output."""
    code = regular_code(96)
    n_frac = 0
    for gamma in _frames(code, [snr], 8, 131):
        a = orc.alp_decode(code, gamma)
        r = orc.decode(code, gamma)
        fun, _ = refs.feldman_lp(code, gamma)
        scale = 1.0 + abs(fun - gamma[gamma < 0].sum())
        assert a.status == 0 and a.flag == r.flag
        assert abs(a.objective - fun) <= 1e-6 * scale and abs(a.objective - r.objective) <= 1e-6 * scale
        assert np.array_equal(a.xhat, r.xhat)
        assert a.malp_iters <= code.n
        assert np.all(np.diff(a.trace_obj) > 0)
        bounds = np.concatenate([[0], a.trace_p])
        for k in range(a.malp_iters):
            new = a.cuts[bounds[k]:bounds[k + 1], 0]
            assert 1 <= len(new) <= code.m and np.all(np.diff(new) > 0)
        for j, V in a.cuts:
            arow, b = refs.cut_row_u(code, int(j), int(V))
            assert arow @ a.u <= b + 1e-6
        n_frac += a.flag == 0
    if snr == 1.0:
        assert n_frac >= 2


def test_alp_keeps_every_cut_and_solves_larger_lps(orc):
    """ALP never removes a cut, so its LPs grow monotonically, and its largest LP is at least
    as large as MALP-A's last one on the same frame (MALP keeps one cut per check)."""
    code = regular_code(240)
    for gamma in _frames(code, [1.5, 2.0], 6, 132):
        a = orc.alp_decode(code, gamma)
        r = orc.decode(code, gamma)
        if a.malp_iters == 0:
            assert r.malp_iters == 0
            continue
        assert np.all(np.diff(a.trace_p) > 0)
        assert a.p_max == a.trace_p[-1] >= r.p_final
        assert len({(int(j), int(V)) for j, V in a.cuts}) == len(a.cuts)
