"""Independent reference computations used to pin the oracle (and, through it, the GPU).

Nothing here calls the oracle or the GPU library: these are brute-force searches, the full
LP-decoding relaxation handed to SciPy's HiGHS solver, and graph checks written from the
definitions in the paper (parity inequalities, stopping sets, peeling).
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linprog


def odd_subsets(d: int):
    for r in range(1, d + 1, 2):
        for V in itertools.combinations(range(d), r):
            yield V


def cut_row_u(code, j: int, vmask: int) -> tuple[np.ndarray, float]:
    """Parity inequality of check j with odd set V (bit k = k-th neighbour) in the form
    a^T u <= b of eq. (constraints): sum_V u_i - sum_{N(j)\\V} u_i <= |V| - 1."""
    N = code.row(j)
    a = np.zeros(code.n)
    a[N] = -1.0
    vsz = 0
    for k, i in enumerate(N):
        if (vmask >> k) & 1:
            a[i] = 1.0
            vsz += 1
    return a, float(vsz - 1)


def feldman_lp(code, gamma):
    """LP decoding over the fundamental polytope with every parity inequality (eq. LP
    decoding): returns (objective, u)."""
    rows, rhs = [], []
    for j in range(code.m):
        N = code.row(j)
        for V in odd_subsets(len(N)):
            a = np.zeros(code.n)
            a[N] = -1.0
            a[N[list(V)]] = 1.0
            rows.append(a)
            rhs.append(len(V) - 1.0)
    res = linprog(gamma, A_ub=np.array(rows), b_ub=np.array(rhs), bounds=[(0.0, 1.0)] * code.n,
                  method="highs", options={"primal_feasibility_tolerance": 1e-10,
                                           "dual_feasibility_tolerance": 1e-10})
    assert res.status == 0, res.message
    return float(res.fun), res.x


def cutset_lp(code, gamma, masks):
    """The LP of one adaptive iteration in the standard form of Sec. III-A: the given cuts
    plus one box constraint per variable (u_i >= 0 if gamma_i >= 0, else u_i <= 1)."""
    rows, rhs = [], []
    for j in range(code.m):
        if masks[j]:
            a, b = cut_row_u(code, j, int(masks[j]))
            rows.append(a)
            rhs.append(b)
    bounds = [(0.0, None) if g >= 0 else (None, 1.0) for g in gamma]
    res = linprog(gamma, A_ub=np.array(rows) if rows else None, b_ub=np.array(rhs) if rows else None,
                  bounds=bounds, method="highs",
                  options={"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10})
    assert res.status == 0, res.message
    return float(res.fun), res.x


def gf2_nullspace(H: np.ndarray) -> np.ndarray:
    """Basis (rows) of the null space of H over GF(2)."""
    H = (np.asarray(H) % 2).astype(np.uint8).copy()
    m, n = H.shape
    piv_cols = []
    r = 0
    for c in range(n):
        piv = [i for i in range(r, m) if H[i, c]]
        if not piv:
            continue
        H[[r, piv[0]]] = H[[piv[0], r]]
        for i in range(m):
            if i != r and H[i, c]:
                H[i] ^= H[r]
        piv_cols.append(c)
        r += 1
        if r == m:
            break
    free = [c for c in range(n) if c not in piv_cols]
    basis = []
    for f in free:
        v = np.zeros(n, dtype=np.uint8)
        v[f] = 1
        for row, pc in enumerate(piv_cols):
            if H[row, f]:
                v[pc] = 1
        basis.append(v)
    return np.array(basis, dtype=np.uint8).reshape(len(basis), n)


def all_codewords(H: np.ndarray) -> np.ndarray:
    B = gf2_nullspace(H)
    k = B.shape[0]
    assert k <= 22, "too many codewords for brute force"
    idx = np.arange(1 << k, dtype=np.int64)
    bits = ((idx[:, None] >> np.arange(k)) & 1).astype(np.uint8)
    return (bits @ B) % 2


def ml_decode(H: np.ndarray, gamma: np.ndarray):
    """Brute-force ML decoding (eq. ML decoding): argmin gamma^T u over all codewords."""
    cw = all_codewords(H)
    cost = cw.astype(np.float64) @ gamma
    k = int(np.argmin(cost))
    return cw[k], float(cost[k]), cw, cost


def peel(code, erased: np.ndarray) -> bool:
    """Peeling (BEC message passing) on the erased set: True iff every erasure is resolved,
    i.e. the set contains no stopping set (Sec. II-A)."""
    E = set(int(i) for i in np.nonzero(erased)[0])
    rows = [set(int(i) for i in code.row(j)) for j in range(code.m)]
    changed = True
    while E and changed:
        changed = False
        for R in rows:
            left = R & E
            if len(left) == 1:
                E -= left
                changed = True
    return not E


def has_stopping_set(code, S: np.ndarray) -> bool:
    """Brute force: does some nonempty subset of S form a stopping set (no check with exactly
    one neighbour in the subset)?"""
    idx = [int(i) for i in np.nonzero(S)[0]]
    rows = [set(int(i) for i in code.row(j)) for j in range(code.m)]
    for r in range(1, len(idx) + 1):
        for sub in itertools.combinations(idx, r):
            s = set(sub)
            if all(len(R & s) != 1 for R in rows):
                return True
    return False


def max_parity_violation(code, u):
    """Largest violation max(0, 1 - LHS) over every odd-set parity inequality of every check
    (brute force over the odd subsets), i.e. how far u is outside the fundamental polytope."""
    worst = 0.0
    u = np.asarray(u, dtype=np.float64)
    by_deg = {}
    for j in range(code.m):
        by_deg.setdefault(len(code.row(j)), []).append(j)
    for d, js in by_deg.items():
        U = np.array([u[code.row(j)] for j in js])            # [checks, d]
        for V in odd_subsets(d):
            mask = np.zeros(d, dtype=bool)
            mask[list(V)] = True
            lhs = (1.0 - U[:, mask]).sum(axis=1) + U[:, ~mask].sum(axis=1)
            worst = max(worst, float(np.max(1.0 - lhs)))
    return max(worst, 0.0)
