"""Random LDPC parity-check matrices (Tanner graphs), seeded and reproducible.

Construction: Gallager-style random edge permutation (configuration model). Variable
sockets and check sockets are laid out by degree, the check sockets are shuffled, and
edges that form a double edge or a cycle of length four are repaired by swapping their
check endpoint with a randomly chosen edge until none is left. The paper's codes are
random (3,6)-regular with 4-cycles removed (Sec. III-D, Sec. VI-B).

The matrix is returned in CSR form (rows = checks, columns = variables), 0-based,
column indices sorted and unique within a row.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

CODE_SEED_BASE = 0x09020657


@dataclass(frozen=True)
class Code:
    m: int
    n: int
    rowptr: np.ndarray  # int32 [m+1]
    col: np.ndarray     # int32 [E]
    name: str = ""

    @property
    def E(self) -> int:
        return int(self.col.shape[0])

    def dense(self) -> np.ndarray:
        H = np.zeros((self.m, self.n), dtype=np.uint8)
        for j in range(self.m):
            H[j, self.col[self.rowptr[j]:self.rowptr[j + 1]]] = 1
        return H

    def row(self, j: int) -> np.ndarray:
        return self.col[self.rowptr[j]:self.rowptr[j + 1]]

    def check_degrees(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def var_degrees(self) -> np.ndarray:
        return np.bincount(self.col, minlength=self.n)


def from_dense(H: np.ndarray, name: str = "") -> Code:
    H = np.asarray(H) != 0
    m, n = H.shape
    rowptr = np.zeros(m + 1, dtype=np.int32)
    cols = []
    for j in range(m):
        c = np.nonzero(H[j])[0]
        cols.append(c)
        rowptr[j + 1] = rowptr[j] + len(c)
    col = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    return Code(m, n, rowptr, col, name)


def _bad_edges(vs: np.ndarray, cs: np.ndarray, m: int, n: int, no4: bool = True) -> np.ndarray:
    """Indices of edges that sit on a double edge or (no4=True) close a cycle of length four."""
    E = vs.shape[0]
    key = cs.astype(np.int64) * n + vs
    order = np.argsort(key, kind="stable")
    ks = key[order]
    bad = np.zeros(E, dtype=bool)
    same = ks[1:] == ks[:-1]
    bad[order[1:][same]] = True
    if not no4:
        return np.nonzero(bad)[0]
    H = sp.csr_matrix((np.ones(E, dtype=np.int32), (cs, vs)), shape=(m, n))
    H.sum_duplicates()
    H.data[:] = 1
    S = (H @ H.T).tocoo()
    mask = (S.row < S.col) & (S.data >= 2)
    for a, b in zip(S.row[mask].tolist(), S.col[mask].tolist()):
        ra = H.indices[H.indptr[a]:H.indptr[a + 1]]
        rb = H.indices[H.indptr[b]:H.indptr[b + 1]]
        common = np.intersect1d(ra, rb)
        # checks a and b share len(common) >= 2 variables; moving all but one of
        # the edges on check a breaks every 4-cycle through this pair
        for v in common[1:].tolist():
            pos = np.searchsorted(ks, a * n + v)
            while pos < E and ks[pos] == a * n + v:
                bad[order[pos]] = True
                pos += 1
    return np.nonzero(bad)[0]


def configuration_code(var_deg: np.ndarray, chk_deg: np.ndarray, seed: int,
                       name: str = "", max_rounds: int = 2000, no4: bool = True) -> Code:
    var_deg = np.asarray(var_deg, dtype=np.int64)
    chk_deg = np.asarray(chk_deg, dtype=np.int64)
    n, m = var_deg.shape[0], chk_deg.shape[0]
    assert var_deg.sum() == chk_deg.sum(), "socket counts differ"
    rng = np.random.Generator(np.random.PCG64(seed))
    vs = np.repeat(np.arange(n, dtype=np.int64), var_deg)
    cs = np.repeat(np.arange(m, dtype=np.int64), chk_deg)
    rng.shuffle(cs)
    E = vs.shape[0]
    for _ in range(max_rounds):
        bad = _bad_edges(vs, cs, m, n, no4)
        if bad.size == 0:
            break
        partners = rng.integers(0, E, size=bad.size)
        for e, f in zip(bad.tolist(), partners.tolist()):
            cs[e], cs[f] = cs[f], cs[e]
    else:
        raise RuntimeError(f"could not remove 4-cycles from {name}")
    order = np.lexsort((vs, cs))
    cs_s, vs_s = cs[order], vs[order]
    rowptr = np.zeros(m + 1, dtype=np.int32)
    np.add.at(rowptr, cs_s + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return Code(m, n, rowptr, vs_s.astype(np.int32), name)


def code_seed(n: int, family: int) -> int:
    return CODE_SEED_BASE ^ (n << 8) ^ family


def regular_code(n: int, dv: int = 3, dc: int = 6, seed: int | None = None,
                 no4: bool = True) -> Code:
    """(dv,dc)-regular code with n variables and n*dv/dc checks; no 4-cycles unless no4=False
    (tiny codes used for brute-force checks cannot avoid them)."""
    assert (n * dv) % dc == 0
    m = n * dv // dc
    if seed is None:
        seed = code_seed(n, dv * 16 + dc)
    return configuration_code(np.full(n, dv), np.full(m, dc), seed, f"reg{dv}{dc}_n{n}", no4=no4)


def irregular_code(n: int = 8192, seed: int | None = None, no4: bool = True) -> Code:
    """Rate-1/2 irregular code: edge fractions lambda_2=.25, lambda_3=.45, lambda_8=.30,
    checks of degree 6 and 7 with the edge count split to match."""
    lam = {2: 0.25, 3: 0.45, 8: 0.30}
    inv = sum(f / d for d, f in lam.items())
    frac = {d: (f / d) / inv for d, f in lam.items()}          # node fractions
    n2 = int(round(frac[2] * n))
    n8 = int(round(frac[8] * n))
    n3 = n - n2 - n8
    var_deg = np.concatenate([np.full(n2, 2), np.full(n3, 3), np.full(n8, 8)])
    E = int(var_deg.sum())
    m = n // 2
    # m checks of degree 6 or 7 with total degree E: a*6 + (m-a)*7 = E
    a = 7 * m - E
    assert 0 <= a <= m, (E, m)
    chk_deg = np.concatenate([np.full(a, 6), np.full(m - a, 7)])
    if seed is None:
        seed = code_seed(n, 0x1B)
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5A5A))
    rng.shuffle(var_deg)
    rng.shuffle(chk_deg)
    return configuration_code(var_deg, chk_deg, seed, f"irr_n{n}", no4=no4)


def code_for_config(n: int, irregular: bool = False) -> Code:
    return irregular_code(n) if irregular else regular_code(n)
