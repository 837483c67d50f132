"""Writes hamming743.json: a parity-check matrix of the (7,4,3) Hamming code for which the
pseudocodeword f = [1, 1/2, 0, 1/2, 0, 0, 1/2] (printed in the remark after Corollary 5,
Sec. III-B, which takes it from Feldman et al.) is a vertex of the fundamental polytope,
and a cost vector gamma that makes f the unique LP-decoding optimum.

Only numpy is used: the polytope is written out from the parity inequalities (eq.
constraints) and the box constraints; f is a vertex when the constraints tight at f have
rank 7; gamma = -sum(w_k a_k) over the tight constraints a_k^T u <= b_k with weights
w_k in [1, 2] lies inside the normal cone of the vertex, so f is the unique minimiser.
"""
import itertools
import json
import os

import numpy as np

F = np.array([1, 0.5, 0, 0.5, 0, 0, 0.5])
BASE = np.array([[int(b) for b in format(c, "03b")] for c in range(1, 8)]).T  # 3 x 7


def constraints(H):
    A, b = [], []
    for j in range(H.shape[0]):
        N = np.nonzero(H[j])[0]
        for r in range(1, len(N) + 1, 2):
            for V in itertools.combinations(N, r):
                a = np.zeros(H.shape[1])
                a[N] = -1.0
                a[list(V)] = 1.0
                A.append(a)
                b.append(len(V) - 1.0)
    for i in range(H.shape[1]):
        e = np.zeros(H.shape[1]); e[i] = -1.0; A.append(e); b.append(0.0)
        e = np.zeros(H.shape[1]); e[i] = 1.0; A.append(e); b.append(1.0)
    return np.array(A), np.array(b)


def main():
    rng = np.random.Generator(np.random.PCG64(743))
    for perm in itertools.permutations(range(7)):
        H = BASE[:, list(perm)]
        A, b = constraints(H)
        slack = b - A @ F
        if slack.min() < -1e-12:
            continue
        tight = np.abs(slack) < 1e-12
        if np.linalg.matrix_rank(A[tight]) != 7:
            continue
        w = rng.uniform(1.0, 2.0, size=int(tight.sum()))
        gamma = -(w @ A[tight])
        out = {
            "citation": "Sec. III-B, remark after Corollary 5: pseudocodeword [1,1/2,0,1/2,0,0,1/2] "
                        "of the (7,4,3) code with m = 3 fractional entries",
            "H": H.tolist(),
            "pseudocodeword": F.tolist(),
            "gamma": gamma.tolist(),
        }
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hamming743.json")
        with open(path, "w") as fh:
            json.dump(out, fh, indent=1)
        print("wrote", path, "perm", perm)
        return
    raise SystemExit("no column order makes f a vertex")


if __name__ == "__main__":
    main()
