"""Seeded channel outputs as log-likelihood ratios gamma_i = log Pr(r_i|0)/Pr(r_i|1)
(the LLR definition of Sec. II-B).

The all-zero codeword is sent. AWGN: BPSK maps bit 0 to +1, y = 1 + sigma*N(0,1),
sigma^2 = 1/(2 R 10^(EbN0/10)), gamma = 2y/sigma^2. BSC with crossover p:
gamma = +-log((1-p)/p), plus a tiny seeded Gaussian perturbation of relative size 1e-3 so
that every LP has a unique optimum (Sec. III-B asks for a small continuous noise on
channels such as the BSC).

Every frame has its own seed, a SplitMix64 hash of (stream id, Eb/N0 index, frame index).
"""
from __future__ import annotations

import math

import numpy as np

_MASK = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One SplitMix64 output for state x (Steele, Lea, Flood 2014)."""
    x = (x + 0x9E3779B97F4A7C15) & _MASK
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def frame_seed(stream: int, snr_index: int, frame: int) -> int:
    return splitmix64(splitmix64(splitmix64(stream) ^ snr_index) ^ frame)


def awgn_sigma2(ebn0_db: float, rate: float) -> float:
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def awgn_llr(n: int, ebn0_db: float, rate: float, seed: int) -> np.ndarray:
    s2 = awgn_sigma2(ebn0_db, rate)
    rng = np.random.Generator(np.random.PCG64(seed))
    y = 1.0 + math.sqrt(s2) * rng.standard_normal(n)
    return 2.0 * y / s2


def bsc_llr(n: int, p: float, seed: int, perturb: float = 1e-3) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    L = math.log((1.0 - p) / p)
    flips = rng.random(n) < p
    g = np.where(flips, -L, L)
    return g + perturb * np.abs(g) * rng.standard_normal(n)


def batch_awgn(n: int, rate: float, ebn0_db: float, nframes: int, stream: int,
               snr_index: int = 0, first_frame: int = 0) -> np.ndarray:
    return np.stack([awgn_llr(n, ebn0_db, rate, frame_seed(stream, snr_index, f))
                     for f in range(first_frame, first_frame + nframes)])


def batch_bsc(n: int, p: float, nframes: int, stream: int, first_frame: int = 0) -> np.ndarray:
    return np.stack([bsc_llr(n, p, frame_seed(stream, 0, f))
                     for f in range(first_frame, first_frame + nframes)])


def uniform_snr_awgn(n: int, lo: float, hi: float, stream: int, frame: int,
                     rate: float = 0.5) -> tuple[float, np.ndarray]:
    """One frame at an Eb/N0 drawn uniformly from [lo, hi] dB: returns (Eb/N0, gamma).
    The Eb/N0 comes from its own seed (SNR index 1), the noise from SNR index 0."""
    u = np.random.Generator(np.random.PCG64(frame_seed(stream, 1, frame))).random()
    e = lo + (hi - lo) * float(u)
    return e, awgn_llr(n, e, rate, frame_seed(stream, 0, frame))
