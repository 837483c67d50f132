"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds no arithmetic of the decoding method: it only builds parity-check
matrices (Tanner graphs) and channel log-likelihood ratios, the inputs the paper's
experiments draw at random (random 4-cycle-free (3,6)-regular codes over AWGN, Sec. III-D
and Sec. VI-B).
"""
from .codes import Code, regular_code, irregular_code, code_for_config  # noqa: F401
from .channel import awgn_llr, bsc_llr, frame_seed, splitmix64, uniform_snr_awgn  # noqa: F401
