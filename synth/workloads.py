"""The benchmark workloads as seeded input batches (codes and channel LLRs only).

    c2: (3,6)-regular n=1024, AWGN at Eb/N0 1.5 / 2.0 / 2.5 dB (171 / 171 / 170 frames),
        512 frames, LLRs rounded to FP32 once
    c3: (3,6)-regular n=4096, AWGN at 1.75 dB, 256 frames
    c4: irregular rate-1/2 n=8192 (variable degrees 2/3/8, checks of degree 6-7), BSC with
        crossover 0.04 plus the small continuous perturbation, 128 frames
    c1: (3,6)-regular n=96, AWGN at 2.0 dB, 200 frames (FP64)
"""
from __future__ import annotations

import numpy as np

from .channel import batch_awgn, batch_bsc
from .codes import irregular_code, regular_code

C2_SNRS, C2_SPLIT, C2_STREAM = (1.5, 2.0, 2.5), (171, 171, 170), 2024


def c1():
    code = regular_code(96)
    return code, batch_awgn(code.n, 0.5, 2.0, 200, stream=1)


def c2():
    code = regular_code(1024)
    G = np.concatenate([batch_awgn(code.n, 0.5, s, k, stream=C2_STREAM, snr_index=i)
                        for i, (s, k) in enumerate(zip(C2_SNRS, C2_SPLIT))]).astype(np.float32)
    return code, G


def c2_group(f: int) -> int:
    """Eb/N0 group (0, 1, 2) of frame f of the c2 batch."""
    return int(np.searchsorted(np.cumsum(C2_SPLIT), f, side="right"))


def c3():
    code = regular_code(4096)
    return code, batch_awgn(code.n, 0.5, 1.75, 256, stream=3)


def c4():
    code = irregular_code(8192)
    return code, batch_bsc(code.n, 0.04, 128, stream=4)


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4}
