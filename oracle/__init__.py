"""FP64 CPU oracle for adaptive LP decoding -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may import this
package. The GPU library in paper_0902_0657_amd/ shares no code with it and never calls it.
"""
from .oracle import (OracleOpts, alp_decode, build, decode, find_cut, ipm, lp_dense, mts, mts_levels,  # noqa: F401
                     mts_levels_any, mts_row, mts_inc, triangulate,
                     newton, normal_solve, pcg)
