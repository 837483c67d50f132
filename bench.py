"""Benchmark: LP-decoded frames/s of the batched decoder on the (3,6)-regular n=1024 code.

One step = one launch of the decoder over a batch of 512 frames (Eb/N0 1.5 / 2.0 / 2.5 dB,
171/171/170 frames, FP32 LLRs, FP64 PCG vectors (--precision fp32: FP32 vectors) with FP64
refinement and FP64 interior-point iterations): every step of the hot path (cut search, cut
update, interior-point iterations, triangular-set search, PCG) runs inside that launch, and
the steps run one after another. Inputs are resident in device memory before timing starts.
Newton systems that PCG does not finish within its cap go to a dense FP64 Cholesky (the
library's default); the method alone is the method_only leg.

Prints one JSON line. Beside the main number:
  roofline        HBM bandwidth of the launch on the method's algorithmic bytes, with the
                  PCG-only figure and the dense fallback's share
  main            flags, parity of all 512 frames against the stored oracle results,
                  per-frame decode times, decode statistics
  method_only     the same batch without the dense fallback (FP64 PCG, cap 2000)
  other_precision the same batch with the other PCG vector precision
  overlapped      successive launches of the batch on three streams (one context each), so
                  that a launch's last frames overlap the next launch's: sustained frames/s
  serving         Poisson arrivals of mixed-length frames through lpdec_server (persistent
                  engines, then the wave scheduler as serving_waves)
  plain_fp64      frames through lpdec_decode (FP64, one frame per launch, host pointers)
  cpu_baseline    the FP64 CPU oracle on the host cores, a time-bounded sample
  config_c3/c4    one launch of the n=4096 / irregular n=8192 workloads, with their rooflines
                  and a time-bounded oracle sample (--no-configs leaves them out)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# HIP's hardware queues per process (read when HIP starts; HIP's default is 4): the server's 8
# streams need a queue each, or their waves serialize behind each other, plus one for the
# other work of this process
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 12:
    os.environ["GPU_MAX_HW_QUEUES"] = "12"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6     # dense FP64 matrix-core peak of the chip
GOLDEN = os.path.join(ROOT, "tests", "golden")
GOLDEN_FILES = {"c2": "c2_n1024.json", "c3": "c3_n4096.json", "c4": "c4_irr8192.json"}
METRIC = "LP-decoded frames/s at n=1024 (3,6) + p50/p99 latency, vs plain FP64 GPU"


def workload(name="c2"):
    from synth.workloads import WORKLOADS
    return WORKLOADS[name]()


def pcg_bytes(st, n, elem):
    """Bytes one PCG iteration must move, summed over the frames: (6e + 3) p + e q with e the
    vector element size (27p + 4q for FP32 vectors: read h, d^2, the row map and the lists,
    write l, update x, r and z; 16-bit indices), q = n + p."""
    rows = st["pcg_rows"].astype(np.float64)
    its = st["pcg_iters"].astype(np.float64)
    return float(np.sum((6 * elem + 3) * rows + elem * (its * n + rows)))


def ipm_bytes(st):
    """FP64 vector passes of the interior-point iterations: 120 q bytes each."""
    return float(np.sum(120 * st["ipm_cols"].astype(np.float64)))


def dense_flops(st):
    """Flops of the dense-fallback Cholesky factorizations: P^3 / 3 per solve (P padded)."""
    return float(st["dense_cube"].astype(np.float64).sum() / 3.0)


def rooflines(st, n, elem, kern_s, ncu, traffic=None, traffic_note=None):
    """The launch's HBM roofline on the method's algorithmic bytes (PCG + IPM vector passes),
    the PCG-only figure, and the dense fallback's flops beside them."""
    pb, ib = pcg_bytes(st, n, elem), ipm_bytes(st)
    alg = pb + ib
    achieved = alg / kern_s / 1e9
    pcg_s = float(st["ticks_pcg"].sum()) / 1e8          # device clock: 100 MHz
    per_frame = pb / pcg_s / 1e9 if pcg_s > 0 else 0.0
    its = int(st["pcg_iters"].sum())
    flops = dense_flops(st)
    return {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": (traffic / 1e9 / kern_s) if traffic is not None else None,
        "traffic_bytes_per_launch": traffic, "traffic_note": traffic_note,
        "algorithmic_bytes_per_launch": alg, "pcg_bytes_per_launch": pb, "ipm_bytes_per_launch": ib,
        "basis": f"per PCG iteration (6e+3)p + eq bytes, e = {elem} (vector element size), q = n + p; "
                 "per IPM iteration 120q bytes; divided by the launch time (HIP events on its stream)",
        "kernel_ms": kern_s * 1e3,
        "pcg_only": {
            "iterations": its, "us_per_iteration": pcg_s * 1e6 / max(1, its),
            "frame_seconds_in_pcg": pcg_s,
            "per_frame_GBps": per_frame,
            "all_cus_GBps": per_frame * ncu, "all_cus_frac": per_frame * ncu / HBM_PEAK_GBS,
            "note": "PCG bytes over the frames' device time inside PCG iterations; all_cus = that "
                    "rate on every compute unit at once (one frame per compute unit)"},
        "dense_fallback": {"bound": "mfma", "achieved": flops / kern_s / 1e12, "peak": FP64_PEAK_TFS,
                           "unit": "TFLOP/s", "frac": flops / kern_s / 1e12 / FP64_PEAK_TFS,
                           "flops_per_launch": flops,
                           "basis": "Cholesky P^3/3 flops per dense-fallback solve (P = LP rows padded to 32), "
                                    "FP64 matrix cores; work outside the method, reported for its share"},
    }


def decode_stats(st, nf):
    tot = max(1, int(st["ticks_total"].sum()))
    newton = int(st["ipm_iters"].sum())
    return {"mean_malp_iters": float(st["malp_iters"].mean()), "max_malp_iters": int(st["malp_iters"].max()),
            "lps_solved": int(st["malp_iters"].sum()),
            "mean_ipm_iters": float(st["ipm_iters"].mean()),
            "mean_pcg_iters": float(st["pcg_iters"].mean()),
            "mean_pcg_per_newton": float(st["pcg_iters"].sum() / max(1, newton)),
            "max_p": int(st["p_max"].max()), "mean_p_max": float(st["p_max"].mean()),
            "max_levels": int(st["max_levels"].max()),
            "pcg_us_per_iteration": float(st["ticks_pcg"].sum() / 100.0 / max(1, st["pcg_iters"].sum())),
            "mts_us_per_ipm_iteration": float(st["ticks_mts"].sum() / 100.0 / max(1, newton)),
            "ref_rounds": int(st["ref_rounds"].sum()), "escalations": int(st["escalations"].sum()),
            "newton_solves": newton, "dense_fallback_solves": int(st["direct_solves"].sum()),
            "newton_solved_by_pcg": 1.0 - float(st["direct_solves"].sum() / max(1, newton)),
            "device_time_share": {"pcg": float(st["ticks_pcg"].sum()) / tot,
                                  "dense_fallback": float(st["ticks_dense"].sum()) / tot,
                                  "mts": float(st["ticks_mts"].sum()) / tot}}


def golden_parity(name, code, G, flags, xhat, objs):
    """Frames of a launch against the stored oracle results (tests/golden, written by an
    oracle-only script): decoded word and flag bit-exact, objective within 1e-6 relative to
    1 + c^T x."""
    path = os.path.join(GOLDEN, GOLDEN_FILES[name])
    if not os.path.exists(path):
        return None
    gold = json.load(open(path))["frames"]
    bad = []
    for k, rec in gold.items():
        f = int(k)
        want = np.unpackbits(np.frombuffer(bytes.fromhex(rec["xhat_hex"]), np.uint8))[:code.n]
        g = G[f].astype(np.float64)
        scale = 1.0 + abs(rec["objective"] - float(g[g < 0].sum()))
        if not (flags[f] == rec["flag"] and np.array_equal(xhat[f], want)
                and abs(objs[f] - rec["objective"]) <= 1e-6 * scale):
            bad.append(f)
    return {"frames": len(gold), "mismatches": len(bad), "mismatched_frames": bad[:20],
            "source": f"tests/golden/{GOLDEN_FILES[name]} (oracle results)"}


_WL = {}


def _oracle_worker(args):
    name, f = args
    import oracle
    if name not in _WL:
        _WL[name] = workload(name)
    code, G = _WL[name]
    t = time.perf_counter()
    r = oracle.decode(code, G[f].astype(np.float64))
    return time.perf_counter() - t, r.xhat, r.flag, r.objective


def host_cores():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    lscpu = None
    try:
        import subprocess
        out = subprocess.run(["lscpu", "-p=CPU"], capture_output=True, text=True, timeout=10).stdout
        lscpu = sum(1 for line in out.splitlines() if line and not line.startswith("#"))
    except Exception:
        pass
    return avail, lscpu


def cpu_baseline(name, frames, budget_s=20.0, max_workers=16):
    """The FP64 CPU oracle on the host cores: one frame per worker process, frames taken in the
    given order until the time budget is used up (the frames in flight then finish). Workers:
    the cores this process may run on, at most max_workers (the host CPU share of one GPU)."""
    from concurrent.futures import ProcessPoolExecutor, FIRST_COMPLETED, wait
    import oracle
    oracle.build(force=False)
    avail, lscpu = host_cores()
    workers = max(1, min(avail, max_workers))
    done, t0 = [], time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        pending, nxt = {}, 0
        while nxt < len(frames) and len(pending) < workers:
            pending[ex.submit(_oracle_worker, (name, frames[nxt]))] = frames[nxt]
            nxt += 1
        while pending:
            fin, _ = wait(list(pending), return_when=FIRST_COMPLETED)
            for f in fin:
                k = pending.pop(f)
                done.append((k, f.result()))
                if nxt < len(frames) and time.perf_counter() - t0 < budget_s:
                    pending[ex.submit(_oracle_worker, (name, frames[nxt]))] = frames[nxt]
                    nxt += 1
    wall = time.perf_counter() - t0
    return {"value": len(done) / wall, "unit": "frames/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(done)} frames of the {name} batch taken in turn from its Eb/N0 groups, "
                      f"{workers} worker processes, {wall:.1f} s wall",
            "single_thread_s_per_frame": float(np.mean([d[1][0] for d in done])),
            "host_cores": {"sched_getaffinity": avail, "lscpu": lscpu, "used": workers}}, done


def cpu_sample_cutoff(name, frames, budget_s=75.0, max_workers=16):
    """The oracle on the host cores for the large workloads, whose frames take minutes each: one
    frame per worker process in index order, and every frame still running when the time
    budget ends is abandoned (the workers are terminated). Rate = frames finished / budget."""
    import multiprocessing as mp
    import oracle
    oracle.build(force=False)
    avail, lscpu = host_cores()
    workers = max(1, min(avail, max_workers))
    ctxp = mp.get_context("fork")
    t0 = time.perf_counter()
    done = []
    pool = ctxp.Pool(workers)
    try:
        it = pool.imap_unordered(_oracle_worker, [(name, f) for f in frames])
        while True:
            left = budget_s - (time.perf_counter() - t0)
            if left <= 0:
                break
            try:
                done.append(it.next(timeout=left))
            except mp.TimeoutError:
                break
            except StopIteration:
                break
    finally:
        pool.terminate()
        pool.join()
    wall = min(time.perf_counter() - t0, budget_s) if len(done) < len(frames) else time.perf_counter() - t0
    return {"value": len(done) / wall, "unit": "frames/s", "cores": workers, "kind": "oracle",
            "sample": f"{name} frames in index order, one per worker process, {workers} workers; "
                      f"{len(done)} finished within {wall:.0f} s, the rest abandoned at the cutoff",
            "single_thread_s_per_frame": float(np.mean([d[0] for d in done])) if done else None,
            "host_cores": {"sched_getaffinity": avail, "lscpu": lscpu, "used": workers}}


def interleaved_c2(k):
    """k frames of the n=1024 batch taken in turn from its three Eb/N0 groups."""
    from synth.workloads import C2_SPLIT
    starts = np.concatenate([[0], np.cumsum(C2_SPLIT)[:-1]])
    out = []
    for r in range(max(C2_SPLIT)):
        for g0, sz in zip(starts, C2_SPLIT):
            if r < sz:
                out.append(int(g0 + r))
    return out[:k]


def plain_fp64(ctx, C, G, frames, budget_s=30.0):
    """lpdec_decode (FP64, one frame per launch) on frames taken in turn from the three Eb/N0
    groups, until the list or the time budget is used up."""
    t0 = time.perf_counter()
    res = []
    for f in frames:
        xh, flag, obj, st, _ = ctx.decode(C, G[f].astype(np.float64))
        res.append((f, xh, flag, obj))
        if time.perf_counter() - t0 > budget_s:
            break
    wall = time.perf_counter() - t0
    return {"value": len(res) / wall, "unit": "frames/s", "frames": len(res),
            "sample": f"{len(res)} frames taken in turn from the 1.5/2.0/2.5 dB groups, lpdec_decode "
                      f"(one frame per launch, host pointers, FP64 PCG, the library's default options), {wall:.1f} s"}, res


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _collect(srv, tickets, label, every_s=20.0):
    """Polls every ticket until all have a result (the server hands results out as frames
    finish), printing progress while frames are outstanding. Returns {ticket: result}."""
    done, last = {}, time.perf_counter()
    while len(done) < len(tickets):
        for t, n, _, _ in tickets:
            if t not in done:
                r = srv.poll(t, n)
                if r is not None:
                    done[t] = r
        if len(done) < len(tickets):
            if time.perf_counter() - last > every_s:
                log(f"{label}: {len(done)} of {len(tickets)} requests done")
                last = time.perf_counter()
            time.sleep(0.005)
    return done


def _poisson(srv, Cs, codes, rng, qps, seconds, stream_id):
    """Poisson arrivals at qps for `seconds`, then drain. Latency = submit to result."""
    from synth.channel import awgn_llr, frame_seed
    t0 = time.perf_counter()
    tickets, t_next, k = [], t0, 0
    while time.perf_counter() - t0 < seconds:
        now = time.perf_counter()
        while t_next <= now:
            ci = int(rng.integers(0, len(codes)))
            e = float(rng.uniform(1.5, 3.0))
            g = awgn_llr(codes[ci].n, e, 0.5, frame_seed(stream_id, ci, k))
            tickets.append((srv.submit(Cs[ci], g), codes[ci].n, e, (stream_id, ci, k)))
            k += 1
            t_next += rng.exponential(1.0 / qps)
        time.sleep(max(0.0, min(t_next - time.perf_counter(), 0.002)))
    res = _collect(srv, tickets, f"poisson {qps:.1f} qps")
    wall = time.perf_counter() - t0
    lat, per, fails = [], {}, []
    for t, n, e, seed in tickets:
        r = res[t]
        lat.append(r[3])
        per.setdefault(n, []).append(r[3])
        if r[1] < 0:
            # enough to rebuild the frame: awgn_llr(n, ebn0, 0.5, frame_seed(*seed))
            fails.append({"n": n, "flag": int(r[1]), "ebn0_db": e, "frame_seed": list(seed)})
    lat = np.array(lat)
    return {"offered_qps": qps, "arrival_s": seconds, "requests": len(lat), "frames_per_s": len(lat) / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "per_code_p50_ms": {str(n): float(np.percentile(v, 50) * 1e3) for n, v in sorted(per.items())},
            "per_code_p99_ms": {str(n): float(np.percentile(v, 99) * 1e3) for n, v in sorted(per.items())},
            "numerical_failures": len(fails), "failure_flags": fails}


def serving(ctx, seconds=8.0, qps=40.0, seed=5, full=False, streams=None, mode=1, burst=384):
    """Frames from a mix of codes, Eb/N0 uniform in [1.5, 3.0] dB, through lpdec_server
    (mode 0: continuous batching over the context's SERVER_STREAMS streams; mode 1: a
    persistent kernel per code that takes each request as a workgroup frees). First the saturated
    throughput of the mix (a burst submitted at once, then drained); then Poisson arrivals
    at a fixed qps and at 0.5x and 0.8x the saturated throughput. Default mix: (3,6) n=256
    and n=1024; full: also (3,6) n=4096 and the irregular n=8192 code (their fractional
    frames take seconds to tens of seconds each)."""
    from paper_0902_0657_amd import Code
    from synth.channel import awgn_llr, frame_seed
    from synth.codes import irregular_code, regular_code
    codes = [regular_code(256), regular_code(1024)]
    if full:
        codes += [regular_code(4096), irregular_code(8192)]
    Cs = [Code.from_synth(ctx, c) for c in codes]
    rng = np.random.Generator(np.random.PCG64(seed))
    if streams:
        ctx.set_option("SERVER_STREAMS", streams)
    prev = ctx.get_option("SERVER_MODE")
    ctx.set_option("SERVER_MODE", mode)
    # the large codes' engines hold a dense-fallback matrix per workgroup (34 MB at n=4096,
    # 134 MB at n=8192): the full mix gets a larger share of the 288 GB
    srv = ctx.server(hbm_budget_bytes=(64 << 30) if full else (8 << 30), max_slots=2048)
    ctx.set_option("SERVER_MODE", prev)
    try:
        t0 = time.perf_counter()
        tk = []
        for k in range(burst):
            ci = int(rng.integers(0, len(codes)))
            e = float(rng.uniform(1.5, 3.0))
            g = awgn_llr(codes[ci].n, e, 0.5, frame_seed(78, ci, k))
            tk.append((srv.submit(Cs[ci], g), codes[ci].n, e, (78, ci, k)))
        res_b = _collect(srv, tk, f"burst of {burst}")
        sat = burst / (time.perf_counter() - t0)
        burst_fails = []
        burst_lat = {}
        for t, n, e, seed in tk:
            r = res_b[t]
            burst_lat.setdefault(n, []).append(r[3])
            if r[1] < 0:
                burst_fails.append({"n": n, "flag": int(r[1]), "ebn0_db": e, "frame_seed": list(seed)})
        log(f"serving mode {mode}: burst of {burst} at {sat:.0f} frames/s")
        res = _poisson(srv, Cs, codes, rng, qps, seconds, 77) if qps > 0 else {}
        if qps > 0:
            log(f"serving mode {mode}: {qps:.0f} qps p50 {res['p50_ms']:.1f} ms p99 {res['p99_ms']:.1f} ms")
        res.update({"burst_latency_max_s": {str(n): float(max(v)) for n, v in sorted(burst_lat.items())},
                    "mode": "persistent" if mode else "waves", "codes": [c.name for c in codes],
                    "streams": int(ctx.get_option("SERVER_STREAMS")) if mode == 0 else len(codes),
                    "saturated_frames_per_s": sat, "burst": burst, "burst_failure_flags": burst_fails,
                    "at_fraction_of_saturated": [dict(fraction=f, **_poisson(srv, Cs, codes, rng, f * sat, seconds,
                                                                               79 + int(10 * f)))
                                                 for f in (0.5, 0.8)]})
    finally:
        srv.close()
    return res


def precond_study(seed=606):
    """The comparison of Sec. VI-B on a synthetic (3,6) n=2000 code: Newton systems of the IPM
    at its 8th and 18th iteration, in the 6th LP of an MALP-A decode, once for a frame decoded
    integral at 1.5 dB and once for a fractional one at 1.0 dB. For each preconditioner the
    relative residual ||w - Q y||^2 / ||w||^2 of FP64 PCG after k iterations (one round, no
    refinement). The systems come from the library itself: the cut set from the decode trace,
    the IPM point from lpdec_ipm_batch stopped after 7 and 17 iterations; w is assembled here
    from that point by the formulas of Sec. IV-B."""
    import torch
    from paper_0902_0657_amd import Code, Context
    from synth.channel import batch_awgn
    from synth.codes import regular_code
    dev = torch.device("cuda:0")
    code = regular_code(2000)
    n, m = code.n, code.m
    H = code.dense().astype(np.float64)
    ctx = Context(0)
    ctx.set_option("PRECISION", 1)
    C = Code.from_synth(ctx, code)
    names = {4: "CG (no preconditioner)", 0: "slack columns (diagonal)", 1: "Algorithm 7 (column-wise)",
             2: "Algorithm 8 (row-wise, diagonal expansion)", 3: "Algorithm 8 (row-wise, triangular expansion)",
             5: "Algorithm 6 (incremental)"}
    steps = (5, 10, 20, 40, 80, 120, 160, 200)
    systems = []
    for label, snr, want in (("integral, 1.5 dB", 1.5, 1), ("fractional, 1.0 dB", 1.0, 0)):
        G = batch_awgn(n, 0.5, snr, 64, stream=seed + int(10 * snr))
        g = torch.as_tensor(G, device=dev)
        tr = ctx.decode_batch_trace(C, g, trace_cap=8)
        torch.cuda.synchronize()
        flag = tr["flag"].cpu().numpy()
        malp = tr["stats"].cpu().numpy()[:, 0]
        cand = [f for f in range(G.shape[0]) if flag[f] == want and malp[f] >= 6]
        if not cand:
            continue
        f = min(cand, key=lambda k: (abs(int(malp[k]) - 6), k))
        vm = tr["trace"].cpu().numpy()[f, 5].astype(np.uint32)
        gam = G[f].astype(np.float64)
        sg = np.where(gam >= 0, 1.0, -1.0)
        rows = np.nonzero(vm)[0]
        p = len(rows)
        # the augmented LP of Sec. IV-B: A = [A_std | I_p], b, c = (|gamma|, 0)
        A = np.zeros((p, n + p))
        b = np.zeros(p)
        for r, j in enumerate(rows):
            cols = np.nonzero(H[j])[0]
            sv = np.array([1.0 if (int(vm[j]) >> k) & 1 else -1.0 for k in range(len(cols))])
            A[r, cols] = sg[cols] * sv
            A[r, n + r] = 1.0
            b[r] = (sv > 0).sum() - 1 - sv[sg[cols] < 0].sum()
        c = np.concatenate([np.abs(gam), np.zeros(p)])
        for it in (8, 18):
            ctx.set_option("IPM_MAX", it - 1)
            vmd = torch.as_tensor(vm[None, :].view(np.int32).copy(), device=dev)
            x, y, z, its, status = ctx.ipm_batch(C, vmd, torch.as_tensor(gam[None, :], device=dev), precision=1)
            ctx.set_option("IPM_MAX", 100)
            x, y, z = x.cpu().numpy()[0], y.cpu().numpy()[0], z.cpu().numpy()[0]
            idx = np.concatenate([np.arange(n), n + rows])
            xa, za, ya = x[idx], z[idx], y[rows]
            d2 = xa / za
            mu = 0.1 * float(xa @ za) / (n + p)
            rb = b - A @ xa
            rc = c - A.T @ ya - za
            re = mu - xa * za
            w = rb + A @ (d2 * rc) - A @ (re / za)
            Q = (A * d2) @ A.T
            ev = np.linalg.eigvalsh(Q)
            d2full = np.zeros(n + m)
            d2full[:n] = d2[:n]
            d2full[n + rows] = d2[n:]
            wfull = np.zeros(m)
            wfull[rows] = w
            sysrec = {"system": label, "frame": int(f), "malp_iterations": int(malp[f]), "ipm_iteration": it,
                      "rows": p, "columns": n + p, "duality_gap": float(xa @ za), "kappa": float(ev[-1] / ev[0]),
                      "residual2": {}}
            for pc in (4, 0, 1, 2, 3, 5):
                ctx.set_option("PRECOND", pc)
                ctx.set_option("REF_MAX", 0)
                ctx.set_option("PCG_TOL", 1e-30)
                curve = []
                for k in steps:
                    ctx.set_option("PCG_MAXIT", k)
                    _, itn, res = ctx.newton_solve_batch(
                        C, vmd, torch.as_tensor(gam[None, :], device=dev), torch.as_tensor(d2full[None, :], device=dev),
                        torch.as_tensor(wfull[None, :], device=dev), precision=1)
                    curve.append([k, float(res.cpu().numpy()[0]) ** 2])
                sysrec["residual2"][names[pc]] = curve
            for key, v in (("PRECOND", 1), ("REF_MAX", 3), ("PCG_TOL", 1e-6), ("PCG_MAXIT", 0)):
                ctx.set_option(key, v)
            systems.append(sysrec)
            log(f"precond study: {label}, IPM iteration {it}, p = {p}")
    ctx.close()
    return {"precond_study": {"code": "(3,6)-regular n=2000, 4-cycle free", "lp": "6th MALP-A iteration",
                              "metric": "||w - Q y||^2 / ||w||^2 after k FP64 PCG iterations", "systems": systems}}


PRECOND_NAMES = {1: "Algorithm 7 (column-wise)", 2: "Algorithm 8 (row-wise, diagonal expansion)",
                 3: "Algorithm 8 (row-wise, triangular expansion)", 5: "Algorithm 6 (incremental)",
                 0: "slack columns (diagonal)", 4: "CG (no preconditioner)"}


def precond_compare(dev, stream, name="c2", preconds=(1, 2, 3, 5, 0, 4), method_only=False, only=None):
    """One launch of a whole workload per preconditioner: the share of Newton systems that PCG
    solves within the automatic cap (the rest go to the dense fallback), PCG iterations per
    PCG-solved system, search cost and launch time; with method_only, no dense fallback (FP64
    PCG, cap 2000) and the PCG iterations per system. Parity against the stored oracle
    results in every row."""
    import torch
    from paper_0902_0657_amd import Code, Context, stats_table
    code, G = workload(name)
    g = torch.as_tensor(G, device=dev)
    rows = []
    for pc in (only or preconds):
        opts = {"PRECOND": pc, "PRECISION": 1}
        if method_only:
            opts.update({"DIRECT_FALLBACK": 0, "PCG_MAXIT": 2000})
        ctx = Context(0, **opts)
        C = Code.from_synth(ctx, code)
        out, ms, _ = run_leg(ctx, C, g, G.shape[0], dev, stream, 1, 0, f"precond {pc}")
        st = stats_table(out["stats"])
        flags, xhat, objs = out["flag"].cpu().numpy(), out["xhat"].cpu().numpy(), out["obj"].cpu().numpy()
        newton = int(st["ipm_iters"].sum())
        dense = int(st["direct_solves"].sum())
        rows.append({"precond": pc, "name": PRECOND_NAMES[pc], "launch_ms": float(ms.mean()),
                     "newton_systems": newton, "solved_by_pcg": 1.0 - dense / max(1, newton),
                     "pcg_iterations": int(st["pcg_iters"].sum()),
                     "pcg_per_newton": float(st["pcg_iters"].sum()) / max(1, newton),
                     "search_us_per_ipm_iteration": float(st["ticks_mts"].sum()) / 100.0 / max(1, newton),
                     "pcg_us_per_iteration": float(st["ticks_pcg"].sum()) / 100.0 / max(1, int(st["pcg_iters"].sum())),
                     "parity_vs_oracle": golden_parity(name, code, G, flags, xhat, objs)})
        log(f"precond {pc}: {ms.mean():.0f} ms, {rows[-1]['solved_by_pcg']:.3f} by PCG")
        ctx.close()
    return {"workload": name, "method_only": method_only, "rows": rows}


def alp_study(dev, stream, name="c2"):
    """Sec. III-D on a whole workload: LPs solved and the size of the largest LP for ALP
    (Algorithm 1), MALP-A and MALP-B, split by integral and fractional output (mean and the
    95% one-sided upper bound), and the size of MALP's largest LP relative to ALP's."""
    import torch
    from paper_0902_0657_amd import Code, Context, stats_table
    code, G = workload(name)
    g = torch.as_tensor(G, device=dev)
    res = {}
    for label, mode in (("MALP-A", 0), ("MALP-B", 1)):
        ctx = Context(0, MALP_MODE=mode)
        C = Code.from_synth(ctx, code)
        out, ms, _ = run_leg(ctx, C, g, G.shape[0], dev, stream, 1, 0, label)
        st = stats_table(out["stats"])
        res[label] = {"flags": out["flag"].cpu().numpy(), "lps": st["malp_iters"], "p": st["p_max"],
                      "ms": float(ms.mean())}
        ctx.close()
    ctx = Context(0)
    C = Code.from_synth(ctx, code)
    t0 = time.perf_counter()
    out = ctx.alp_decode_batch(C, G.astype(np.float64))
    st = stats_table(out["stats"])
    res["ALP"] = {"flags": out["flag"], "lps": st["malp_iters"], "p": st["p_max"],
                  "ms": (time.perf_counter() - t0) * 1e3}
    gold = json.load(open(os.path.join(GOLDEN, GOLDEN_FILES[name])))["frames"]
    integral = np.array([gold[str(f)]["flag"] == 1 for f in range(G.shape[0])])
    summary = {}
    for label, r in res.items():
        rec = {"ms": r["ms"], "flags": {str(k): int(v) for k, v in zip(*np.unique(r["flags"], return_counts=True))},
               "matches_oracle_flags": int(sum(int(r["flags"][f]) == gold[str(f)]["flag"] for f in range(G.shape[0])))}
        for part, sel in (("integral", integral), ("fractional", ~integral)):
            lps, p = r["lps"][sel].astype(float), r["p"][sel].astype(float)
            rec[part] = {"frames": int(sel.sum()), "lps_mean": float(lps.mean()), "lps_p95": float(np.percentile(lps, 95)),
                         "largest_lp_mean": float(p.mean())}
        summary[label] = rec
    for label in ("MALP-A", "MALP-B"):
        for part, sel in (("integral", integral), ("fractional", ~integral)):
            summary[label][part]["largest_lp_vs_alp"] = float(
                np.mean(res[label]["p"][sel].astype(float) / np.maximum(1, res["ALP"]["p"][sel])))
    ctx.close()
    return {"workload": name, "study": "Sec. III-D", "modes": summary}


def sources_digest():
    """SHA-256 over the HIP sources and the C header: identifies the kernel build that a
    stored traffic measurement belongs to."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0902_0657_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".hpp", ".cpp")))
    for f in files + [os.path.join(ROOT, "include", "lpdec.h")]:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()


PROFILE_TAGS = {"c2": "n1024", "c3": "n4096", "c4": "irr8192"}


def traffic_file(name="c2"):
    return os.path.join(ROOT, "profiles", f"lpdec_main_{PROFILE_TAGS[name]}_traffic.md")


def stored_traffic(name="c2"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, when it was taken on
    the current sources (else None). The summary holds one JSON line starting with
    '{"traffic"'."""
    TRAFFIC_FILE = traffic_file(name)
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter summary"
    with open(TRAFFIC_FILE) as fh:
        rec = [json.loads(line) for line in fh if line.startswith('{"traffic"')]
    if not rec:
        return None, "no counter summary"
    t = rec[-1]["traffic"]
    if t.get("sources_sha256") != sources_digest():
        return None, "kernel changed since the counters were taken"
    fetch = t["fetch_kib_per_launch"] * 1024.0 * t["fetch_scale"]
    write = t["write_kib_per_launch"] * 1024.0 * t["write_scale"]
    return fetch + write, "FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factors"


PROFILE_COMMANDS = {
    "c2": "python bench.py --steps 1 --warmup 0 --no-cpu --no-plain --no-legs --no-serve --no-configs --block 256",
    "c3": "python bench.py --only-configs --configs c3 --no-cpu",
    "c4": "python bench.py --only-configs --configs c4 --no-cpu",
}
PROFILE_TITLES = {"c2": "n=1024 (3,6) batch of 512 frames", "c3": "n=4096 (3,6) batch of 256 frames",
                  "c4": "irregular n=8192 batch of 128 frames (BSC)"}


def summarize_profiles(name, base):
    """Writes profiles/lpdec_main_<tag>_kernel_stats.md and _traffic.md from the rocprofv3 CSV
    output of the three runs of PROFILE_COMMANDS[name] (kernel trace, FETCH_SIZE, WRITE_SIZE)
    under base/prof_<name>_{kt,fetch,write}/, and the benchmark line the kernel-trace run
    printed (base/prof_<name>_kt.out)."""
    import csv
    tag, cmd, title = PROFILE_TAGS[name], PROFILE_COMMANDS[name], PROFILE_TITLES[name]
    stats = list(csv.DictReader(open(os.path.join(base, f"prof_{name}_kt", "run_kernel_stats.csv"))))
    line = [ln for ln in open(os.path.join(base, f"prof_{name}_kt.out")) if ln.startswith("{")][-1]
    bench = json.loads(line)
    if name == "c2":
        leg, roof = bench["main"], bench["roofline"]
    else:
        leg = bench[f"config_{name}"]
        roof = leg["roofline"]
    out = [f"# lpdec_main, {title}: rocprofv3 kernel statistics", "",
           "Command (from the repository root, on an MI355X):", "",
           f"    rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/prof_{name}_kt -o run -- {cmd}", "",
           "| kernel | calls | total ns | average ns | min ns | max ns | share % |", "|---|---|---|---|---|---|---|"]
    for r in stats:
        out.append(f"| `{r['Name']}` | {r['Calls']} | {r['TotalDurationNs']} | {float(r['AverageNs']):.0f} | "
                   f"{r['MinNs']} | {r['MaxNs']} | {float(r['Percentage']):.2f} |")
    out += ["", f"bench.py in the same run: kernel time from HIP events {roof['kernel_ms']:.1f} ms, "
                f"{leg['value']:.2f} frames/s; algorithmic bytes {roof['algorithmic_bytes_per_launch']:.4g} "
                f"(PCG {roof['pcg_bytes_per_launch']:.4g}, IPM {roof['ipm_bytes_per_launch']:.4g}); "
                f"PCG {roof['pcg_only']['us_per_iteration']:.1f} us per iteration; Newton systems solved by PCG "
                f"{leg['decode_stats']['newton_solved_by_pcg']:.3f}; parity with the stored oracle frames: "
                f"{leg['parity_vs_oracle']['mismatches']} of {leg['parity_vs_oracle']['frames']} differ.", ""]
    open(os.path.join(ROOT, "profiles", f"lpdec_main_{tag}_kernel_stats.md"), "w").write("\n".join(out))
    kib = {}
    for cnt in ("fetch", "write"):
        rows = list(csv.DictReader(open(os.path.join(base, f"prof_{name}_{cnt}", "run_counter_collection.csv"))))
        main = [r for r in rows if r["Kernel_Name"].startswith("void lpdec::lpdec_main")]
        copy = [r for r in rows if r["Kernel_Name"] == "__amd_rocclr_copyBuffer"]
        kib[cnt] = (float(main[-1]["Counter_Value"]), max(float(r["Counter_Value"]) for r in copy))
    copy_bytes = 256 << 20
    fs = copy_bytes / 1024.0 / kib["fetch"][1]
    ws = copy_bytes / 1024.0 / kib["write"][1]
    hbm = kib["fetch"][0] * 1024 * fs + kib["write"][0] * 1024 * ws
    alg = roof["algorithmic_bytes_per_launch"]
    rec = {"traffic": {"sources_sha256": sources_digest(), "fetch_kib_per_launch": kib["fetch"][0],
                       "write_kib_per_launch": kib["write"][0], "fetch_scale": fs, "write_scale": ws,
                       "copy_fetch_kib": kib["fetch"][1], "copy_write_kib": kib["write"][1], "copy_bytes": copy_bytes}}
    out = [f"# lpdec_main, {title}: HBM traffic counters", "", "Two counter runs (from the repository root, on an MI355X):", "",
           f"    rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/prof_{name}_fetch -o run -- {cmd} --calib-copy",
           f"    rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/prof_{name}_write -o run -- {cmd} --calib-copy", "",
           "`--calib-copy` runs one 256 MiB device-to-device copy first; the counters of that copy",
           "kernel give the scale factors (bytes moved / counter reading).", "",
           "| counter | decode launch (KiB) | 256 MiB copy (KiB) | scale |", "|---|---|---|---|",
           f"| FETCH_SIZE | {kib['fetch'][0]:.0f} | {kib['fetch'][1]:.0f} | {fs:.4f} |",
           f"| WRITE_SIZE | {kib['write'][0]:.0f} | {kib['write'][1]:.0f} | {ws:.4f} |", "",
           f"HBM bytes per decode launch: {hbm:.4g}; algorithmic bytes {alg:.4g}; counters / algorithmic = "
           f"{hbm / alg:.3f}; {hbm / (roof['kernel_ms'] / 1e3) / 1e9:.0f} GB/s over the launch.", "",
           "Machine-readable (bench.py uses it while the sources hash matches):", "", json.dumps(rec), ""]
    open(os.path.join(ROOT, "profiles", f"lpdec_main_{tag}_traffic.md"), "w").write("\n".join(out))
    print(f"{name}: counters {hbm:.4g} B, algorithmic {alg:.4g} B, ratio {hbm / alg:.3f}")


def copy_calibration(dev, nbytes=256 << 20):
    """One plain device-to-device copy of known size, for scaling the HBM counters."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {nbytes} bytes read and written")


def run_leg(ctx, C, g, nf, dev, stream, steps=1, warmup=0, label=""):
    """Times `steps` launches of the batch with HIP events on the launch stream."""
    import torch
    out = ctx.batch_outputs(C, nf, dev)
    for w in range(warmup):
        ctx.decode_batch(C, g, out=out, stream=stream)
        torch.cuda.synchronize()
        log(f"{label} warmup {w + 1} done")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        ctx.decode_batch(C, g, out=out, stream=stream)
        ev[k + 1].record(stream)
        ev[k + 1].synchronize()
        log(f"{label} step {k + 1}: {ev[k].elapsed_time(ev[k + 1]):.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    return out, step_ms, wall


def overlapped_leg(code, G, dev, opts, ncu, ref, streams=3, launches=6):
    """Launches of the same 512-frame batch issued in turn on `streams` streams, each with its
    own context (workspace, outputs): a launch ends with its slowest frame, and meanwhile the
    compute units its finished workgroups free take the next launch's frames. Reports the
    sustained rate (launches x frames / wall time), each launch's duration (HIP events on its
    stream) and whether every output equals the single-launch result."""
    import torch
    from paper_0902_0657_amd import Code, Context, stats_table
    g = torch.as_tensor(G, device=dev)
    nf = G.shape[0]
    ctxs = [Context(0, **opts) for _ in range(streams)]
    Cs = [Code.from_synth(c, code) for c in ctxs]
    sts = [torch.cuda.Stream(dev) for _ in range(streams)]
    outs = [ctxs[i].batch_outputs(Cs[i], nf, dev) for i in range(streams)]
    for i in range(streams):
        ctxs[i].decode_batch(Cs[i], g, out=outs[i], stream=sts[i])
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(launches)]
    t0 = time.perf_counter()
    for k in range(launches):
        i = k % streams
        ev[k][0].record(sts[i])
        ctxs[i].decode_batch(Cs[i], g, out=outs[i], stream=sts[i])
        ev[k][1].record(sts[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    same = all(np.array_equal(outs[i][key].cpu().numpy(), ref[key]) for i in range(streams) for key in ref)
    busy = sum(float(stats_table(outs[i]["stats"])["ticks_total"].sum()) / 1e8 for i in range(streams))
    for c in ctxs:
        c.close()
    log(f"overlapped: {launches} launches on {streams} streams in {wall:.2f} s")
    return {"value": launches * nf / wall, "unit": "frames/s", "streams": streams, "launches": launches,
            "frames_per_launch": nf, "wall_s": wall, "options": opts,
            "launch_ms": {"p50": float(np.percentile(lat, 50)), "max": float(lat.max()),
                          "note": "each launch from its start on its stream to its end (HIP events)"},
            "cu_busy_fraction": busy / len(ctxs) * launches / (wall * ncu),
            "same_results_as_single_launch": bool(same)}


def leg_summary(name, ctx_opts, code, G, out, step_ms, ncu, elem, traffic=None, traffic_note=None):
    from paper_0902_0657_amd import stats_table
    st = stats_table(out["stats"])
    flags, xhat, objs = out["flag"].cpu().numpy(), out["xhat"].cpu().numpy(), out["obj"].cpu().numpy()
    nf = G.shape[0]
    kern_s = float(step_ms.mean()) / 1e3
    frame_ms = st["ticks_total"].astype(np.float64) / 1e5   # 100 MHz device clock
    busy = float(frame_ms.sum()) / 1e3
    return {
        "value": nf / kern_s, "unit": "frames/s", "ms_per_step": float(step_ms.mean()), "options": ctx_opts,
        "flags": {str(k): int(v) for k, v in zip(*np.unique(flags, return_counts=True))},
        "parity_vs_oracle": golden_parity(name, code, G, flags, xhat, objs),
        "frame_decode_ms": {"p50": float(np.percentile(frame_ms, 50)), "p99": float(np.percentile(frame_ms, 99)),
                            "max": float(frame_ms.max()), "note": "in-kernel decode time of each frame (device clock)"},
        "cu_busy_fraction": busy / (kern_s * ncu),
        "decode_stats": decode_stats(st, nf),
        "roofline": rooflines(st, code.n, elem, kern_s, ncu, traffic, traffic_note),
    }, st, flags, xhat, objs


def config_leg(name, dev, stream, opts, label, cpu=True):
    """One launch of a whole workload (c3: n=4096, 256 frames; c4: irregular n=8192, 128
    frames) with its roofline, parity on the stored oracle frames and decode statistics."""
    import torch
    from paper_0902_0657_amd import Code, Context
    code, G = workload(name)
    ctx = Context(0, **opts)
    C = Code.from_synth(ctx, code)
    g = torch.as_tensor(G, device=dev)
    out, step_ms, _ = run_leg(ctx, C, g, G.shape[0], dev, stream, 1, 0, f"{name} {label}")
    elem = 8 if int(ctx.get_option("PRECISION")) != 0 else 4
    traffic, note = stored_traffic(name)
    res, *_ = leg_summary(name, opts, code, G, out, step_ms, ctx_ncu(), elem, traffic, note)
    ctx.close()
    if cpu:
        res["cpu_baseline"] = cpu_sample_cutoff(name, list(range(G.shape[0])))
        log(f"{name} cpu sample: {res['cpu_baseline']['sample']}")
    return res


def ctx_ncu():
    import torch
    return int(torch.cuda.get_device_properties(0).multi_processor_count)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp64",
                    help="PCG vector precision of the main leg (fp64, the library's default: with FP32 "
                         "vectors PCG finishes far fewer of the late Newton systems within the cap; "
                         "the FP32 form is the other_precision leg)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the method-only and other-precision legs")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving legs")
    ap.add_argument("--serve-full", action="store_true",
                    help="serving mix over n = 256, 1024, 4096 and the irregular 8192 code")
    ap.add_argument("--configs", default="c3,c4",
                    help="comma list of extra whole-workload launches (c3, c4)")
    ap.add_argument("--no-configs", action="store_true", help="leave out the c3 / c4 launches")
    ap.add_argument("--summarize-profiles", default="",
                    help="DIR: write the profiles/ summaries from rocprofv3 output under DIR (no GPU)")
    ap.add_argument("--only-configs", action="store_true",
                    help="run only the --configs launches (for profiling them alone); prints their legs")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 256 MiB copy first (HBM counter calibration under rocprofv3)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--precond-study", action="store_true",
                    help="print the preconditioner comparison of Sec. VI-B (n=2000 code) instead of the benchmark")
    ap.add_argument("--precond-compare", default="",
                    help="print the preconditioners' Newton-system shares on a whole workload (c2 or c3) instead "
                         "of the benchmark; with --method-only, without the dense fallback")
    ap.add_argument("--method-only", action="store_true")
    ap.add_argument("--preconds", default="", help="comma list of PRECOND values for --precond-compare")
    ap.add_argument("--alp-study", action="store_true",
                    help="print ALP / MALP-A / MALP-B LP counts and sizes on the n=1024 batch (Sec. III-D)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (one GPU's share of the batch); "
                                   "frames are independent LPs and would shard by frame index with no "
                                   "exchange: run with --gpus 1"}))
        sys.exit(2)

    if args.precond_study:
        print(json.dumps(precond_study()))
        return
    if args.summarize_profiles:
        for name in ("c2", "c3", "c4"):
            if os.path.exists(os.path.join(args.summarize_profiles, f"prof_{name}_kt")):
                summarize_profiles(name, args.summarize_profiles)
        return
    if args.only_configs:
        import torch
        dev = torch.device("cuda:0")
        stream = torch.cuda.current_stream(dev)
        if args.calib_copy:
            copy_calibration(dev)
        opts = {"PRECISION": 1 if args.precision == "fp64" else 0}
        print(json.dumps({f"config_{c}": config_leg(c, dev, stream, opts, "main", cpu=not args.no_cpu)
                          for c in args.configs.split(",") if c}))
        return
    if args.precond_compare or args.alp_study:
        import torch
        dev = torch.device("cuda:0")
        stream = torch.cuda.current_stream(dev)
        if args.precond_compare:
            only = [int(x) for x in args.preconds.split(",")] if args.preconds else None
            print(json.dumps(precond_compare(dev, stream, args.precond_compare, method_only=args.method_only,
                                             only=only)))
        if args.alp_study:
            print(json.dumps(alp_study(dev, stream)))
        return
    import torch
    from paper_0902_0657_amd import Code, Context, _lib
    if not os.path.exists(_lib.LIB_PATH):
        raise SystemExit(f"{_lib.LIB_PATH} is missing: run `python -c 'import __graft_entry__ as g; g.build()'`")
    code, G = workload("c2")
    dev = torch.device("cuda:0")
    ncu = ctx_ncu()
    if args.calib_copy:
        copy_calibration(dev)
    fp64 = args.precision == "fp64"
    main_opts = {"PRECISION": 1 if fp64 else 0}
    if args.block:
        main_opts["BLOCK"] = args.block
    ctx = Context(0, **main_opts)
    C = Code.from_synth(ctx, code)
    g = torch.as_tensor(G, device=dev)
    stream = torch.cuda.current_stream(dev)
    nf = G.shape[0]
    tune = None
    c2_opts = dict(main_opts)
    if not args.block:
        # threads per frame picked by the launch-shape tuner on 128 frames of the batch
        from paper_0902_0657_amd import autotune
        tune = autotune.tune_block(ctx, C, g[interleaved_c2(128)].contiguous())
        c2_opts["BLOCK"] = int(tune["block"])
        log(f"autotune: BLOCK {tune['block']} ({', '.join(f'{b}: {t:.0f} ms' for b, t in tune['ms'].items())})")
    out, step_ms, wall = run_leg(ctx, C, g, nf, dev, stream, args.steps, args.warmup, "main")
    traffic, traffic_note = stored_traffic()
    main_res, st, flags, xhat, objs = leg_summary("c2", c2_opts, code, G, out, step_ms, ncu, 8 if fp64 else 4,
                                                  traffic, traffic_note)
    if tune is not None:
        main_res["autotune"] = {"block": int(tune["block"]), "ms_on_128_frames": {str(b): float(t) for b, t in tune["ms"].items()}}
    value = main_res["value"]
    roof = main_res.pop("roofline")
    roof["kernel"] = f"lpdec_main<{'double' if fp64 else 'float'}, LDS, DECODE>"
    res = {
        "metric": METRIC,
        "value": value, "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": float(step_ms.mean()), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if fp64 else "f32 PCG / f64 IPM", "data": "synthetic",
        "config": {"workload": "(3,6)-regular LDPC n=1024 m=512, AWGN Eb/N0 1.5/2.0/2.5 dB "
                               "(171/171/170 frames), FP32 LLRs, 512 frames per launch, MALP-A; Newton systems "
                               "by " + ("FP64" if fp64 else "FP32") + " PCG (Algorithm 4, Algorithm 7 "
                               "preconditioner) with FP64 refinement; a system PCG does not finish within "
                               "max(300, p^2/3500) iterations, and the rest of its LP's systems, go to a dense "
                               "FP64 Cholesky on the matrix cores (share in main.decode_stats."
                               "newton_solved_by_pcg; the method alone in method_only)",
                   "global_batch": nf, "parallelism": "one workgroup per frame"},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "note": "batch mode: a frame's result is available when its launch ends"},
        "wall_s_timed": wall,
        "roofline": roof,
        "main": main_res,
    }
    # serving first among the extra legs, while the process holds no other device work
    if not args.no_serve:
        if args.serve_full:
            # the irregular n=8192 code's fractional frames take about 2 minutes each over AWGN
            # (hundreds of dense solves at p up to 4096): a burst of 64 gives the saturated rate,
            # then 20 s of arrivals at each fraction of it, each drained
            res["serving"] = serving(ctx, mode=1, full=True, seconds=20.0, qps=0.0, burst=64)
        else:
            res["serving"] = serving(ctx, mode=1)
            res["serving_waves"] = serving(ctx, mode=0)
        log("serving done")
    if not args.no_legs:
        # the method alone: no dense fallback, FP64 PCG with a fixed cap of 2000 iterations
        legs = [("method_only", {"DIRECT_FALLBACK": 0, "PCG_MAXIT": 2000, "PRECISION": 1}),
                ("other_precision", {"PRECISION": 0 if fp64 else 1})]
        for lname, opts in legs:
            c2x = Context(0, **opts)
            Cx = Code.from_synth(c2x, code)
            ox, msx, _ = run_leg(c2x, Cx, g, nf, dev, stream, 1, 0, lname)
            res[lname], *_ = leg_summary("c2", opts, code, G, ox, msx, ncu, 8 if opts["PRECISION"] == 1 else 4)
            log(f"{lname}: {msx.mean():.1f} ms")
            c2x.close()
    if not args.no_legs:
        ref = {"flag": flags, "xhat": xhat, "obj": objs}
        res["overlapped"] = overlapped_leg(code, G, dev, c2_opts, ncu, ref)
    for name in [c for c in args.configs.split(",") if c and not args.no_configs]:
        res[f"config_{name}"] = config_leg(name, dev, stream, main_opts, "main", cpu=not args.no_cpu)
        log(f"config {name}: {res[f'config_{name}']['ms_per_step']:.0f} ms")
    if not args.no_plain:
        frames = interleaved_c2(24)
        pf, plain_res = plain_fp64(ctx, C, G, frames)
        log(f"plain FP64: {pf['frames']} frames")
        res["plain_fp64"] = pf
        res["speedup_vs_plain"] = value / pf["value"]
        res["plain_fp64"]["mismatch_vs_batch"] = len([f for f, xh, fl, ob in plain_res
                                                      if not (np.array_equal(xh, xhat[f]) and fl == flags[f])])
    if not args.no_cpu:
        cb, done = cpu_baseline("c2", interleaved_c2(nf))
        log(f"cpu baseline: {len(done)} frames")
        res["cpu_baseline"] = cb
        mism = [k for k, (t, xh, fl, ob) in done
                if not (np.array_equal(xh, xhat[k]) and fl == flags[k]
                        and abs(ob - objs[k]) <= 1e-6 * (1.0 + abs(ob - float(G[k][G[k] < 0].sum()))))]
        res["cpu_baseline"]["mismatches_vs_main"] = len(mism)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
