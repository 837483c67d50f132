"""Benchmark: LP-decoded frames/s of the batched decoder on the (3,6)-regular n=1024 code.

One step = one launch of the decoder over a batch of 512 frames (Eb/N0 1.5 / 2.0 / 2.5 dB,
171/171/170 frames, FP32 LLRs, FP64 PCG with the dense FP64 fallback): every step of the hot path
(cut search, cut update, interior-point iterations, triangular-set search, PCG) runs inside
that launch. Inputs are resident in device memory before timing starts.

Prints one JSON line. Extra legs, each reported beside the main number:
  plain_fp64   the same frames through lpdec_decode (FP64, one frame per launch, host
               pointers), a bounded sample;
  cpu_baseline the FP64 CPU oracle on the host cores, a time-bounded sample;
  roofline     effective bandwidth of the decode kernel on its algorithmic bytes;
  serving      Poisson arrivals of mixed-length frames through lpdec_server (persistent
               engines, then the wave scheduler as serving_waves).
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

N, SNRS, SPLIT = 1024, (1.5, 2.0, 2.5), (171, 171, 170)
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6     # dense FP64 matrix-core peak of the chip


def workload():
    from synth.channel import batch_awgn
    from synth.codes import regular_code
    code = regular_code(N)
    G = np.concatenate([batch_awgn(code.n, 0.5, s, k, stream=2024, snr_index=i)
                        for i, (s, k) in enumerate(zip(SNRS, SPLIT))]).astype(np.float32)
    return code, G


def algorithmic_bytes(st, n):
    """Bytes the method must move per frame: per PCG iteration 27p + 4q
    (q = n + p, FP32 vectors), per interior-point iteration 120q (FP64 vector passes)."""
    pcg_rows = st["pcg_rows"].astype(np.float64)
    pcg_its = st["pcg_iters"].astype(np.float64)
    ipm_cols = st["ipm_cols"].astype(np.float64)
    return float(np.sum(27 * pcg_rows + 4 * (pcg_its * n + pcg_rows) + 120 * ipm_cols))


def dense_flops(st):
    """Flops of the dense-fallback Cholesky factorizations: P^3 / 3 per solve (P padded)."""
    return float(st["dense_cube"].astype(np.float64).sum() / 3.0)


def _oracle_worker(args):
    code_spec, gamma = args
    import oracle
    from synth.codes import regular_code
    code = regular_code(code_spec)
    t = time.perf_counter()
    r = oracle.decode(code, gamma)
    return time.perf_counter() - t, r.xhat, r.flag, r.objective


def cpu_baseline(G, budget_s=12.0):
    from concurrent.futures import ProcessPoolExecutor, FIRST_COMPLETED, wait
    import oracle
    oracle.build(force=False)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(avail, 16))
    done, t0 = [], time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        pending, nxt = {}, 0
        while nxt < G.shape[0] and len(pending) < workers:
            pending[ex.submit(_oracle_worker, (N, G[nxt].astype(np.float64)))] = nxt
            nxt += 1
        while pending:
            fin, _ = wait(list(pending), return_when=FIRST_COMPLETED)
            for f in fin:
                k = pending.pop(f)
                done.append((k, f.result()))
                if nxt < G.shape[0] and time.perf_counter() - t0 < budget_s:
                    pending[ex.submit(_oracle_worker, (N, G[nxt].astype(np.float64)))] = nxt
                    nxt += 1
    wall = time.perf_counter() - t0
    return {"value": len(done) / wall, "unit": "frames/s", "cores": workers, "kind": "oracle",
            "sample": f"first {len(done)} frames of the benchmark batch (n=1024, 1.5/2.0/2.5 dB), "
                      f"{workers} worker processes, {wall:.1f} s wall",
            "single_thread_s_per_frame": float(np.mean([d[1][0] for d in done]))}, done


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
                      f"(FP64 PCG, one frame per launch), {wall:.1f} s"}, res


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _poisson(srv, Cs, codes, rng, qps, seconds, stream_id):
    """Poisson arrivals at qps for `seconds`, then drain. Latency = submit to result."""
    from synth.channel import awgn_llr, frame_seed
    t0 = time.perf_counter()
    tickets, t_next, k = [], t0, 0
    while time.perf_counter() - t0 < seconds:
        now = time.perf_counter()
        while t_next <= now:
            ci = int(rng.integers(0, len(codes)))
            g = awgn_llr(codes[ci].n, float(rng.uniform(1.5, 3.0)), 0.5, frame_seed(stream_id, ci, k))
            tickets.append((srv.submit(Cs[ci], g), codes[ci].n))
            k += 1
            t_next += rng.exponential(1.0 / qps)
        time.sleep(max(0.0, min(t_next - time.perf_counter(), 0.002)))
    srv.drain()
    wall = time.perf_counter() - t0
    lat, per, fails = [], {}, []
    for t, n in tickets:
        r = srv.poll(t, n)
        lat.append(r[3])
        per.setdefault(n, []).append(r[3])
        if r[1] < 0:
            fails.append({"n": n, "flag": int(r[1])})
    lat = np.array(lat)
    return {"offered_qps": qps, "arrival_s": seconds, "requests": len(lat), "frames_per_s": len(lat) / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "per_code_p50_ms": {str(n): float(np.percentile(v, 50) * 1e3) for n, v in sorted(per.items())},
            "per_code_p99_ms": {str(n): float(np.percentile(v, 99) * 1e3) for n, v in sorted(per.items())},
            "numerical_failures": len(fails), "failure_flags": fails}


def serving(ctx, seconds=8.0, qps=40.0, seed=5, full=False, streams=None, mode=1):
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
    srv = ctx.server(hbm_budget_bytes=8 << 30, max_slots=2048)
    ctx.set_option("SERVER_MODE", prev)
    try:
        burst = 384
        t0 = time.perf_counter()
        tk = []
        for k in range(burst):
            ci = int(rng.integers(0, len(codes)))
            g = awgn_llr(codes[ci].n, float(rng.uniform(1.5, 3.0)), 0.5, frame_seed(78, ci, k))
            tk.append((srv.submit(Cs[ci], g), codes[ci].n))
        srv.drain()
        sat = burst / (time.perf_counter() - t0)
        for t, n in tk:
            srv.poll(t, n)
        log(f"serving mode {mode}: burst of {burst} at {sat:.0f} frames/s")
        res = _poisson(srv, Cs, codes, rng, qps, seconds, 77)
        log(f"serving mode {mode}: {qps:.0f} qps p50 {res['p50_ms']:.1f} ms p99 {res['p99_ms']:.1f} ms")
        res.update({"mode": "persistent" if mode else "waves", "codes": [c.name for c in codes],
                    "streams": int(ctx.get_option("SERVER_STREAMS")) if mode == 0 else len(codes),
                    "saturated_frames_per_s": sat, "burst": burst,
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
             2: "Algorithm 8 (row-wise, diagonal expansion)", 3: "Algorithm 8 (row-wise, triangular expansion)"}
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
            for pc in (4, 0, 1, 2, 3):
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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lpdec_main_n1024_traffic.md")


def stored_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, when it was taken on
    the current sources (else None). The summary holds one JSON line starting with
    '{"traffic"'."""
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp64",
                    help="PCG vector precision of the main leg (fp64: the library's batch default)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-PCG leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-pcg-primary", action="store_true",
                    help="skip the leg with a fixed PCG cap of 500 (dense solves only for systems PCG fails)")
    ap.add_argument("--serve-full", action="store_true",
                    help="serving leg over n = 256, 1024, 4096 and the irregular 8192 code")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a 256 MiB copy first (HBM counter calibration under rocprofv3)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--precond-study", action="store_true",
                    help="print the preconditioner comparison of Sec. VI-B (n=2000 code) instead of the benchmark")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU: frames are independent LPs and the "
                                   "multi-GPU form is a per-frame shard with no exchange; "
                                   "run with --gpus 1"}))
        sys.exit(2)

    if args.precond_study:
        print(json.dumps(precond_study()))
        return
    import torch
    from paper_0902_0657_amd import Code, Context, _lib, stats_table
    if not os.path.exists(_lib.LIB_PATH):
        from paper_0902_0657_amd import build as B
        B.build()
    code, G = workload()
    dev = torch.device("cuda:0")
    if args.calib_copy:
        copy_calibration(dev)
    ctx = Context(0)
    if args.block:
        ctx.set_option("BLOCK", args.block)
    fp64 = args.precision == "fp64"
    ctx.set_option("PRECISION", 1 if fp64 else 0)
    C = Code.from_synth(ctx, code)
    g = torch.as_tensor(G, device=dev)
    stream = torch.cuda.current_stream(dev)
    nf = G.shape[0]
    out = ctx.batch_outputs(C, nf, dev)
    for w in range(args.warmup):
        ctx.decode_batch(C, g, out=out)
        torch.cuda.synchronize()
        log(f"warmup {w + 1} done")
    # HIP events on the stream the decode kernel is launched on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        ctx.decode_batch(C, g, out=out, stream=stream)
        ev[k + 1].record(stream)
        ev[k + 1].synchronize()
        log(f"step {k + 1}: {ev[k].elapsed_time(ev[k + 1]):.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    total_s = float(step_ms.sum()) / 1e3
    value = nf * args.steps / total_s
    st = stats_table(out["stats"])
    flags = out["flag"].cpu().numpy()
    xhat = out["xhat"].cpu().numpy()
    objs = out["obj"].cpu().numpy()
    alg = algorithmic_bytes(st, code.n)
    kern_s = float(step_ms.mean()) / 1e3
    achieved = alg / kern_s / 1e9
    traffic, traffic_note = stored_traffic()
    frame_ms = st["ticks_total"].astype(np.float64) / 1e5   # 100 MHz device clock
    flops = dense_flops(st)
    tf = flops / kern_s / 1e12
    pcg_share = float(st["ticks_pcg"].sum() / max(1, st["ticks_total"].sum()))
    dense_share = float(st["ticks_dense"].sum() / max(1, st["ticks_total"].sum()))
    hbm_view = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": (traffic / 1e9 / kern_s) if traffic is not None else None,
                "traffic_bytes_per_launch": traffic, "traffic_note": traffic_note,
                "algorithmic_bytes_per_launch": alg,
                "basis": "PCG iterations 27p + 4q bytes, IPM iterations 120q bytes"}
    mfma_view = {"bound": "mfma", "achieved": tf, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                 "frac": tf / FP64_PEAK_TFS, "traffic": None, "algorithmic_flops_per_launch": flops,
                 "basis": "dense-fallback Cholesky, P^3/3 flops per solve, FP64 matrix cores"}
    # the roofline of the work that takes most of the device time; the other one beside it
    primary, secondary = (mfma_view, hbm_view) if dense_share > pcg_share else (hbm_view, mfma_view)
    kname = f"lpdec_main<{'double' if fp64 else 'float'}, LDS, DECODE>"
    primary.update({"kernel": kname, "kernel_ms": kern_s * 1e3})
    res = {
        "metric": "LP-decoded frames/s at n=1024 (3,6) + p50/p99 latency, vs plain FP64 GPU",
        "value": value, "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": float(step_ms.mean()), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if fp64 else "f32 PCG / f64 IPM", "data": "synthetic",
        "config": {"workload": "(3,6)-regular LDPC n=1024 m=512, AWGN Eb/N0 1.5/2.0/2.5 dB "
                               "(171/171/170 frames), FP32 LLRs, 512 frames per launch, MALP-A, "
                               + ("FP64 PCG" if fp64 else "FP32 PCG") + " (Algorithm 4, Algorithm 7 "
                               "preconditioner) with FP64 refinement first; once PCG misses its goal within "
                               "the automatic cap (max(100, p^2/3500) iterations, one round) the LP's remaining Newton systems "
                               "go to dense FP64 Cholesky on the matrix cores",
                   "global_batch": nf, "parallelism": "one workgroup per frame"},
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "note": "batch mode: a frame's result is available when its launch ends"},
        "frame_decode_ms": {"p50": float(np.percentile(frame_ms, 50)), "p99": float(np.percentile(frame_ms, 99)),
                            "max": float(frame_ms.max()),
                            "note": "in-kernel decode time of each frame (device clock)"},
        "wall_s_timed": wall,
        "decode_stats": {"flags": {str(k): int(v) for k, v in zip(*np.unique(flags, return_counts=True))},
                         "mean_malp_iters": float(st["malp_iters"].mean()),
                         "mean_ipm_iters": float(st["ipm_iters"].mean()),
                         "mean_pcg_iters": float(st["pcg_iters"].mean()),
                         "mean_pcg_per_newton": float(st["pcg_iters"].sum() / max(1, st["ipm_iters"].sum())),
                         "max_p": int(st["p_max"].max()), "max_levels": int(st["max_levels"].max()),
                         "pcg_us_per_iteration": float(st["ticks_pcg"].sum() / 100.0 / max(1, st["pcg_iters"].sum())),
                         "mts_us_per_ipm_iteration": float(st["ticks_mts"].sum() / 100.0 / max(1, st["ipm_iters"].sum())),
                         "ref_rounds": int(st["ref_rounds"].sum()),
                         "dense_fallback_solves": int(st["direct_solves"].sum()),
                         "newton_solves": int(st["ipm_iters"].sum()),
                         "newton_solved_by_pcg": 1.0 - float(st["direct_solves"].sum() / max(1, st["ipm_iters"].sum())),
                         "device_time_share": {"pcg": pcg_share, "dense_fallback": dense_share,
                                               "mts": float(st["ticks_mts"].sum() / max(1, st["ticks_total"].sum()))}},
        "roofline": primary,
        "roofline_other": secondary,
    }
    # serving first among the extra legs, while the process holds no other device work
    if not args.no_serve:
        res["serving"] = serving(ctx, full=args.serve_full, mode=1)
        log(f"serving: {res['serving']['requests']} requests")
        res["serving_waves"] = serving(ctx, full=args.serve_full, mode=0)
        log(f"serving (waves): {res['serving_waves']['requests']} requests")
    if not args.no_fp32 and fp64:
        c32 = Context(0)
        c32.set_option("PRECISION", 0)
        C32 = Code.from_synth(c32, code)
        o32 = c32.batch_outputs(C32, nf, dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        c32.decode_batch(C32, g, out=o32, stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms32 = e0.elapsed_time(e1)
        f32, x32 = o32["flag"].cpu().numpy(), o32["xhat"].cpu().numpy()
        res["fp32_pcg"] = {"value": nf / (ms32 / 1e3), "unit": "frames/s", "ms_per_step": ms32,
                           "flags": {str(k): int(v) for k, v in zip(*np.unique(f32, return_counts=True))},
                           "differs_from_main": int(sum(1 for f in range(nf) if f32[f] != flags[f]
                                                        or not np.array_equal(x32[f], xhat[f])))}
        log(f"fp32 PCG leg: {ms32:.1f} ms")
        c32.close()
    if not args.no_pcg_primary:
        cp = Context(0)
        cp.set_option("PCG_MAXIT", 500)
        Cp = Code.from_synth(cp, code)
        op = cp.batch_outputs(Cp, nf, dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cp.decode_batch(Cp, g, out=op, stream=stream)
        e1.record(stream)
        e1.synchronize()
        msp = e0.elapsed_time(e1)
        sp = stats_table(op["stats"])
        fp_, xp = op["flag"].cpu().numpy(), op["xhat"].cpu().numpy()
        res["pcg_primary"] = {"value": nf / (msp / 1e3), "unit": "frames/s", "ms_per_step": msp,
                              "pcg_maxit": 500,
                              "newton_solved_by_pcg": 1.0 - float(sp["direct_solves"].sum() / max(1, sp["ipm_iters"].sum())),
                              "differs_from_main": int(sum(1 for f in range(nf) if fp_[f] != flags[f]
                                                           or not np.array_equal(xp[f], xhat[f])))}
        log(f"PCG-primary leg: {msp:.1f} ms")
        cp.close()
    if not args.no_plain:
        frames = [g0 + k for k in range(8) for g0 in (0, 171, 342)]
        pf, plain_res = plain_fp64(ctx, C, G, frames)
        log(f"plain FP64: {pf['frames']} frames")
        res["plain_fp64"] = pf
        res["speedup_vs_plain"] = value / pf["value"]
        mism = [f for f, xh, fl, ob in plain_res if not (np.array_equal(xh, xhat[f]) and fl == flags[f])]
        res["plain_fp64"]["mismatch_vs_batch"] = len(mism)
    if not args.no_cpu:
        cb, done = cpu_baseline(G)
        log(f"cpu baseline: {len(done)} frames")
        res["cpu_baseline"] = cb
        mism = [k for k, (t, xh, fl, ob) in done
                if not (np.array_equal(xh, xhat[k]) and fl == flags[k]
                        and abs(ob - objs[k]) <= 1e-6 * (1.0 + abs(ob - float(G[k][G[k] < 0].sum()))))]
        res["parity_sample"] = {"frames": len(done), "mismatches": len(mism)}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
