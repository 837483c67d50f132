"""MI355X-native adaptive LP decoding (Taghavi, Shokrollahi, Siegel).

Thin Python layer over the C ABI of liblpdec.so (include/lpdec.h). Device buffers are torch
CUDA (HIP) tensors; every step of the decoder runs in the library's HIP kernels. There is no
CPU fallback: a missing library raises at the first call.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import OPT, STATS_FIELDS, Stats

STATS_WORDS = C.sizeof(Stats) // 4   # int32 words per lpdec_stats


def stats_table(stats_i32):
    """Decodes an int32 tensor/array [nframes, STATS_WORDS] of lpdec_stats into a dict of
    numpy arrays."""
    a = np.ascontiguousarray(stats_i32.cpu().numpy() if hasattr(stats_i32, "cpu") else stats_i32)
    rec = a.view(np.dtype([(f, np.int32) for f in STATS_FIELDS[:10]] + [(f, np.int64) for f in STATS_FIELDS[10:]]))
    return {f: rec[f].reshape(-1) for f in STATS_FIELDS}

__all__ = ["Context", "Code", "LpdecError", "OPT", "STATS_FIELDS"]


class LpdecError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lpdec status {status}: {msg}")
        self.status = status


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A decoding context on one HIP device (lpdec_ctx)."""

    def __init__(self, device: int = 0, **options):
        self.L = _lib.load()
        h = C.c_void_p()
        st = self.L.lpdec_ctx_create(device, C.byref(h))
        if st != 0:
            raise LpdecError(st, f"lpdec_ctx_create(device={device}) failed")
        self.h = h
        self.device = device
        for k, v in options.items():
            self.set_option(k, v)

    def _check(self, st):
        if st != 0:
            raise LpdecError(st, self.L.lpdec_last_error(self.h).decode())

    def set_option(self, key, value):
        k = OPT[key.upper()] if isinstance(key, str) else int(key)
        self._check(self.L.lpdec_set_option(self.h, k, float(value)))

    def get_option(self, key):
        k = OPT[key.upper()] if isinstance(key, str) else int(key)
        v = C.c_double()
        self._check(self.L.lpdec_get_option(self.h, k, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "h", None):
            self.L.lpdec_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ codes
    def code(self, m, n, rowptr, col) -> "Code":
        return Code(self, m, n, rowptr, col)

    # ------------------------------------------------------------------ decoding
    def decode(self, code: "Code", gamma):
        """One frame from host memory (lpdec_decode). Returns (xhat, flag, objective, stats, u)."""
        g = np.ascontiguousarray(gamma, dtype=np.float64)
        assert g.shape == (code.n,)
        xhat = np.zeros(code.n, dtype=np.uint8)
        u = np.zeros(code.n, dtype=np.float64)
        flag = C.c_int32()
        obj = C.c_double()
        st = Stats()
        self._check(self.L.lpdec_decode(self.h, code.h, g.ctypes.data_as(C.c_void_p),
                                        xhat.ctypes.data_as(C.c_void_p), C.byref(flag), C.byref(obj),
                                        C.byref(st), u.ctypes.data_as(C.c_void_p)))
        return xhat, int(flag.value), float(obj.value), {f: getattr(st, f) for f in STATS_FIELDS}, u

    def alp_decode_batch(self, code: "Code", gamma):
        """ALP decoding (lpdec_alp_decode_batch) of frames from host memory: gamma [nframes, n].
        Returns a dict of numpy arrays: xhat, flag, obj, u and stats (lpdec_stats rows)."""
        g = np.ascontiguousarray(gamma, dtype=np.float64)
        assert g.ndim == 2 and g.shape[1] == code.n
        nf = g.shape[0]
        xhat = np.zeros((nf, code.n), dtype=np.uint8)
        flag = np.zeros(nf, dtype=np.int32)
        obj = np.zeros(nf, dtype=np.float64)
        u = np.zeros((nf, code.n), dtype=np.float64)
        st = (Stats * max(nf, 1))()
        self._check(self.L.lpdec_alp_decode_batch(self.h, code.h, nf, g.ctypes.data_as(C.c_void_p),
                                                  xhat.ctypes.data_as(C.c_void_p), flag.ctypes.data_as(C.c_void_p),
                                                  obj.ctypes.data_as(C.c_void_p), C.cast(st, C.c_void_p),
                                                  u.ctypes.data_as(C.c_void_p)))
        stats = np.frombuffer(bytes(st), dtype=np.int32).reshape(max(nf, 1), STATS_WORDS)[:nf].copy()
        return {"xhat": xhat, "flag": flag, "obj": obj, "u": u, "stats": stats}

    @staticmethod
    def batch_outputs(code: "Code", nf, device, want_u=False, want_stats=True):
        """Output tensors of decode_batch for nf frames (allocated, not filled)."""
        import torch
        out = {
            "xhat": torch.empty((nf, code.n), dtype=torch.uint8, device=device),
            "flag": torch.empty(nf, dtype=torch.int32, device=device),
            "obj": torch.empty(nf, dtype=torch.float64, device=device),
        }
        if want_stats:
            out["stats"] = torch.empty((nf, STATS_WORDS), dtype=torch.int32, device=device)
        if want_u:
            out["u"] = torch.empty((nf, code.n), dtype=torch.float64, device=device)
        return out

    def decode_batch(self, code: "Code", gamma, out=None, want_u=False, want_stats=True, stream=None,
                     noalloc=False):
        """gamma: CUDA tensor [nframes, n] (float32 or float64). Asynchronous on `stream`
        (default: torch's current stream). Returns a dict of output tensors. noalloc=True calls
        lpdec_decode_batch_noalloc (the library's fixed device region as workspace; pass `out`
        to allocate nothing here either)."""
        import torch
        assert gamma.is_cuda and gamma.is_contiguous() and gamma.dim() == 2 and gamma.shape[1] == code.n
        nf = gamma.shape[0]
        dev = gamma.device
        if out is None:
            out = self.batch_outputs(code, nf, dev, want_u=want_u, want_stats=want_stats)
        gdt = 1 if gamma.dtype == torch.float64 else 0
        assert gamma.dtype in (torch.float32, torch.float64)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        fn = self.L.lpdec_decode_batch_noalloc if noalloc else self.L.lpdec_decode_batch
        self._check(fn(self.h, code.h, nf, _ptr(gamma), gdt, _ptr(out["xhat"]),
                                              _ptr(out["flag"]), _ptr(out.get("obj")), _ptr(out.get("stats")),
                                              _ptr(out.get("u")), C.c_void_p(s.cuda_stream)))
        return out

    def decode_batch_trace(self, code: "Code", gamma, trace_cap: int):
        import torch
        nf = gamma.shape[0]
        dev = gamma.device
        out = {
            "xhat": torch.empty((nf, code.n), dtype=torch.uint8, device=dev),
            "flag": torch.empty(nf, dtype=torch.int32, device=dev),
            "obj": torch.empty(nf, dtype=torch.float64, device=dev),
            "stats": torch.empty((nf, STATS_WORDS), dtype=torch.int32, device=dev),
            "u": torch.empty((nf, code.n), dtype=torch.float64, device=dev),
            "trace": torch.zeros((nf, trace_cap, code.m), dtype=torch.int32, device=dev),
        }
        gdt = 1 if gamma.dtype == torch.float64 else 0
        torch.cuda.synchronize(dev)
        self._check(self.L.lpdec_decode_batch_trace(self.h, code.h, nf, _ptr(gamma), gdt, _ptr(out["xhat"]),
                                                    _ptr(out["flag"]), _ptr(out["obj"]), _ptr(out["stats"]),
                                                    _ptr(out["u"]), _ptr(out["trace"]), trace_cap))
        return out

    # ------------------------------------------------------------------ steps
    def cut_search_batch(self, code, u):
        import torch
        nf = u.shape[0]
        vm = torch.empty((nf, code.m), dtype=torch.int32, device=u.device)
        viol = torch.empty((nf, code.m), dtype=torch.uint8, device=u.device)
        lhs = torch.empty((nf, code.m), dtype=torch.float64, device=u.device)
        torch.cuda.synchronize(u.device)
        self._check(self.L.lpdec_cut_search_batch(self.h, code.h, nf, _ptr(u), _ptr(vm), _ptr(viol), _ptr(lhs)))
        return vm, viol, lhs

    def mts_batch(self, code, hascut, w):
        import torch
        nf = hascut.shape[0]
        dev = hascut.device
        pair = torch.empty((nf, code.m), dtype=torch.int32, device=dev)
        lb = torch.empty((nf, code.m), dtype=torch.int32, device=dev)
        lf = torch.empty((nf, code.m), dtype=torch.int32, device=dev)
        rounds = torch.empty(nf, dtype=torch.int32, device=dev)
        torch.cuda.synchronize(dev)
        self._check(self.L.lpdec_mts_batch(self.h, code.h, nf, _ptr(hascut), _ptr(w), _ptr(pair), _ptr(lb),
                                           _ptr(lf), _ptr(rounds)))
        return pair, lb, lf, rounds

    def normal_matvec_batch(self, code, vmask, gamma, d2, h, precision=0):
        import torch
        nf = vmask.shape[0]
        l = torch.empty((nf, code.m), dtype=torch.float64, device=vmask.device)
        torch.cuda.synchronize(vmask.device)
        self._check(self.L.lpdec_normal_matvec_batch(self.h, code.h, nf, _ptr(vmask), _ptr(gamma), _ptr(d2),
                                                     _ptr(h), _ptr(l), precision))
        return l

    def newton_solve_batch(self, code, vmask, gamma, d2, w, precision=0):
        import torch
        nf = vmask.shape[0]
        dev = vmask.device
        y = torch.empty((nf, code.m), dtype=torch.float64, device=dev)
        its = torch.empty(nf, dtype=torch.int32, device=dev)
        res = torch.empty(nf, dtype=torch.float64, device=dev)
        torch.cuda.synchronize(dev)
        self._check(self.L.lpdec_newton_solve_batch(self.h, code.h, nf, _ptr(vmask), _ptr(gamma), _ptr(d2),
                                                    _ptr(w), _ptr(y), _ptr(its), _ptr(res), precision))
        return y, its, res

    def ipm_batch(self, code, vmask, gamma, precision=0):
        import torch
        nf = vmask.shape[0]
        dev = vmask.device
        q = code.n + code.m
        x = torch.empty((nf, q), dtype=torch.float64, device=dev)
        z = torch.empty((nf, q), dtype=torch.float64, device=dev)
        y = torch.empty((nf, code.m), dtype=torch.float64, device=dev)
        its = torch.empty(nf, dtype=torch.int32, device=dev)
        status = torch.empty(nf, dtype=torch.int32, device=dev)
        torch.cuda.synchronize(dev)
        self._check(self.L.lpdec_ipm_batch(self.h, code.h, nf, _ptr(vmask), _ptr(gamma), _ptr(x), _ptr(y),
                                           _ptr(z), _ptr(its), _ptr(status), precision))
        return x, y, z, its, status

    # ------------------------------------------------------------------ serving
    def server(self, hbm_budget_bytes: int, max_slots: int) -> "Server":
        return Server(self, hbm_budget_bytes, max_slots)


class Code:
    """A parity-check matrix registered with a context (lpdec_code)."""

    def __init__(self, ctx: Context, m, n, rowptr, col):
        self.ctx = ctx
        self.m, self.n = int(m), int(n)
        self._rp = np.ascontiguousarray(rowptr, dtype=np.int32)
        self._cl = np.ascontiguousarray(col, dtype=np.int32)
        h = C.c_void_p()
        ctx._check(ctx.L.lpdec_code_create(ctx.h, self.m, self.n, self._rp.ctypes.data_as(C.c_void_p),
                                           self._cl.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.h = h

    @classmethod
    def from_synth(cls, ctx: Context, code) -> "Code":
        return cls(ctx, code.m, code.n, code.rowptr, code.col)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.L.lpdec_code_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (lpdec_server)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int):
        self.ctx = ctx
        h = C.c_void_p()
        ctx._check(ctx.L.lpdec_server_create(ctx.h, int(hbm_budget_bytes), int(max_slots), C.byref(h)))
        self.h = h

    def submit(self, code: Code, gamma) -> int:
        g = np.ascontiguousarray(gamma, dtype=np.float64)
        t = C.c_uint64()
        st = self.ctx.L.lpdec_server_submit(self.h, code.h, g.ctypes.data_as(C.c_void_p), C.byref(t))
        if st != 0:
            raise LpdecError(st, "submit failed")
        return int(t.value)

    def poll(self, ticket: int, n: int):
        """Returns None while busy, else (xhat, flag, objective, latency_s)."""
        xh = np.zeros(n, dtype=np.uint8)
        flag = C.c_int32()
        obj = C.c_double()
        lat = C.c_double()
        st = self.ctx.L.lpdec_server_poll(self.h, ticket, xh.ctypes.data_as(C.c_void_p), C.byref(flag),
                                          C.byref(obj), C.byref(lat))
        if st == _lib.EBUSY:
            return None
        if st != 0:
            raise LpdecError(st, f"poll({ticket}) failed")
        return xh, int(flag.value), float(obj.value), float(lat.value)

    def drain(self):
        self.ctx.L.lpdec_server_drain(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.L.lpdec_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
