"""Helpers shared by the GPU tests (marshalling only)."""
import numpy as np


def cuda(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def make_ctx(**opts):
    from paper_0902_0657_amd import Context
    c = Context(0)
    # caps that bound the run time of a test on a faulty build (the PCG cap keeps its
    # automatic default, the production setting)
    base = {"MALP_MAX": 80, "IPM_MAX": 100}
    base.update(opts)
    for k, v in base.items():
        c.set_option(k, v)
    return c


def obj_close(a, b, gamma, rel=1e-6):
    """LP objectives gamma^T u agree to `rel` relative to the scale on which the interior-point
    method measures its duality gap, 1 + c^T x with c = |gamma| and x the flipped variables
    (c^T x = gamma^T u - sum of the negative gamma_i). A relative test against |gamma^T u|
    alone is meaningless near gamma^T u = 0, the value of every correctly decoded frame."""
    g = np.asarray(gamma, dtype=np.float64)
    scale = 1.0 + abs(b - float(g[g < 0].sum()))
    return abs(a - b) <= rel * scale


def snapshot_d2(orc, code, gamma, masks, ipm_iter):
    """D^2 = X Z^-1 of the oracle's interior-point iterate after ipm_iter iterations on the LP
    of a cut set (a realistic, increasingly ill-conditioned normal matrix), in the
    check-space layout [n standard | slack of check j at n+j]. The iterate is never past the
    last one at which the oracle itself solves a Newton system."""
    _, _, _, _, its = orc.ipm(code, gamma, masks)
    o = orc.OracleOpts(ipm_max=max(0, min(ipm_iter, its - 1)))
    rc, x, y, z, its = orc.ipm(code, gamma, masks, o)
    rows = np.nonzero(masks)[0]
    d2 = np.ones(code.n + code.m)
    d2[:code.n] = x[:code.n] / z[:code.n]
    d2[code.n + rows] = x[code.n:] / z[code.n:]
    return d2
