"""lpdec_decode_batch_noalloc (the library's fixed device region as workspace, no allocation)
against lpdec_decode_batch on the same frames: decoded words, flags, objectives, LP points and
iteration counts identical. Two calls in a row, the second with fewer frames, so the second
runs over the region the first left behind."""
import numpy as np
import pytest

from synth.channel import batch_awgn
from synth.codes import irregular_code, regular_code
from tests.gpu_util import cuda, host, make_ctx

pytestmark = pytest.mark.gpu


def _same(a, b):
    for key in ("xhat", "flag", "obj", "u"):
        assert np.array_equal(host(a[key]), host(b[key])), key
    assert np.array_equal(host(a["stats"])[:, :10], host(b["stats"])[:, :10])   # counts; ticks vary


@pytest.mark.parametrize("n,block", [(256, 0), (1024, 0)])
def test_noalloc_matches_decode_batch(n, block):
    import torch
    from paper_0902_0657_amd import Code
    ctx = make_ctx(BLOCK=block)
    code = regular_code(n)
    C = Code.from_synth(ctx, code)
    calls = [batch_awgn(code.n, 0.5, 1.5, 300, stream=700 + n), batch_awgn(code.n, 0.5, 2.0, 40, stream=800 + n)]
    for k, G in enumerate(calls):
        print(f"[noalloc] n={n} call {k}: {G.shape[0]} frames", flush=True)
        g = cuda(G, torch.float64)
        ref = ctx.decode_batch(C, g, want_u=True)
        torch.cuda.synchronize()
        out = ctx.batch_outputs(C, G.shape[0], g.device, want_u=True)
        ctx.decode_batch(C, g, out=out, noalloc=True)
        torch.cuda.synchronize()
        _same(out, ref)
    ctx.close()


def test_noalloc_rejects_a_frame_larger_than_the_region():
    """The irregular n=8192 code with the dense fallback needs 134 MB for one frame's dense
    system alone: the call is refused on the host, nothing is launched."""
    import torch
    from paper_0902_0657_amd import Code, LpdecError
    ctx = make_ctx()
    code = irregular_code(8192)
    C = Code.from_synth(ctx, code)
    g = cuda(np.ones((2, code.n)), torch.float64)
    with pytest.raises(LpdecError) as e:
        ctx.decode_batch(C, g, noalloc=True)
        torch.cuda.synchronize()
    assert e.value.status == -1 and "fixed region" in str(e.value)
    ctx.close()
