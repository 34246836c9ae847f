"""The adjoint entry point for callers that cannot allocate
(eamfe_adjoint_theta_noalloc): through the C ABI it gives what
eamfe_adjoint_theta gives on the same context, on two calls in a row, the
second with a smaller system (the fixed scratch keeps the first call's
contents and must be cleared), with and without the replica reduction, and
refuses a call whose scratch would exceed its fixed size."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import make_ctx, say
from paper_2201_04622_amd import inputs as I

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _noalloc(ctx, x, out, reduce, w=None):
    import paper_2201_04622_amd.eamfe as E
    wp = None if w is None else np.ascontiguousarray(w, dtype=np.float64).ctypes.data_as(C.POINTER(C.c_double))
    return E.lib().eamfe_adjoint_theta_noalloc(ctx._h, C.c_void_p(x.data_ptr()), wp, int(reduce),
                                                C.c_void_p(out.data_ptr()))


@pytest.mark.parametrize("prec", [FP64, FP32])
def test_noalloc_adjoint_matches_the_allocating_entry_point(prec):
    import torch

    import paper_2201_04622_amd.eamfe as E
    systems = [
        [I.Replica("bcc", 6, I.A_BCC_STABLE, 300.0, 5.0, 1), I.Replica("fcc", 5, I.A_FCC_STABLE, 300.0, 5.0, 2),
         I.Replica("bcc", 4, I.A_BCC_VERBATIM, 100.0, 5.0, 3)],
        [I.Replica("bcc", 4, I.A_BCC_VERBATIM, 200.0, 5.0, 4)],      # the second call: smaller
    ]
    n = I.N_KNOTS
    for call, reps in enumerate(systems):
        ctx, x0, arrs = make_ctx(reps, prec)
        x = E.to_soa(I.displaced(arrs["x0"], 0.05, seed=20 + call))
        w = np.linspace(1.0, -0.5, len(reps))
        for reduce in (0, 1):
            shape = (3, n) if reduce else (len(reps), 3, n)
            ref = torch.zeros(shape, dtype=torch.float64, device="cuda")
            ctx.adjoint_theta(x, ref, weights=w, reduce=bool(reduce))
            got = torch.zeros_like(ref)
            code = _noalloc(ctx, x, got, reduce, w)
            assert code == 0, E.lib().eamfe_last_error(ctx._h)
            torch.cuda.synchronize()
            say(f"call {call} prec {prec} reduce {reduce}: max |diff| {float((got - ref).abs().max()):.3e}")
            assert torch.equal(got, ref)     # the same kernels on fixed-point bins: bitwise
        ctx.close()


def test_noalloc_adjoint_refuses_scratch_beyond_its_size():
    import torch

    import paper_2201_04622_amd.eamfe as E
    reps = [I.Replica("bcc", 4, I.A_BCC_VERBATIM, 100.0, 5.0, s) for s in range(180)]   # 180 * 192 KB of bins
    ctx, x0, _ = make_ctx(reps, FP32)
    out = torch.zeros(3, I.N_KNOTS, dtype=torch.float64, device="cuda")
    code = _noalloc(ctx, x0, out, 1)
    msg = E.lib().eamfe_last_error(ctx._h).decode()
    say(f"refused: {code} {msg}")
    assert code == 1 and "scratch" in msg
    assert float(out.abs().max()) == 0.0
    ctx.close()
