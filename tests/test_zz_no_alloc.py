"""GPU test of rsr_eval_unknown_noalloc (the evaluation entry point that
allocates nothing) against rsr_eval_unknown, through the C ABI: the same Y
and the same number of system-function evaluations, on two calls in a row,
the second with a smaller input (so a stale counter or list from the first
call would show), for s-t connectivity and max-flow systems; sizes beyond
the scratch are rejected."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2604_17066_amd as R
import workloads as WL
from paper_2604_17066_amd import _abi as A

pytestmark = pytest.mark.gpu

P = R.api._ptr


def _run(ctx, fn, system, xs, N, flags, which):
    Y = torch.full((N,), 7, dtype=torch.uint8, device="cuda")
    nev = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.check(fn(ctx.h, system.h, P(xs), N, P(flags) if flags is not None else None, which,
                 P(Y), P(nev)))
    torch.cuda.synchronize()
    return Y.cpu().numpy(), int(nev.cpu()[0])


@pytest.mark.parametrize("kind", ["st", "flow"])
def test_noalloc_equals_eval_unknown(rsr_ctx, kind):
    lib = A.lib()
    if kind == "st":
        cfg = WL.configs.graph2(N=1)
        K, level, rows = 2, 1, (cfg["lower"][:500], cfg["upper"][:500])
        p = cfg["p"]
    else:
        cfg = WL.configs.multi(N=1, R_per_level=600)
        K, level = 3, 2
        rows = (cfg["levels"][2]["lower"], cfg["levels"][2]["upper"])
        p = cfg["p"]
    n = cfg["n"]
    model = R.Model(rsr_ctx, p)
    refs = R.Refs(rsr_ctx, n, K, rows[0], rows[1])
    system = R.System(rsr_ctx, cfg["graph"], K=K, level=level, kind=kind)
    for N, seed in ((300_001, 5), (77_777, 6)):
        xs = R.rsr_sample(rsr_ctx, model, seed, 0, 0, N)
        flags = R.rsr_classify(rsr_ctx, refs, xs, N)
        for which in (R.RSR_UNKNOWN_ONLY, R.RSR_ALL):
            fl = flags if which == R.RSR_UNKNOWN_ONLY else None
            Y0, n0 = _run(rsr_ctx, lib.rsr_eval_unknown, system, xs, N, fl, which)
            Y1, n1 = _run(rsr_ctx, lib.rsr_eval_unknown_noalloc, system, xs, N, fl, which)
            np.testing.assert_array_equal(Y1, Y0, err_msg=f"N={N} which={which}")
            assert n1 == n0 and n0 > 0, (N, which, n0, n1)


def test_noalloc_rejects_sizes_beyond_its_scratch(rsr_ctx):
    lib = A.lib()
    cfg = WL.configs.tiny(N=1)
    system = R.System(rsr_ctx, cfg["graph"])
    dummy = torch.zeros(16, dtype=torch.int32, device="cuda")
    st = lib.rsr_eval_unknown_noalloc(rsr_ctx.h, system.h, P(dummy), (1 << 22) + 1, P(dummy),
                                      R.RSR_UNKNOWN_ONLY, P(dummy), None)
    assert st == A.RSR_EINVAL
    assert b"scratch" in lib.rsr_last_error(rsr_ctx.h)
