"""GPU parity at the workloads' full sizes, against the oracle.

* Multi-state workload (295 three-state edges, 5e4 reference rows per
  level, N = 1e6): every Y of both levels equals the oracle's plain Monte
  Carlo, flags on sampled indices equal the oracle's Algorithm 1, P is
  bit-exact and the fp32 gradient is within 1e-5 of the fp64 oracle.  The
  LABEL flags of the popcount cascade and of the persistent cascade equal
  the automatic form's on every sample.
* The 1250-edge graph with 4.5e4 + 4.5e4 reference rows: the automatic
  form's FP4 round over rows 8 192..45 000 wants 71 chunks of 512 rows and
  is held to the cap of 64, the popcount form's round over rows
  20 000..45 000 wants 195 chunks of 128 rows and is held to its cap of
  128; both equal the persistent cascade and the oracle.
* One job of the batched workload at its full reference-set size (the
  647-edge graph, 2.2e4 + 2.2e4 rows) inside a plan, against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_17066_amd as R
import workloads as WL
from helpers import unpack_states

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-5


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _grad_close(G32, G64):
    nz = G64 != 0
    assert np.all(G32[~nz] == 0.0)
    rel = np.abs(G32[nz].astype(np.float64) - G64[nz]) / np.abs(G64[nz])
    assert rel.max() <= GRAD_RTOL, rel.max()


def test_multistate_config_size(rsr_ctx):
    cfg = WL.configs.multi()
    N, n, K = cfg["N"], cfg["n"], cfg["K"]
    g = cfg["graph"]
    model = R.Model(rsr_ctx, cfg["p"])
    x = oracle.sample(cfg["p"], cfg["seed"], 0, 0, N)
    rng = np.random.default_rng(44)
    idx = np.unique(np.concatenate([rng.integers(0, N, 4000), [0, N - 1]]))
    for level in (1, 2):
        lv = cfg["levels"][level]
        refs = R.Refs(rsr_ctx, n, K, lv["lower"], lv["upper"])
        assert refs.consistent and max(refs.R_L, refs.R_U) > 16_384
        system = R.System(rsr_ctx, g, K=K, level=level)
        est, buf = R.stage2(rsr_ctx, model, refs, system, N, cfg["seed"])
        G, counts = R.rsr_grad(rsr_ctx, model, buf.samples, buf.Y, N, want_counts=True)
        np.testing.assert_array_equal(unpack_states(_np(buf.samples)[:, idx], n, K), x[idx])
        fl, _, _ = oracle.classify(lv["lower"], lv["upper"], x[idx], mode=0)
        np.testing.assert_array_equal(_np(buf.flags)[idx], fl, err_msg=f"level {level}")
        auto = _np(buf.flags).copy()
        for form in (R.RSR_POPCOUNT, R.RSR_PERSIST):
            other = R.rsr_classify(rsr_ctx, refs, buf.samples, N, R.RSR_LABEL, form)
            np.testing.assert_array_equal(_np(other), auto, err_msg=f"level {level}, form {form}")
        Y, _ = oracle.eval_unknown(g, x, None, which=1, level=level)
        np.testing.assert_array_equal(_np(buf.Y), Y, err_msg=f"level {level}")
        assert est["P"] == float(Y.sum(dtype=np.int64)) / N
        assert est["n_both"] == 0
        c, G64 = oracle.grad(cfg["p"], x, Y)
        np.testing.assert_array_equal(_np(counts).view(np.uint64), c)
        _grad_close(_np(G), G64)


def test_wide_graph_chunk_caps(rsr_ctx):
    cfg = WL.configs.batched(n_scen=1, N=1, graphs=[7], ref_scale=0.45)
    sd, jd = cfg["systems"][0], cfg["jobs"][0]
    n, N = sd["n"], 20_000
    refs = R.Refs(rsr_ctx, n, 2, sd["lower"], sd["upper"])
    # Both rounds exceed their caps: (R - 8192) / 512 > 64, (R - 20000) / 128 > 128.
    assert refs.consistent and min(refs.R_L, refs.R_U) >= 42_000
    m = R.Model(rsr_ctx, jd["p"])
    xs = R.rsr_sample(rsr_ctx, m, jd["seed"], 0, 0, N)
    flags = {f: _np(R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, f)).copy()
             for f in (R.RSR_AUTO, R.RSR_POPCOUNT, R.RSR_PERSIST)}
    np.testing.assert_array_equal(flags[R.RSR_POPCOUNT], flags[R.RSR_AUTO])
    np.testing.assert_array_equal(flags[R.RSR_PERSIST], flags[R.RSR_AUTO])
    idx = np.unique(np.random.default_rng(71).integers(0, N, 400))
    x = oracle.sample_at(jd["p"], jd["seed"], 0, idx.astype(np.uint64))
    want, _, _ = oracle.classify(sd["lower"], sd["upper"], x, mode=0)
    np.testing.assert_array_equal(flags[R.RSR_AUTO][idx], want)
    print("unclassified", int((flags[R.RSR_AUTO] == 0).sum()), "of", N)


def test_batched_job_full_reference_size(rsr_ctx):
    N = 1 << 18
    cfg = WL.configs.batched(n_scen=2, N=N, graphs=[5], ref_scale=1.0)
    sd = cfg["systems"][0]
    n = sd["n"]
    refs = R.Refs(rsr_ctx, n, 2, sd["lower"], sd["upper"])
    system = R.System(rsr_ctx, sd["graph"])
    jobs = []
    for jd in cfg["jobs"]:
        jobs.append({"model": R.Model(rsr_ctx, jd["p"]), "refs": refs, "system": system,
                     "seed": jd["seed"], "N": N, "buffers": R.Buffers(rsr_ctx, n, 2, N),
                     "p": jd["p"]})
    plan = R.Plan(rsr_ctx, jobs, tune=False)
    plan.run()
    est, grads = plan.results()
    for k, jb in enumerate(jobs):
        x = oracle.sample(jb["p"], jb["seed"], 0, 0, N)
        Y, _ = oracle.eval_unknown(sd["graph"], x, None, which=1)
        np.testing.assert_array_equal(_np(jb["buffers"].Y), Y, err_msg=f"job {k}")
        idx = np.unique(np.random.default_rng(k).integers(0, N, 1500))
        fl, _, _ = oracle.classify(sd["lower"], sd["upper"], x[idx], mode=0)
        np.testing.assert_array_equal(_np(jb["buffers"].flags)[idx], fl, err_msg=f"job {k}")
        assert est[k]["P"] == float(Y.sum(dtype=np.int64)) / N
        _, G64 = oracle.grad(jb["p"], x, Y)
        _grad_close(grads[k], G64)
    plan.close()
