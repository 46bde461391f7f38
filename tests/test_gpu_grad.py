"""GPU tests of the score-function gradient through the autograd wrapper:

* exact importances on the tiny graph (brute force over 2^20 states): every
  dP/dp_i within 3 standard errors, and the z-scores calibrated (mean z^2
  near 1);
* common-random-number central differences: P is multilinear in each p_i,
  so (P(p_i + d) - P(p_i - d)) / 2d is an unbiased estimate of dP/dp_i with
  no truncation error; it must agree with the score-function value within
  3 combined standard errors.
(The fp32 gradient's 1e-5 relative agreement with the fp64 oracle is tested
in test_gpu_parity.py.)"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2604_17066_amd as R
import workloads as WL

pytestmark = pytest.mark.gpu


def _sf_se(counts, p, N):
    """Standard error of the score-function estimate of dP/dp_i for a binary
    component: the per-sample term is Y (1{x=1}/p - 1{x=0}/(1-p))."""
    c0 = counts[:, 0].astype(np.float64)
    c1 = counts[:, 1].astype(np.float64)
    q = 1.0 - p
    mean = c1 / (N * p) - c0 / (N * q)
    second = c1 / (N * p * p) + c0 / (N * q * q)
    return np.sqrt(np.maximum(second - mean * mean, 0.0) / N)


def test_importance_against_exact_tiny(rsr_ctx):
    cfg = WL.configs.tiny()
    N = 1 << 20
    lower, upper = cfg["lower"][:-3], cfg["upper"][:-12]
    refs = R.Refs(rsr_ctx, cfg["n"], 2, lower, upper)
    system = R.System(rsr_ctx, cfg["graph"])
    p = torch.tensor(cfg["p"][:, 1], dtype=torch.float64, requires_grad=True)
    P = R.rsr_probability(p, refs, system, N, seed=123, rsr_ctx=rsr_ctx)
    P.backward()
    grad = p.grad.numpy()
    table = oracle.phi_table_st(cfg["graph"])
    P_exact, Gx = oracle.exact(cfg["p"], table)
    I_exact = Gx[:, 1] - Gx[:, 0]
    # standard errors from the gradient counts of the same samples
    model = R.Model(rsr_ctx, cfg["p"])
    est, buf = R.stage2(rsr_ctx, model, refs, system, N, 123)
    _, counts = R.rsr_grad(rsr_ctx, model, buf.samples, buf.Y, N, want_counts=True)
    torch.cuda.synchronize()
    se = _sf_se(counts.cpu().numpy().view(np.uint64), cfg["p"][:, 1], N)
    z = (grad - I_exact) / se
    print("max |z| =", np.abs(z).max(), "mean z^2 =", np.mean(z * z))
    assert float(P) == est["P"]
    assert abs(float(P) - P_exact) <= 3 * est["se"]
    assert np.all(np.abs(z) <= 3.0)
    assert 0.2 <= np.mean(z * z) <= 3.0


def test_importance_against_crn_differences(rsr_ctx):
    cfg = WL.configs.graph2(N=1)
    N = 1 << 20
    refs = R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"][:4000], cfg["upper"][:4000])
    system = R.System(rsr_ctx, cfg["graph"])
    p0 = cfg["p"][:, 1].copy()
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    P = R.rsr_probability(p, refs, system, N, seed=77, rsr_ctx=rsr_ctx)
    P.backward()
    grad = p.grad.numpy()
    model = R.Model(rsr_ctx, cfg["p"])
    _, buf = R.stage2(rsr_ctx, model, refs, system, N, 77)
    _, counts = R.rsr_grad(rsr_ctx, model, buf.samples, buf.Y, N, want_counts=True)
    torch.cuda.synchronize()
    se_sf = _sf_se(counts.cpu().numpy().view(np.uint64), p0, N)
    order = np.argsort(-np.abs(grad))
    picks = list(order[:4]) + [int(order[len(order) // 2])]
    delta = 0.02
    for i in picks:
        Ys = []
        for sign in (+1, -1):
            q = p0.copy()
            q[i] = min(1.0, max(0.0, q[i] + sign * delta))
            m = R.Model(rsr_ctx, WL.configs.binary_model(q))
            _, b = R.stage2(rsr_ctx, m, refs, system, N, 77, grad=False, estimate=False)
            torch.cuda.synchronize()
            Ys.append(b.Y.cpu().numpy().astype(np.int64))
        span = min(1.0, p0[i] + delta) - max(0.0, p0[i] - delta)
        d = Ys[0] - Ys[1]
        assert d.min() >= 0      # common random numbers: raising p_i never lowers Y
        fd = d.mean() / span
        se_fd = math.sqrt(d.mean() * (1 - d.mean()) / N) / span
        tol = 3.0 * math.hypot(se_fd, se_sf[i])
        print(f"i={i}: score-function {grad[i]:.5f}, CRN difference {fd:.5f}, tol {tol:.5f}")
        assert abs(fd - grad[i]) <= tol


def test_importance_config_size_against_oracle(rsr_ctx):
    """Binary Birnbaum importance on the graph2 workload at its full size
    (N = 1e6, 1e4 + 1e4 rows): rsr_importance against the fp64 oracle's
    G[i][1] - G[i][0], held to |I32 - I64| <= 1e-5 (|G1| + |G0|) (the
    difference can cancel, so the bound is relative to the two terms); the
    library forms both quotients in fp64, so the result is the fp64 value
    rounded once."""
    cfg = WL.configs.graph2()
    N = cfg["N"]
    model = R.Model(rsr_ctx, cfg["p"])
    refs = R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"], cfg["upper"])
    system = R.System(rsr_ctx, cfg["graph"])
    est, buf = R.stage2(rsr_ctx, model, refs, system, N, cfg["seed"], grad=False)
    I = R.rsr_importance(rsr_ctx, model, buf.samples, buf.Y, N)
    torch.cuda.synchronize()
    x = oracle.sample(cfg["p"], cfg["seed"], 0, 0, N)
    Y, _ = oracle.eval_unknown(cfg["graph"], x, None, which=1)
    np.testing.assert_array_equal(buf.Y.cpu().numpy(), Y)
    _, G = oracle.grad(cfg["p"], x, Y)
    I64 = G[:, 1] - G[:, 0]
    I32 = I.cpu().numpy().astype(np.float64)
    err = np.abs(I32 - I64)
    bound = 1e-5 * (np.abs(G[:, 1]) + np.abs(G[:, 0]))
    print("max |I32 - I64| / (|G1| + |G0|) =", np.max(err / np.maximum(bound * 1e5, 1e-300)))
    assert np.all(err <= bound)
    np.testing.assert_array_equal(I.cpu().numpy(), I64.astype(np.float32))


def test_model_update_equals_fresh_model(rsr_ctx):
    """rsr_model_update followed by the hot path gives exactly what a model
    created with the new probabilities gives, and the update is ordered after
    work enqueued before it."""
    cfg = WL.configs.graph2(N=50_000)
    N = cfg["N"]
    refs = R.Refs(rsr_ctx, cfg["n"], 2, cfg["lower"][:2000], cfg["upper"][:2000])
    system = R.System(rsr_ctx, cfg["graph"])
    rng = np.random.default_rng(5)
    q = WL.configs.binary_model(rng.uniform(0.7, 0.99, cfg["n"]))
    m = R.Model(rsr_ctx, cfg["p"])
    xs_old = R.rsr_sample(rsr_ctx, m, 9, 0, 0, N)      # enqueued before the update
    m.update(q)
    est_u, buf_u = R.stage2(rsr_ctx, m, refs, system, N, 9)
    fresh = R.Model(rsr_ctx, q)
    est_f, buf_f = R.stage2(rsr_ctx, fresh, refs, system, N, 9)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(buf_u.samples.cpu().numpy(), buf_f.samples.cpu().numpy())
    np.testing.assert_array_equal(buf_u.G.cpu().numpy(), buf_f.G.cpu().numpy())
    assert est_u == est_f
    old = R.rsr_sample(rsr_ctx, R.Model(rsr_ctx, cfg["p"]), 9, 0, 0, N)
    np.testing.assert_array_equal(xs_old.cpu().numpy(), old.cpu().numpy())
    with pytest.raises(R.RSRError):
        m.update(np.full((cfg["n"], 2), 0.7))      # rows do not sum to 1
    est_again, _ = R.stage2(rsr_ctx, m, refs, system, N, 9)
    assert est_again == est_u                    # a rejected update leaves the model as it was


def test_autograd_float32_multistate_rows(rsr_ctx):
    """A float32 [n][3] probability tensor (rows sum to 1 only up to float32
    rounding) is accepted; the gradient is rsr_grad's G at the rows
    renormalised in fp64."""
    cfg = WL.configs.multi(N=1, R_per_level=2000)
    n = cfg["n"]
    lv = cfg["levels"][1]
    refs = R.Refs(rsr_ctx, n, 3, lv["lower"], lv["upper"])
    system = R.System(rsr_ctx, cfg["graph"], K=3, level=1)
    p32 = torch.tensor(cfg["p"], dtype=torch.float32, requires_grad=True)
    assert float(torch.abs(p32.detach().double().sum(dim=1) - 1.0).max()) > 1e-9
    N = 1 << 16
    P = R.rsr_probability(p32, refs, system, N, seed=4, rsr_ctx=rsr_ctx)
    P.backward()
    pm = p32.detach().double()
    pm = (pm / pm.sum(dim=1, keepdim=True)).numpy()
    m = R.Model(rsr_ctx, pm)
    est, buf = R.stage2(rsr_ctx, m, refs, system, N, 4)
    torch.cuda.synchronize()
    assert float(P) == est["P"]
    np.testing.assert_array_equal(p32.grad.numpy(), buf.G.cpu().numpy())
    # A second forward reuses the pooled model (no new model is created).
    pool = rsr_ctx.__dict__["_autograd_models"][(n, 3)]
    assert len(pool) == 1
    P2 = R.rsr_probability(p32, refs, system, N, seed=4, rsr_ctx=rsr_ctx)
    assert float(P2) == float(P) and len(pool) == 0
