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
