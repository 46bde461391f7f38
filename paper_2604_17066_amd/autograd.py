"""torch.autograd wrapper: P(S >= level) as a differentiable function of the
component-state probabilities.

Forward runs the Stage-2 hot path (sample, classify, evaluate, estimate) in
the library's kernels; backward calls rsr_grad, whose score-function
estimator gives dP/dp[i][s] = E[Y 1{x_i = s}] / p[i][s] (independent
components make P multilinear in the state probabilities), or, for a binary
input p [n] of survival probabilities (state matrix (1 - p, p)),
rsr_importance, which forms dP/dp_i = G[i][1] - G[i][0] in the library.

Input rows are renormalised in fp64 before use, so float32 probabilities
(whose rows sum to 1 only up to float32 rounding) are accepted; the gradient
is the unconstrained partial at the renormalised point.  Models are reused
from a per-context pool and refreshed with rsr_model_update, so a forward
pass allocates no model.
"""
import torch

from . import _abi as A
from . import api


def _take_model(rsr_ctx, pm):
    n, K = pm.shape
    pool = rsr_ctx.__dict__.setdefault("_autograd_models", {}).setdefault((n, K), [])
    if pool:
        model = pool.pop()
        model.update(pm)
        return model
    return api.Model(rsr_ctx, pm)


def _return_model(rsr_ctx, model):
    rsr_ctx.__dict__.setdefault("_autograd_models", {}).setdefault(
        (model.n, model.K), []).append(model)


class RSRProbability(torch.autograd.Function):
    @staticmethod
    def forward(ctx_, p, refs, system, N, seed, rsr_ctx, stream_id=0, form=A.RSR_AUTO):
        p_cpu = p.detach().to("cpu", torch.float64)
        binary = p_cpu.dim() == 1
        pm = torch.stack([1.0 - p_cpu, p_cpu], dim=1) if binary else p_cpu
        pm = pm / pm.sum(dim=1, keepdim=True)
        model = _take_model(rsr_ctx, pm.contiguous().numpy())
        est, buf = api.stage2(rsr_ctx, model, refs, system, int(N), int(seed), stream_id=stream_id,
                              form=form, grad=False)
        ctx_.rsr = (rsr_ctx, model, buf, int(N), binary)
        return torch.tensor(est["P"], dtype=torch.float64, device=p.device)

    @staticmethod
    def backward(ctx_, grad_out):
        rsr_ctx, model, buf, N, binary = ctx_.rsr
        if binary:
            g = api.rsr_importance(rsr_ctx, model, buf.samples, buf.Y, N).to(torch.float64)
        else:
            g = api.rsr_grad(rsr_ctx, model, buf.samples, buf.Y, N).to(torch.float64)
        # The kernels above are ordered before any later update of the model on
        # the context stream, so it can go back to the pool now.
        _return_model(rsr_ctx, model)
        ctx_.rsr = None
        g = g.to(grad_out.device) * grad_out
        return (g, None, None, None, None, None, None, None)


def rsr_probability(p, refs, system, N, seed, rsr_ctx, stream_id=0, form=A.RSR_AUTO):
    return RSRProbability.apply(p, refs, system, N, seed, rsr_ctx, stream_id, form)
