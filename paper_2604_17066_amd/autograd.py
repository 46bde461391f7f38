"""torch.autograd wrapper: P(S >= level) as a differentiable function of the
component-state probabilities.

Forward runs the Stage-2 hot path (sample, classify, evaluate, estimate) in
the library's kernels; backward calls rsr_grad, whose score-function
estimator gives dP/dp[i][s] = E[Y 1{x_i = s}] / p[i][s] (independent
components make P multilinear in the state probabilities).  For a binary
input p [n] of survival probabilities the state matrix is (1 - p, p), so
dP/dp_i = G[i][1] - G[i][0].
"""
import torch

from . import _abi as A
from . import api


class RSRProbability(torch.autograd.Function):
    @staticmethod
    def forward(ctx_, p, refs, system, N, seed, rsr_ctx, stream_id=0, form=A.RSR_AUTO):
        p_cpu = p.detach().to("cpu", torch.float64)
        binary = p_cpu.dim() == 1
        pm = torch.stack([1.0 - p_cpu, p_cpu], dim=1) if binary else p_cpu
        model = api.Model(rsr_ctx, pm.numpy())
        est, buf = api.stage2(rsr_ctx, model, refs, system, int(N), int(seed), stream_id=stream_id,
                              form=form, grad=False)
        ctx_.rsr = (rsr_ctx, model, buf, int(N), binary)
        return torch.tensor(est["P"], dtype=torch.float64, device=p.device)

    @staticmethod
    def backward(ctx_, grad_out):
        rsr_ctx, model, buf, N, binary = ctx_.rsr
        G = api.rsr_grad(rsr_ctx, model, buf.samples, buf.Y, N).to(torch.float64)
        g = G[:, 1] - G[:, 0] if binary else G
        g = g.to(grad_out.device) * grad_out
        return (g, None, None, None, None, None, None, None)


def rsr_probability(p, refs, system, N, seed, rsr_ctx, stream_id=0, form=A.RSR_AUTO):
    return RSRProbability.apply(p, refs, system, N, seed, rsr_ctx, stream_id, form)
