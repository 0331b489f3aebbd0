"""torch.autograd wrapper: FEPE as a differentiable function of density scales.

The forward pass runs the score-function transport (gadep_run_grad), which
returns FEPE per energy together with the Jacobian dFEPE/ds estimated from
the same histories; the backward pass applies the chain rule with that
Jacobian.  Torch only carries the tensors.
"""
from __future__ import annotations

import numpy as np
import torch


class GadepFEPE(torch.autograd.Function):
    """fepe = GadepFEPE.apply(scales, engine, job)

    scales: tensor [G] of density scales (one per region scale group)
    engine: a gadep.Context with the scene and cross sections loaded
    job:    dict(source=..., energies=[...], n_histories=N, seed=S[, first_history=0])
    returns tensor [E] (float64) on the device of `scales`
    """

    @staticmethod
    def forward(ctx, scales, engine, job):
        s = scales.detach().to("cpu", torch.float32).numpy()
        r = engine.run_grad(job["source"], job["energies"], job["n_histories"], job["seed"], s,
                            first_history=job.get("first_history", 0))
        fepe = torch.as_tensor(np.asarray(r.fepe()), dtype=torch.float64, device=scales.device)
        jac = torch.as_tensor(r.grad, dtype=torch.float64, device=scales.device)
        ctx.save_for_backward(jac)
        ctx.in_dtype = scales.dtype
        return fepe

    @staticmethod
    def backward(ctx, grad_fepe):
        (jac,) = ctx.saved_tensors
        g = grad_fepe.to(jac.dtype).reshape(1, -1) @ jac
        return g.reshape(-1).to(ctx.in_dtype), None, None


def fepe(scales, engine, job):
    return GadepFEPE.apply(scales, engine, job)
