"""torch.autograd.Function over the checkpointed ADER-MOOD forward run and
its hand-written adjoint.

    x_T = LagrangianRun.apply(mu, v_cell, v_node, ctx, workload, nsteps, ckpt_every)

runs `nsteps` CFL-controlled steps from the initial state built from
(mu, v_cell, v_node) and returns the final node positions; backward calls
the library's reverse sweep (dt and cascade choice frozen as recorded) and
returns dL/dmu, dL/dv_cell, dL/dv_node.  All compute happens in
libhyperlag's kernels; the tensors are CUDA float64.
"""
from __future__ import annotations

import torch

from . import hyperlag as H


class LagrangianRun(torch.autograd.Function):
    @staticmethod
    def forward(actx, mu, v_cell, v_node, hctx, workload, nsteps, ckpt_every):
        w = workload
        dev = mu.device
        as_dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev).contiguous()
        hctx.init_state(as_dev(w.rho0), mu.detach().contiguous(), as_dev(w.lam),
                        v_cell.detach().contiguous(), v_node.detach().contiguous(), hctx.params)
        hctx.forward_record(int(nsteps), int(ckpt_every))
        x = torch.empty((w.n_nodes, w.dim), dtype=torch.float64, device=dev)
        hctx.query("x", out=x)
        actx.hctx = hctx
        actx.generation = hctx.record_generation
        return x

    @staticmethod
    def backward(actx, grad_x):
        # the context holds one recorded run: a later forward on the same
        # context replaced the tape this backward would need
        if actx.hctx.record_generation != actx.generation:
            raise RuntimeError("the context recorded another forward run since this one; give each "
                               "differentiated run its own context")
        gmu, gvc, gvn = actx.hctx.adjoint_run(grad_x.contiguous())
        return gmu, gvc, gvn, None, None, None, None


def run(mu, v_cell, v_node, hctx, workload, nsteps, ckpt_every=20):
    return LagrangianRun.apply(mu, v_cell, v_node, hctx, workload, nsteps, ckpt_every)
