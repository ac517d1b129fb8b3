"""Differentiable unrolled ACCORD-FBS: the held-out loss after K fixed-step iterations
as a torch.autograd.Function, with the reverse pass in the library's kernels.

Orchestration only: every step of the forward and reverse pass runs in libaccord
(accord_fit to record the steps, accord_fbs_replay, accord_val_loss_grad,
accord_fbs_adjoint_step); this module chooses checkpoints and moves tensors.

Forward: record the step sizes tau_t with a backtracking fit (Alg. 1) unless they
are given, then replay the K steps with those sizes held fixed, keeping Omega_t
every `checkpoint_every` steps.  Loss: the held-out pseudolikelihood
    l_val(Omega_K) = -sum_j log Omega_jj + ||X_v Omega_K||_F^2 / (2 n_v).
Backward: for each checkpoint segment, last first, replay the segment storing its
iterates, then apply the reverse step from its last iterate back to its first.
Gradients are returned for X (the training data) and lambda; tau_t are constants.
"""
from __future__ import annotations

import torch

from . import accord


class UnrolledValLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X, lam, Xv, iters: int, checkpoint_every: int, taus):
        lam_v = float(lam)
        n, p = X.shape
        ws = torch.empty(max(accord.accord_adjoint_workspace_bytes(max(n, Xv.shape[0]), p), 256),
                         dtype=torch.uint8, device=X.device)
        if taus is None:
            _, _, tr = accord.accord_fit(X, lam_v, iters, trace=True)
            taus = tr[1:, 3].cpu().tolist()
        taus = [float(t) for t in taus][:iters]
        om = torch.eye(p, dtype=torch.float32, device=X.device)
        ckpts = [om.clone()]
        for s in range(0, len(taus), checkpoint_every):
            accord.accord_fbs_replay(X, om, taus[s:s + checkpoint_every], lam_v, ws=ws)
            if s + checkpoint_every < len(taus):
                ckpts.append(om.clone())
        out, obar = accord.accord_val_loss_grad(Xv, om, ws=ws)
        ctx.save_for_backward(X)
        ctx.ckpts, ctx.taus, ctx.lam, ctx.every = ckpts, taus, lam_v, checkpoint_every
        ctx.obar, ctx.ws = obar, ws
        ctx.lam_meta = (lam.dtype, lam.device) if torch.is_tensor(lam) else None
        return out[2].clone()

    @staticmethod
    def backward(ctx, grad_out):
        (X,) = ctx.saved_tensors
        n, p = X.shape
        ws, taus, lam, every = ctx.ws, ctx.taus, ctx.lam, ctx.every
        obar = ctx.obar * float(grad_out)
        lbar = torch.zeros(1, dtype=torch.float64, device=X.device)
        xbar = torch.zeros_like(X)
        seq = torch.empty((every, p, p), dtype=torch.float32, device=X.device)
        starts = list(range(0, len(taus), every))
        for c in range(len(starts) - 1, -1, -1):
            s = starts[c]
            steps = taus[s:s + every]
            om = ctx.ckpts[c].clone()
            accord.accord_fbs_replay(X, om, steps, lam, seq=seq[:len(steps)], ws=ws)
            for k in range(len(steps) - 1, -1, -1):
                # (iterates inside `seq` start p*p floats apart: copy to an aligned tensor)
                om_t = ctx.ckpts[c] if k == 0 else seq[k - 1].clone()
                accord.accord_fbs_adjoint_step(X, om_t, steps[k], lam, obar, lbar, xbar, ws=ws)
        glam = None
        if ctx.lam_meta is not None:
            dtype, device = ctx.lam_meta
            glam = lbar.reshape(()).to(dtype=dtype, device=device)
        return xbar, glam, None, None, None, None


def unrolled_val_loss(X: torch.Tensor, lam, Xv: torch.Tensor, iters: int = 50,
                      checkpoint_every: int = 10, taus=None) -> torch.Tensor:
    """Held-out pseudolikelihood after `iters` FP32 ACCORD-FBS steps on X (steps
    recorded by a backtracking fit unless `taus` is given, then held fixed).
    Differentiable with respect to X and lambda (a 0-dim tensor)."""
    return UnrolledValLoss.apply(X, lam, Xv, iters, checkpoint_every, taus)
