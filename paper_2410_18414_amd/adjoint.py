"""Reverse-mode gradients through the HIP path (torch.autograd.Function).

    ctx = pic.Context(pic.make_config(..., dtype="f64", scheme="bdf",
                                      flags=pic.FLAG_ADJOINT, max_particles=n))
    W = field_energy(ctx, x0, y0, P0, nsteps=20, every=5)   # 0-dim tensor
    W.backward()                                             # x0.grad, y0.grad, P0.grad

The forward runs `nsteps` steps from the cold start of init_particles and
returns the field energy of the final level (pic_diagnostics out[5]).  The
backward walks the run in reverse with libpic's discrete adjoint
(adjoint_seed_energy, step_adjoint, adjoint_initial): the state is kept every
`every` steps during the forward (checkpoints: particles + spectral history);
each segment is replayed forward from its checkpoint to recover the states
inside it, then the adjoint steps through the segment backwards.  every=1
stores every state (no replay).  Only argument marshalling happens here:
every step and every adjoint step runs in the library's kernels.
"""

import torch

from . import pic


class _FieldEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x0, y0, P0, ctx, nsteps, every):
        pic.init_particles(ctx, x0.detach(), y0.detach(), P0.detach())
        ckpts = []
        s = 0
        while s < nsteps:
            ckpts.append((s, pic.get_particles(ctx), pic.get_history(ctx)))
            k = min(every, nsteps - s)
            pic.step(ctx, k)
            s += k
        final = (pic.get_particles(ctx), pic.get_history(ctx))
        W = pic.diagnostics(ctx)["energy"]
        fctx.sim = ctx
        fctx.ckpts = ckpts
        fctx.final = final
        fctx.nsteps = nsteps
        fctx.every = every
        fctx.save_for_backward(P0)
        return torch.tensor(W, dtype=torch.float64, device=x0.device)

    @staticmethod
    def backward(fctx, gW):
        ctx = fctx.sim
        (P0,) = fctx.saved_tensors
        n = ctx.n
        # the seed needs the final history loaded
        pic.set_particles(ctx, fctx.final[0])
        pic.set_history(ctx, fctx.final[1])
        lam = torch.zeros((11, n), dtype=torch.float64, device=ctx.device)
        lam_hist = pic.adjoint_seed_energy(ctx, float(gW))
        for s0, parts, hist in reversed(fctx.ckpts):
            seg = min(fctx.every, fctx.nsteps - s0)
            states = [(parts, hist)]
            if seg > 1:
                pic.set_particles(ctx, parts)
                pic.set_history(ctx, hist)
                for _ in range(1, seg):
                    pic.step(ctx, 1)
                    states.append((pic.get_particles(ctx), pic.get_history(ctx)))
            for parts_j, hist_j in reversed(states):
                pic.set_particles(ctx, parts_j)
                pic.set_history(ctx, hist_j)
                pic.step_adjoint(ctx, lam, lam_hist)
        pic.adjoint_initial(ctx, P0.detach(), lam)
        return lam[0].clone(), lam[1].clone(), lam[2:5].clone(), None, None, None


def field_energy(ctx, x0, y0, P0, nsteps, every=5):
    """Field energy after `nsteps` steps from (x0 [n], y0 [n], P0 [3, n]),
    differentiable with respect to all three (float64 device tensors)."""
    if nsteps < 1 or every < 1:
        raise ValueError("nsteps and every must be >= 1")
    return _FieldEnergy.apply(x0, y0, P0, ctx, int(nsteps), int(every))
