"""Reverse-mode gradients through the HIP path (torch.autograd.Function).

    ctx = pic.Context(pic.make_config(..., dtype="f64", scheme="bdf",
                                      flags=pic.FLAG_ADJOINT, max_particles=n))
    W = field_energy(ctx, x0, y0, P0, nsteps=20, every=5)   # 0-dim tensor
    W.backward()                                             # x0.grad, y0.grad, P0.grad

The forward runs `nsteps` steps from the cold start of init_particles and
returns the field energy of the final level (pic_diagnostics out[5]).  The
backward walks the run in reverse with libpic's discrete adjoint
(adjoint_seed_energy, step_adjoint, adjoint_initial): the state is kept every
`every` steps during the forward (checkpoints: pic_save_state, the context's
raw device state -- particles in their sorted order, tile metadata, history
ring); each segment is replayed forward from its checkpoint, step by step as
deposit_current, field_solve and gather_push, saving the state after each
solve (phase SOLVED: the new positions and fields step_adjoint needs,
so it recomputes nothing) into a pool of saved states (the last one stays in
the context); then the adjoint steps through the segment backwards, loading
each state with pic_load_state_h (no conversion and no re-sort; the header
kept on the host, so no synchronisation); the particle adjoint stays inside
the context in slot order for the whole sweep.  every=1 keeps every state,
saved after its step's deposit and solve (no replay, no recompute).  Only
argument marshalling happens here: every step and every adjoint step runs in
the library's kernels.
"""

import torch

from . import pic


class _FieldEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x0, y0, P0, ctx, nsteps, every):
        pic.init_particles(ctx, x0.detach(), y0.detach(), P0.detach())
        ckpts = []
        if every == 1:
            # every state kept, each after its step's deposit and solve (phase
            # SOLVED), so the adjoint steps recompute nothing
            for s in range(nsteps):
                pic.deposit_current(ctx)
                pic.field_solve(ctx)
                ckpts.append((s, pic.save_state(ctx)))
                pic.gather_push(ctx)
        else:
            s = 0
            while s < nsteps:
                ckpts.append((s, pic.save_state(ctx)))
                k = min(every, nsteps - s)
                pic.step(ctx, k)
                s += k
        final = pic.save_state(ctx)
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
        # the seed needs the final history loaded
        pic.load_state(ctx, fctx.final, trust_header=True)
        pic.adjoint_set_particles(ctx, None)  # the particle adjoint of W is zero
        lam_hist = pic.adjoint_seed_energy(ctx, float(gW))
        # each segment is replayed from its checkpoint; the state after each
        # step's deposit and solve goes into a pool of saved states
        pool = []
        for s0, ck in reversed(fctx.ckpts):
            if fctx.every == 1:  # a solved state per step: no replay
                pic.load_state(ctx, ck, trust_header=True)
                pic.step_adjoint(ctx, None, lam_hist)
                continue
            seg = min(fctx.every, fctx.nsteps - s0)
            pic.load_state(ctx, ck, trust_header=True)
            states = []
            for j in range(seg):
                pic.deposit_current(ctx)
                pic.field_solve(ctx)
                if j < seg - 1:  # the segment's last solved state stays in the context
                    if len(pool) <= j:
                        pool.append(pic.State(ctx))
                    states.append(pic.save_state(ctx, pool[j]))
                    pic.gather_push(ctx)
            pic.step_adjoint(ctx, None, lam_hist)
            for st in reversed(states):
                pic.load_state(ctx, st, trust_header=True)
                pic.step_adjoint(ctx, None, lam_hist)
        lam = pic.adjoint_get_particles(ctx)
        pic.adjoint_initial(ctx, P0.detach(), lam)
        return lam[0].clone(), lam[1].clone(), lam[2:5].clone(), None, None, None


def field_energy(ctx, x0, y0, P0, nsteps, every=5):
    """Field energy after `nsteps` steps from (x0 [n], y0 [n], P0 [3, n]),
    differentiable with respect to all three (float64 device tensors)."""
    if nsteps < 1 or every < 1:
        raise ValueError("nsteps and every must be >= 1")
    return _FieldEnergy.apply(x0, y0, P0, ctx, int(nsteps), int(every))
