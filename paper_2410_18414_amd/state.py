"""Checkpoints and diagnostics logs on top of the C ABI (argument marshalling only).

    save_state(ctx, "run.npz")          # particles + spectral history of the selected instance
    load_state(ctx, "run.npz")          # into a context created with the same configuration
    run_logged(ctx, 200, 10, "diag.jsonl")   # step, writing the residuals every 10 steps

A checkpoint holds the particle state [11, n] (x, y, P, v^n, v^{n-1}, float64,
original order), the spectral history in pic.h's export order, and the
configuration fields that must match on load.  Files are plain `numpy.savez`
archives without pickled objects (`numpy.load(..., allow_pickle=False)` reads
them).  With PIC_FLAG_DETERMINISTIC a run resumed from a checkpoint repeats the
uninterrupted run bit for bit.
"""

import json

import numpy as np
import torch

from . import pic

# configuration fields a checkpoint must agree on
_KEYS = ("nx", "ny", "lx", "ly", "spline_degree", "scheme", "bdf_order", "particle_dtype", "dt", "c", "eps0",
         "mu0", "q", "m", "flags")


def _cfg_fields(cfg):
    return {k: getattr(cfg, k) for k in _KEYS}


def save_state(ctx, path):
    """Write the selected instance's particles and spectral history to `path`."""
    cfg = ctx.cfgs[ctx.sel]
    parts = pic.get_particles(ctx).cpu().numpy()
    hist = pic.get_history(ctx).cpu().numpy()
    fields = _cfg_fields(cfg)
    np.savez(path, particles=parts, history=hist,
             config_keys=np.array(list(fields.keys())),
             config_values=np.array([float(v) for v in fields.values()], dtype=np.float64))


def load_state(ctx, path):
    """Load a checkpoint into the selected instance (same configuration)."""
    with np.load(path, allow_pickle=False) as z:
        parts, hist = z["particles"], z["history"]
        saved = dict(zip([str(k) for k in z["config_keys"]], z["config_values"].tolist()))
    cfg = ctx.cfgs[ctx.sel]
    for k, v in _cfg_fields(cfg).items():
        if not np.isclose(saved.get(k, np.nan), float(v), rtol=1e-15, atol=0.0):
            raise ValueError("checkpoint configuration differs in %s: %r vs %r" % (k, saved.get(k), v))
    n = parts.shape[1]
    if n > cfg.max_particles:
        raise ValueError("checkpoint holds %d particles, capacity %d" % (n, cfg.max_particles))
    dev = ctx.device
    # load the count (positions and momenta of the checkpoint), then the full state
    pic.init_particles(ctx, torch.as_tensor(parts[0], device=dev), torch.as_tensor(parts[1], device=dev),
                       torch.as_tensor(np.ascontiguousarray(parts[2:5]), device=dev))
    pic.set_particles(ctx, torch.as_tensor(parts, device=dev))
    pic.set_history(ctx, torch.as_tensor(hist, device=dev))


def run_logged(ctx, nsteps, every, path):
    """Step `nsteps` times, appending the diagnostics (pic.h's residuals,
    charge, energies, as relative residuals too) to the JSON-lines file
    `path` after every `every` steps."""
    done = 0
    with open(path, "a") as f:
        while done < nsteps:
            k = min(every, nsteps - done)
            pic.step(ctx, k)
            done += k
            d = pic.diagnostics(ctx, allow_nonfinite=True)
            rec = dict(step=done, **{key: float(v) for key, v in d.items()})
            rec["gauge_rel"] = d["gauge_l2"] / d["gauge_scale"] if d["gauge_scale"] else 0.0
            rec["gauss_rel"] = d["gauss_l2"] / d["gauss_scale"] if d["gauss_scale"] else 0.0
            f.write(json.dumps(rec) + "\n")
    return done
