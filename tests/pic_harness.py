"""Shared helpers for the GPU parity tests: build the oracle and the HIP
context from the same seeded workload, convert state between them, and
measure normwise relative errors.

Inputs flow one way only: workload -> both sides, or oracle -> GPU.  No value
read back from the GPU is ever fed to the oracle.
"""

import numpy as np

from oracle import pic as opic

DT_TOL = {"f64": 1e-10, "f32": 1e-4}


def oracle_params(w, degree, scheme, bdf_order=2, naive=False, jvstar=False, dirk_substep=False):
    return opic.Params(w["nx"], w["ny"], w["lx"], w["ly"], degree, scheme, w["dt"],
                       c=w.get("c", 1.0), eps0=w.get("eps0", 1.0), mu0=w.get("mu0", 1.0),
                       q=w["q"], m=w["m"], bdf_order=bdf_order, naive=naive, jvstar=jvstar,
                       dirk_substep=dirk_substep)


def make_oracle(w, degree, scheme, bdf_order=2, naive=False, jvstar=False, dirk_substep=False):
    p = oracle_params(w, degree, scheme, bdf_order, naive, jvstar, dirk_substep)
    return opic.State(p, w["x"], w["y"], w["P"])


def make_gpu(w, degree, scheme, dtype, bdf_order=2, flags=0, max_particles=None, sort_interval=0):
    import torch
    from paper_2410_18414_amd import pic
    n = w["x"].shape[0]
    cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=degree,
                          scheme=scheme, bdf_order=bdf_order, dtype=dtype,
                          c=w.get("c", 1.0), eps0=w.get("eps0", 1.0), mu0=w.get("mu0", 1.0),
                          q=w["q"], m=w["m"], max_particles=max(1, max_particles or n),
                          flags=flags, sort_interval=sort_interval)
    ctx = pic.Context(cfg)
    dev = ctx.device
    pic.init_particles(ctx, torch.as_tensor(w["x"], device=dev),
                       torch.as_tensor(w["y"], device=dev),
                       torch.as_tensor(np.ascontiguousarray(w["P"].T), device=dev))
    return ctx


def gpu_parts(ctx):
    """GPU particle state as the oracle's dict (float64 numpy, original order)."""
    from paper_2410_18414_amd import pic
    a = pic.get_particles(ctx).cpu().numpy()
    return dict(x=a[0], y=a[1], P=a[2:5].T, v=a[5:8].T, vprev=a[8:11].T)


def set_gpu_parts(ctx, part):
    import torch
    from paper_2410_18414_amd import pic
    a = np.concatenate([part["x"][None], part["y"][None], part["P"].T, part["v"].T,
                        part["vprev"].T])
    pic.set_particles(ctx, torch.as_tensor(a))


def hist_to_flat(p, hist):
    """Oracle history dict -> [nfield, ny, nx/2+1] in pic.h's export order."""
    out = []
    out += list(hist["rho"])
    out += list(hist["phi"])
    if p.scheme in ("dirk2", "dirk3"):
        out.append(hist["vphi"])
    for A in hist["A"]:
        out += [A[0], A[1], A[2]]
    if p.scheme in ("dirk2", "dirk3"):
        out += [hist["vA"][0], hist["vA"][1], hist["vA"][2]]
        out += [hist["J"][0], hist["J"][1], hist["J"][2]]
    if p.scheme in ("cdf2", "cdf2_semi", "cdf2_explicit"):
        for J in hist["J"]:
            out += [J[0], J[1], J[2]]
    return np.stack(out)


def flat_to_hist_bdf(p, flat):
    """[nfield, ny, nx/2+1] in pic.h's BDF-k export order -> oracle history dict."""
    k = p.bdf_order
    flat = np.asarray(flat, np.complex128)
    rho = [flat[j] for j in range(k)]
    phi = [flat[k + j] for j in range(2 * k)]
    A = [np.stack([flat[3 * k + 3 * j + l] for l in range(3)]) for j in range(2 * k)]
    return dict(rho=rho, phi=phi, A=A)


def oracle_from_gpu(p, ctx, w):
    """An oracle State holding the GPU context's particles and BDF-k history
    (promoted to float64)."""
    from paper_2410_18414_amd import pic
    s = opic.State(p, w["x"], w["y"], w["P"])
    a = pic.get_particles(ctx).cpu().numpy()
    s.part = dict(x=a[0].copy(), y=a[1].copy(), P=a[2:5].T.copy(), v=a[5:8].T.copy(), vprev=a[8:11].T.copy())
    s.hist = flat_to_hist_bdf(p, pic.get_history(ctx).cpu().numpy())
    return s


def rel(a, b):
    """Normwise relative error ||a - b||_inf / ||b||_inf (absolute if b == 0)."""
    a, b = np.asarray(a), np.asarray(b)
    s = np.abs(b).max() if b.size else 0.0
    d = np.abs(a - b).max() if b.size else 0.0
    return d / s if s > 0 else d


def rel_periodic(a, b, L):
    """Like rel for positions: differences taken modulo the period L."""
    d = np.asarray(a) - np.asarray(b)
    d = d - L * np.round(d / L)
    return np.abs(d).max() / L if d.size else 0.0


def compare_particles(gp, op, lx, ly, tol):
    errs = dict(x=rel_periodic(gp["x"], op["x"], lx), y=rel_periodic(gp["y"], op["y"], ly),
                P=rel(gp["P"], op["P"]), v=rel(gp["v"], op["v"]), vprev=rel(gp["vprev"], op["vprev"]))
    bad = {k: v for k, v in errs.items() if not v <= tol}
    return errs, bad
