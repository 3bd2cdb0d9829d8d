"""Shared helpers for the GPU parity tests: build the oracle and the HIP
context from the same seeded workload, convert state between them, and
measure normwise relative errors.

Inputs come from the seeded workloads, which both sides receive.  The one
exception is shadow stepping (the parity protocol for long float32 runs, whose
chaotic growth amplifies rounding differences beyond the tolerance): there
the oracle is loaded with the GPU's state, promoted to float64
(`oracle_from_gpu`, `shadow_step`), and one step of each is compared.  No
expected value is ever taken from the GPU.
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


def flat_to_hist(p, flat):
    """[nfield, ny, nx/2+1] in pic.h's export order -> oracle history dict
    (every stepper: the inverse of hist_to_flat)."""
    flat = np.asarray(flat, np.complex128)
    if p.scheme == "bdf":
        return flat_to_hist_bdf(p, flat)
    it = iter(range(flat.shape[0]))

    def take(count):
        return [flat[next(it)] for _ in range(count)]

    def take3(levels):
        return [np.stack(take(3)) for _ in range(levels)]
    if p.scheme in ("cdf2", "cdf2_semi", "cdf2_explicit"):
        return dict(rho=take(3), phi=take(3), A=take3(2), J=take3(2))
    h = dict(rho=take(2), phi=take(2))
    h["vphi"] = take(1)[0]
    h["A"] = take3(2)
    h["vA"] = take3(1)[0]
    h["J"] = take3(1)[0]
    return h


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


def _workers():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def chunked_deposit(p, x, y, v, chunks=64):
    """oracle deposit_current over the whole particle set, summed over
    particle chunks deposited on host threads (each chunk is the oracle's own
    float64 deposit; only the order of the final summation differs from one
    pass over all particles)."""
    from concurrent.futures import ThreadPoolExecutor
    n = x.shape[0]
    bounds = [(i * n // chunks, (i + 1) * n // chunks) for i in range(chunks)]
    with ThreadPoolExecutor(_workers()) as ex:
        parts = list(ex.map(lambda b: opic.deposit_current(p, x[b[0]:b[1]], y[b[0]:b[1]], v[b[0]:b[1]]), bounds))
    J = parts[0]
    for q in parts[1:]:
        J = J + q
    return J


def chunked_gather(p, fields, x, y, chunks=32):
    """oracle gather of the mesh fields at the given particles, by chunks on
    host threads (each particle's interpolation is the oracle's own)."""
    from concurrent.futures import ThreadPoolExecutor
    n = x.shape[0]
    bounds = [(i * n // chunks, (i + 1) * n // chunks) for i in range(chunks)]
    with ThreadPoolExecutor(_workers()) as ex:
        parts = list(ex.map(lambda b: opic.gather(p, fields, x[b[0]:b[1]], y[b[0]:b[1]]), bounds))
    return np.concatenate(parts)


def shadow_step(p, x, y, v, hist, sample, P_s, vprev_s):
    """One oracle step (Algorithm 1) from a particle state and history: the
    position update and J deposit over every particle (positions x, y and
    velocities v of all of them), the field update and spectral gradients,
    then the gather and IAEM push of the particles in `sample` only, whose
    momenta P_s and older velocities vprev_s are given (the other particles'
    pushes do not affect any output of this step).  Returns (history after
    the step, particle dict of the sample after the step)."""
    from oracle import spectral
    x1, y1 = opic.position_update(p, x, y, v)
    J = chunked_deposit(p, x1, y1, v)
    Jh = np.stack([spectral.fft2(J[c]) for c in range(3)])
    hist1, phi_t, A = opic.field_update(p, hist, Jh)
    fields = opic.gradient_fields(p, phi_t, A)
    g = chunked_gather(p, fields, x1[sample], y1[sample])
    Pn, vn = opic.push(p, P_s, v[sample], vprev_s, g)
    return hist1, dict(x=x1[sample], y=y1[sample], P=Pn, v=vn, vprev=v[sample])
