"""Seeded synthetic particle inputs for the workloads (no method arithmetic).

Only sampling lives here: positions and momenta of one species of
macro-electrons, plus the physical constants of the run.  Both the HIP path
and the FP64 test oracle receive the same arrays; neither module's arithmetic
is in this file.

Units are normalised: c = eps0 = mu0 = 1, the electron plasma frequency of the
mean density is 1, electron q/m = -1.  With N_p macro-particles on an
lx * ly box, omega_pe^2 = n q^2 / (eps0 m) = 1 gives the macro charge
q = -lx*ly/N_p and mass m = lx*ly/N_p.  The time step is dt = 0.5 dx / c.

Workload shapes (the paper's experiments use no dataset; these stand in for
the drifting electron cloud of Sec. 5.2 and the anisotropic relativistic
Weibel setup of Sec. 5.1):

  cloud     -- Gaussian cloud N(L/2, (0.1 L)^2) per axis, proper velocity
               u = (0.1c, 0.1c, 0) + N(0, (0.01c)^2) in x and y, u_z = 0.
  weibel    -- uniform positions; bi-Maxwellian proper velocity with
               sigma_z = 0.3c hot and sigma_x = sigma_y = 0.3c/sqrt(a),
               anisotropy a = T_z/T_x = 25; an optional counter-streaming
               drift +-u_d along x on alternate particles.
"""

import numpy as np


def _box(nx, ny, dx):
    return dict(nx=int(nx), ny=int(ny), lx=nx * dx, ly=ny * dx, dt=0.5 * dx)


def _species(lx, ly, n):
    w = lx * ly / n
    return dict(q=-w, m=w, c=1.0, eps0=1.0, mu0=1.0)


def cloud(nx=32, ny=32, ppc=4, seed=1001, L=1.0, sigma=0.1, drift=0.1, vth=0.01):
    """Drifting Gaussian electron cloud on a fixed neutralising background."""
    rng = np.random.default_rng(seed)
    n = nx * ny * ppc
    box = dict(nx=nx, ny=ny, lx=L, ly=L * ny / nx, dt=0.5 * L / nx)
    x = np.mod(rng.normal(0.5 * box["lx"], sigma * box["lx"], n), box["lx"])
    y = np.mod(rng.normal(0.5 * box["ly"], sigma * box["ly"], n), box["ly"])
    u = np.zeros((n, 3))
    u[:, 0] = drift + vth * rng.standard_normal(n)
    u[:, 1] = drift + vth * rng.standard_normal(n)
    sp = _species(box["lx"], box["ly"], n)
    return dict(box, **sp, x=x, y=y, P=sp["m"] * u, seed=seed, name="cloud")


def weibel_normals(nx, ny, ppc, seed):
    """The fixed normals (xi) and positions of the anisotropic workload."""
    rng = np.random.default_rng(seed)
    n = nx * ny * ppc
    pos = rng.random((2, n))
    xi = rng.standard_normal((n, 3))
    return pos, xi


def weibel(nx=128, ny=128, ppc=64, seed=1002, dx=0.1, vth=0.3, aniso=25.0, drift=0.0):
    """Anisotropic bi-Maxwellian (T_z/T_x = aniso), uniform in space."""
    box = _box(nx, ny, dx)
    pos, xi = weibel_normals(nx, ny, ppc, seed)
    n = pos.shape[1]
    x = pos[0] * box["lx"]
    y = pos[1] * box["ly"]
    u = np.empty((n, 3))
    sgn = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    u[:, 0] = sgn * drift + vth / np.sqrt(aniso) * xi[:, 0]
    u[:, 1] = vth / np.sqrt(aniso) * xi[:, 1]
    u[:, 2] = vth * xi[:, 2]
    sp = _species(box["lx"], box["ly"], n)
    return dict(box, **sp, x=x, y=y, P=sp["m"] * u, seed=seed, name="weibel")


def maxwellian_cloud(nx, ny, ppc, seed, dx=0.1, sigma=0.1, vth=0.05):
    """Isotropic Maxwellian Gaussian cloud (ensemble members)."""
    rng = np.random.default_rng(seed)
    box = _box(nx, ny, dx)
    n = nx * ny * ppc
    x = np.mod(rng.normal(0.5 * box["lx"], sigma * box["lx"], n), box["lx"])
    y = np.mod(rng.normal(0.5 * box["ly"], sigma * box["ly"], n), box["ly"])
    u = vth * rng.standard_normal((n, 3))
    sp = _species(box["lx"], box["ly"], n)
    return dict(box, **sp, x=x, y=y, P=sp["m"] * u, seed=seed, name="mcloud")


def ensemble(count=64, draw_seed=4999, seed_base=4000, sizes=(32, 64, 128, 256), ppc_range=(4, 64)):
    """The uneven ensemble: `count` Maxwellian clouds (sigma = 0.1 L, v_th =
    0.05c) whose grid sides are drawn independently from `sizes` (a tuple of
    sides, or a (lo, hi) range given as a slice for uniform integers in
    [lo, hi]) and whose particles per cell are uniform integers in
    `ppc_range`; the draws use `draw_seed`, member i samples its particles
    with seed seed_base + i."""
    rng = np.random.default_rng(draw_seed)
    if isinstance(sizes, slice):
        nx = rng.integers(sizes.start, sizes.stop + 1, count)
        ny = rng.integers(sizes.start, sizes.stop + 1, count)
    else:
        nx = rng.choice(sizes, count)
        ny = rng.choice(sizes, count)
    ppc = rng.integers(ppc_range[0], ppc_range[1] + 1, count)
    return [maxwellian_cloud(int(nx[i]), int(ny[i]), int(ppc[i]), seed_base + i, dx=0.1, sigma=0.1, vth=0.05)
            for i in range(count)]


# The named workloads: (generator, kwargs, spline degree, stepper, BDF order,
# particle precision, steps).
CONFIGS = {
    "cloud32": dict(gen="cloud", kw=dict(nx=32, ny=32, ppc=4, seed=1001), degree=2,
                    scheme="bdf", bdf_order=1, dtype="f64", steps=50),
    "weibel128": dict(gen="weibel", kw=dict(nx=128, ny=128, ppc=64, seed=1002), degree=3,
                      scheme="bdf", bdf_order=2, dtype="f32", steps=200),
    "weibel512": dict(gen="weibel", kw=dict(nx=512, ny=512, ppc=256, seed=1003), degree=3,
                      scheme="dirk2", bdf_order=2, dtype="f32", steps=100),
    "weibel128-drift": dict(gen="weibel", kw=dict(nx=128, ny=128, ppc=64, seed=1005, drift=0.1),
                            degree=3, scheme="bdf", bdf_order=2, dtype="f64", steps=20),
}


def make(name, **override):
    cfg = dict(CONFIGS[name])
    kw = dict(cfg["kw"], **override)
    gen = {"cloud": cloud, "weibel": weibel}[cfg["gen"]]
    out = gen(**kw)
    out.update(degree=cfg["degree"], scheme=cfg["scheme"],
               bdf_order=cfg["bdf_order"], dtype=cfg["dtype"], steps=cfg["steps"])
    return out
