"""Seeded synthetic workloads (problem descriptions and initial conditions).

This module holds no arithmetic of the numerical method: it only builds the
plain problem description (grid, system, boundary conditions, coefficients)
and the initial state on the host in FP64 with numpy.  Both the GPU library's
binding and the CPU oracle consume what it returns, so the two sides always
start from the same bytes.

Initial conditions are point values at cell centres; random draws come from
``numpy.random.default_rng(seed)`` (PCG64).  For single-precision runs the
initial state is rounded to FP32 once and the oracle starts from those
rounded values.

The problem description is a dict:

    ndim, n (nx, ny, nz), lower, upper           grid (x fastest in memory)
    system   "acoustics" | "shallow_water" | "burgers"
    meqn     acoustics 1 + ndim (p, u, v[, w]); shallow water 3 (h, hu, hv);
             Burgers 1
    coef     Burgers: flux coefficient per direction (flux coef_d q^2 / 2)
    solver   "builtin" (default) or "generic": the GPU library solves shallow
             water through its point-wise plug-in interface instead of its
             specialised sweep
    limiter  "mc" | "none" (phi = 1) | "first_order"
    efix     shallow water entropy fix on/off
    bc_lo, bc_hi   per direction "extrap" | "wall" | "periodic"
    rho, bulk      acoustics coefficients when has_aux is False
    has_aux        acoustics: per-cell (rho, K) given in aux[2, nz, ny, nx]
    grav           shallow water gravity
    cfl_desired, cfl_max, dt_max, nsteps, dtype
"""
import math

import numpy as np

__all__ = ["problem", "CONFIGS", "cell_centers", "round_to", "random_states"]


def _base(ndim, n, lower, upper, system, meqn, bc, **kw):
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    prob = {
        "ndim": ndim,
        "n": n,
        "lower": tuple(float(v) for v in lower) + (0.0,) * (3 - len(lower)),
        "upper": tuple(float(v) for v in upper) + (1.0,) * (3 - len(upper)),
        "system": system,
        "meqn": meqn,
        "limiter": "mc",
        "efix": True,
        "bc_lo": (bc,) * 3,
        "bc_hi": (bc,) * 3,
        "rho": 1.0,
        "bulk": 1.0,
        "grav": 1.0,
        "has_aux": False,
        "cfl_desired": 0.9,
        "cfl_max": 1.0,
        "dt_max": float("inf"),
        "nsteps": 1,
        "dtype": "f64",
    }
    prob.update(kw)
    return prob


def cell_centers(prob):
    """Cell-centre coordinate arrays (x, y, z), each shaped (nz, ny, nx)."""
    nx, ny, nz = prob["n"]
    axes = []
    for k, m in enumerate((nx, ny, nz)):
        lo, hi = prob["lower"][k], prob["upper"][k]
        dx = (hi - lo) / m
        axes.append(lo + (np.arange(m, dtype=np.float64) + 0.5) * dx)
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return x, y, z


def round_to(q, dtype):
    """The initial state as the given precision sees it, returned in FP64."""
    if dtype in ("f32", np.float32):
        return np.ascontiguousarray(q, dtype=np.float32).astype(np.float64)
    return np.ascontiguousarray(q, dtype=np.float64)


def acoustics2d_pulse(n=128, dtype="f64", nsteps=100):
    """2D linear acoustics, 128 x 128 on [0,1]^2, rho = 1, K = 4 (c = 2),
    p0 = exp(-((x-.5)^2 + (y-.5)^2) / 0.01), u = v = 0, extrapolation
    boundaries, MC limiter, CFL 0.9, 100 steps."""
    prob = _base(2, (n, n), (0, 0), (1, 1), "acoustics", 3, "extrap", rho=1.0, bulk=4.0,
                 nsteps=nsteps, dtype=dtype, name="acoustics2d_pulse")
    x, y, _ = cell_centers(prob)
    q = np.zeros((3,) + x.shape)
    q[0] = np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2) / 0.01)
    return prob, round_to(q, dtype), None


def sw_radial_dam(n=2048, dtype="f32", nsteps=1000, noise=True, seed=0, h_in=2.0, h_out=1.0):
    """2D shallow water, n x n on [-2.5, 2.5]^2, g = 1; radial dam break
    h = h_in (2) for r < 0.5 else h_out (1), plus seeded U(-1e-3, 1e-3) per
    cell on h (drawn in memory order, y-major); hu = hv = 0; reflecting walls,
    CFL 0.9.  With h_in = 1, h_out = 0.1 the outflow is supercritical and the
    rarefactions are transonic in both directions (1-waves on the far side of
    the centre, 3-waves on the near side)."""
    prob = _base(2, (n, n), (-2.5, -2.5), (2.5, 2.5), "shallow_water", 3, "wall", grav=1.0,
                 nsteps=nsteps, dtype=dtype, name="sw_radial_dam", seed=seed, noise=noise)
    x, y, _ = cell_centers(prob)
    r = np.sqrt(x * x + y * y)
    q = np.zeros((3,) + x.shape)
    q[0] = np.where(r < 0.5, float(h_in), float(h_out))
    if noise:
        rng = np.random.default_rng(seed)
        q[0] += rng.uniform(-1e-3, 1e-3, size=x.shape)
    return prob, round_to(q, dtype), None


def acoustics3d_layers(n=256, dtype="f32", nsteps=200, seed=0):
    """3D linear acoustics, n^3 on [0,1]^3, q = (p, u, v, w); two-layer medium
    rho = 1, K = 1 for z < 0.5 and rho = 4, K = 1 above (by cell centre);
    p = exp(-|x - x0|^2 / 0.05^2) with x0 ~ U[0.2, 0.8]^3 (seeded);
    extrapolation boundaries, 200 steps."""
    prob = _base(3, (n, n, n), (0, 0, 0), (1, 1, 1), "acoustics", 4, "extrap", has_aux=True,
                 nsteps=nsteps, dtype=dtype, name="acoustics3d_layers", seed=seed)
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.2, 0.8, size=3)
    x, y, z = cell_centers(prob)
    q = np.zeros((4,) + x.shape)
    q[0] = np.exp(-((x - x0[0]) ** 2 + (y - x0[1]) ** 2 + (z - x0[2]) ** 2) / 0.05 ** 2)
    aux = np.empty((2,) + x.shape)
    aux[0] = np.where(z < 0.5, 1.0, 4.0)
    aux[1] = 1.0
    prob["x0"] = tuple(float(v) for v in x0)
    return prob, round_to(q, dtype), round_to(aux, dtype)


def sw_ensemble(count=256, seed=0, nmin=128, nmax=1024, dtype="f32", nsteps=500, sides=None):
    """Ensemble of 2D shallow-water problems on [0,1]^2 (L = 1), reflecting
    walls, g = 1, MC, CFL 0.9: side n_k ~ U{nmin..nmax}, hump
    h = 1 + A exp(-r^2 / w^2) with A ~ U[0.1, 0.5], centre ~ U[0.25, 0.75]^2,
    w ~ U[0.05, 0.2] L, zero momentum; all draws from default_rng(seed) in the
    order sides, A, centres, widths.  Returns a list of (prob, q0)."""
    rng = np.random.default_rng(seed)
    if sides is None:
        sides = rng.integers(nmin, nmax + 1, size=count)
    else:
        sides = np.asarray(sides)
        count = len(sides)
    amp = rng.uniform(0.1, 0.5, size=count)
    centre = rng.uniform(0.25, 0.75, size=(count, 2))
    width = rng.uniform(0.05, 0.2, size=count)
    out = []
    for k in range(count):
        n = int(sides[k])
        prob = _base(2, (n, n), (0, 0), (1, 1), "shallow_water", 3, "wall", grav=1.0,
                     nsteps=nsteps, dtype=dtype, name="sw_ensemble", member=k)
        x, y, _ = cell_centers(prob)
        q = np.zeros((3,) + x.shape)
        r2 = (x - centre[k, 0]) ** 2 + (y - centre[k, 1]) ** 2
        q[0] = 1.0 + amp[k] * np.exp(-r2 / width[k] ** 2)
        out.append((prob, round_to(q, dtype)))
    return out


def sw_hump(n=1024, seed=0, dtype="f32", nsteps=500):
    """One member of the Gaussian-hump family of sw_ensemble at a given side n
    (training and evaluation runs of the learned coarse correction): A, centre
    and w drawn from default_rng(seed) in that order, same ranges, walls, g = 1."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.1, 0.5)
    centre = rng.uniform(0.25, 0.75, size=2)
    width = rng.uniform(0.05, 0.2)
    prob = _base(2, (n, n), (0, 0), (1, 1), "shallow_water", 3, "wall", grav=1.0,
                 nsteps=nsteps, dtype=dtype, name="sw_hump", seed=seed)
    x, y, _ = cell_centers(prob)
    q = np.zeros((3,) + x.shape)
    q[0] = 1.0 + amp * np.exp(-((x - centre[0]) ** 2 + (y - centre[1]) ** 2) / width ** 2)
    return prob, round_to(q, dtype), None


def burgers2d(n=1024, seed=0, dtype="f64", nsteps=200, coef=(1.0, 0.5), bc="periodic",
              nbumps=4):
    """2D scalar Burgers-type law q_t + (c_x q^2/2)_x + (c_y q^2/2)_y = 0 on
    [0,1]^2, periodic, MC, CFL 0.9: q0 = 0.1 + sum of nbumps Gaussians
    A exp(-r^2 / w^2) with A ~ U[-1, 1], centre ~ U[0.2, 0.8]^2,
    w ~ U[0.05, 0.15], drawn from default_rng(seed) in that order per bump.
    Signs of q change across the domain, so shocks, rarefactions and transonic
    rarefactions all occur."""
    prob = _base(2, (n, n), (0, 0), (1, 1), "burgers", 1, bc, coef=tuple(float(c) for c in coef)
                 + (0.0,) * (3 - len(coef)), nsteps=nsteps, dtype=dtype, name="burgers2d", seed=seed)
    rng = np.random.default_rng(seed)
    x, y, _ = cell_centers(prob)
    q = np.full((1,) + x.shape, 0.1)
    for _ in range(nbumps):
        a = rng.uniform(-1.0, 1.0)
        c = rng.uniform(0.2, 0.8, size=2)
        w = rng.uniform(0.05, 0.15)
        q[0] += a * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / w ** 2)
    return prob, round_to(q, dtype), None


def burgers3d(n=64, seed=0, dtype="f64", nsteps=50, coef=(1.0, 0.5, -0.75), bc="periodic"):
    """The 3D analogue of burgers2d on [0,1]^3 with three signed bumps."""
    prob = _base(3, (n, n, n), (0, 0, 0), (1, 1, 1), "burgers", 1, bc,
                 coef=tuple(float(c) for c in coef), nsteps=nsteps, dtype=dtype, name="burgers3d",
                 seed=seed)
    rng = np.random.default_rng(seed)
    x, y, z = cell_centers(prob)
    q = np.full((1,) + x.shape, 0.1)
    for _ in range(3):
        a = rng.uniform(-1.0, 1.0)
        c = rng.uniform(0.2, 0.8, size=3)
        w = rng.uniform(0.08, 0.2)
        q[0] += a * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / w ** 2)
    return prob, round_to(q, dtype), None


def lc_init_params(seed=0, hidden=64, nin=12, nout=3, out_gain=0.1):
    """Seeded initial parameters of the two correction networks (x faces,
    then y faces), each 12-64-64-3 and flat in the order W1 (64, 12), b1,
    W2 (64, 64), b2, W3 (3, 64), b3: weights normal with standard deviation
    sqrt(2 / fan_in) (the last layer scaled by out_gain), biases zero; drawn
    from default_rng(seed), x network first; rounded to FP32, returned in FP64."""
    rng = np.random.default_rng(seed)
    nets = []
    for _ in range(2):
        w1 = rng.normal(0.0, math.sqrt(2.0 / nin), size=(hidden, nin))
        w2 = rng.normal(0.0, math.sqrt(2.0 / hidden), size=(hidden, hidden))
        w3 = rng.normal(0.0, out_gain * math.sqrt(2.0 / hidden), size=(nout, hidden))
        nets.append(np.concatenate([w1.ravel(), np.zeros(hidden), w2.ravel(), np.zeros(hidden),
                                    w3.ravel(), np.zeros(nout)]))
    return np.concatenate(nets).astype(np.float32).astype(np.float64)


def lc_norm(mu_h=1.0, sl=(0.1, 0.03, 0.03), sd1=(1e-3, 3e-4, 3e-4), sd2=(6e-5, 1.5e-5, 1.5e-5),
            sd3=(4e-6, 1e-6, 1e-6), s_out=(1e-4, 1e-4, 1e-4)):
    """Input and output scales of the correction network (a plain dict): per
    channel (h, m_n, m_t) the scales of the stencil's level, slope, curvature
    and third difference, and of the outputs.  The defaults are the typical
    magnitudes over the Gaussian-hump family at side 512, the same for both
    momentum channels and kept well above FP32 rounding of the states."""
    t = lambda v: tuple(float(x) for x in v)  # noqa: E731
    return {"mu_h": float(mu_h), "sl": t(sl), "sd1": t(sd1), "sd2": t(sd2), "sd3": t(sd3), "s_out": t(s_out)}


def problem(name, **kw):
    """(prob, q0, aux) for a named workload; keyword arguments override sizes."""
    return CONFIGS[name](**kw)


CONFIGS = {
    "acoustics2d_pulse": acoustics2d_pulse,
    "sw_radial_dam": sw_radial_dam,
    "acoustics3d_layers": acoustics3d_layers,
    "burgers2d": burgers2d,
    "burgers3d": burgers3d,
}


def random_states(system, count, seed, meqn=3, depth=(0.5, 2.0), vel=0.5):
    """Seeded random valid cell states (count, meqn) for interface-level tests:
    shallow water depths in the given range and velocities up to vel (with
    depth (0.1, 2) and vel 2 many neighbouring pairs are transonic); acoustics
    pressures and velocities in [-1, 1]."""
    rng = np.random.default_rng(seed)
    if system == "shallow_water":
        h = rng.uniform(depth[0], depth[1], size=count)
        u = rng.uniform(-vel, vel, size=count)
        v = rng.uniform(-vel, vel, size=count)
        return np.stack([h, h * u, h * v], axis=1)
    return rng.uniform(-1.0, 1.0, size=(count, meqn))


def dx_of(prob, k):
    return (prob["upper"][k] - prob["lower"][k]) / prob["n"][k]


def cell_count(prob):
    return int(math.prod(prob["n"]))
