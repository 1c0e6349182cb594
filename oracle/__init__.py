"""CPU oracle of the dimension-split wave-propagation step (TEST INFRASTRUCTURE).

A thin ctypes wrapper over ``liboracle.so`` (plain FP64 C, see claw_oracle.c).
Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package; the product library never does.

Problems are described by the plain dict of ``paper_1805_08846_amd.inputs``
(grid, system, limiter, boundary conditions, coefficients); states are numpy
arrays ``q[meqn, nz, ny, nx]`` and ``aux[2, nz, ny, nx]`` (rho, K).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))

_SYSTEM = {"acoustics": 0, "shallow_water": 1, "burgers": 2}
_BC = {"extrap": 0, "wall": 1, "periodic": 2}
_LIM = {"mc": 0, "none": 1, "first_order": 2, "minmod": 3, "superbee": 4, "vanleer": 5}

STATUS = {0: "ok", 1: "invalid description", 5: "non-physical state", 6: "step control failed"}


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where}: {STATUS.get(code, code)} (code {code})")
        self.code = code


class _Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_long * 3),
        ("lower", ctypes.c_double * 3),
        ("upper", ctypes.c_double * 3),
        ("meqn", ctypes.c_int),
        ("system", ctypes.c_int),
        ("limiter", ctypes.c_int),
        ("efix", ctypes.c_int),
        ("bc_lo", ctypes.c_int * 3),
        ("bc_hi", ctypes.c_int * 3),
        ("has_aux", ctypes.c_int),
        ("rho", ctypes.c_double),
        ("bulk", ctypes.c_double),
        ("grav", ctypes.c_double),
        ("splitting", ctypes.c_int),
        ("coef", ctypes.c_double * 3),
    ]


_libs = {}
_dp = ctypes.POINTER(ctypes.c_double)


def _lib(precision="f64"):
    if precision not in _libs:
        _build.ensure_built()
        name = "liboracle.so" if precision == "f64" else "liboracle_f32.so"
        lib = ctypes.CDLL(os.path.join(_HERE, name))
        vp = ctypes.c_void_p
        lib.oracle_mc_phi.restype = ctypes.c_double
        lib.oracle_mc_phi.argtypes = [ctypes.c_double]
        lib.oracle_phi.restype = ctypes.c_double
        lib.oracle_phi.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.oracle_riemann_acoustics.argtypes = [vp, vp] + [ctypes.c_double] * 4 + [
            ctypes.c_int, ctypes.c_int, vp, vp, vp, vp]
        lib.oracle_riemann_sw.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                          vp, vp, vp, vp]
        lib.oracle_riemann_burgers.argtypes = [ctypes.c_double] * 3 + [vp] * 4
        lib.oracle_sweep.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_double, vp, vp]
        lib.oracle_step.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp, vp]
        lib.oracle_speeds.argtypes = [vp, vp, vp, vp]
        lib.oracle_advance.argtypes = [vp, vp, vp, ctypes.c_long, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       vp, vp, vp, vp, ctypes.c_long]
        lib.oracle_advance_fixed.argtypes = [vp, vp, vp, ctypes.c_long, vp, vp]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _libs[precision] = lib
    return _libs[precision]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def make_desc(prob):
    d = _Desc()
    d.ndim = int(prob["ndim"])
    n = list(prob["n"]) + [1] * (3 - len(prob["n"]))
    for k in range(3):
        d.n[k] = int(n[k])
        d.lower[k] = float(prob["lower"][k]) if k < len(prob["lower"]) else 0.0
        d.upper[k] = float(prob["upper"][k]) if k < len(prob["upper"]) else 1.0
        d.bc_lo[k] = _BC[prob["bc_lo"][k]] if k < len(prob["bc_lo"]) else 0
        d.bc_hi[k] = _BC[prob["bc_hi"][k]] if k < len(prob["bc_hi"]) else 0
    d.meqn = int(prob["meqn"])
    d.system = _SYSTEM[prob["system"]]
    d.limiter = _LIM[prob.get("limiter", "mc")]
    d.splitting = {"godunov": 0, "strang": 1}[prob.get("splitting", "godunov")]
    d.efix = 1 if prob.get("efix", True) else 0
    d.has_aux = 1 if prob.get("has_aux", False) else 0
    d.rho = float(prob.get("rho", 1.0))
    d.bulk = float(prob.get("bulk", 1.0))
    d.grav = float(prob.get("grav", 1.0))
    coef = tuple(prob.get("coef", (1.0, 1.0, 1.0))) + (0.0,) * 3
    for k in range(3):
        d.coef[k] = float(coef[k])
    return d


def _state(prob, q):
    n = list(prob["n"]) + [1] * (3 - len(prob["n"]))
    shape = (int(prob["meqn"]), n[2], n[1], n[0])
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(shape)
    return q


def _aux(prob, aux):
    if not prob.get("has_aux", False):
        return None
    return np.ascontiguousarray(aux, dtype=np.float64)


def num_threads(precision="f64"):
    return _lib(precision).oracle_num_threads()


def set_num_threads(n, precision="f64"):
    _lib(precision).oracle_set_num_threads(int(n))


def mc_phi(theta, precision="f64"):
    return _lib(precision).oracle_mc_phi(float(theta))


def phi(limiter, theta, precision="f64"):
    """phi(theta) of a named limiter ("mc", "minmod", "superbee", "vanleer", "none", "first_order")."""
    return _lib(precision).oracle_phi(_LIM[limiter], float(theta))


def riemann_acoustics(ql, qr, Zl, cl, Zr, cr, normal, precision="f64"):
    """Waves (2, meqn), speeds (2,), A-dQ, A+dQ for one acoustics interface."""
    ql = np.ascontiguousarray(ql, dtype=np.float64)
    qr = np.ascontiguousarray(qr, dtype=np.float64)
    meqn = ql.size
    W = np.zeros((2, meqn))
    s = np.zeros(2)
    am = np.zeros(meqn)
    ap = np.zeros(meqn)
    rc = _lib(precision).oracle_riemann_acoustics(_ptr(ql), _ptr(qr), Zl, cl, Zr, cr, meqn,
                                                  normal, _ptr(W), _ptr(s), _ptr(am), _ptr(ap))
    if rc:
        raise OracleError(rc, "riemann_acoustics")
    return W, s, am, ap


def riemann_sw(ql, qr, grav, normal, efix=True, precision="f64"):
    """Waves (3, 3), speeds (3,), A-dQ, A+dQ for one shallow-water interface."""
    ql = np.ascontiguousarray(ql, dtype=np.float64)
    qr = np.ascontiguousarray(qr, dtype=np.float64)
    W = np.zeros((3, 3))
    s = np.zeros(3)
    am = np.zeros(3)
    ap = np.zeros(3)
    rc = _lib(precision).oracle_riemann_sw(_ptr(ql), _ptr(qr), grav, normal, 1 if efix else 0,
                                           _ptr(W), _ptr(s), _ptr(am), _ptr(ap))
    if rc:
        raise OracleError(rc, "riemann_sw")
    return W, s, am, ap


def riemann_burgers(ql, qr, coef, precision="f64"):
    """Burgers-type Riemann problem with flux coef q^2/2: (W, s, amdq, apdq)."""
    out = [np.zeros(1) for _ in range(4)]
    rc = _lib(precision).oracle_riemann_burgers(float(ql), float(qr), float(coef),
                                                *[_ptr(a) for a in out])
    if rc:
        raise OracleError(rc, "riemann_burgers")
    return tuple(float(a[0]) for a in out)


def sweep(prob, q, aux, direction, dt, precision="f64"):
    """One directional sweep; returns (q_new, largest |s|)."""
    d = make_desc(prob)
    q = _state(prob, q)
    aux = _aux(prob, aux)
    out = np.empty_like(q)
    sm = ctypes.c_double(0)
    rc = _lib(precision).oracle_sweep(ctypes.byref(d), _ptr(q), _ptr(aux), int(direction),
                                      float(dt), _ptr(out), ctypes.byref(sm))
    if rc:
        raise OracleError(rc, "sweep")
    return out, sm.value


def step(prob, q, aux, dt, precision="f64"):
    """One split step; returns (q_new, smax per direction (3,), cfl)."""
    d = make_desc(prob)
    q = _state(prob, q)
    aux = _aux(prob, aux)
    out = np.empty_like(q)
    smax = np.zeros(3)
    cfl = ctypes.c_double(0)
    rc = _lib(precision).oracle_step(ctypes.byref(d), _ptr(q), _ptr(aux), float(dt), _ptr(out),
                                     _ptr(smax), ctypes.byref(cfl))
    if rc:
        raise OracleError(rc, "step")
    return out, smax, cfl.value


def speeds(prob, q, aux, precision="f64"):
    """Largest |s| per direction of the speed-only pass on q."""
    d = make_desc(prob)
    q = _state(prob, q)
    aux = _aux(prob, aux)
    smax = np.zeros(3)
    rc = _lib(precision).oracle_speeds(ctypes.byref(d), _ptr(q), _ptr(aux), _ptr(smax))
    if rc:
        raise OracleError(rc, "speeds")
    return smax


def sigma(prob, q, aux, precision="f64"):
    """max_d smax_d / dx_d of the speed-only pass."""
    sm = speeds(prob, q, aux, precision)
    s = 0.0
    for k in range(int(prob["ndim"])):
        dx = (prob["upper"][k] - prob["lower"][k]) / prob["n"][k]
        s = max(s, sm[k] / dx)
    return s


def advance(prob, q, aux, nsteps, dt0=0.0, cfl_desired=None, cfl_max=None, dt_max=None,
            precision="f64", max_log=None):
    """Adaptive stepping with revert.  Returns dict(q, t, nreject, dts, accepted_flags)."""
    d = make_desc(prob)
    q = _state(prob, q).copy()
    aux = _aux(prob, aux)
    cd = prob.get("cfl_desired", 0.9) if cfl_desired is None else cfl_desired
    cm = prob.get("cfl_max", 1.0) if cfl_max is None else cfl_max
    dm = prob.get("dt_max", float("inf")) if dt_max is None else dt_max
    max_log = int(2 * nsteps + 64) if max_log is None else int(max_log)
    dts = np.zeros(max_log)
    acc = np.zeros(max_log, dtype=np.int32)
    t = ctypes.c_double(0)
    nrej = ctypes.c_long(0)
    rc = _lib(precision).oracle_advance(ctypes.byref(d), _ptr(q), _ptr(aux), int(nsteps),
                                        float(dt0), float(cd), float(cm), float(dm),
                                        ctypes.byref(t), ctypes.byref(nrej), _ptr(dts), _ptr(acc),
                                        max_log)
    if rc:
        raise OracleError(rc, "advance")
    ntrial = int(nsteps) + nrej.value
    return {"q": q, "t": t.value, "nreject": nrej.value, "dts": dts[:ntrial].copy(),
            "accepted": acc[:ntrial].astype(bool)}


def advance_fixed(prob, q, aux, dts, precision="f64"):
    """Applies one split step per entry of dts; returns (q, cfl per step)."""
    d = make_desc(prob)
    q = _state(prob, q).copy()
    aux = _aux(prob, aux)
    dts = np.ascontiguousarray(dts, dtype=np.float64)
    cfl = np.zeros(max(dts.size, 1))
    rc = _lib(precision).oracle_advance_fixed(ctypes.byref(d), _ptr(q), _ptr(aux), dts.size,
                                              _ptr(dts), _ptr(cfl))
    if rc:
        raise OracleError(rc, "advance_fixed")
    return q, cfl[:dts.size]
