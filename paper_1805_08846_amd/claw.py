"""ctypes binding of the C ABI in include/claw.h (argument marshalling only).

Every function here forwards to the function of the same name in
``libclaw.so``; all numerical work runs in the library's HIP kernels.  PyTorch
supplies device memory (q, aux, the workspace) and the stream.  The library
must have been built (``python -m paper_1805_08846_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CLAW_LIBRARY names another build of the same library (A/B timing of kernel
# variants); by default the in-tree build is loaded
_LIB_PATH = os.environ.get("CLAW_LIBRARY") or os.path.join(_HERE, "libclaw.so")

CLAW_OK, CLAW_E_INVALID, CLAW_E_UNSUPPORTED, CLAW_E_HIP, CLAW_E_CFL, CLAW_E_NONPHYSICAL, \
    CLAW_E_STATE = range(7)
CLAW_FP32, CLAW_FP64 = 0, 1
CLAW_RP_ACOUSTICS, CLAW_RP_SHALLOW_WATER = 0, 1
CLAW_RP_PLUGIN_BASE = 16
CLAW_RP_BURGERS, CLAW_RP_SHALLOW_WATER_GENERIC = 16, 17  # plug-in solvers
CLAW_BC_EXTRAP, CLAW_BC_WALL, CLAW_BC_PERIODIC = 0, 1, 2
CLAW_LIM_MC, CLAW_LIM_NONE, CLAW_FIRST_ORDER, CLAW_LIM_MINMOD, CLAW_LIM_SUPERBEE, CLAW_LIM_VANLEER = range(6)
CLAW_FLAG_FUSED_STEP = 1
CLAW_FLAG_STRANG = 2
CLAW_FLAG_SPLIT_STEP = 4

_BC = {"extrap": CLAW_BC_EXTRAP, "wall": CLAW_BC_WALL, "periodic": CLAW_BC_PERIODIC}
_LIM = {"mc": CLAW_LIM_MC, "none": CLAW_LIM_NONE, "first_order": CLAW_FIRST_ORDER, "minmod": CLAW_LIM_MINMOD,
        "superbee": CLAW_LIM_SUPERBEE, "vanleer": CLAW_LIM_VANLEER}

EXPORTED = ["claw_desc_init", "claw_plugin_info", "claw_workspace_bytes", "claw_create", "claw_cfl", "claw_step",
            "claw_sweep", "claw_sweep_noalloc", "claw_advance", "claw_advance_fixed", "claw_advance_timed",
            "claw_sync_state", "claw_get_control", "claw_set_control", "claw_destroy",
            "claw_batch_workspace_bytes", "claw_batch_create", "claw_batch_tune",
            "claw_batch_set_tiles", "claw_batch_advance", "claw_batch_destroy",
            "claw_lc_sizes", "claw_lc_init", "claw_lc_forward", "claw_lc_loss_grad", "claw_lc_adam",
            "claw_lc_apply", "claw_lc_coarsen", "claw_lc_advance", "claw_lc_perturb", "claw_lc_scales",
            "claw_stream_bench", "claw_debug_take", "claw_status_string", "claw_last_error"]

CLAW_LC_NET = 5187
CLAW_LC_NPARAM = 2 * CLAW_LC_NET  # x-face network, then y-face network


class claw_desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("meqn", ctypes.c_int32),
        ("mwaves", ctypes.c_int32),
        ("maux", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("lower", ctypes.c_double * 3),
        ("upper", ctypes.c_double * 3),
        ("riemann", ctypes.c_int32),
        ("limiter", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("efix", ctypes.c_int32),
        ("bc_lo", ctypes.c_int32 * 3),
        ("bc_hi", ctypes.c_int32 * 3),
        ("num_ghost", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("rho", ctypes.c_double),
        ("bulk", ctypes.c_double),
        ("grav", ctypes.c_double),
        ("cfl_desired", ctypes.c_double),
        ("cfl_max", ctypes.c_double),
        ("dt_max", ctypes.c_double),
        ("param", ctypes.c_double * 4),
    ]


class claw_lc_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("mu_h", ctypes.c_float),
        ("sl", ctypes.c_float * 3),
        ("sd1", ctypes.c_float * 3),
        ("sd2", ctypes.c_float * 3),
        ("sd3", ctypes.c_float * 3),
        ("s_out", ctypes.c_float * 3),
    ]


class ClawError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where}: {message} (status {status})")
        self.status = status


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(
            f"{_LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_1805_08846_amd.build); there is no CPU fallback")
    # torch first: the library must bind to the HIP runtime torch has loaded
    # (loaded the other way round, the process holds two runtimes and the
    # library's calls see no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "claw_desc_init": (None, [P(claw_desc)]),
        "claw_plugin_info": (i32, [i32, P(i32), P(i32), P(i32), P(i32), P(ctypes.c_char_p)]),
        "claw_workspace_bytes": (i32, [P(claw_desc), P(ctypes.c_size_t)]),
        "claw_create": (i32, [P(claw_desc), vp, vp, vp, ctypes.c_size_t, vp, P(vp)]),
        "claw_cfl": (i32, [vp, P(dbl), P(dbl)]),
        "claw_step": (i32, [vp, dbl, P(dbl)]),
        "claw_sweep": (i32, [vp, i32, dbl, P(dbl)]),
        "claw_sweep_noalloc": (i32, [P(claw_desc), vp, vp, vp, i32, dbl, vp, vp]),
        "claw_advance": (i32, [vp, i64, dbl, P(dbl), P(i64)]),
        "claw_advance_fixed": (i32, [vp, i64, P(dbl), P(dbl)]),
        "claw_advance_timed": (i32, [vp, i64, P(dbl), P(i64)]),
        "claw_sync_state": (i32, [vp]),
        "claw_get_control": (i32, [vp, P(dbl), P(dbl), P(i64), P(i64)]),
        "claw_set_control": (i32, [vp, dbl, dbl]),
        "claw_destroy": (i32, [vp]),
        "claw_stream_bench": (i32, [vp, vp, ctypes.c_size_t, i32, vp, P(dbl)]),
        "claw_batch_workspace_bytes": (i32, [P(claw_desc), i32, P(ctypes.c_size_t)]),
        "claw_batch_create": (i32, [P(claw_desc), i32, P(vp), vp, ctypes.c_size_t, vp, P(vp)]),
        "claw_batch_tune": (i32, [vp, ctypes.c_char_p, P(i32), P(i32), P(i32), P(dbl)]),
        "claw_batch_set_tiles": (i32, [vp, i32, i32, i32]),
        "claw_batch_advance": (i32, [vp, i64, P(dbl), P(i64)]),
        "claw_batch_destroy": (i32, [vp]),
        "claw_lc_sizes": (i32, [P(claw_lc_desc), P(ctypes.c_size_t), P(ctypes.c_size_t)]),
        "claw_lc_init": (i32, [vp, vp]),
        "claw_lc_forward": (i32, [P(claw_lc_desc), vp, vp, vp, vp, vp]),
        "claw_lc_loss_grad": (i32, [P(claw_lc_desc), vp, vp, vp, vp, dbl, dbl, P(dbl), vp, vp, vp, vp]),
        "claw_lc_adam": (i32, [vp, vp, i64, dbl, dbl, dbl, dbl, vp]),
        "claw_lc_apply": (i32, [P(claw_lc_desc), vp, vp, vp, vp, dbl, dbl, dbl, dbl, vp, vp, vp, vp, vp]),
        "claw_lc_coarsen": (i32, [i64, i64, vp, vp, vp]),
        "claw_lc_advance": (i32, [vp, P(claw_lc_desc), vp, i64, dbl, dbl, dbl, vp]),
        "claw_lc_perturb": (i32, [i64, i64, vp, vp, P(ctypes.c_float), ctypes.c_uint32, ctypes.c_uint32, vp]),
        "claw_lc_scales": (i32, [P(dbl), i64, dbl, i32, P(ctypes.c_float), P(dbl)]),
        "claw_debug_take": (i32, [P(ctypes.c_uint64), P(ctypes.c_uint32)]),
        "claw_status_string": (ctypes.c_char_p, [i32]),
        "claw_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def library_path():
    return _LIB_PATH


def claw_debug_take():
    """(failed range checks since the last call, source line of the first) of
    a debug build; raises ClawError(CLAW_E_UNSUPPORTED) on a release build."""
    n, line = ctypes.c_uint64(0), ctypes.c_uint32(0)
    _check(_lib.claw_debug_take(ctypes.byref(n), ctypes.byref(line)), "claw_debug_take")
    return int(n.value), int(line.value)


def _check(status, where):
    if status != CLAW_OK:
        msg = _lib.claw_last_error().decode(errors="replace")
        raise ClawError(status, where, msg or _lib.claw_status_string(status).decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------
# Thin wrappers with the C names
# --------------------------------------------------------------------------

def claw_desc_init():
    d = claw_desc()
    _lib.claw_desc_init(ctypes.byref(d))
    return d


def claw_plugin_info(pid):
    """dict(meqn, mwaves, ndim_max, vec_field, name) of a compiled plug-in solver."""
    v = [ctypes.c_int32(0) for _ in range(4)]
    name = ctypes.c_char_p()
    _check(_lib.claw_plugin_info(int(pid), *[ctypes.byref(x) for x in v], ctypes.byref(name)),
           "claw_plugin_info")
    return {"meqn": v[0].value, "mwaves": v[1].value, "ndim_max": v[2].value,
            "vec_field": v[3].value, "name": name.value.decode()}


def claw_workspace_bytes(desc):
    n = ctypes.c_size_t(0)
    _check(_lib.claw_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)), "claw_workspace_bytes")
    return n.value


def claw_create(desc, q, aux, workspace, stream_handle):
    h = ctypes.c_void_p(None)
    _check(_lib.claw_create(ctypes.byref(desc), _ptr(q), _ptr(aux), _ptr(workspace),
                            workspace.numel() * workspace.element_size(),
                            ctypes.c_void_p(stream_handle), ctypes.byref(h)), "claw_create")
    return h


def claw_cfl(h):
    sigma = ctypes.c_double(0)
    smax = (ctypes.c_double * 3)()
    _check(_lib.claw_cfl(h, ctypes.byref(sigma), smax), "claw_cfl")
    return sigma.value, list(smax)


def claw_step(h, dt, sync=True):
    """Returns (status, cfl); status CLAW_E_CFL means the step was reverted."""
    if not sync:
        _check(_lib.claw_step(h, float(dt), None), "claw_step")
        return CLAW_OK, None
    cfl = ctypes.c_double(0)
    st = _lib.claw_step(h, float(dt), ctypes.byref(cfl))
    if st not in (CLAW_OK, CLAW_E_CFL):
        _check(st, "claw_step")
    return st, cfl.value


def claw_sweep(h, direction, dt):
    sm = ctypes.c_double(0)
    _check(_lib.claw_sweep(h, int(direction), float(dt), ctypes.byref(sm)), "claw_sweep")
    return sm.value


def claw_sweep_noalloc(desc, src, dst, aux, direction, dt, smax_dev, stream_handle):
    """One sweep src -> dst with no handle or workspace (scratch in the
    library's static device memory); smax_dev: a device float64 tensor of one
    element or None.  Enqueued, no synchronisation."""
    import torch
    n = desc.meqn * desc.n[0] * desc.n[1] * desc.n[2]
    dt_ = torch.float32 if desc.dtype == CLAW_FP32 else torch.float64
    _need(src, "src", n, dt_)
    _need(dst, "dst", n, dt_)
    if desc.maux:
        _need(aux, "aux", desc.maux * desc.n[0] * desc.n[1] * desc.n[2], dt_)
    if smax_dev is not None:
        _need(smax_dev, "smax_dev", 1, torch.float64)
    _check(_lib.claw_sweep_noalloc(ctypes.byref(desc), _ptr(src), _ptr(dst), _ptr(aux) if desc.maux else None,
                                   int(direction), float(dt), _ptr(smax_dev), ctypes.c_void_p(stream_handle)),
           "claw_sweep_noalloc")


def claw_advance(h, nsteps, dt0=0.0):
    t = ctypes.c_double(0)
    nrej = ctypes.c_int64(0)
    _check(_lib.claw_advance(h, int(nsteps), float(dt0), ctypes.byref(t), ctypes.byref(nrej)),
           "claw_advance")
    return t.value, nrej.value


def claw_advance_fixed(h, dts, log=True):
    """Steps of the given sizes; returns the Courant number of each step, or
    None with log=False (equal steps then replay a captured graph)."""
    dts = np.ascontiguousarray(dts, dtype=np.float64)
    cfl = np.zeros(max(dts.size, 1)) if log else None
    _check(_lib.claw_advance_fixed(h, dts.size, dts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   None if cfl is None else cfl.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "claw_advance_fixed")
    return None if cfl is None else cfl[:dts.size]


def claw_advance_timed(h, nsteps):
    ms = (ctypes.c_double * 4)()
    cnt = (ctypes.c_int64 * 4)()
    _check(_lib.claw_advance_timed(h, int(nsteps), ms, cnt), "claw_advance_timed")
    return list(ms), list(cnt)


def claw_sync_state(h):
    _check(_lib.claw_sync_state(h), "claw_sync_state")


def claw_get_control(h):
    t, dtn = ctypes.c_double(0), ctypes.c_double(0)
    acc, rej = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(_lib.claw_get_control(h, ctypes.byref(t), ctypes.byref(dtn), ctypes.byref(acc),
                                 ctypes.byref(rej)), "claw_get_control")
    return {"t": t.value, "dt_next": dtn.value, "accepted": acc.value, "rejected": rej.value}


def claw_set_control(h, t, dt_next):
    _check(_lib.claw_set_control(h, float(t), float(dt_next)), "claw_set_control")


def claw_destroy(h):
    _check(_lib.claw_destroy(h), "claw_destroy")


def claw_stream_bench(a, b, reps, stream_handle):
    """Achievable bandwidth (GB/s) of copy, copy-nt, read, write, write-nt streams
    over the device tensors a (zero-filled) and b of equal byte size."""
    out = (ctypes.c_double * 5)()
    nbytes = min(a.numel() * a.element_size(), b.numel() * b.element_size())
    _check(_lib.claw_stream_bench(_ptr(a), _ptr(b), nbytes, int(reps),
                                  ctypes.c_void_p(stream_handle), out), "claw_stream_bench")
    return dict(zip(["copy", "copy_nt", "read", "write", "write_nt"], list(out)))


def claw_batch_workspace_bytes(descs):
    arr = (claw_desc * len(descs))(*descs)
    n = ctypes.c_size_t(0)
    _check(_lib.claw_batch_workspace_bytes(arr, len(descs), ctypes.byref(n)),
           "claw_batch_workspace_bytes")
    return n.value


def claw_batch_create(descs, qs, workspace, stream_handle):
    arr = (claw_desc * len(descs))(*descs)
    ptrs = (ctypes.c_void_p * len(qs))(*[q.data_ptr() for q in qs])
    h = ctypes.c_void_p(None)
    _check(_lib.claw_batch_create(arr, len(descs), ptrs, _ptr(workspace),
                                  workspace.numel() * workspace.element_size(),
                                  ctypes.c_void_p(stream_handle), ctypes.byref(h)), "claw_batch_create")
    return h


def claw_batch_tune(h, cache_path=None):
    c, s, r, us = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0)
    _check(_lib.claw_batch_tune(h, cache_path.encode() if cache_path else None, ctypes.byref(c),
                                ctypes.byref(s), ctypes.byref(r), ctypes.byref(us)), "claw_batch_tune")
    return {"chunk": c.value, "schedule": s.value, "rows_per_wave": r.value, "us_per_step": us.value}


def claw_batch_set_tiles(h, chunk, schedule, rows_per_wave=8):
    _check(_lib.claw_batch_set_tiles(h, int(chunk), int(schedule), int(rows_per_wave)), "claw_batch_set_tiles")


def claw_batch_advance(h, count, nsteps):
    t = (ctypes.c_double * count)()
    rej = (ctypes.c_int64 * count)()
    _check(_lib.claw_batch_advance(h, int(nsteps), t, rej), "claw_batch_advance")
    return list(t), list(rej)


def claw_batch_destroy(h):
    _check(_lib.claw_batch_destroy(h), "claw_batch_destroy")


class BatchSolver:
    """An ensemble of 2D shallow-water problems advanced together; qs are torch
    device tensors, one per problem (same dtype).  Problems with fused_step=True
    (all or none) run the batched fused 2D step."""

    def __init__(self, probs, qs, stream=None):
        import torch
        self.probs = probs
        self.descs = [desc_from_problem(p) for p in probs]
        if len(qs) != len(self.descs):
            raise ValueError(f"{len(self.descs)} problems but {len(qs)} state tensors")
        for i, (d, q) in enumerate(zip(self.descs, qs)):
            _need(q, f"qs[{i}]", d.meqn * d.n[0] * d.n[1] * d.n[2],
                  torch.float32 if d.dtype == CLAW_FP32 else torch.float64)
        self.qs = qs
        dev = qs[0].device
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        nbytes = claw_batch_workspace_bytes(self.descs)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.h = claw_batch_create(self.descs, qs, self.workspace, self.stream.cuda_stream)

    def tune(self, cache_path=None):
        return claw_batch_tune(self.h, cache_path)

    def set_tiles(self, chunk, schedule, rows_per_wave=8):
        claw_batch_set_tiles(self.h, chunk, schedule, rows_per_wave)

    def advance(self, nsteps):
        return claw_batch_advance(self.h, len(self.qs), nsteps)

    def close(self):
        if self.h is not None:
            claw_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# Learned coarse-grid flux correction
# --------------------------------------------------------------------------

def lc_desc(nx, ny, norm):
    """claw_lc_desc from a grid and a normalisation dict (mu_h, sl, sd1, sd2, sd3, s_out)."""
    d = claw_lc_desc()
    d.nx, d.ny = int(nx), int(ny)
    d.mu_h = float(norm["mu_h"])
    for key in ("sl", "sd1", "sd2", "sd3", "s_out"):
        arr = getattr(d, key)
        for c in range(3):
            arr[c] = float(norm[key][c])
    return d


def claw_lc_sizes(desc):
    pb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_lib.claw_lc_sizes(ctypes.byref(desc), ctypes.byref(pb), ctypes.byref(wb)), "claw_lc_sizes")
    return pb.value, wb.value


def claw_lc_init(params, stream_handle):
    _check(_lib.claw_lc_init(_ptr(params), ctypes.c_void_p(stream_handle)), "claw_lc_init")


def claw_lc_forward(desc, params, q, dF, dG, stream_handle):
    _check(_lib.claw_lc_forward(ctypes.byref(desc), _ptr(params), _ptr(q), _ptr(dF), _ptr(dG),
                                ctypes.c_void_p(stream_handle)), "claw_lc_forward")


def claw_lc_loss_grad(desc, params, q, target, plain, nux, nuy, w, work, grad, loss, stream_handle):
    wv = (ctypes.c_double * 3)(*[float(v) for v in w])
    _check(_lib.claw_lc_loss_grad(ctypes.byref(desc), _ptr(params), _ptr(q), _ptr(target), _ptr(plain),
                                  float(nux), float(nuy), wv, _ptr(work), _ptr(grad), _ptr(loss),
                                  ctypes.c_void_p(stream_handle)), "claw_lc_loss_grad")


def claw_lc_adam(params, grad, step, lr, beta1, beta2, eps, stream_handle):
    _check(_lib.claw_lc_adam(_ptr(params), _ptr(grad), int(step), float(lr), float(beta1), float(beta2),
                             float(eps), ctypes.c_void_p(stream_handle)), "claw_lc_adam")


def claw_lc_apply(desc, qn, plain, dF, dG, nux, nuy, tau, kappa, out, keep_x, keep_y, work, stream_handle):
    _check(_lib.claw_lc_apply(ctypes.byref(desc), _ptr(qn), _ptr(plain), _ptr(dF), _ptr(dG), float(nux),
                              float(nuy), float(tau), float(kappa), _ptr(out), _ptr(keep_x), _ptr(keep_y),
                              _ptr(work), ctypes.c_void_p(stream_handle)), "claw_lc_apply")


def claw_lc_coarsen(nx, ny, fine, coarse, stream_handle):
    import torch
    _need(fine, "fine", 3 * (2 * int(ny)) * (2 * int(nx)), torch.float32)
    _need(coarse, "coarse", 3 * int(ny) * int(nx), torch.float32)
    _check(_lib.claw_lc_coarsen(int(nx), int(ny), _ptr(fine), _ptr(coarse), ctypes.c_void_p(stream_handle)),
           "claw_lc_coarsen")


def claw_lc_perturb(nx, ny, q, out, sigma, seed, call, stream_handle):
    import torch
    _need(q, "q", 3 * int(ny) * int(nx), torch.float32)
    _need(out, "out", 3 * int(ny) * int(nx), torch.float32)
    sg = (ctypes.c_float * 3)(*[float(v) for v in sigma])
    _check(_lib.claw_lc_perturb(int(nx), int(ny), _ptr(q), _ptr(out), sg, int(seed) & 0xFFFFFFFF,
                                int(call) & 0xFFFFFFFF, ctypes.c_void_p(stream_handle)), "claw_lc_perturb")


def claw_lc_scales(r2, ncell, nu, correct_depth=True):
    """(s_out, w): output scales and loss weights from residual energies r2 (3 sums)."""
    r = (ctypes.c_double * 3)(*[float(v) for v in r2])
    so = (ctypes.c_float * 3)()
    w = (ctypes.c_double * 3)()
    _check(_lib.claw_lc_scales(r, int(ncell), float(nu), 1 if correct_depth else 0, so, w), "claw_lc_scales")
    return tuple(float(v) for v in so), tuple(float(v) for v in w)


def claw_lc_advance(h, desc, params, nsteps, dt, tau, kappa, work):
    _check(_lib.claw_lc_advance(h, ctypes.byref(desc), _ptr(params), int(nsteps), float(dt), float(tau),
                                float(kappa), _ptr(work)), "claw_lc_advance")


def _need(t, name, numel, dtype):
    """Checks a device buffer before its pointer goes to the library: the C
    calls take plain pointers, so a tensor of the wrong size or type would
    become an out-of-bounds access on the GPU instead of an error here."""
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype or t.numel() != numel:
        where = "device" if t.is_cuda else "host"
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor of {numel} elements "
                         f"(got {tuple(t.shape)} {t.dtype} on the {where})")


class LearnedCorrection:
    """Parameter block and workspace (torch device buffers) of the learned
    correction on an nx x ny grid; every method forwards to one C call."""

    def __init__(self, nx, ny, norm, theta, device="cuda", stream=None):
        import torch
        self.desc = lc_desc(nx, ny, norm)
        self.nx, self.ny = int(nx), int(ny)
        pbytes, wbytes = claw_lc_sizes(self.desc)
        self.params = torch.zeros(pbytes // 4, dtype=torch.float32, device=device)
        self.work = torch.empty(wbytes, dtype=torch.uint8, device=device)
        self.grad = torch.zeros(CLAW_LC_NPARAM, dtype=torch.float32, device=device)
        self.loss = torch.zeros(4, dtype=torch.float64, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.step_count = 0
        self.set_theta(theta)

    def set_theta(self, theta):
        import torch
        t = torch.as_tensor(np.asarray(theta, dtype=np.float32))
        self.params[:CLAW_LC_NPARAM].copy_(t)
        claw_lc_init(self.params, self.stream.cuda_stream)
        self.step_count = 0

    def theta(self):
        return self.params[:CLAW_LC_NPARAM].double().cpu().numpy()

    def _cells(self, name, t):
        import torch
        _need(t, name, 3 * self.nx * self.ny, torch.float32)

    def _faces(self, dF, dG):
        import torch
        _need(dF, "dF", 3 * self.ny * (self.nx + 1), torch.float32)
        _need(dG, "dG", 3 * (self.ny + 1) * self.nx, torch.float32)

    def forward(self, q, dF, dG):
        self._cells("q", q)
        self._faces(dF, dG)
        claw_lc_forward(self.desc, self.params, q, dF, dG, self.stream.cuda_stream)

    def loss_grad(self, q, target, plain, nux, nuy, w):
        for name, t in (("q", q), ("target", target), ("plain", plain)):
            self._cells(name, t)
        claw_lc_loss_grad(self.desc, self.params, q, target, plain, nux, nuy, w, self.work, self.grad,
                          self.loss, self.stream.cuda_stream)

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        claw_lc_adam(self.params, self.grad, self.step_count, lr, beta1, beta2, eps, self.stream.cuda_stream)

    def apply(self, qn, plain, dF, dG, nux, nuy, tau, kappa, out, keep_x=None, keep_y=None):
        import torch
        for name, t in (("qn", qn), ("plain", plain), ("out", out)):
            self._cells(name, t)
        self._faces(dF, dG)
        if keep_x is not None:
            _need(keep_x, "keep_x", self.ny * (self.nx + 1), torch.uint8)
        if keep_y is not None:
            _need(keep_y, "keep_y", (self.ny + 1) * self.nx, torch.uint8)
        claw_lc_apply(self.desc, qn, plain, dF, dG, nux, nuy, tau, kappa, out, keep_x, keep_y, self.work,
                      self.stream.cuda_stream)

    def advance(self, solver, nsteps, dt, tau, kappa):
        claw_lc_advance(solver.h, self.desc, self.params, nsteps, dt, tau, kappa, self.work)


def claw_status_string(status):
    return _lib.claw_status_string(int(status)).decode()


def claw_last_error():
    return _lib.claw_last_error().decode(errors="replace")


# --------------------------------------------------------------------------
# Convenience layer over torch tensors
# --------------------------------------------------------------------------

def desc_from_problem(prob):
    """claw_desc for a problem description dict (see inputs.py)."""
    d = claw_desc_init()
    d.ndim = int(prob["ndim"])
    n = list(prob["n"]) + [1] * (3 - len(prob["n"]))
    for k in range(3):
        d.n[k] = int(n[k])
        d.lower[k] = float(prob["lower"][k])
        d.upper[k] = float(prob["upper"][k])
        d.bc_lo[k] = _BC[prob["bc_lo"][k]]
        d.bc_hi[k] = _BC[prob["bc_hi"][k]]
    d.meqn = int(prob["meqn"])
    if prob["system"] == "acoustics":
        d.riemann = CLAW_RP_ACOUSTICS
        d.mwaves = 2
        d.maux = 2 if prob.get("has_aux", False) else 0
    elif prob["system"] == "burgers":
        d.riemann = CLAW_RP_BURGERS
        d.mwaves = 1
        d.maux = 0
        coef = tuple(prob.get("coef", (1.0, 1.0, 1.0))) + (0.0,) * 4
        for k in range(4):
            d.param[k] = float(coef[k]) if k < 3 else 0.0
    elif prob.get("solver", "builtin") == "generic":
        d.riemann = CLAW_RP_SHALLOW_WATER_GENERIC
        d.mwaves = 3
        d.maux = 0
        d.param[0] = float(prob.get("grav", 1.0))
        d.param[1] = 1.0 if prob.get("efix", True) else 0.0
    else:
        d.riemann = CLAW_RP_SHALLOW_WATER
        d.mwaves = 3
        d.maux = 0
    d.limiter = _LIM[prob.get("limiter", "mc")]
    d.dtype = CLAW_FP32 if prob.get("dtype", "f64") in ("f32", "float32") else CLAW_FP64
    d.efix = 1 if prob.get("efix", True) else 0
    d.rho = float(prob.get("rho", 1.0))
    d.bulk = float(prob.get("bulk", 1.0))
    d.grav = float(prob.get("grav", 1.0))
    d.cfl_desired = float(prob.get("cfl_desired", 0.9))
    d.cfl_max = float(prob.get("cfl_max", 1.0))
    dm = prob.get("dt_max", float("inf"))
    d.dt_max = float(dm) if dm is not None else math.inf
    fs = prob.get("fused_step")  # True: fused, False: x and y sweeps, None: the library's choice
    d.flags = (CLAW_FLAG_FUSED_STEP if fs else (CLAW_FLAG_SPLIT_STEP if fs is False else 0)) | \
        (CLAW_FLAG_STRANG if prob.get("splitting", "godunov") == "strang" else 0)
    return d


class Solver:
    """A solver bound to torch device tensors q[meqn, nz, ny, nx] (and aux).

    The workspace is allocated here with torch (the library never allocates);
    all calls enqueue on the given torch stream (default: current stream)."""

    def __init__(self, prob, q, aux=None, stream=None):
        import torch
        self.prob = prob
        self.desc = desc_from_problem(prob)
        want = torch.float32 if self.desc.dtype == CLAW_FP32 else torch.float64
        if q.dtype != want or not q.is_cuda or not q.is_contiguous():
            raise ValueError(f"q must be a contiguous {want} device tensor")
        if aux is not None and (aux.dtype != want or not aux.is_contiguous()):
            raise ValueError(f"aux must be a contiguous {want} device tensor")
        ncell = self.desc.n[0] * self.desc.n[1] * self.desc.n[2]
        _need(q, "q", self.desc.meqn * ncell, want)
        if self.desc.maux > 0:
            _need(aux, "aux", self.desc.maux * ncell, want)
        elif aux is not None:
            raise ValueError("aux given for a problem without aux fields")
        self.q = q
        self.aux = aux
        self.stream = stream if stream is not None else torch.cuda.current_stream(q.device)
        nbytes = claw_workspace_bytes(self.desc)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=q.device)
        self.h = claw_create(self.desc, q, aux, self.workspace, self.stream.cuda_stream)

    def cfl(self):
        return claw_cfl(self.h)

    def step(self, dt, sync=True):
        return claw_step(self.h, dt, sync)

    def sweep(self, direction, dt):
        return claw_sweep(self.h, direction, dt)

    def advance(self, nsteps, dt0=0.0):
        return claw_advance(self.h, nsteps, dt0)

    def advance_fixed(self, dts, log=True):
        return claw_advance_fixed(self.h, dts, log)

    def advance_timed(self, nsteps):
        return claw_advance_timed(self.h, nsteps)

    def sync_state(self):
        claw_sync_state(self.h)

    def control(self):
        return claw_get_control(self.h)

    def set_control(self, t, dt_next):
        claw_set_control(self.h, t, dt_next)

    def close(self):
        if self.h is not None:
            claw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
