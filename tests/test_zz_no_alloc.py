"""claw_sweep_noalloc, the sweep that allocates nothing (its step state,
speed maxima and derived coefficients live in the library's static device
scratch array), against claw_sweep of a solver bound to the same state: the
same kernels run, so the results must agree bitwise, and the reported
largest speed must be equal.  Two calls in a row per case, the second on a
smaller grid, so the second call runs on scratch the first one left behind.
"""
import zlib

import numpy as np
import pytest

from paper_1805_08846_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def claw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_08846_amd import claw as c
    return c


def _tdt(prob):
    return torch.float64 if prob["dtype"] == "f64" else torch.float32


def _dev(a, prob):
    return torch.tensor(np.ascontiguousarray(a), dtype=_tdt(prob), device="cuda").contiguous()


def _sw(n, dtype, seed):
    prob = inputs._base(2, n, (-1.0, -0.5), (1.2, 0.9), "shallow_water", 3, "wall", dtype=dtype)
    prob["bc_lo"] = ("periodic", "extrap", "wall")
    prob["bc_hi"] = ("periodic", "wall", "wall")
    rng = np.random.default_rng(seed)
    nx, ny = n
    q0 = np.empty((3, ny, nx))
    q0[0] = rng.uniform(0.3, 2.0, (ny, nx))
    q0[1] = q0[0] * rng.uniform(-1.5, 1.5, (ny, nx))  # transonic pairs occur
    q0[2] = q0[0] * rng.uniform(-1.5, 1.5, (ny, nx))
    return prob, inputs.round_to(q0, dtype), None


def _ac3d(n, dtype, seed):
    prob, q0, aux = inputs.acoustics3d_layers(n=8, dtype=dtype, nsteps=1, seed=seed)
    nx, ny, nz = n
    prob["n"] = (nx, ny, nz)
    prob["bc_lo"] = ("wall", "extrap", "periodic")
    prob["bc_hi"] = ("extrap", "wall", "periodic")
    rng = np.random.default_rng(seed)
    q0 = rng.uniform(-1, 1, (4, nz, ny, nx))
    aux = np.stack([rng.uniform(0.5, 4.0, (nz, ny, nx)), rng.uniform(0.5, 2.0, (nz, ny, nx))])
    return prob, inputs.round_to(q0, dtype), inputs.round_to(aux, dtype)


def _reference(claw, prob, q0, aux, direction, dt):
    """claw_sweep on a solver over q0 (state left in q by claw_sync_state)."""
    q = _dev(q0, prob)
    a = _dev(aux, prob) if aux is not None else None
    s = claw.Solver(prob, q, a)
    smax = s.sweep(direction, dt)
    s.sync_state()
    torch.cuda.synchronize()
    out = q.clone()
    s.close()
    return out, smax


def _noalloc(claw, prob, q0, aux, direction, dt):
    d = claw.desc_from_problem(prob)
    src = _dev(q0, prob)
    dst = torch.full_like(src, float("nan"))
    a = _dev(aux, prob) if aux is not None else None
    sm = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    claw.claw_sweep_noalloc(d, src, dst, a, direction, dt, sm, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return src, dst, float(sm.item())


CASES = [
    ("sw", "f32", (300, 70), (67, 45)),
    ("sw", "f64", (129, 127), (33, 9)),
    ("ac3d", "f32", (37, 21, 13), (9, 11, 5)),
    ("ac3d", "f64", (20, 17, 24), (6, 7, 9)),
]


@pytest.mark.parametrize("kind,dtype,big,small", CASES)
def test_noalloc_sweep_equals_solver_sweep(claw, kind, dtype, big, small):
    make = _sw if kind == "sw" else _ac3d
    ndim = 2 if kind == "sw" else 3
    for n in (big, small):
        seed = zlib.crc32(repr((kind, dtype, n)).encode())
        prob, q0, aux = make(n, dtype, seed)
        for direction in range(ndim):
            dt = 0.4 * inputs.dx_of(prob, direction) / 2.5
            print(f"# noalloc {kind} {dtype} n={n} dir={direction}", flush=True)
            ref, smax_ref = _reference(claw, prob, q0, aux, direction, dt)
            src, got, smax = _noalloc(claw, prob, q0, aux, direction, dt)
            assert torch.equal(src, _dev(q0, prob)), "src must be left unchanged"
            assert torch.equal(got, ref), f"{kind} {dtype} {n} dir {direction}: results differ"
            assert smax == smax_ref and smax > 0


def test_noalloc_reports_nonphysical_depth(claw):
    prob, q0, _ = _sw((40, 30), "f32", 3)
    q0 = q0.copy()
    q0[0, 10, 10] = -0.5
    _, _, smax = _noalloc(claw, prob, q0, None, 0, 1e-3)
    assert np.isnan(smax)
    # the next call clears the flag it left behind
    prob, q0, _ = _sw((40, 30), "f32", 4)
    _, _, smax = _noalloc(claw, prob, q0, None, 1, 1e-3)
    assert np.isfinite(smax) and smax > 0
