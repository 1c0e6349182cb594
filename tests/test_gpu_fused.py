"""The fused 2D shallow-water step (CLAW_FLAG_FUSED_STEP: rows x-swept into
LDS, then y-swept out of it, one kernel per step) against the CPU oracle and
against the two-kernel path: same tolerances as the two-kernel path (FP64
1e-12, FP32 1e-5 relative L-infinity of the whole state); strip and chunk
edges in x and y, ragged strips, FP32 and FP64 strip widths, walls,
extrapolation and periodic boundaries in y; the library's automatic choice
of the fused step for large states."""
import numpy as np
import pytest

import oracle
from paper_1805_08846_amd import inputs
from helpers import rel_linf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def claw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_08846_amd import claw as c
    return c


def _run(claw, prob, q0, fused, steps=None, dts=None):
    prob = dict(prob, fused_step=fused)
    dt = torch.float64 if prob["dtype"] == "f64" else torch.float32
    q = torch.tensor(q0, dtype=dt, device="cuda").contiguous()
    s = claw.Solver(prob, q)
    if dts is None:
        t, nrej = s.advance(steps)
    else:
        s.advance_fixed(dts)
        t, nrej = s.control()["t"], 0
    torch.cuda.synchronize()
    out = q.double().cpu().numpy()
    ms, cnt = s.advance_timed(1)
    s.close()
    return out, t, nrej, cnt


@pytest.mark.parametrize("dtype,n", [("f64", 200), ("f32", 333), ("f64", 131), ("f32", 64)])
def test_fused_adaptive_matches_oracle(claw, dtype, n):
    prob, q0, _ = inputs.sw_radial_dam(n=n, dtype=dtype, nsteps=60, seed=3)
    out, t, nrej, cnt = _run(claw, prob, q0, True, steps=60)
    assert cnt[0] >= 1 and cnt[1] == 0  # one kernel per step
    ref = oracle.advance(prob, q0, None, 60)
    err, per = rel_linf(out, ref["q"])
    print(f"fused {dtype} {n}^2: rel {err:.2e} per field {per}")
    assert nrej == ref["nreject"]
    assert err <= TOL[dtype]
    assert t == pytest.approx(ref["t"], rel=1e-12 if dtype == "f64" else 1e-6)


@pytest.mark.parametrize("bc", ["extrap", "wall"])
def test_fused_rectangular_and_boundaries(claw, bc):
    prob, q0, _ = inputs.sw_radial_dam(n=96, dtype="f64", nsteps=30, seed=4)
    prob["n"] = (250, 37, 1)
    prob["bc_lo"] = ("wall", bc, bc)
    prob["bc_hi"] = ("extrap", bc, bc)
    rng = np.random.default_rng(4)
    q0 = np.zeros((3, 1, 37, 250))
    q0[0] = 1.0 + 0.5 * rng.uniform(size=(1, 37, 250))
    q0[1] = 0.1 * rng.uniform(-1, 1, size=(1, 37, 250))
    q0[2] = 0.1 * rng.uniform(-1, 1, size=(1, 37, 250))
    out, _, _, _ = _run(claw, prob, q0, True, steps=30)
    split, _, _, _ = _run(claw, prob, q0, False, steps=30)
    ref = oracle.advance(prob, q0, None, 30)
    err, _ = rel_linf(out, ref["q"])
    assert err <= 1e-12
    assert rel_linf(out, split)[0] <= 1e-13


def test_fused_prescribed_steps_fp32(claw):
    prob, q0, _ = inputs.sw_radial_dam(n=257, dtype="f32", nsteps=40, seed=8)
    ref = oracle.advance(prob, q0, None, 40)
    dts = ref["dts"][ref["accepted"]]
    out, _, _, _ = _run(claw, prob, q0, True, dts=dts)
    qf, _ = oracle.advance_fixed(prob, q0, None, dts)
    assert rel_linf(out, qf)[0] <= 1e-5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_periodic_y(claw, dtype):
    # ghost rows of a periodic y boundary come from the far end of the grid
    prob, q0, _ = inputs.sw_radial_dam(n=64, dtype=dtype, nsteps=5, seed=1)
    prob["n"] = (300, 45, 1)
    prob["bc_lo"] = ("wall", "periodic", "periodic")
    prob["bc_hi"] = ("wall", "periodic", "periodic")
    rng = np.random.default_rng(12)
    q0 = np.zeros((3, 1, 45, 300))
    q0[0] = 1.0 + 0.5 * rng.uniform(size=(1, 45, 300))
    q0[1] = 0.2 * rng.uniform(-1, 1, size=(1, 45, 300))
    q0[2] = 0.2 * rng.uniform(-1, 1, size=(1, 45, 300))
    if dtype == "f32":
        q0 = q0.astype(np.float32).astype(np.float64)
    out, _, _, cnt = _run(claw, prob, q0, True, steps=25)
    assert cnt[0] >= 1 and cnt[1] == 0  # one kernel per step
    ref = oracle.advance(prob, q0, None, 25)
    assert rel_linf(out, ref["q"])[0] <= TOL[dtype]
    split, _, _, _ = _run(claw, prob, q0, False, steps=25)
    assert rel_linf(out, split)[0] <= (1e-13 if dtype == "f64" else 1e-6)


def test_large_states_take_the_fused_step_by_default(claw):
    # 4800^2 FP32 (264 MiB of state, above CLAW_FUSED_AUTO_BYTES): the library
    # chooses the fused step by itself; same result as the forced split path
    prob, q0, _ = inputs.sw_radial_dam(n=4800, dtype="f32", nsteps=4, seed=2)
    prob = dict(prob, fused_step=None)
    out, _, _, cnt = _run(claw, prob, q0, None, steps=4)
    assert cnt[0] >= 1 and cnt[1] == 0
    split, _, _, cnt2 = _run(claw, prob, q0, False, steps=4)
    assert cnt2[1] >= 1
    assert rel_linf(out, split)[0] <= 1e-6
    small, qs, _ = inputs.sw_radial_dam(n=512, dtype="f32", nsteps=2, seed=2)
    _, _, _, cnt3 = _run(claw, small, qs, None, steps=2)
    assert cnt3[1] >= 1  # a small state keeps the x and y sweep kernels


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fused_advance_in_pieces_equals_one_call_bitwise(claw, dtype):
    # the fused step plans each trial's result buffer so that an adaptive call
    # ends in the caller's array: calls of 1, 2, 3 and 5 steps (a one-step call
    # from buffer 0 still ends elsewhere and is copied) equal one call of 11
    prob, q0, _ = inputs.sw_radial_dam(n=200, dtype=dtype, nsteps=11, seed=9)
    prob = dict(prob, fused_step=True)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    q = torch.tensor(q0, dtype=tdt, device="cuda").contiguous()
    s = claw.Solver(prob, q)
    t_one, rej_one = s.advance(11)
    torch.cuda.synchronize()
    one = q.double().cpu().numpy()
    s.close()
    q = torch.tensor(q0, dtype=tdt, device="cuda").contiguous()
    s = claw.Solver(prob, q)
    rej = 0
    for k in (1, 2, 3, 5):
        t, r = s.advance(k)
        rej += r
    torch.cuda.synchronize()
    pieces = q.double().cpu().numpy()
    ms, cnt = s.advance_timed(1)
    s.close()
    assert cnt[0] >= 1 and cnt[1] == 0
    assert np.array_equal(pieces, one)
    assert t == t_one and rej == rej_one
    ref = oracle.advance(prob, q0, None, 11)
    assert rel_linf(one, ref["q"])[0] <= TOL[dtype]
