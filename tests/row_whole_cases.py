"""Acoustics x sweeps on rows of exactly 64 cells per wavefront (256 FP32 or
128 FP64 cells) with extrapolation at both ends: the rows the whole-row
sweep kernel takes.

run(claw) returns, per case, the state after one x sweep and the largest
speed it reported, and the state, time and rejection count after a few
adaptive 3D steps.  As a script (python tests/row_whole_cases.py OUT.npz)
it writes them to OUT.npz: tests/test_gpu_row_whole.py runs it in a child
process with CLAW_ROW_WHOLE=0 (the segment kernels) and compares.
"""
import os
import sys
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (nx, ny, nz or None, aux, dtype, limiter)
SWEEPS = [(256, 67, None, False, "f32", "mc"), (128, 45, None, False, "f64", "mc"), (256, 13, 7, True, "f32", "mc"),
          (128, 9, 5, True, "f64", "mc"), (256, 5, 3, False, "f32", "mc"), (256, 1, None, False, "f32", "mc"),
          (256, 9, 4, True, "f32", "superbee"), (128, 7, None, False, "f64", "minmod")]


def seed(*case):
    return zlib.crc32(repr(case).encode())


def sweep_case(nx, ny, nz, aux, dtype, limiter):
    """Problem, initial state and coefficients of one single-sweep case."""
    from paper_1805_08846_amd import inputs
    rng = np.random.default_rng(seed(nx, ny, nz, aux, dtype))
    bcs = ["extrap", "wall", "periodic"]
    if nz is None:
        prob = inputs._base(2, (nx, ny), (0, 0), (1.0, 1.5), "acoustics", 3, "extrap", rho=1.7, bulk=2.9,
                            dtype=dtype)
        shape, meqn = (1, ny, nx), 3
    else:
        prob = inputs._base(3, (nx, ny, nz), (0, 0, 0), (1.0, 0.8, 0.6), "acoustics", 4, "extrap", rho=1.7,
                            bulk=2.9, has_aux=aux, dtype=dtype)
        shape, meqn = (nz, ny, nx), 4
    prob["bc_lo"] = ("extrap",) + tuple(rng.choice(bcs) for _ in range(2))
    prob["bc_hi"] = ("extrap",) + tuple(rng.choice(bcs) for _ in range(2))
    prob["limiter"] = limiter
    q0 = inputs.round_to(rng.uniform(-1, 1, (meqn,) + shape), dtype)
    a0 = inputs.round_to(rng.uniform(0.5, 2.0, (2,) + shape), dtype) if aux else None
    cmax = 2.0 if aux else (2.9 / 1.7) ** 0.5
    dt = 0.7 * (prob["upper"][0] - prob["lower"][0]) / nx / cmax
    return prob, q0, a0, dt


def advance_case(dtype):
    """A 3D layered acoustics problem 256 (128 in FP64) cells wide in x."""
    from paper_1805_08846_amd import inputs
    nx = 256 if dtype == "f32" else 128
    rng = np.random.default_rng(seed("advance", dtype))
    prob = inputs._base(3, (nx, 12, 10), (0, 0, 0), (1.0, 0.6, 0.5), "acoustics", 4, "extrap", rho=1.0, bulk=1.0,
                        has_aux=True, dtype=dtype)
    prob["bc_lo"] = ("extrap", "wall", "periodic")
    prob["bc_hi"] = ("extrap", "extrap", "periodic")
    shape = (10, 12, nx)
    x = (np.arange(nx) + 0.5) / nx
    q0 = np.zeros((4,) + shape)
    q0[0] = np.exp(-200.0 * (x - 0.4) ** 2)[None, None, :] * (1 + 0.1 * rng.uniform(size=shape))
    a0 = np.empty((2,) + shape)
    a0[0] = np.where(x < 0.55, 1.0, 2.5)[None, None, :]
    a0[1] = np.where(x < 0.55, 1.0, 0.6)[None, None, :]
    return prob, inputs.round_to(q0, dtype), inputs.round_to(a0, dtype)


def run(claw):
    import torch

    def dev(a, dtype):
        return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64 if dtype == "f64" else torch.float32,
                            device="cuda").contiguous()

    out = {}
    for case in SWEEPS:
        prob, q0, a0, dt = sweep_case(*case)
        dtype = case[4]
        q = dev(q0, dtype)
        s = claw.Solver(prob, q, None if a0 is None else dev(a0, dtype))
        sm = s.sweep(0, dt)
        s.sync_state()
        torch.cuda.synchronize()
        name = "sweep_" + "_".join(str(c) for c in case)
        out[name] = q.double().cpu().numpy()
        out[name + "_smax"] = np.array([sm])
        s.close()
    for dtype in ("f32", "f64"):
        prob, q0, a0 = advance_case(dtype)
        q = dev(q0, dtype)
        s = claw.Solver(prob, q, dev(a0, dtype))
        t, nrej = s.advance(8)
        torch.cuda.synchronize()
        out[f"advance_{dtype}"] = q.double().cpu().numpy()
        out[f"advance_{dtype}_t"] = np.array([t, nrej])
        s.close()
    return out


def main(path):
    from paper_1805_08846_amd import claw
    out = run(claw)
    np.savez(path, **out)
    print(f"# {len(out)} arrays written", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
