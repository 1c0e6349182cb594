"""Small runs of every kernel family, for the range-checked debug build.

run(claw) executes single sweeps (2D shallow water and acoustics, 3D
acoustics with per-cell coefficients) on ragged grids with a random boundary
rule per side, fused steps, a batched ensemble, a plug-in solver, the learned
correction's passes and the sweep that allocates nothing; it returns every
final state keyed by case name.  With a debug library it also records the
range checks each case failed (claw_debug_take).

Run as a script (python tests/debug_cases.py OUT.npz) it loads whatever
library CLAW_LIBRARY names and writes the states plus, per case, the count
and first source line of failed checks; tests/test_gpu_debug.py runs it on
the debug build in a child process and compares with the release build run
in its own process.
"""
import os
import sys
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _seed(*case):
    return zlib.crc32(repr(case).encode())


def run(claw, take=None):
    import torch

    from paper_1805_08846_amd import inputs

    out, checks = {}, {}

    def dev(a, dtype):
        return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64 if dtype == "f64" else torch.float32,
                            device="cuda").contiguous()

    def host(t):
        torch.cuda.synchronize()
        return t.double().cpu().numpy()

    def done(name, arr):
        out[name] = arr
        if take is not None:
            checks[name] = take()

    bcs = ["extrap", "wall", "periodic"]
    # single sweeps in 2D
    for n in ((300, 70), (129, 127), (251, 5)):
        for system in ("shallow_water", "acoustics"):
            for dtype in ("f32", "f64"):
                for direction in (0, 1):
                    rng = np.random.default_rng(_seed(n, system, dtype, direction))
                    prob = inputs._base(2, n, (0, 0), (1.0, 1.5), system, 3, "extrap", dtype=dtype, grav=1.3,
                                        rho=1.7, bulk=2.9)
                    prob["bc_lo"] = tuple(rng.choice(bcs) for _ in range(3))
                    prob["bc_hi"] = tuple(rng.choice(bcs) for _ in range(3))
                    if system == "shallow_water":
                        q0 = inputs.random_states("shallow_water", n[0] * n[1], seed=3, depth=(0.1, 2.0),
                                                  vel=2.0).T.reshape(3, 1, n[1], n[0])
                    else:
                        q0 = rng.uniform(-1, 1, (3, 1, n[1], n[0]))
                    q0 = inputs.round_to(q0, dtype)
                    q = dev(q0, dtype)
                    s = claw.Solver(prob, q)
                    dx = (prob["upper"][direction] - prob["lower"][direction]) / n[direction]
                    s.sweep(direction, 0.2 * dx)
                    s.sync_state()
                    done(f"sweep2d_{system}_{dtype}_{n[0]}x{n[1]}_d{direction}", host(q))
                    s.close()
    # single sweeps in 3D, per-cell coefficients
    for n in ((37, 21, 13), (5, 70, 3)):
        for dtype in ("f32", "f64"):
            for direction in (0, 1, 2):
                rng = np.random.default_rng(_seed(n, dtype, direction))
                prob = inputs._base(3, n, (0, 0, 0), (1.0, 0.8, 0.6), "acoustics", 4, "extrap", rho=1.7, bulk=2.9,
                                    has_aux=True, dtype=dtype)
                prob["bc_lo"] = tuple(rng.choice(bcs) for _ in range(3))
                prob["bc_hi"] = tuple(rng.choice(bcs) for _ in range(3))
                shape = (n[2], n[1], n[0])
                q = dev(inputs.round_to(rng.uniform(-1, 1, (4,) + shape), dtype), dtype)
                a = dev(inputs.round_to(rng.uniform(0.5, 2.0, (2,) + shape), dtype), dtype)
                s = claw.Solver(prob, q, a)
                dx = (prob["upper"][direction] - prob["lower"][direction]) / n[direction]
                s.sweep(direction, 0.3 * dx / 2.0)
                s.sync_state()
                done(f"sweep3d_{dtype}_{n[0]}x{n[1]}x{n[2]}_d{direction}", host(q))
                s.close()
    # acoustics x sweeps on rows of 64 cells per wavefront, extrapolation at both ends (whole-row kernel)
    for nx, dtype in ((256, "f32"), (128, "f64")):
        rng = np.random.default_rng(_seed("whole", nx, dtype))
        prob = inputs._base(3, (nx, 5, 3), (0, 0, 0), (1.0, 0.8, 0.6), "acoustics", 4, "extrap", rho=1.7, bulk=2.9,
                            has_aux=True, dtype=dtype)
        shape = (3, 5, nx)
        q = dev(inputs.round_to(rng.uniform(-1, 1, (4,) + shape), dtype), dtype)
        a = dev(inputs.round_to(rng.uniform(0.5, 2.0, (2,) + shape), dtype), dtype)
        s = claw.Solver(prob, q, a)
        s.sweep(0, 0.3 / nx / 2.0)
        s.sync_state()
        done(f"sweep3d_whole_{dtype}_{nx}", host(q))
        s.close()
    # fused x and y steps of 3D acoustics (rows of 64 cells per wavefront), adaptive
    for nx, ny, aux, dtype, ybc in ((256, 5, True, "f32", "wall"), (128, 3, False, "f64", "periodic")):
        rng = np.random.default_rng(_seed("fused3", nx, dtype))
        prob = inputs._base(3, (nx, ny, 3), (0, 0, 0), (1.0, 0.8, 0.6), "acoustics", 4, "extrap", rho=1.7,
                            bulk=2.9, has_aux=aux, dtype=dtype)
        prob["bc_lo"] = ("extrap", ybc, "wall")
        prob["bc_hi"] = ("extrap", ybc, "periodic")
        prob["fused_step"] = True
        shape = (3, ny, nx)
        q = dev(inputs.round_to(rng.uniform(-1, 1, (4,) + shape), dtype), dtype)
        a = dev(inputs.round_to(rng.uniform(0.5, 2.0, (2,) + shape), dtype), dtype) if aux else None
        s = claw.Solver(prob, q, a)
        s.advance(3)
        done(f"fused3_{dtype}_{nx}x{ny}", host(q))
        s.close()
    # fused steps (walls, and periodic in y), adaptive
    for dtype in ("f32", "f64"):
        for ybc in ("wall", "periodic"):
            prob, q0, _ = inputs.sw_radial_dam(n=97, dtype=dtype, nsteps=6, seed=1)
            prob["fused_step"] = True
            prob["bc_lo"] = ("wall", ybc, "wall")
            prob["bc_hi"] = ("wall", ybc, "wall")
            q = dev(q0, dtype)
            s = claw.Solver(prob, q)
            s.advance(6)
            done(f"fused_{dtype}_{ybc}", host(q))
            s.close()
    # batched ensemble
    probs, qs = [], []
    for k, side in enumerate((64, 77, 128)):
        p, q0, _ = inputs.sw_hump(n=side, seed=10 + k, dtype="f32")
        probs.append(p)
        qs.append(dev(q0, "f32"))
    b = claw.BatchSolver(probs, qs)
    b.advance(5)
    for k, q in enumerate(qs):
        done(f"batch_{k}", host(q))
    b.close()
    # batched fused steps
    probs, qs = [], []
    for k, side in enumerate((64, 77, 300)):
        p, q0, _ = inputs.sw_hump(n=side, seed=20 + k, dtype="f32")
        p["fused_step"] = True
        probs.append(p)
        qs.append(dev(q0, "f32"))
    b = claw.BatchSolver(probs, qs)
    b.advance(4)
    for k, q in enumerate(qs):
        done(f"batch_fused_{k}", host(q))
    b.close()
    # plug-in solver (Burgers-type law)
    prob, q0, _ = inputs.burgers2d(n=80, seed=1, dtype="f64", nsteps=5)
    q = dev(q0, "f64")
    s = claw.Solver(prob, q)
    s.advance(5)
    done("plugin_burgers_f64", host(q))
    s.close()
    # learned correction: forward pass, fallback and application, learned steps
    from paper_1805_08846_amd import learned
    nx, ny = 130, 70
    th = inputs.lc_init_params(seed=11, out_gain=1.0)
    lc = claw.LearnedCorrection(nx, ny, learned.default_norm(), th)
    p, q0, _ = inputs.sw_hump(n=128, seed=4, dtype="f32")
    rng = np.random.default_rng(5)
    qn = dev(1.0 + 0.1 * rng.uniform(size=(3, ny, nx)), "f32")
    dF = torch.zeros((3, ny, nx + 1), device="cuda")
    dG = torch.zeros((3, ny + 1, nx), device="cuda")
    lc.forward(qn, dF, dG)
    done("learned_dF", host(dF))
    done("learned_dG", host(dG))
    res = torch.empty_like(qn)
    lc.apply(qn, qn, dF, dG, 0.1, 0.1, learned.TAU, learned.KAPPA, res)
    done("learned_apply", host(res))
    lc2 = claw.LearnedCorrection(128, 128, learned.default_norm(), inputs.lc_init_params(seed=12, out_gain=0.05))
    q = dev(q0, "f32")
    s = claw.Solver(p, q)
    lc2.advance(s, 4, 2 * learned.fine_dt(256), learned.TAU, learned.KAPPA)
    done("learned_advance", host(q))
    s.close()
    # the sweep that allocates nothing
    prob = inputs._base(2, (300, 70), (-1.0, -0.5), (1.2, 0.9), "shallow_water", 3, "wall", dtype="f32")
    q0 = inputs.round_to(inputs.random_states("shallow_water", 300 * 70, seed=8).T.reshape(3, 1, 70, 300), "f32")
    src, dst = dev(q0, "f32"), torch.empty((3, 1, 70, 300), dtype=torch.float32, device="cuda")
    d = claw.desc_from_problem(prob)
    claw.claw_sweep_noalloc(d, src, dst, None, 1, 0.2 / 70, None, torch.cuda.current_stream().cuda_stream)
    done("noalloc", host(dst))
    return out, checks


def main(path):
    from paper_1805_08846_amd import claw
    out, checks = run(claw, take=claw.claw_debug_take)
    arrays = {f"q_{k}": v for k, v in out.items()}
    arrays.update({f"chk_{k}": np.array(v, dtype=np.int64) for k, v in checks.items()})
    np.savez(path, **arrays)
    print(f"# {len(out)} cases, failed range checks: {sum(v[0] for v in checks.values())}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
