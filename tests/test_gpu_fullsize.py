"""Full-size parity: the HIP path at the benchmark's sizes against stored
oracle results (tests/golden/*.npz, written by make_golden.py, which calls
only the CPU oracle).

The oracle cannot be rerun here in seconds at these sizes, so its final states
are compared on 4096 seeded sample cells plus whole lines, with the norm's
denominator (max |q| over all fields and cells) taken from the full oracle
state.  FP64: 1e-12 relative L-infinity; FP32: 1e-5.
"""
import math
import os

import numpy as np
import pytest

from paper_1805_08846_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def claw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_08846_amd import claw as c
    return c


def _golden(name):
    return dict(np.load(os.path.join(GOLD, name + ".npz"), allow_pickle=False))


def _compare(q, g):
    """Relative L-inf on samples + lines; returns (global, per-field list)."""
    meqn = q.shape[0]
    flat = q.reshape(meqn, -1)
    diffs = [np.abs(flat[:, g["sample_idx"]] - g["sample_val"]).max(axis=1)]
    nz = q.shape[1]
    rows = q[:, nz // 2, g["lines_y"], :]
    diffs.append(np.abs(rows - g["rows"]).reshape(meqn, -1).max(axis=1))
    col = q[:, nz // 2, :, q.shape[3] // 2]
    diffs.append(np.abs(col - g["col"]).max(axis=1))
    d = np.max(np.stack(diffs), axis=0)
    top = g["fieldmax"].max()
    per = [float(d[m] / max(g["fieldmax"][m], 1e-3 * top)) for m in range(meqn)]
    return float(d.max() / top), per


def _run(claw, prob, q0, aux, dts=None):
    dt = torch.float64 if prob["dtype"] == "f64" else torch.float32
    q = torch.tensor(q0, dtype=dt, device="cuda").contiguous()
    a = torch.tensor(aux, dtype=dt, device="cuda").contiguous() if aux is not None else None
    s = claw.Solver(prob, q, a)
    if dts is None:
        t, nrej = s.advance(prob["nsteps"])
    else:
        s.advance_fixed(dts)
        t, nrej = s.control()["t"], 0
    torch.cuda.synchronize()
    out = q.double().cpu().numpy()
    s.close()
    return out, t, nrej


def test_sw2048_fp64_1000_adaptive_steps(claw):
    g = _golden("sw2048_f64")
    prob, q0, _ = inputs.sw_radial_dam(n=2048, dtype="f64", nsteps=1000, seed=0)
    out, t, nrej = _run(claw, prob, q0, None)
    err, per = _compare(out, g)
    print(f"sw2048 fp64: rel Linf {err:.3e} per field {per}, t {t!r} vs {float(g['t'])!r}")
    assert nrej == int(g["nreject"])
    assert err <= 1e-12
    assert t == pytest.approx(float(g["t"]), rel=1e-13)
    mass = math.fsum(out[0].ravel())
    assert abs(mass - g["sums"][0]) <= 1e-12 * g["sums"][0]


def test_sw2048_fp32_1000_prescribed_steps(claw):
    g = _golden("sw2048_f32")
    prob, q0, _ = inputs.sw_radial_dam(n=2048, dtype="f32", nsteps=1000, seed=0)
    dts = g["dts"][g["accepted"].astype(bool)]
    assert dts.size == 1000
    out, _, _ = _run(claw, prob, q0, None, dts=dts)
    err, per = _compare(out, g)
    print(f"sw2048 fp32 (oracle dt list): rel Linf {err:.3e} per field {per}")
    assert err <= 1e-5


def test_sw2048_fp32_1000_adaptive_steps(claw):
    g = _golden("sw2048_f32")
    prob, q0, _ = inputs.sw_radial_dam(n=2048, dtype="f32", nsteps=1000, seed=0)
    out, t, nrej = _run(claw, prob, q0, None)
    err, per = _compare(out, g)
    print(f"sw2048 fp32 adaptive: rel Linf {err:.3e} per field {per}, t {t} vs {float(g['t'])}")
    assert nrej == int(g["nreject"])
    assert t == pytest.approx(float(g["t"]), rel=1e-6)
    assert err <= 1e-5


def test_acoustics3d_256_fp32_200_steps(claw):
    g = _golden("ac3d256_f32")
    prob, q0, aux = inputs.acoustics3d_layers(n=256, dtype="f32", nsteps=200, seed=0)
    out, t, nrej = _run(claw, prob, q0, aux)
    err, per = _compare(out, g)
    print(f"acoustics3d 256^3 fp32: rel Linf {err:.3e} per field {per}, t {t!r}")
    assert nrej == 0
    assert t == float(g["t"]) and abs(t - 0.703125) <= 1e-12
    assert err <= 1e-5
