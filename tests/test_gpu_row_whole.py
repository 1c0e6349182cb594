"""Acoustics x sweeps on rows of 64 CPL cells with extrapolation at both ends
(the rows of the 256^3 acoustics workload), which the whole-row sweep kernel
takes: each single sweep against the oracle's sweep, a few adaptive 3D steps
against the oracle, and every result against the segment kernels (the
general row sweep, selected by CLAW_ROW_WHOLE=0 in a child process) value
for value.  The two kernels do the same arithmetic per face; they can differ
only in the sign of a zero, which a comparison of values ignores.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from helpers import rel_linf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, HERE)
import row_whole_cases as cases  # noqa: E402


@pytest.fixture(scope="module")
def claw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_08846_amd import claw as c
    return c


@pytest.fixture(scope="module")
def results(claw):
    return cases.run(claw)


@pytest.mark.parametrize("case", cases.SWEEPS, ids=lambda c: "_".join(str(x) for x in c))
def test_whole_row_sweep_matches_oracle(results, case):
    prob, q0, a0, dt = cases.sweep_case(*case)
    name = "sweep_" + "_".join(str(c) for c in case)
    ref, sm_ref = oracle.sweep(prob, q0, a0, 0, dt)
    err, per = rel_linf(results[name].reshape(ref.shape), ref)
    f64 = case[4] == "f64"
    assert err <= (1e-13 if f64 else 2e-6), per
    assert results[name + "_smax"][0] == pytest.approx(sm_ref, rel=1e-14 if f64 else 1e-6)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_whole_row_advance_matches_oracle(results, dtype):
    prob, q0, a0 = cases.advance_case(dtype)
    ref = oracle.advance(prob, q0, a0, 8)
    err, per = rel_linf(results[f"advance_{dtype}"].reshape(ref["q"].shape), ref["q"])
    assert err <= (1e-12 if dtype == "f64" else 2e-5), per
    t, nrej = results[f"advance_{dtype}_t"]
    assert nrej == ref["nreject"]
    assert t == pytest.approx(ref["t"], rel=1e-12 if dtype == "f64" else 1e-5)


def test_whole_row_equals_segment_kernels(results, tmp_path):
    out = tmp_path / "segment.npz"
    env = dict(os.environ, CLAW_ROW_WHOLE="0")
    print("# child: the same cases on the segment row kernels", flush=True)
    r = subprocess.run([sys.executable, os.path.join(HERE, "row_whole_cases.py"), str(out)], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:], flush=True)
    assert r.returncode == 0
    seg = np.load(out)
    assert sorted(seg.files) == sorted(results)
    for name, v in results.items():
        assert np.isfinite(v).all(), name
        assert np.array_equal(seg[name], v), f"{name}: whole-row and segment kernels differ"
