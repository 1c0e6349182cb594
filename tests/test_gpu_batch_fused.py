"""Batched ensembles on the fused 2D step (every instance with
CLAW_FLAG_FUSED_STEP): one opening launch (one thread per instance) and one
fused launch per trial for the whole batch.  Every instance must equal the
single-grid fused step bit for bit, whatever rows per workgroup or schedule
the tuner picks, and match the CPU oracle."""
import re

import numpy as np
import pytest

import oracle
from paper_1805_08846_amd import inputs
from helpers import rel_linf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIDES = [37, 64, 129, 100, 256, 300, 128, 513]


@pytest.fixture(scope="module")
def claw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_08846_amd import claw as c
    return c


def _members(seed, dtype, nsteps, sides=SIDES):
    members = inputs.sw_ensemble(sides=sides, seed=seed, dtype=dtype, nsteps=nsteps)
    for p, _ in members:
        p["fused_step"] = True
    return members


def _single(claw, prob, q0, nsteps):
    tdt = torch.float32 if prob["dtype"] == "f32" else torch.float64
    q = torch.tensor(q0, dtype=tdt, device="cuda").contiguous()
    s = claw.Solver(prob, q)
    t, nrej = s.advance(nsteps)
    torch.cuda.synchronize()
    out = q.double().cpu().numpy()
    ms, cnt = s.advance_timed(1)  # one more step, timed by kernel: which kernels ran
    s.close()
    assert cnt[0] >= 1 and cnt[1] == 0  # the single grid ran the fused step
    return out, t, nrej


def _batch(claw, members, dtype, nsteps, tiles=None, tune_path=None):
    tdt = torch.float32 if dtype == "f32" else torch.float64
    qs = [torch.tensor(q0, dtype=tdt, device="cuda").contiguous() for _, q0 in members]
    b = claw.BatchSolver([p for p, _ in members], qs)
    tuned = None
    if tiles:
        b.set_tiles(*tiles)
    if tune_path:
        tuned = b.tune(tune_path)
    t, nrej = b.advance(nsteps)
    torch.cuda.synchronize()
    outs = [q.double().cpu().numpy() for q in qs]
    b.close()
    return outs, t, nrej, tuned


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fused_batch_equals_single_fused_step_bitwise(claw, dtype):
    members = _members(3, dtype, 50)
    outs, ts, rejs, _ = _batch(claw, members, dtype, 50)
    for k, (prob, q0) in enumerate(members):
        ref, t, nrej = _single(claw, prob, q0, 50)
        assert np.array_equal(outs[k], ref), f"instance {k} (n={prob['n'][0]}) differs"
        assert ts[k] == t and rejs[k] == nrej


def test_fused_batch_rows_and_schedules_do_not_change_results(claw):
    members = _members(4, "f32", 30)
    base, _, _, _ = _batch(claw, members, "f32", 30, tiles=(32, 0, 8))
    for tiles in [(16, 1, 8), (48, 0, 8), (64, 1, 8), (24, 0, 8)]:
        outs, _, _, _ = _batch(claw, members, "f32", 30, tiles=tiles)
        for a, b in zip(outs, base):
            assert np.array_equal(a, b), tiles


def test_fused_batch_matches_oracle(claw):
    members = _members(11, "f32", 40, sides=[128, 333, 600])
    outs, ts, rejs, _ = _batch(claw, members, "f32", 40)
    for k, (prob, q0) in enumerate(members):
        ref = oracle.advance(prob, q0, None, 40)
        err, per = rel_linf(outs[k], ref["q"])
        print(f"fused batch side {prob['n'][0]}: rel Linf {err:.3e}", flush=True)
        assert err <= 1e-5, per
        assert rejs[k] == ref["nreject"]
        assert ts[k] == pytest.approx(ref["t"], rel=1e-6)


def test_fused_batch_tuner(claw, tmp_path):
    members = _members(5, "f32", 20)
    cache = str(tmp_path / "tune.json")
    outs, _, _, tuned = _batch(claw, members, "f32", 20, tune_path=cache)
    assert tuned["chunk"] in (16, 24, 32, 48, 64) and tuned["schedule"] in (0, 1)
    assert re.search(r'"gfx950/f32/sw-fused/n8/', open(cache).read())
    base, _, _, _ = _batch(claw, members, "f32", 20)
    for a, b in zip(outs, base):
        assert np.array_equal(a, b)
