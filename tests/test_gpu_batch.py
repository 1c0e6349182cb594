"""Batched shallow-water ensembles through the C ABI (claw_batch_*).

Every instance of a batch must equal the single-grid GPU path bitwise (the
batched kernels run the same sweep bodies), whatever tiles or schedule the
autotuner picks, and the small instances must match the CPU oracle.
"""
import os

import re

import numpy as np
import pytest

import oracle
from paper_1805_08846_amd import inputs
from helpers import rel_linf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def claw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_08846_amd import claw as c
    return c


SIDES = [37, 64, 129, 100, 256, 300, 128]


def _tensors(members, dtype):
    tdt = torch.float32 if dtype == "f32" else torch.float64
    return [torch.tensor(q0, dtype=tdt, device="cuda").contiguous() for _, q0 in members]


def _single(claw, prob, q0, nsteps):
    tdt = torch.float32 if prob["dtype"] == "f32" else torch.float64
    q = torch.tensor(q0, dtype=tdt, device="cuda").contiguous()
    s = claw.Solver(prob, q)
    t, nrej = s.advance(nsteps)
    torch.cuda.synchronize()
    out = q.double().cpu().numpy()
    s.close()
    return out, t, nrej


def _batch(claw, members, dtype, nsteps, tiles=None, tune_path=None):
    qs = _tensors(members, dtype)
    b = claw.BatchSolver([p for p, _ in members], qs)
    if tiles:
        b.set_tiles(*tiles)
    if tune_path:
        b.tune(tune_path)
    t, nrej = b.advance(nsteps)
    torch.cuda.synchronize()
    outs = [q.double().cpu().numpy() for q in qs]
    b.close()
    return outs, t, nrej


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_equals_single_grid_bitwise(claw, dtype):
    members = inputs.sw_ensemble(sides=SIDES, seed=3, dtype=dtype, nsteps=60)
    outs, ts, rejs = _batch(claw, members, dtype, 60)
    for k, (prob, q0) in enumerate(members):
        ref, t, nrej = _single(claw, prob, q0, 60)
        assert np.array_equal(outs[k], ref), f"instance {k} (n={SIDES[k]}) differs"
        assert ts[k] == t and rejs[k] == nrej


def test_tiles_and_schedules_do_not_change_results(claw):
    members = inputs.sw_ensemble(sides=SIDES, seed=4, dtype="f32", nsteps=40)
    base, _, _ = _batch(claw, members, "f32", 40, tiles=(32, 0, 8))
    for tiles in [(16, 1, 2), (128, 0, 4), (64, 1, 8), (32, 0, 2)]:
        outs, _, _ = _batch(claw, members, "f32", 40, tiles=tiles)
        for a, b in zip(outs, base):
            assert np.array_equal(a, b), tiles


PERSISTENT_SKIP = ("one persistent launch per trial (schedules 2 and 3) was removed: its first GPU run, "
                   "tiles (32, 2, 8), did not finish (killed after 180 s without output) and no cause "
                   "was shown; the library rejects these schedules")


@pytest.mark.skip(reason=PERSISTENT_SKIP)
def test_persistent_schedules_do_not_change_results(claw):
    members = inputs.sw_ensemble(sides=SIDES, seed=4, dtype="f32", nsteps=40)
    base, _, _ = _batch(claw, members, "f32", 40, tiles=(32, 0, 8))
    for tiles in [(32, 2, 8), (16, 3, 4), (128, 2, 2)]:
        outs, _, _ = _batch(claw, members, "f32", 40, tiles=tiles)
        for a, b in zip(outs, base):
            assert np.array_equal(a, b), tiles


@pytest.mark.skip(reason=PERSISTENT_SKIP)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_persistent_trials_equal_single_grids_bitwise(claw, dtype):
    # one launch per trial for the whole batch: each instance still equals its
    # single grid bit for bit, across many trials and adaptive steps
    members = inputs.sw_ensemble(sides=SIDES, seed=13, dtype=dtype, nsteps=80)
    outs, ts, rejs = _batch(claw, members, dtype, 80, tiles=(32, 3, 4))
    for k, (prob, q0) in enumerate(members):
        ref, t, nrej = _single(claw, prob, q0, 80)
        assert np.array_equal(outs[k], ref), f"instance {k} (n={SIDES[k]}) differs"
        assert ts[k] == t and rejs[k] == nrej


def test_batch_graph_replays_with_eager_work_between(claw):
    # three advance calls of the batch (captured graphs replayed) with
    # unrelated eager GPU work and synchronisations between them; after each
    # call every instance equals its single grid advanced eagerly, bitwise
    members = inputs.sw_ensemble(sides=[37, 64, 129], seed=9, dtype="f32", nsteps=120)
    qs = _tensors(members, "f32")
    b = claw.BatchSolver([p for p, _ in members], qs)
    singles = []
    for prob, q0 in members:
        q = torch.tensor(q0, dtype=torch.float32, device="cuda").contiguous()
        singles.append((claw.Solver(prob, q), q))
    for k in range(3):
        b.advance(40)
        for s, _ in singles:
            s.advance_timed(40)
        torch.cuda.synchronize()
        for i, (_, q) in enumerate(singles):
            assert torch.equal(qs[i], q), (k, i)
        junk = torch.randn(1 << 20, device="cuda")
        float((junk * junk).sum())
        torch.cuda.synchronize()
    b.close()
    for s, _ in singles:
        s.close()


def test_autotuner_cache_roundtrip(claw, tmp_path):
    members = inputs.sw_ensemble(sides=SIDES, seed=5, dtype="f32", nsteps=30)
    base, _, _ = _batch(claw, members, "f32", 30)
    cache = str(tmp_path / "tune.json")
    tuned, _, _ = _batch(claw, members, "f32", 30, tune_path=cache)
    for a, b in zip(tuned, base):
        assert np.array_equal(a, b)
    text = open(cache).read()
    assert "gfx950/f32/sw/n7/" in text and "chunk" in text and "rows_per_wave" in text
    qs = _tensors(members, "f32")
    b = claw.BatchSolver([p for p, _ in members], qs)
    first = b.tune(cache)
    again = b.tune(cache)
    b.close()
    assert first == again and first["chunk"] in (16, 32, 64, 128) and first["rows_per_wave"] in (2, 4, 8)
    # a damaged entry (chunk 0) is not used: the tuner times the candidates again
    with open(cache, "w") as fh:
        fh.write(re.sub(r'"chunk":\s*\d+', '"chunk": 0', text))
    b = claw.BatchSolver([p for p, _ in members], qs)
    retuned = b.tune(cache)
    b.close()
    assert retuned["chunk"] in (16, 32, 64, 128)
    assert '"chunk": 0' not in open(cache).read()


def test_batch_matches_oracle(claw):
    members = inputs.sw_ensemble(sides=[48, 64], seed=6, dtype="f32", nsteps=50)
    outs, ts, rejs = _batch(claw, members, "f32", 50)
    for k, (prob, q0) in enumerate(members):
        ref = oracle.advance(prob, q0, None, 50)
        err, per = rel_linf(outs[k], ref["q"])
        assert err <= 1e-5, per
        assert rejs[k] == ref["nreject"]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_matches_oracle_across_the_size_range(claw, dtype):
    # instances across the ensemble's side range 128 .. 1024 (one above 512,
    # one ragged), FP32 and FP64, 40 adaptive steps each, every cell compared
    members = inputs.sw_ensemble(sides=[128, 333, 600, 1024], seed=11, dtype=dtype, nsteps=40)
    outs, ts, rejs = _batch(claw, members, dtype, 40)
    tol = 1e-12 if dtype == "f64" else 1e-5
    for k, (prob, q0) in enumerate(members):
        ref = oracle.advance(prob, q0, None, 40)
        err, per = rel_linf(outs[k], ref["q"])
        print(f"batch {dtype} side {prob['n'][0]}: rel Linf {err:.3e} per field {per}", flush=True)
        assert err <= tol, per
        assert rejs[k] == ref["nreject"]
        assert ts[k] == pytest.approx(ref["t"], rel=1e-12 if dtype == "f64" else 1e-6)
