"""The range-checked debug build (libclaw_debug.so, CLAW_DEBUG) on small runs
of every kernel family: no buffer access and no boundary index of any kernel
leaves its field, and the debug build computes the same states as the
release build, bit for bit (the checks add no arithmetic).

The debug build runs in a child process (tests/debug_cases.py: the binding
loads one library per process); the release build runs the same cases here.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEBUG_LIB = os.path.join(ROOT, "paper_1805_08846_amd", "libclaw_debug.so")


@pytest.fixture(scope="module")
def claw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_08846_amd import claw as c
    return c


def test_debug_build_has_no_range_failures_and_matches_release(claw, tmp_path):
    if not os.path.exists(DEBUG_LIB):
        pytest.fail("libclaw_debug.so is not built (python -m paper_1805_08846_amd.build --debug)")
    out = tmp_path / "debug_cases.npz"
    env = dict(os.environ, CLAW_LIBRARY=DEBUG_LIB)
    print("# child: debug build on every kernel family", flush=True)
    r = subprocess.run([sys.executable, os.path.join(HERE, "debug_cases.py"), str(out)], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=500)
    print(r.stdout[-2000:], r.stderr[-4000:], flush=True)
    assert r.returncode == 0
    dbg = np.load(out)
    sys.path.insert(0, HERE)
    import debug_cases
    rel, _ = debug_cases.run(claw)
    failed = {k[4:]: tuple(dbg[k]) for k in dbg.files if k.startswith("chk_") and dbg[k][0] != 0}
    assert not failed, f"failed range checks (count, first source line) per case: {failed}"
    assert sorted(k[2:] for k in dbg.files if k.startswith("q_")) == sorted(rel)
    for name, q in rel.items():
        d = dbg["q_" + name]
        assert np.isfinite(q).all(), name
        assert np.array_equal(d.view(np.uint64), q.view(np.uint64)), f"{name}: debug and release builds differ"
