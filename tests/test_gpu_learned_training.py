"""What the trained network gains over the plain method: a short training on
the GPU (the project's own forward/backward/Adam kernels, data from the plain
method's fine runs), then held-out measurements against the coarse-grained
fine run.

Asserted: training lowers its loss; on held-out runs the corrected one-step
update is closer to the coarse-grained fine solution than the plain coarse
step (momentum error down by at least 5 %, depth error not up by more than
5 %); a corrected run of 50 steps stays finite and conserves mass.  The multi-step errors against the
4x-finer reference are printed, not asserted (they are reported by the
benchmark's learned workload).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def trained():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_08846_amd import learned
    tr = learned.Trainer(n_fine=1024, total_samples=40 * 250)
    for k in range(40):
        tr.run(seed=1000 + k)
    yield tr
    tr.close()


def test_training_lowers_the_loss(trained):
    first = np.mean(trained.losses[:5])
    last = np.mean(trained.losses[-5:])
    print(f"loss (in units of the first samples' residual energy): {first:.3f} -> {last:.3f}")
    assert last < 0.5 * first


def test_one_step_gain_on_held_out_runs(trained):
    from paper_1805_08846_amd import learned
    plain, corrected = learned.one_step_gain(trained.lc, seeds=[1, 2])
    print("one-step L1 per field (h, hu, hv): plain", plain, "learned", corrected)
    assert corrected[1] < 0.95 * plain[1] and corrected[2] < 0.95 * plain[2]
    assert corrected[0] < 1.05 * plain[0]


def test_corrected_run_is_stable_and_conservative(trained):
    from paper_1805_08846_amd import learned
    res = learned.evaluate(trained.lc, seeds=[3], steps_coarse=50)
    row = res["rows"][0]
    print("50 steps, L1 per field: plain 512", row["plain"][512]["l1_fields"], "plain 1024",
          row["plain"][1024]["l1_fields"], "learned 512", row["learned"]["l1_fields"])
    assert np.isfinite(row["learned"]["l1"])
    assert row["learned"]["l1"] < 10 * row["plain"][512]["l1"]
    assert row["learned"]["mass_drift"] <= 1e-6
