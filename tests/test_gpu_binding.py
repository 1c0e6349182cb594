"""The Python binding refuses device buffers whose size, type or layout differ
from what the descriptor implies, before any pointer reaches the library (the
C calls take plain pointers and cannot check them)."""
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


def test_solver_checks_state_and_aux(claw):
    prob, q0, _ = inputs.sw_radial_dam(n=32, dtype="f32", nsteps=1)
    q = torch.tensor(q0, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError, match="q must be"):
        claw.Solver(prob, q[:, :, :31].contiguous())  # one row short
    with pytest.raises(ValueError, match="aux given"):
        claw.Solver(prob, q, torch.zeros(2 * 32 * 32, device="cuda"))
    s = claw.Solver(prob, q)  # the right buffers are accepted
    s.close()
    aprob, a0, aux = inputs.acoustics3d_layers(n=12, dtype="f32", nsteps=1)
    qa = torch.tensor(a0, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError, match="aux must be"):
        claw.Solver(aprob, qa, torch.tensor(aux, dtype=torch.float32, device="cuda")[:1].contiguous())
    with pytest.raises(ValueError, match="aux is required"):
        claw.Solver(aprob, qa, None)


def test_batch_checks_each_state(claw):
    members = inputs.sw_ensemble(sides=[16, 24], seed=1, dtype="f32", nsteps=1)
    probs = [p for p, _ in members]
    qs = [torch.tensor(q, dtype=torch.float32, device="cuda") for _, q in members]
    with pytest.raises(ValueError, match="qs\\[1\\]"):
        claw.BatchSolver(probs, [qs[0], qs[0]])  # 16^2 state for the 24^2 grid
    with pytest.raises(ValueError, match="2 problems but 1"):
        claw.BatchSolver(probs, qs[:1])
    with pytest.raises(ValueError, match="qs\\[0\\]"):
        claw.BatchSolver(probs, [qs[0].double(), qs[1]])


def test_learned_checks_buffers(claw):
    nx, ny = 20, 12
    lc = claw.LearnedCorrection(nx, ny, inputs.lc_norm(), np.zeros(claw.CLAW_LC_NPARAM))
    q = torch.ones((3, ny, nx), device="cuda")
    dF = torch.zeros((3, ny, nx + 1), device="cuda")
    dG = torch.zeros((3, ny + 1, nx), device="cuda")
    with pytest.raises(ValueError, match="dF must be"):
        lc.forward(q, dG, dG)
    with pytest.raises(ValueError, match="q must be"):
        lc.forward(q.double(), dF, dG)
    out = torch.empty_like(q)
    with pytest.raises(ValueError, match="keep_y must be"):
        lc.apply(q, q, dF, dG, 0.1, 0.1, 0.3, 10.0, out, None,
                 torch.zeros((ny, nx), dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError, match="fine must be"):
        claw.claw_lc_coarsen(nx, ny, q, out, lc.stream.cuda_stream)
    lc.forward(q, dF, dG)  # the right buffers run
    torch.cuda.synchronize()
