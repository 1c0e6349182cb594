"""GPU parity of the learned coarse-grid correction against the CPU oracle
(oracle/learned.py), through the C ABI.

Network outputs and gradients: the device forms the features and sums the
BF16 products in FP32, the oracle in FP64 with the same BF16 rounding points,
so an input or activation next to a BF16 rounding boundary can round the other
way (one BF16 step is 2^-8 of that value).  Outputs: all but 0.1 % of the
faces (or 4 faces on small grids) agree to 1e-4 of the largest output (the
median to ~1e-9), every face to 1e-2.
Gradients, sums over all faces: 1e-3 relative per parameter tensor.  Application and fallback decisions
are FP32 on both sides from the same inputs: bitwise.
"""
import numpy as np
import pytest

from oracle import learned as L
from paper_1805_08846_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def claw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_08846_amd import claw as c
    return c


def _norm():
    return inputs.lc_norm(mu_h=1.1, sl=(0.2, 0.1, 0.1), sd1=(0.02, 0.01, 0.01), sd2=(0.03, 0.01, 0.01),
                          sd3=(0.05, 0.02, 0.02), s_out=(0.01, 0.02, 0.03))


def _state(ny, nx, seed):
    """A smooth hump plus seeded noise (FP32 values)."""
    rng = np.random.default_rng(seed)
    y, x = np.meshgrid((np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx, indexing="ij")
    h = 1.0 + 0.3 * np.exp(-((x - 0.4) ** 2 + (y - 0.6) ** 2) / 0.05) + 0.01 * rng.uniform(size=(ny, nx))
    hu = 0.1 * np.sin(3 * x + 1) * h + 0.005 * rng.uniform(-1, 1, size=(ny, nx))
    hv = 0.1 * np.cos(2 * y) * h + 0.005 * rng.uniform(-1, 1, size=(ny, nx))
    return np.stack([h, hu, hv]).astype(np.float32)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


SHAPES = [(70, 130), (17, 64), (2, 2), (65, 3)]


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_forward_matches_oracle(claw, ny, nx):
    q = _state(ny, nx, seed=nx + ny)
    th = inputs.lc_init_params(seed=11, out_gain=1.0)
    lc = claw.LearnedCorrection(nx, ny, _norm(), th)
    dF = torch.full((3, ny, nx + 1), float("nan"), device="cuda")
    dG = torch.full((3, ny + 1, nx), float("nan"), device="cuda")
    lc.forward(_dev(q), dF, dG)
    torch.cuda.synchronize()
    rF, rG = L.face_corrections(th, _norm(), q.astype(np.float64))
    gF, gG = dF.double().cpu().numpy(), dG.double().cpu().numpy()
    assert np.isfinite(gF).all() and np.isfinite(gG).all()  # wall faces written too
    assert not gF[:, :, [0, nx]].any() and not gG[:, [0, ny], :].any()
    for got, ref in ((gF, rF), (gG, rG)):
        scale = np.abs(ref).max()
        err = np.abs(got - ref)
        print(f"{ny}x{nx}: max {err.max() / scale:.2e}, median {np.median(err) / scale:.2e}")
        assert err.max() <= 1e-2 * scale
        assert np.sum(err > 1e-4 * scale) <= max(12, 1e-3 * err.size)  # a few faces (3 components each)
        assert np.median(err) <= 1e-6 * scale


@pytest.mark.parametrize("ny,nx,seed", [(70, 130, 0), (33, 40, 1)])
def test_loss_gradient_matches_oracle(claw, ny, nx, seed):
    rng = np.random.default_rng(seed)
    q = _state(ny, nx, seed)
    plain = (q + 0.002 * rng.normal(size=q.shape)).astype(np.float32)
    target = (plain + 1e-4 * rng.normal(size=q.shape)).astype(np.float32)
    th = inputs.lc_init_params(seed=seed, out_gain=1.0)
    nux, nuy, w = 0.31, 0.27, (1.0, 2.0, 3.0)
    lc = claw.LearnedCorrection(nx, ny, _norm(), th)
    lc.loss_grad(_dev(q), _dev(target), _dev(plain), nux, nuy, w)
    torch.cuda.synchronize()
    got = lc.grad.double().cpu().numpy()
    loss = lc.loss.cpu().numpy()
    ref_loss, ref = L.loss_grad(th, _norm(), q.astype(np.float64), target.astype(np.float64),
                                plain.astype(np.float64), nux, nuy, w)
    assert loss[0] == pytest.approx(ref_loss, rel=1e-4)
    r = target.astype(np.float64) - plain
    assert np.allclose(loss[1:], (r * r).sum(axis=(1, 2)), rtol=1e-5)
    o = 0
    for net in ("x", "y"):
        for name, shape in L.SHAPES:
            k = int(np.prod(shape))
            g, e = got[o:o + k], ref[o:o + k]
            rel = np.abs(g - e).max() / np.abs(e).max()
            print(f"{net} {name}: rel {rel:.2e}")
            assert rel <= 1e-3, (net, name)
            o += k
    assert o == L.NPARAM


def test_adam_matches_oracle(claw):
    rng = np.random.default_rng(3)
    th = inputs.lc_init_params(seed=3, out_gain=1.0)
    lc = claw.LearnedCorrection(16, 16, _norm(), th)
    ref, m, v = th.copy(), np.zeros(L.NPARAM), np.zeros(L.NPARAM)
    for step in range(1, 4):
        g = (rng.normal(size=L.NPARAM) * 10.0 ** rng.integers(-6, 0, size=L.NPARAM)).astype(np.float32)
        lc.grad.copy_(torch.tensor(g))
        lc.adam(1e-3)
        ref, m, v = L.adam(ref, m, v, g.astype(np.float64), step, 1e-3)
    torch.cuda.synchronize()
    got = lc.theta()
    assert np.abs(got - ref).max() <= 1e-6
    # the BF16 copies follow the new masters: forward equals the oracle at the new weights
    q = _state(16, 16, 4)
    dF = torch.empty((3, 16, 17), device="cuda")
    dG = torch.empty((3, 17, 16), device="cuda")
    lc.forward(_dev(q), dF, dG)
    torch.cuda.synchronize()
    rF, _ = L.face_corrections(got, _norm(), q.astype(np.float64))
    err = np.abs(dF.double().cpu().numpy() - rF)
    assert err.max() <= 1e-2 * np.abs(rF).max() and np.median(err) <= 1e-6 * np.abs(rF).max()


def _apply_case(ny, nx, seed, big=False, scale=1.0):
    rng = np.random.default_rng(seed)
    qn = _state(ny, nx, seed)
    qn[0, ny // 2, nx // 3] = 2.5  # a jump for the shock indicator
    plain = (qn + 0.01 * rng.normal(size=qn.shape)).astype(np.float32)
    plain[0] = np.maximum(plain[0], 0.5)
    scale = 1e30 if big else scale
    dF = (scale * 0.02 * rng.normal(size=(3, ny, nx + 1)) ** 3).astype(np.float32)
    dG = (scale * 0.02 * rng.normal(size=(3, ny + 1, nx)) ** 3).astype(np.float32)
    dF[:, :, [0, nx]] = 0
    dG[:, [0, ny], :] = 0
    return qn, plain, dF, dG


# kappa 1: the magnitude test decides; kappa 1000 with 50x larger
# corrections: the positivity pass decides
@pytest.mark.parametrize("ny,nx,seed,kappa,scale", [(70, 130, 0, 1.0, 1.0), (70, 130, 1, 1000.0, 50.0),
                                                    (9, 5, 1, 1.0, 1.0), (2, 2, 2, 1.0, 1.0)])
def test_apply_matches_oracle_bitwise(claw, ny, nx, seed, kappa, scale):
    qn, plain, dF, dG = _apply_case(ny, nx, seed, scale=scale)
    nux, nuy, tau = 0.45, 0.4, 0.3
    lc = claw.LearnedCorrection(nx, ny, _norm(), np.zeros(L.NPARAM))
    out = torch.empty((3, ny, nx), device="cuda")
    kx = torch.full((ny, nx + 1), 7, dtype=torch.uint8, device="cuda")
    ky = torch.full((ny + 1, nx), 7, dtype=torch.uint8, device="cuda")
    lc.apply(_dev(qn), _dev(plain), _dev(dF), _dev(dG), nux, nuy, tau, kappa, out, kx, ky)
    torch.cuda.synchronize()
    ref, rkx, rky = L.apply(qn, plain, dF, dG, nux, nuy, tau, kappa, _norm()["s_out"])
    assert np.array_equal(kx.cpu().numpy().astype(bool), rkx)
    assert np.array_equal(ky.cpu().numpy().astype(bool), rky)
    assert np.array_equal(out.cpu().numpy(), ref)
    if ny > 2:
        assert 0.05 < rkx.mean() < 0.95  # both outcomes occur
    # in place (out aliases plain) gives the same bytes
    pl = _dev(plain)
    lc.apply(_dev(qn), pl, _dev(dF), _dev(dG), nux, nuy, tau, kappa, pl)
    torch.cuda.synchronize()
    assert np.array_equal(pl.cpu().numpy(), ref)


def test_huge_corrections_give_the_plain_step_bitwise(claw):
    qn, plain, dF, dG = _apply_case(40, 50, 5, big=True)
    lc = claw.LearnedCorrection(50, 40, _norm(), np.zeros(L.NPARAM))
    out = torch.empty((3, 40, 50), device="cuda")
    lc.apply(_dev(qn), _dev(plain), _dev(dF), _dev(dG), 0.4, 0.4, 0.3, 0.01, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), plain)


def test_coarsen_matches_oracle(claw):
    rng = np.random.default_rng(6)
    fine = rng.uniform(0.5, 1.5, size=(3, 34, 50)).astype(np.float32)
    coarse = torch.empty((3, 17, 25), device="cuda")
    claw.claw_lc_coarsen(25, 17, _dev(fine), coarse, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    ref = L.coarsen(fine.astype(np.float64))
    assert np.abs(coarse.double().cpu().numpy() - ref).max() <= 2e-7 * np.abs(ref).max()


def test_learned_advance_replays_with_eager_work_between(claw):
    # three calls of 20 steps (a captured graph of 16 replayed each call) with
    # unrelated eager GPU work between them; after every call the state equals
    # the composition of the separate entry points, bitwise
    n, dt = 48, 0.4 / 48
    prob, q0, _ = inputs.sw_hump(n=n, seed=4, dtype="f32", nsteps=60)
    th = inputs.lc_init_params(seed=4, out_gain=1.0)
    lc = claw.LearnedCorrection(n, n, inputs.lc_norm(s_out=(2e-3, 2e-3, 2e-3)), th)
    tau, kappa = 0.5, 5.0
    qa, qb = _dev(q0), _dev(q0)
    sa, sb = claw.Solver(prob, qa), claw.Solver(prob, qb)
    dF = torch.empty((3, n, n + 1), device="cuda")
    dG = torch.empty((3, n + 1, n), device="cuda")
    for k in range(3):
        lc.advance(sa, 20, dt, tau, kappa)
        for _ in range(20):
            qn = qb.clone()
            sb.advance_fixed([dt])
            lc.forward(qn, dF, dG)
            lc.apply(qn, qb, dF, dG, dt * n, dt * n, tau, kappa, qb)
        torch.cuda.synchronize()
        assert torch.equal(qa, qb), k
        junk = torch.randn(1 << 20, device="cuda")
        float((junk * junk).sum())
        torch.cuda.synchronize()
    sa.close()
    sb.close()


@pytest.mark.parametrize("steps", [6, 40])  # 40: two captured graphs of 16 and 8 eager steps
def test_learned_advance_equals_composition_and_conserves(claw, steps):
    n, dt = 64, 0.4 / 64
    prob, q0, _ = inputs.sw_hump(n=n, seed=9, dtype="f32", nsteps=steps)
    th = inputs.lc_init_params(seed=9, out_gain=1.0)
    norm = inputs.lc_norm(s_out=(2e-3, 2e-3, 2e-3))
    tau, kappa = 0.5, 5.0
    # fused: plain step + correction from Q^n, on the device, no host round trip
    qa = _dev(q0)
    sa = claw.Solver(prob, qa)
    lc = claw.LearnedCorrection(n, n, norm, th)
    lc.advance(sa, steps, dt, tau, kappa)
    torch.cuda.synchronize()
    # composed from the separate entry points
    qb = _dev(q0)
    sb = claw.Solver(prob, qb)
    dF = torch.empty((3, n, n + 1), device="cuda")
    dG = torch.empty((3, n + 1, n), device="cuda")
    for _ in range(steps):
        qn = qb.clone()
        sb.advance_fixed([dt])
        lc.forward(qn, dF, dG)
        lc.apply(qn, qb, dF, dG, dt * n, dt * n, tau, kappa, qb)
    torch.cuda.synchronize()
    a, b = qa.cpu().numpy(), qb.cpu().numpy()
    assert np.array_equal(a, b)
    m0 = np.sum(q0[0].astype(np.float64))
    assert abs(np.sum(a[0].astype(np.float64)) - m0) <= 2e-6 * m0
    # the correction did something
    qc = _dev(q0)
    sc = claw.Solver(prob, qc)
    sc.advance_fixed([dt] * steps)
    torch.cuda.synchronize()
    assert not np.array_equal(qc.cpu().numpy(), a)
    for s in (sa, sb, sc):
        s.close()


def test_fixed_steps_graph_path_equals_eager_path(claw):
    prob, q0, _ = inputs.sw_hump(n=96, seed=2, dtype="f32", nsteps=70)
    dt = 0.5 / 96
    qa, qb = _dev(q0), _dev(q0)
    sa, sb = claw.Solver(prob, qa), claw.Solver(prob, qb)
    assert sa.advance_fixed([dt] * 70, log=False) is None  # 2 graphs of 32 + 6 eager
    cfl = sb.advance_fixed([dt] * 70)
    torch.cuda.synchronize()
    assert np.array_equal(qa.cpu().numpy(), qb.cpu().numpy())
    assert sa.control()["t"] == sb.control()["t"]
    assert 0.3 < cfl.max() < 1.0
    sa.close()
    sb.close()


def test_training_noise_matches_philox_box_muller(claw):
    # claw_lc_perturb against the published generator written out in numpy
    # (tests/helpers.philox4x32_10) and the Box-Muller transform in FP64
    from helpers import philox4x32_10
    ny, nx = 37, 29
    rng = np.random.default_rng(3)
    q = rng.uniform(0.5, 1.5, (3, ny, nx)).astype(np.float32)
    sigma = (1e-5, 3e-5, 2e-5)
    seed, call = 12345, 7
    out = torch.empty((3, ny, nx), dtype=torch.float32, device="cuda")
    claw.claw_lc_perturb(nx, ny, _dev(q), out, sigma, seed, call, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    n = 3 * ny * nx
    k = np.arange((n + 1) // 2, dtype=np.uint64)
    w = philox4x32_10(k, call, 0, 0, seed, 0)
    u0 = (w[0].astype(np.float64) + 0.5) * 2.0 ** -32
    u1 = (w[1].astype(np.float64) + 0.5) * 2.0 ** -32
    rad = np.sqrt(-2 * np.log(u0))
    z = np.stack([rad * np.cos(2 * np.pi * u1), rad * np.sin(2 * np.pi * u1)], axis=1).ravel()[:n]
    sg = np.repeat(np.asarray(sigma), ny * nx)
    want = q.astype(np.float64).ravel() + sg * z
    err = np.abs(got.ravel() - want)
    assert np.all(err <= 1e-5 * sg * (1 + np.abs(z)) + 2 * np.spacing(np.float32(2.0)))
    zz = (got.ravel() - q.astype(np.float64).ravel()) / sg
    assert abs(zz.mean()) < 0.1 and 0.9 < zz.std() < 1.1
    # in place gives the same values; another call number gives others
    qq = _dev(q)
    claw.claw_lc_perturb(nx, ny, qq, qq, sigma, seed, call, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(qq, out)
    claw.claw_lc_perturb(nx, ny, qq, qq, sigma, seed, call + 1, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert not torch.equal(qq, out)
