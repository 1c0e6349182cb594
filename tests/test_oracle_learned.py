"""Pins of the learned-correction oracle (oracle/learned.py) against things
other than itself: torch's own BF16 conversion, finite differences of the
loss, conservation of the flux difference, special cases (zero network, huge
corrections), the transpose symmetry of the x/y frames, a hand-built stencil,
the closed form of Adam's first step and the mean of the 2 x 2 coarsening."""
import numpy as np
import pytest

from oracle import learned as L
from paper_1805_08846_amd import inputs


def _state(ny=10, nx=12, seed=3):
    rng = np.random.default_rng(seed)
    h = 1.0 + 0.3 * rng.uniform(size=(ny, nx))
    hu = 0.2 * rng.uniform(-1, 1, size=(ny, nx))
    hv = 0.2 * rng.uniform(-1, 1, size=(ny, nx))
    return np.stack([h, hu, hv])


def _norm():
    return inputs.lc_norm(mu_h=1.1, sl=(0.2, 0.1, 0.1), sd1=(0.1, 0.05, 0.05), sd2=(0.1, 0.05, 0.05),
                          sd3=(0.2, 0.1, 0.1), s_out=(0.01, 0.02, 0.02))


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-20, 20, size=4000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40]])
    # exact ties between two BF16 neighbours, both parities of the kept bit
    base = rng.integers(0x3F800000 >> 16, 0x40800000 >> 16, size=200).astype(np.uint32) << 16
    ties = (base | 0x8000).view(np.float32).astype(np.float64)
    x = np.concatenate([x, ties, -ties])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    got = L.bf16(x)
    assert np.array_equal(got, ref)


def test_param_layout():
    th = inputs.lc_init_params(seed=1)
    assert L.NET == 5187 and th.size == L.NPARAM == 2 * L.NET
    for net in (th[:L.NET], th[L.NET:]):
        p = L.unpack(net)
        assert p["W1"].shape == (64, 12) and p["W3"].shape == (3, 64)
        assert np.array_equal(L.pack(p), net)
    assert not np.array_equal(th[:L.NET], th[L.NET:])  # two networks, drawn one after the other


def test_stencil_by_hand():
    # 1 x 4 grid: cells 0..3 along x, faces 1..3; face 1 needs the mirror of cell 0
    q = np.zeros((3, 1, 4))
    q[0, 0] = [1.0, 2.0, 3.0, 4.0]
    q[1, 0] = [0.1, 0.2, 0.3, 0.4]
    q[2, 0] = [5.0, 6.0, 7.0, 8.0]
    st = L.stencils(q, 0)  # (3, 1, 3, 4)
    assert np.array_equal(st[0, 0, 0], [1.0, 1.0, 2.0, 3.0])
    assert np.array_equal(st[1, 0, 0], [-0.1, 0.1, 0.2, 0.3])  # mirrored normal momentum
    assert np.array_equal(st[2, 0, 0], [5.0, 5.0, 6.0, 7.0])
    assert np.array_equal(st[0, 0, 2], [2.0, 3.0, 4.0, 4.0])
    assert np.array_equal(st[1, 0, 2], [0.2, 0.3, 0.4, -0.4])
    # along y the frame is (h, hv, hu)
    qt = np.transpose(q[[0, 2, 1]], (0, 2, 1))  # 4 x 1 grid with hu <-> hv
    sty = L.stencils(qt, 1)
    assert np.array_equal(sty, st)


@pytest.mark.parametrize("kind", ["linear", "quadratic", "cubic"])
def test_features_reproduce_polynomials(kind):
    # depth a polynomial of the cell index along x: slope, curvature and third
    # difference of the stencil are exact (cells k-2 .. k+1 around face k-1/2)
    nx = 10
    x = np.arange(nx, dtype=np.float64)
    coef = {"linear": (0.01, 0, 0), "quadratic": (0, 0.002, 0), "cubic": (0, 0, 0.0003)}[kind]
    q = np.zeros((3, 2, nx))
    q[0] = 1.0 + coef[0] * x + coef[1] * x ** 2 + coef[2] * x ** 3
    f = L.features(q, 0, inputs.lc_norm(mu_h=1.0, sl=(1, 1, 1), sd1=(1, 1, 1), sd2=(1, 1, 1), sd3=(1, 1, 1)))
    inner = f.reshape(2, nx - 1, 12)[:, 1:-1]  # faces k = 2 .. nx-2, away from the walls
    k = np.arange(2, nx - 1, dtype=np.float64)
    level = coef[0] * (k - 0.5) + coef[1] * ((k - 1) ** 2 + k ** 2) / 2 + coef[2] * ((k - 1) ** 3 + k ** 3) / 2
    slope = coef[0] + coef[1] * (2 * k - 1) + coef[2] * (3 * k * k - 3 * k + 1)
    assert np.allclose(inner[..., 0], level, atol=1e-12)
    assert np.allclose(inner[..., 1], slope, atol=1e-12)
    assert np.allclose(inner[..., 2], 4 * coef[1] + coef[2] * (12 * k - 6), atol=1e-12)
    assert np.allclose(inner[..., 3], 6 * coef[2], atol=1e-12)
    assert np.allclose(inner[..., 4:], 0.0)


@pytest.mark.parametrize("seed", [0, 1])
def test_loss_gradient_finite_differences(seed):
    rng = np.random.default_rng(seed)
    q = _state(seed=seed)
    th = inputs.lc_init_params(seed=seed, out_gain=1.0) + 0.01 * rng.normal(size=L.NPARAM)
    plain = q + 0.01 * rng.normal(size=q.shape)
    target = plain + 0.001 * rng.normal(size=q.shape)
    args = (_norm(), q, target, plain, 0.3, 0.25, (1.0, 2.0, 3.0))
    loss, g = L.loss_grad(th, *args, bf=False)
    assert loss == pytest.approx(L.loss(th, *args, bf=False), rel=1e-14)
    one = [rng.choice(768, 6, replace=False), 768 + rng.choice(64, 3, replace=False),
           832 + rng.choice(4096, 8, replace=False), 4928 + rng.choice(64, 3, replace=False),
           4992 + rng.choice(192, 5, replace=False), [5184, 5185, 5186]]
    idx = np.concatenate(one + [L.NET + np.asarray(i) for i in one])  # both networks
    for i in idx:
        eps = 1e-6 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (L.loss(tp, *args, bf=False) - L.loss(tm, *args, bf=False)) / (2 * eps)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9 * np.abs(g).max()), i


def test_bf16_gradient_close_to_exact():
    rng = np.random.default_rng(5)
    q = _state(seed=5)
    th = inputs.lc_init_params(seed=5, out_gain=1.0)
    plain = q + 0.01 * rng.normal(size=q.shape)
    target = plain + 0.001 * rng.normal(size=q.shape)
    args = (_norm(), q, target, plain, 0.3, 0.25, (1.0, 1.0, 1.0))
    _, g0 = L.loss_grad(th, *args, bf=False)
    _, g1 = L.loss_grad(th, *args, bf=True)
    assert np.abs(g1 - g0).max() <= 0.05 * np.abs(g0).max()
    assert np.abs(g1 - g0).max() > 0  # the rounding points are active


def test_flux_difference_conserves():
    rng = np.random.default_rng(2)
    ny, nx = 9, 11
    dF = rng.normal(size=(3, ny, nx + 1))
    dG = rng.normal(size=(3, ny + 1, nx))
    dF[:, :, 0] = dF[:, :, -1] = 0
    dG[:, 0, :] = dG[:, -1, :] = 0
    p = L.flux_difference(dF, dG, 0.4, 0.3)
    assert np.abs(p.sum(axis=(1, 2))).max() <= 1e-13


def test_zero_network_and_huge_corrections_give_plain():
    rng = np.random.default_rng(4)
    q = _state(seed=4).astype(np.float32)
    plain = (q + 0.01 * rng.normal(size=q.shape)).astype(np.float32)
    dF, dG = L.face_corrections(np.zeros(L.NPARAM), _norm(), q)
    assert not dF.any() and not dG.any()
    out, _, _ = L.apply(q, plain, dF, dG, 0.3, 0.3, 0.5, 0.01, _norm()["s_out"])
    assert np.array_equal(out, plain)
    big = np.full_like(dF, 1e30)
    big[:, :, 0] = big[:, :, -1] = 0
    bigG = np.full_like(dG, -1e30)
    bigG[:, 0, :] = bigG[:, -1, :] = 0
    out, kF, kG = L.apply(q, plain, big, bigG, 0.3, 0.3, 0.5, 0.01, _norm()["s_out"])
    assert not kF.any() and not kG.any()
    assert np.array_equal(out, plain)


def test_apply_conserves_and_falls_back():
    rng = np.random.default_rng(6)
    q = _state(ny=16, nx=16, seed=6).astype(np.float32)
    q[0, 5, 5] = 3.0  # a jump that the shock indicator must catch
    plain = q.copy()
    dF = (1e-3 * rng.normal(size=(3, 16, 17))).astype(np.float32)
    dG = (1e-3 * rng.normal(size=(3, 17, 16))).astype(np.float32)
    dF[:, :, 0] = dF[:, :, -1] = 0
    dG[:, 0, :] = dG[:, -1, :] = 0
    out, kF, kG = L.apply(q, plain, dF, dG, 0.3, 0.3, 0.5, 1.0, _norm()["s_out"])
    assert not kF[5, 5] and not kF[5, 6] and not kG[5, 5] and not kG[6, 5]
    assert kF[:, 1:16].mean() > 0.8
    mass = np.sum(out[0].astype(np.float64)) - np.sum(plain[0].astype(np.float64))
    assert abs(mass) <= 1e-6 * np.sum(plain[0].astype(np.float64)) / 256
    # a cell whose corrected depth would drop below half its plain depth
    dF2 = np.zeros_like(dF)
    dF2[0, 8, 8] = -0.9 / 0.3  # face 8 takes 0.9 of depth out of cell 8 and gives it to cell 7
    out2, kF2, _ = L.apply(q, plain, dF2, np.zeros_like(dG), 0.3, 0.3, 0.5, 1000.0, _norm()["s_out"])
    assert not kF2[8, 8]
    assert np.array_equal(out2, plain)
    # the magnitude test counts in output scales, per frame channel: a y face's
    # hu component is its tangential channel
    so = _norm()["s_out"]  # (h, m_n, m_t) = (0.01, 0.02, 0.02)
    dG3 = np.zeros_like(dG)
    dG3[1, 8, 3] = 1.5 * so[2]
    dG3[2, 8, 4] = 0.5 * so[1]
    _, _, kG3 = L.apply(q, plain, np.zeros_like(dF), dG3, 0.3, 0.3, 10.0, 1.0, (0.01, 0.02, 0.015))
    assert not kG3[8, 3] and kG3[8, 4]


def test_fallback_keeps_every_depth_at_half_its_plain_value():
    # Cell 8 of row 8 takes depth in through its left face and gives the same
    # amount out through its right face (net zero).  Cell 7 loses 0.6 of its
    # depth 1 through the shared face, so that face must go; judged on the
    # full correction, cell 8 would look safe, keep its right face alone and
    # end at 0.4.  Judged on its depth-lowering faces alone it is bad itself,
    # so it keeps its plain depth.
    q = np.zeros((3, 16, 16), dtype=np.float32)
    q[0] = 1.0
    plain = q.copy()
    dF = np.zeros((3, 16, 17), dtype=np.float32)
    dF[0, 8, 8] = dF[0, 8, 9] = 0.6 / 0.3
    out, kF, _ = L.apply(q, plain, dF, np.zeros((3, 17, 16), np.float32), 0.3, 0.3, 0.5, 1000.0,
                         _norm()["s_out"])
    assert not kF[8, 8] and not kF[8, 9]
    assert out[0, 8, 8] == plain[0, 8, 8] and out[0, 8, 7] == plain[0, 8, 7]
    # random corrections large enough to push many cells below half their
    # depth: after the fallback none is
    rng = np.random.default_rng(9)
    for k in range(20):
        q = _state(ny=24, nx=20, seed=100 + k).astype(np.float32)
        plain = (q + 0.01 * rng.normal(size=q.shape)).astype(np.float32)
        plain[0] = np.maximum(plain[0], 0.3)
        dF = (0.6 * rng.normal(size=(3, 24, 21))).astype(np.float32)
        dG = (0.6 * rng.normal(size=(3, 25, 20))).astype(np.float32)
        dF[:, :, [0, 20]] = 0
        dG[:, [0, 24], :] = 0
        out, kF, kG = L.apply(q, plain, dF, dG, 0.4, 0.4, 10.0, 1e6, _norm()["s_out"])
        assert 0.05 < kF[:, 1:20].mean() < 0.95
        assert np.all(out[0] >= np.float32(0.5) * plain[0] * np.float32(1 - 1e-6))


def test_transpose_symmetry():
    # swapping x <-> y (and hu <-> hv) in the state swaps the roles of the
    # two networks: the x-face network of the swapped state sees what the
    # y-face network of the original would see
    q = _state(ny=9, nx=11, seed=7)
    qt = np.transpose(q[[0, 2, 1]], (0, 2, 1))
    th = inputs.lc_init_params(seed=7, out_gain=1.0)
    swapped = np.concatenate([th[L.NET:], th[:L.NET]])
    dF, dG = L.face_corrections(swapped, _norm(), q)
    dFt, dGt = L.face_corrections(th, _norm(), qt)
    assert np.array_equal(dGt[[0, 2, 1]], np.transpose(dF, (0, 2, 1)))
    assert np.array_equal(dFt[[0, 2, 1]], np.transpose(dG, (0, 2, 1)))
    # and the x faces use only the first network
    dF2, dG2 = L.face_corrections(np.concatenate([th[:L.NET], np.zeros(L.NET)]), _norm(), q)
    dF3, _ = L.face_corrections(th, _norm(), q)
    assert np.array_equal(dF2, dF3) and not dG2.any()


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(8)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = L.adam(th, np.zeros(50), np.zeros(50), g, 1, 1e-3, eps=0.0)
    assert np.allclose(new, th - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_coarsen_mean():
    rng = np.random.default_rng(9)
    qf = rng.normal(size=(3, 8, 6))
    qc = L.coarsen(qf)
    assert qc.shape == (3, 4, 3)
    assert qc[1, 2, 1] == pytest.approx(np.mean(qf[1, 4:6, 2:4]), rel=1e-15)
    assert np.allclose(4 * qc.sum(axis=(1, 2)), qf.sum(axis=(1, 2)), rtol=1e-14)
