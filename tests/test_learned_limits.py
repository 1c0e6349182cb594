"""Why the learned coarse correction gains little on depth (CPU, oracle only).

The correction is a flux difference computed from the four-cell stencil of
each face of the coarse state Q^n (include/claw.h, claw_lc_*).  Its target
is the one-step residual r = C(Q_f^{n+2}) - S_c(Q_c^n) between the
coarse-grained fine run and the plain coarse step.  Measured here on the
Gaussian-hump family at fine side 256 (coarse 128), with the oracle's plain
method for both grids:

* the depth residual's energy sits mostly at the grid scale (wavenumbers
  above a quarter cycle per cell), where a coarse state carries no
  information about the fine run's sub-cell structure;
* the best linear correction on the network's own inputs (the 12 stencil
  features and a bias per face direction, fitted by least squares on
  training runs) cuts the held-out one-step L1 error of both momenta by
  more than a third, but that of the depth by less than 5 %.

So a per-face network can learn the momentum part of the residual and not
the depth part, which is the quantity the evaluation scores.
"""
import numpy as np
import pytest

import oracle
from oracle import learned as OL
from paper_1805_08846_amd import inputs

NF, NC = 256, 128
DTF = 0.9 / (NF * 1.6)  # the training recipe's fixed fine step (global speed bound 1.6)
DTC = 2 * DTF
NU = DTC * NC


def _step(prob, q, dt):
    out, _, _ = oracle.step(prob, q, None, dt)
    return out.reshape(3, q.shape[-2], q.shape[-1])


def _coarsen(q):
    return q.reshape(3, q.shape[-2] // 2, 2, q.shape[-1] // 2, 2).mean(axis=(2, 4))


def _samples(seed, every):
    pf, qf, _ = inputs.sw_hump(n=NF, seed=seed, dtype="f64")
    pc, _, _ = inputs.sw_hump(n=NC, seed=seed, dtype="f64")
    qf = qf.reshape(3, NF, NF)
    out = []
    for k in range(NF // 2):
        qc = _coarsen(qf)
        plain = _step(pc, qc, DTC)
        qf = _step(pf, _step(pf, qf, DTF), DTF)
        if k % every == every // 2:
            out.append((qc, _coarsen(qf) - plain))
    return out


def _design(qc, norm):
    """Linear map from per-direction coefficients (12 features + bias each)
    to the cell-level flux difference -nu (dF_{i+1/2} - dF_{i-1/2}) - nu (dG ...)."""
    Fx = np.concatenate([OL.features(qc, 0, norm), np.ones(((NC - 1) * NC, 1))], 1).reshape(NC, NC - 1, 13)
    Fy = np.concatenate([OL.features(qc, 1, norm), np.ones(((NC - 1) * NC, 1))], 1).reshape(NC, NC - 1, 13)
    A = np.zeros((NC, NC, 26))
    A[:, :-1, :13] -= NU * Fx
    A[:, 1:, :13] += NU * Fx
    Fyt = Fy.transpose(1, 0, 2)
    A[:-1, :, 13:] -= NU * Fyt
    A[1:, :, 13:] += NU * Fyt
    return A.reshape(NC * NC, 26)


@pytest.fixture(scope="module")
def data():
    norm = inputs.lc_norm()
    train = [s for seed in (1000, 1001, 1002) for s in _samples(seed, 4)]
    test = _samples(1, 8)
    return norm, train, test


def test_depth_residual_is_mostly_grid_scale(data):
    _, _, test = data
    k = np.fft.fftfreq(NC)
    K = np.hypot(*np.meshgrid(k, k))
    shares = []
    for _, r in test:
        e = np.abs(np.fft.fft2(r[0])) ** 2
        shares.append(e[K > 0.25].sum() / e.sum())
    print("grid-scale share of the depth residual's energy:", np.round(shares, 2))
    assert np.median(shares) > 0.5


def test_best_linear_correction_helps_momenta_not_depth(data):
    norm, train, test = data
    AtA = np.zeros((26, 26))
    Atb = np.zeros((3, 26))
    for qc, r in train:
        A = _design(qc, norm)
        AtA += A.T @ A
        Atb += np.stack([A.T @ r[f].ravel() for f in range(3)])
    reg = 1e-10 * np.trace(AtA) / 26 * np.eye(26)
    W = np.stack([np.linalg.solve(AtA + reg, Atb[f]) for f in range(3)])
    e_plain, e_corr = np.zeros(3), np.zeros(3)
    for qc, r in test:
        A = _design(qc, norm)
        for f in range(3):
            e_plain[f] += np.abs(r[f]).mean()
            e_corr[f] += np.abs(r[f].ravel() - A @ W[f]).mean()
    gain = 1 - e_corr / e_plain
    print("held-out one-step L1 reduction (h, hu, hv):", np.round(gain, 3))
    assert gain[1] > 0.33 and gain[2] > 0.33
    assert gain[0] < 0.05
