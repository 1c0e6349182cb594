"""Pins of the oracle's Burgers-type law, the example of a user-supplied
point-wise Riemann solver (no GPU).

The solver is checked against the exact Godunov flux of the scalar Riemann
problem (a closed form independent of the wave/fluctuation split), the sweep
against exact solutions (a moving shock, a transonic rarefaction that only
opens with the entropy fix, a smooth solution before it breaks, in 1D and
along an oblique direction in 2D), mirror symmetry for a negative flux
coefficient, conservation under periodic boundaries and the maximum
principle.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1805_08846_amd import inputs
from helpers import observed_order


def _flux(c, q):
    return c * q * q / 2.0


def _godunov_flux(c, ql, qr):
    """Flux of the exact Riemann solution at x/t = 0 for f(q) = c q^2 / 2:
    min of f over [ql, qr] if ql <= qr, else max over [qr, ql]; f has its only
    extremum at q = 0."""
    lo, hi = min(ql, qr), max(ql, qr)
    cand = [_flux(c, ql), _flux(c, qr)]
    if lo < 0.0 < hi:
        cand.append(0.0)
    return min(cand) if ql <= qr else max(cand)


def _line_problem(n, coef=(1.0, 0.0), bc="extrap", limiter="mc", ny=1, splitting="godunov"):
    prob = inputs._base(2, (n, ny), (0, 0), (1, 1), "burgers", 1, bc, coef=tuple(coef) + (0.0,),
                        limiter=limiter, splitting=splitting)
    prob["bc_lo"] = (bc, "periodic", "periodic")
    prob["bc_hi"] = (bc, "periodic", "periodic")
    return prob


def _run_to(prob, q, t_end, cfl, smax):
    dx = min(inputs.dx_of(prob, k) for k in range(prob["ndim"]))
    nsteps = int(math.ceil(t_end * smax / (cfl * dx)))
    dts = np.full(nsteps, t_end / nsteps)
    out, _ = oracle.advance_fixed(prob, q, None, dts)
    return out


# ---------------------------------------------------------------------------
# Riemann solver
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("c", [1.0, 0.5, -0.75, -1.3])
def test_fluctuations_are_the_exact_godunov_split(c):
    rng = np.random.default_rng(5)
    pairs = rng.uniform(-2.0, 2.0, size=(400, 2))
    # exact special cases: steady shock, both transonic orientations, equal states
    pairs = np.vstack([pairs, [[1.0, -1.0], [-1.0, 1.0], [-1.0, 2.0], [0.7, 0.7], [0.0, 1.0]]])
    for ql, qr in pairs:
        W, s, am, ap = oracle.riemann_burgers(ql, qr, c)
        fg = _godunov_flux(c, ql, qr)
        scale = max(1.0, abs(_flux(c, ql)), abs(_flux(c, qr)))
        assert W == qr - ql
        assert abs(s - c * (ql + qr) / 2.0) <= 1e-15 * max(1.0, abs(s))
        assert abs(am - (fg - _flux(c, ql))) <= 2e-15 * scale, (ql, qr, c)
        assert abs(ap - (_flux(c, qr) - fg)) <= 2e-15 * scale, (ql, qr, c)


def test_non_finite_state_is_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.riemann_burgers(float("nan"), 1.0, 1.0)


# ---------------------------------------------------------------------------
# Exact solutions in 1D (a line of cells, the y sweep sees a single cell)
# ---------------------------------------------------------------------------

def test_steady_shock_is_exactly_steady():
    n = 64
    prob = _line_problem(n)
    x = (np.arange(n) + 0.5) / n
    q0 = np.where(x < 0.5, 1.0, -1.0).reshape(1, 1, 1, n)
    out = _run_to(prob, q0, 0.5, 0.9, 1.0)
    assert np.array_equal(out, q0)


def test_moving_shock_has_the_rankine_hugoniot_speed():
    # q = 2 left of x = 0.25, 0 right: the shock moves at (2 + 0) / 2 = 1
    errs, ns = [], [200, 400]
    for n in ns:
        prob = _line_problem(n)
        x = (np.arange(n) + 0.5) / n
        q0 = np.where(x < 0.25, 2.0, 0.0).reshape(1, 1, 1, n)
        t = 0.3
        out = _run_to(prob, q0, t, 0.8, 2.0)[0, 0, 0]
        exact = np.where(x < 0.25 + t, 2.0, 0.0)
        errs.append(np.abs(out - exact).sum() / n)
        # the shock stays sharp: at most a few cells between the two states
        assert np.count_nonzero((out > 0.05) & (out < 1.95)) <= 6
    assert errs[-1] < 3.0 / ns[-1]


def test_transonic_rarefaction_opens_only_through_the_entropy_fix():
    # q = -1 left, +1 right: the exact solution is the fan q = (x - 1/2) / t;
    # a solver that left the jump as one wave of speed 0 would keep it forever
    errs, ns = [], [200, 400, 800]
    for n in ns:
        prob = _line_problem(n)
        x = (np.arange(n) + 0.5) / n
        q0 = np.where(x < 0.5, -1.0, 1.0).reshape(1, 1, 1, n)
        t = 0.25
        out = _run_to(prob, q0, t, 0.8, 1.0)[0, 0, 0]
        exact = np.clip((x - 0.5) / t, -1.0, 1.0)
        errs.append(np.abs(out - exact).sum() / n)
    assert errs[-1] < 0.01
    assert errs[0] > errs[1] > errs[2]
    assert observed_order(errs, ns) > 0.6


def test_negative_coefficient_is_the_mirror_image():
    n = 96
    rng = np.random.default_rng(3)
    q0 = rng.uniform(-1.0, 1.0, size=n)
    pos = _line_problem(n, coef=(1.0, 0.0))
    neg = _line_problem(n, coef=(-1.0, 0.0))
    a = _run_to(pos, q0.reshape(1, 1, 1, n), 0.2, 0.8, 1.0)[0, 0, 0]
    b = _run_to(neg, q0[::-1].copy().reshape(1, 1, 1, n), 0.2, 0.8, 1.0)[0, 0, 0]
    assert np.max(np.abs(a - b[::-1])) <= 1e-14


def _smooth_exact(x, t, a, g, amp):
    """q(x, t) = g(x - a q t) for q0 = g along the line, by Newton iteration
    (before breaking the map q -> g(x - a q t) has a unique fixed point)."""
    q = g(x)
    for _ in range(60):
        arg = x - a * q * t
        r = q - g(arg)
        dr = 1.0 + a * t * amp * 2 * math.pi * np.cos(2 * math.pi * arg)
        q = q - r / dr
    return q


def test_smooth_solution_converges_at_second_order():
    amp = 0.4
    g = lambda s: 0.5 + amp * np.sin(2 * math.pi * s)  # noqa: E731
    t = 0.2  # breaking time 1 / (2 pi amp) ~ 0.398
    errs, ns = [], [100, 200, 400]
    for n in ns:
        prob = _line_problem(n, bc="periodic")
        x = (np.arange(n) + 0.5) / n
        out = _run_to(prob, g(x).reshape(1, 1, 1, n), t, 0.8, 0.9)[0, 0, 0]
        errs.append(np.abs(out - _smooth_exact(x, t, 1.0, g, amp)).sum() / n)
    assert observed_order(errs, ns) > 1.6


def test_oblique_smooth_solution_in_2d_converges_with_strang_splitting():
    # q0 = g(x + 2y) is transported along xi = x + 2y with speed (c_x + 2 c_y) q
    amp = 0.3
    cx, cy = 1.0, 0.5
    g = lambda s: 0.5 + amp * np.sin(2 * math.pi * s)  # noqa: E731
    t = 0.15
    errs, ns = [], [64, 128]
    for n in ns:
        prob = inputs._base(2, (n, n), (0, 0), (1, 1), "burgers", 1, "periodic", coef=(cx, cy, 0.0),
                            splitting="strang")
        x, y, _ = inputs.cell_centers(prob)
        q0 = g(x + 2 * y).reshape(1, 1, n, n)
        out = _run_to(prob, q0, t, 0.8, 0.8)[0, 0]
        exact = _smooth_exact(x[0] + 2 * y[0], t, cx + 2 * cy, g, amp)
        errs.append(np.abs(out - exact).sum() / (n * n))
    assert observed_order(errs, ns) > 1.6


# ---------------------------------------------------------------------------
# Invariants of the 2D and 3D sweeps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bc", ["periodic", "wall"])
def test_conservation_and_maximum_principle_2d(bc):
    # A scalar law has no normal component: a wall mirrors the state, so the
    # boundary interface carries no fluctuation and the interior cell's flux
    # leaves through it; only periodic boundaries conserve the total.
    prob, q0, _ = inputs.burgers2d(n=96, seed=2, bc=bc)
    res = oracle.advance(prob, q0, None, 30)
    q = res["q"]
    if bc == "periodic":
        assert abs(q.sum() - q0.sum()) <= 1e-12 * np.abs(q0).sum()
    assert q.max() <= q0.max() + 1e-12 and q.min() >= q0.min() - 1e-12
    assert res["t"] > 0


def test_conservation_3d():
    prob, q0, _ = inputs.burgers3d(n=24, seed=1)
    res = oracle.advance(prob, q0, None, 10)
    assert abs(res["q"].sum() - q0.sum()) <= 1e-12 * np.abs(q0).sum()


def test_zero_coefficient_leaves_that_direction_alone():
    prob, q0, _ = inputs.burgers2d(n=48, seed=4, coef=(0.0, 1.0))
    out, sm = oracle.sweep(prob, q0, None, 0, 0.01)
    assert np.array_equal(out, q0) and sm == 0.0
    out, sm = oracle.sweep(prob, q0, None, 1, 0.01)
    assert not np.array_equal(out, q0) and sm > 0.0
