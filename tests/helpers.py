"""Shared test helpers: norms and textbook exact solutions.

Nothing here calls the GPU library or the oracle; these are the independent
mathematical references the oracle is pinned against.
"""
import math

import numpy as np


def rel_linf(a, b):
    """Relative L-infinity error of state a against reference b (shape (meqn, ...)):
    max|a - b| over all fields and cells divided by max|b| over all fields and
    cells (the relative L-infinity norm of the whole state vector).  Returns
    (that value, per-field list max|a_m - b_m| / max(||b_m||_inf, 1e-3 ||b||_inf))
    where the per-field figures are reported for diagnosis."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.array([np.max(np.abs(b[m])) for m in range(b.shape[0])])
    top = scale.max() if scale.max() > 0 else 1.0
    per = []
    worst = 0.0
    for m in range(b.shape[0]):
        d = float(np.max(np.abs(a[m] - b[m])))
        worst = max(worst, d)
        per.append(d / max(scale[m], 1e-3 * top))
    return worst / top, per


def sw_flux(q, g, normal):
    """Physical shallow-water flux in the direction of component `normal`."""
    tng = 3 - normal
    h, mn, mt = q[0], q[normal], q[tng]
    f = np.zeros(3)
    f[0] = mn
    f[normal] = mn * mn / h + 0.5 * g * h * h
    f[tng] = mn * mt / h
    return f


def sw_dam_break_exact(hl, hr, g=1.0):
    """Exact 1D dam break (u_l = u_r = 0, hl > hr): left rarefaction, right shock.
    Newton on the middle depth h_m of
      u_m = 2 (sqrt(g hl) - sqrt(g h_m))                      (1-rarefaction)
      u_m = (h_m - hr) sqrt(g/2 (1/h_m + 1/hr))               (2-shock)
    Returns dict(hm, um, shock, head, tail) and a sampler h(xi), u(xi)."""
    def f(h):
        return 2 * (math.sqrt(g * hl) - math.sqrt(g * h)) - (h - hr) * math.sqrt(
            0.5 * g * (1 / h + 1 / hr))

    h = 0.5 * (hl + hr)
    for _ in range(100):
        eps = 1e-7 * h
        d = (f(h + eps) - f(h - eps)) / (2 * eps)
        step = f(h) / d
        h -= step
        if abs(step) < 1e-15 * h:
            break
    hm = h
    um = 2 * (math.sqrt(g * hl) - math.sqrt(g * hm))
    shock = hm * um / (hm - hr)
    head = -math.sqrt(g * hl)
    tail = um - math.sqrt(g * hm)
    cl = math.sqrt(g * hl)

    def sample(xi):
        xi = np.asarray(xi, dtype=np.float64)
        h_out = np.empty_like(xi)
        u_out = np.empty_like(xi)
        left = xi <= head
        fan = (xi > head) & (xi <= tail)
        mid = (xi > tail) & (xi <= shock)
        right = xi > shock
        h_out[left] = hl
        u_out[left] = 0.0
        c = (2 * cl - xi[fan]) / 3.0
        h_out[fan] = c * c / g
        u_out[fan] = xi[fan] + c
        h_out[mid] = hm
        u_out[mid] = um
        h_out[right] = hr
        u_out[right] = 0.0
        return h_out, u_out

    return {"hm": hm, "um": um, "shock": shock, "head": head, "tail": tail}, sample


def observed_order(errors, ns):
    """Least-squares slope of -log(error) against log(n) for the finest pair."""
    e1, e2 = errors[-2], errors[-1]
    n1, n2 = ns[-2], ns[-1]
    return math.log(e1 / e2) / math.log(n2 / n1)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 of Salmon et al. (SC 2011) on numpy uint32 arrays (or
    scalars): ten rounds of the 4x32 S-box with multipliers 0xD2511F53,
    0xCD9E8D57 and key increments 0x9E3779B9, 0xBB67AE85.  Returns the four
    32-bit output words as uint64 arrays."""
    u = np.uint64
    c = [np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3)]
    k0, k1 = np.asarray(k0, dtype=np.uint64), np.asarray(k1, dtype=np.uint64)
    m32 = u(0xFFFFFFFF)
    for _ in range(10):
        p0 = u(0xD2511F53) * c[0]
        p1 = u(0xCD9E8D57) * c[2]
        c = [(p1 >> u(32)) ^ c[1] ^ k0, p1 & m32, (p0 >> u(32)) ^ c[3] ^ k1, p0 & m32]
        k0 = (k0 + u(0x9E3779B9)) & m32
        k1 = (k1 + u(0xBB67AE85)) & m32
    return c
