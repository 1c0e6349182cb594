"""CPU oracle of the learned coarse-grid flux correction (TEST INFRASTRUCTURE).

Plain numpy in FP64.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product library never does.

What is computed.  The method's conservative update (section 3, equation
LW-update) changes a cell only through differences of interface fluxes.  The
learned part adds a second flux difference on a grid twice as coarse as the
reference run: a small network maps the four-cell stencil around each
interior interface to a correction dF (three components), and the corrected
coarse step is

    Q^{n+1} = S(Q^n) - nu_x (dF_{i+1/2} - dF_{i-1/2}) - nu_y (dG_{j+1/2} - dG_{j-1/2})

with S the plain split step and nu = dt/dx.  Corrections on wall faces are
zero, so the sum of every field changes by nothing but rounding.  The network
is this project's extension of the method; the paper has no such part, so
every definition here is the project's own and the pins are finite
differences, invariants and special cases (tests/test_oracle_learned.py).

Networks.  One per sweep direction (x faces, y faces): the split step
sweeps x then y, so the two directions carry different errors and share no
weights.  Each is 12 -> 64 -> 64 -> 3 with ReLU, parameters
    W1 (64, 12), b1 (64), W2 (64, 64), b2 (64), W3 (3, 64), b3 (3)
flattened in that order (row-major) into 5187 numbers; the parameter vector
is the x-face network followed by the y-face network (10374 numbers).

Interface frame.  An interface along direction d sees its stencil in the
channels (h, m_n, m_t): depth, momentum along d, momentum across d.  x faces
take (h, hu, hv); y faces take (h, hv, hu), and the network output
(dh, dm_n, dm_t) is mapped back the same way.  Stencil cells k-2, k-1, k, k+1
around face k-1/2; a cell outside the grid is the mirror image across the
wall with m_n negated (reflecting walls, the same rule as the ghost cells of
the plain method).

Features (channel c, stencil values a, b, e, f): the level, slope, curvature
and third difference of the stencil at the face, each over its own scale,
    x[4c+0] = ((b + e) / 2 - mu_c) / sl_c          (mu = (mu_h, 0, 0))
    x[4c+1] = (e - b) / sd1_c
    x[4c+2] = ((a + f) - (b + e)) / sd2_c
    x[4c+3] = ((f - a) - 3 (e - b)) / sd3_c
(an invertible linear map of the four stencil values; separate scales keep
each at full BF16 relative precision, where raw differences of nearly equal
values would lose the higher differences to rounding).
Output: d = s_out * y, per channel.

Rounding points (BF16 operands, FP32-or-better accumulation), emulated when
``bf16=True``: the features x; the weights W1, W2, W3 (biases stay wide);
the activations h1 = bf16(relu(z1)), h2 = bf16(relu(z2)); in the backward
pass the output gradient dy and the pre-activation gradients dz2, dz1 where
they enter a product.  The ReLU derivative is taken as [h > 0] on the
rounded activation.  Bias gradients sum the unrounded gradients.  Values are
rounded FP64 -> FP32 -> BF16 (round to nearest even), as a device rounding its
FP32 values would.

Loss (training).  Per cell c and field f, with residual r = target - S(Q^n)
and correction p = -nu_x (dF_{i+1/2} - dF_{i-1/2}) - nu_y (dG_{j+1/2} - dG_{j-1/2}):
    L = sum_{c,f} w_f (p_{c,f} - r_{c,f})^2 / (3 N)

Fallback (inference).  A face keeps its correction only if
    |h_R - h_L| <= tau * min(h_L, h_R)       (no shock across it)
    |d_c| <= kappa * s_out_c for all three components c of the face frame
                                             (the output within kappa of its
                                             training scale)
and neither neighbour is a bad cell.  A cell is bad when the depth it would
get from only those of its kept faces that lower it,
    p - [(max(nu_x dF_r, 0) - min(nu_x dF_l, 0)) + (max(nu_y dG_t, 0) - min(nu_y dG_b, 0))],
is below half its plain depth p or not positive.  That worst case bounds the
depth after any of its faces are dropped, so every cell ends at least at half
its plain depth (a bad cell loses all its faces and keeps its plain depth).
These decisions are taken in FP32 arithmetic on FP32 data, in this order, as
the device takes them.
"""
import numpy as np

H1 = 64
H2 = 64
NIN = 12
NOUT = 3
SHAPES = (("W1", (H1, NIN)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)),
          ("W3", (NOUT, H2)), ("b3", (NOUT,)))
NET = sum(int(np.prod(s)) for _, s in SHAPES)  # 5187 per network
NPARAM = 2 * NET  # x-face network, then y-face network


def unpack(theta):
    """Parameters of one network (NET numbers) -> dict of arrays (views, FP64)."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to bfloat16 (through FP32, nearest even), returned as FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


# ---------------------------------------------------------------------------
# Stencils and features
# ---------------------------------------------------------------------------
def _frame(q, axis):
    """(h, m_n, m_t) of a state q[3, ny, nx] for faces along `axis` (0 = x, 1 = y),
    with the face direction moved to the last array axis."""
    h, hu, hv = (np.asarray(q[k], dtype=np.float64) for k in range(3))
    if axis == 0:
        return np.stack([h, hu, hv])            # (3, ny, nx): faces along x
    return np.stack([h.T, hv.T, hu.T])          # (3, nx, ny): faces along y


def _padded(fr):
    """Frame state with one mirrored wall ghost on each end of the last axis."""
    n = fr.shape[-1]
    out = np.empty(fr.shape[:-1] + (n + 2,))
    out[..., 1:n + 1] = fr
    out[..., 0] = fr[..., 0]
    out[..., n + 1] = fr[..., n - 1]
    out[1, :, 0] *= -1.0
    out[1, :, n + 1] *= -1.0
    return out


def stencils(q, axis):
    """Stencil values of the interior faces along `axis`: array (3, L, n-1, 4)
    with L lines and faces k = 1 .. n-1 (face k between cells k-1 and k);
    the last index runs over cells k-2, k-1, k, k+1."""
    p = _padded(_frame(q, axis))  # padded index = cell + 1
    n = p.shape[-1] - 2
    k = np.arange(1, n)
    cols = [p[..., k - 2 + 1 + s] for s in range(4)]
    return np.stack(cols, axis=-1)


def features(q, axis, norm):
    """Network inputs (L * (n-1), 12) of the interior faces along `axis`."""
    st = stencils(q, axis)
    mu = np.array([norm["mu_h"], 0.0, 0.0])
    sl, s1, s2, s3 = (np.asarray(norm[k], dtype=np.float64) for k in ("sl", "sd1", "sd2", "sd3"))
    a, b, e, f = (st[..., s] for s in range(4))
    cols = []
    for c in range(3):
        cols += [((b[c] + e[c]) * 0.5 - mu[c]) / sl[c], (e[c] - b[c]) / s1[c],
                 ((a[c] + f[c]) - (b[c] + e[c])) / s2[c], ((f[c] - a[c]) - 3 * (e[c] - b[c])) / s3[c]]
    return np.stack([x.ravel() for x in cols], axis=1)


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------
def forward(theta, x, bf=True):
    """Forward pass of one network (NET parameters) on inputs x (N, 12).
    Returns a dict of every intermediate."""
    p = unpack(theta)
    xb = _r(x, bf)
    W1, W2, W3 = _r(p["W1"], bf), _r(p["W2"], bf), _r(p["W3"], bf)
    z1 = xb @ W1.T + p["b1"]
    h1 = _r(np.maximum(z1, 0.0), bf)
    z2 = h1 @ W2.T + p["b2"]
    h2 = _r(np.maximum(z2, 0.0), bf)
    y = h2 @ W3.T + p["b3"]
    return {"x": xb, "W1": W1, "W2": W2, "W3": W3, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "y": y}


def backward(fw, dy, bf=True):
    """Gradients of sum(dy * y) with respect to one network's parameters,
    given its forward record `fw`; flat vector in the parameter order."""
    dyr = _r(dy, bf)
    dh2 = dyr @ fw["W3"]
    dz2 = dh2 * (fw["h2"] > 0)
    dz2r = _r(dz2, bf)
    dh1 = dz2r @ fw["W2"]
    dz1 = dh1 * (fw["h1"] > 0)
    dz1r = _r(dz1, bf)
    g = {
        "W3": dyr.T @ fw["h2"], "b3": dy.sum(axis=0),
        "W2": dz2r.T @ fw["h1"], "b2": dz2.sum(axis=0),
        "W1": dz1r.T @ fw["x"], "b1": dz1.sum(axis=0),
    }
    return pack(g)


def face_corrections(theta, norm, q, bf=True):
    """Corrections on every face: dF (3, ny, nx+1) and dG (3, ny+1, nx), in the
    state's component order (h, hu, hv); wall faces are zero."""
    _, ny, nx = q.shape
    s_out = np.asarray(norm["s_out"], dtype=np.float64)
    dF = np.zeros((3, ny, nx + 1))
    dG = np.zeros((3, ny + 1, nx))
    theta = np.asarray(theta, dtype=np.float64)
    yx = forward(theta[:NET], features(q, 0, norm), bf)["y"] * s_out  # (ny*(nx-1), 3) frame (h, hu, hv)
    yy = forward(theta[NET:], features(q, 1, norm), bf)["y"] * s_out  # (nx*(ny-1), 3) frame (h, hv, hu)
    yx = yx.reshape(ny, nx - 1, 3)
    yy = yy.reshape(nx, ny - 1, 3)
    dF[0, :, 1:nx] = yx[..., 0]
    dF[1, :, 1:nx] = yx[..., 1]
    dF[2, :, 1:nx] = yx[..., 2]
    dG[0, 1:ny, :] = yy[..., 0].T
    dG[2, 1:ny, :] = yy[..., 1].T
    dG[1, 1:ny, :] = yy[..., 2].T
    return dF, dG


def flux_difference(dF, dG, nux, nuy):
    """p = -nu_x (dF_{i+1/2} - dF_{i-1/2}) - nu_y (dG_{j+1/2} - dG_{j-1/2})."""
    return -nux * (dF[:, :, 1:] - dF[:, :, :-1]) - nuy * (dG[:, 1:, :] - dG[:, :-1, :])


def loss(theta, norm, q, target, plain, nux, nuy, w, bf=True):
    dF, dG = face_corrections(theta, norm, q, bf)
    p = flux_difference(dF, dG, nux, nuy)
    r = np.asarray(target, dtype=np.float64) - np.asarray(plain, dtype=np.float64)
    n = q.shape[1] * q.shape[2]
    w = np.asarray(w, dtype=np.float64).reshape(3, 1, 1)
    return float(np.sum(w * (p - r) ** 2) / (3 * n))


def loss_grad(theta, norm, q, target, plain, nux, nuy, w, bf=True):
    """(loss, flat gradient) of `loss` by the chain rule written out:
    cell gradient g = 2 w (p - r) / (3N); face gradient dL/dF_{k-1/2} =
    nu (g_k - g_{k-1}); output gradient dy = s_out * (face gradient in the
    face frame); then each network's backward pass over its faces."""
    _, ny, nx = q.shape
    s_out = np.asarray(norm["s_out"], dtype=np.float64)
    dF, dG = face_corrections(theta, norm, q, bf)
    p = flux_difference(dF, dG, nux, nuy)
    r = np.asarray(target, dtype=np.float64) - np.asarray(plain, dtype=np.float64)
    n = ny * nx
    wv = np.asarray(w, dtype=np.float64).reshape(3, 1, 1)
    L = float(np.sum(wv * (p - r) ** 2) / (3 * n))
    g = 2.0 * wv * (p - r) / (3 * n)
    # x faces k = 1..nx-1: cell k gets +nu dF_{k-1/2}, cell k-1 gets -nu dF_{k-1/2}
    gFx = nux * (g[:, :, 1:] - g[:, :, :-1])           # (3, ny, nx-1), components (h, hu, hv)
    gGy = nuy * (g[:, 1:, :] - g[:, :-1, :])           # (3, ny-1, nx)
    dyx = np.stack([gFx[0], gFx[1], gFx[2]], axis=-1).reshape(-1, 3) * s_out
    dyy = np.stack([gGy[0].T, gGy[2].T, gGy[1].T], axis=-1).reshape(-1, 3) * s_out
    theta = np.asarray(theta, dtype=np.float64)
    gx = backward(forward(theta[:NET], features(q, 0, norm), bf), dyx, bf)
    gy = backward(forward(theta[NET:], features(q, 1, norm), bf), dyy, bf)
    return L, np.concatenate([gx, gy])


def adam(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------------------
# Inference: fallback and application
# ---------------------------------------------------------------------------
def apply(qn, plain, dF, dG, nux, nuy, tau, kappa, s_out):
    """Corrected coarse state from Q^n (qn), the plain step S(Q^n) (plain) and
    face corrections dF, dG (state component order), with the fallback rules
    of the module docstring.  FP32 arithmetic throughout, as on the device.
    Returns (q_out, keepF, keepG)."""
    f32 = np.float32
    qn = np.asarray(qn, dtype=f32)
    plain = np.asarray(plain, dtype=f32)
    dF = np.asarray(dF, dtype=f32).copy()
    dG = np.asarray(dG, dtype=f32).copy()
    nux, nuy, tau, kappa = f32(nux), f32(nuy), f32(tau), f32(kappa)
    _, ny, nx = qn.shape
    h = qn[0]
    keepF = np.zeros((ny, nx + 1), dtype=bool)
    keepG = np.zeros((ny + 1, nx), dtype=bool)
    so = [f32(v) for v in s_out]
    # bound per state component: x faces (h, hu, hv) = frame (h, m_n, m_t);
    # y faces (h, hu, hv) = frame (h, m_t, m_n)
    bx = [kappa * so[0], kappa * so[1], kappa * so[2]]
    by = [kappa * so[0], kappa * so[2], kappa * so[1]]
    hl, hr = h[:, :-1], h[:, 1:]
    ok = np.abs(hr - hl) <= tau * np.minimum(hl, hr)
    for c in range(3):
        ok &= np.abs(dF[c, :, 1:nx]) <= bx[c]
    keepF[:, 1:nx] = ok
    hb, ht = h[:-1, :], h[1:, :]
    ok = np.abs(ht - hb) <= tau * np.minimum(hb, ht)
    for c in range(3):
        ok &= np.abs(dG[c, 1:ny, :]) <= by[c]
    keepG[1:ny, :] = ok

    def corrected(kF, kG):
        F = np.where(kF[None], dF, f32(0))
        G = np.where(kG[None], dG, f32(0))
        cx = nux * (F[:, :, 1:] - F[:, :, :-1])
        cy = nuy * (G[:, 1:, :] - G[:, :-1, :])
        return plain - (cx + cy)

    # worst case of each cell's depth: only the kept faces that lower it
    F0 = np.where(keepF, dF[0], f32(0))
    G0 = np.where(keepG, dG[0], f32(0))
    tl, tr = nux * F0[:, :-1], nux * F0[:, 1:]
    tb, tt = nuy * G0[:-1, :], nuy * G0[1:, :]
    f0 = f32(0)
    lower = (np.maximum(tr, f0) - np.minimum(tl, f0)) + (np.maximum(tt, f0) - np.minimum(tb, f0))
    worst = plain[0] - lower
    bad = (worst < f32(0.5) * plain[0]) | (worst <= f0)
    keepF[:, :-1] &= ~bad
    keepF[:, 1:] &= ~bad
    keepG[:-1, :] &= ~bad
    keepG[1:, :] &= ~bad
    return corrected(keepF, keepG), keepF, keepG


def coarsen(qf):
    """2 x 2 cell averages of a fine state (meqn, 2ny, 2nx) -> (meqn, ny, nx)."""
    qf = np.asarray(qf, dtype=np.float64)
    m, ny2, nx2 = qf.shape
    return qf.reshape(m, ny2 // 2, 2, nx2 // 2, 2).mean(axis=(2, 4))
