"""Training and evaluation of the learned coarse-grid flux correction.

A thin driver over the C ABI (``claw.py``): every numerical step of training
and of the corrected runs executes in the library's kernels (plain split
steps, 2 x 2 coarsening, the network's forward and backward passes, the loss,
Adam, fallback and application).  Python only sequences the calls, keeps the
torch buffers, and, for evaluation, measures errors on the host.

Data (the plain method generates it).  A training run starts from a seeded
Gaussian hump on an n_f x n_f grid (the ensemble family: h = 1 + A
exp(-r^2/w^2), walls, g = 1) and takes fixed steps dt_f = cfl / (n_f s_max)
with a global speed bound s_max.  Every second fine step gives one sample on
the grid of side n_f / 2:
    Q_c^n = C(Q_f^{2n}),  plain = S_c(Q_c^n) (one plain step of 2 dt_f),
    target = C(Q_f^{2n+2}),
with C the 2 x 2 average.  Samples stream straight into the training pass
(no data set is stored).

Evaluation.  The reference is the plain method at 4x the coarse resolution
(its dt halved), coarse-grained; every run starts from the cell averages of
the reference's initial state.  The error is the L1 norm of depth, mean over
coarse cells.  Plain runs at several resolutions give error and time as
functions of n; the learned run's speedup at equal error is
T_plain(n_eq) / T_learned, n_eq where the plain error equals the learned one
(log-log interpolation).
"""
import math
import time

import numpy as np

from . import claw, inputs

S_MAX = 1.6  # bound on |u| + sqrt(g h) over the hump family's runs (checked per run: CFL <= 1)
CFL = 0.9
# Training input noise per field (h, hu, hv): the network sees Q^n perturbed
# at about the level by which a coarse run drifts from the coarse-grained fine
# run, so that it does not build on grid-scale detail its own corrections
# would feed back (without it the corrected runs go unstable).
NOISE = (1e-5, 3e-5, 3e-5)
TAU = 0.3      # shock test: relative depth jump across a face
KAPPA = 1000.0  # magnitude test, in output scales (only far-out outputs fall back)


def fine_dt(n_fine):
    return CFL / (n_fine * S_MAX)


def default_norm():
    """Input scales of the hump family at side 512 (inputs.lc_norm's
    defaults); the output scales are replaced from the residuals of the first
    samples."""
    return inputs.lc_norm()


def _torch():
    import torch
    return torch


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def _dev(a):
    torch = _torch()
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def coarsen(fine, nc):
    """C(fine) on the device (one claw_lc_coarsen call)."""
    torch = _torch()
    out = torch.empty((3, nc, nc), dtype=torch.float32, device="cuda")
    claw.claw_lc_coarsen(nc, nc, fine, out, _stream())
    return out


class Trainer:
    """Streams samples of fine runs at side n_fine into Adam steps of the
    correction network on side n_fine / 2."""

    def __init__(self, n_fine=1024, norm=None, theta0=None, init_seed=0, lr=1e-3, lr_final=3e-5,
                 total_samples=None, resync=1, tau=0.3, kappa=KAPPA, noise=NOISE, noise_seed=0,
                 correct_depth=True):
        torch = _torch()
        self.nf = int(n_fine)
        self.nc = self.nf // 2
        self.dt_f = fine_dt(self.nf)
        self.dt_c = 2 * self.dt_f
        self.nu = self.dt_c * self.nc  # dt / dx on the unit square
        self.norm = dict(norm or default_norm())
        theta0 = inputs.lc_init_params(seed=init_seed) if theta0 is None else theta0
        self.lc = claw.LearnedCorrection(self.nc, self.nc, self.norm, theta0)
        self.w = (1.0, 1.0, 1.0)
        self.lr, self.lr_final = lr, lr_final
        self.total = total_samples
        self.resync, self.tau, self.kappa = int(resync), tau, kappa
        self.correct_depth = bool(correct_depth)
        # input noise per field, drawn on the device by claw_lc_perturb
        # (counter-based: seed and a per-sample call counter)
        self.noise = tuple(float(v) for v in noise)
        self.noise_seed = int(noise_seed)
        self.noise_calls = 0
        self.samples = 0
        self.losses = []
        self.scaled = False
        c = (3, self.nc, self.nc)
        self.dF = torch.empty((3, self.nc, self.nc + 1), dtype=torch.float32, device="cuda")
        self.dG = torch.empty((3, self.nc + 1, self.nc), dtype=torch.float32, device="cuda")
        self.qcn = torch.empty(c, dtype=torch.float32, device="cuda")
        self.target = torch.empty(c, dtype=torch.float32, device="cuda")
        self.plain = torch.empty(c, dtype=torch.float32, device="cuda")
        self.qin = torch.empty(c, dtype=torch.float32, device="cuda")
        pc, _, _ = inputs.sw_hump(n=self.nc, seed=0, dtype="f32")
        self.coarse = claw.Solver(pc, self.plain)

    def _lr(self):
        if not self.total:
            return self.lr
        f = min(self.samples / self.total, 1.0)
        return self.lr_final + 0.5 * (self.lr - self.lr_final) * (1 + math.cos(math.pi * f))

    def _set_scales(self, r2):
        """Output scales and loss weights from the residual energy of the
        first samples (sum r_f^2 over cells, per field), by claw_lc_scales;
        correct_depth False gives momentum-only corrections."""
        s_out, w = claw.claw_lc_scales(r2, self.nc * self.nc, self.nu, self.correct_depth)
        self.norm["s_out"] = s_out
        self.lc.desc = claw.lc_desc(self.nc, self.nc, self.norm)
        self.w = w
        self.scaled = True

    def run(self, seed, steps_fine=500):
        """One training run: steps_fine fine steps, steps_fine / 2 samples.

        With resync = 1 every sample starts from the coarse-grained fine state
        (teacher forcing).  With resync = K > 1 the coarse state is the
        corrected coarse run itself, set back to the coarse-grained fine state
        every K samples, so the network also sees the states its own
        corrections produce and the drift they must undo."""
        torch = _torch()
        pf, qf0, _ = inputs.sw_hump(n=self.nf, seed=seed, dtype="f32", nsteps=steps_fine)
        qf = _dev(qf0)
        fine = claw.Solver(pf, qf)
        claw.claw_lc_coarsen(self.nc, self.nc, qf, self.qcn, _stream())
        first = []
        for k in range(steps_fine // 2):
            self.plain.copy_(self.qcn)
            self.coarse.advance_fixed([self.dt_c], log=False)
            fine.advance_fixed([self.dt_f, self.dt_f], log=False)
            claw.claw_lc_coarsen(self.nc, self.nc, qf, self.target, _stream())
            if any(self.noise) and self.scaled:
                # the network sees a perturbed Q^n; the plain step and the target do not
                claw.claw_lc_perturb(self.nc, self.nc, self.qcn, self.qin, self.noise, self.noise_seed,
                                     self.noise_calls, _stream())
                self.noise_calls += 1
                qin = self.qin
            else:
                qin = self.qcn
            self.lc.loss_grad(qin, self.target, self.plain, self.nu, self.nu, self.w)
            if not self.scaled:
                first.append(self.lc.loss[1:].cpu().numpy().copy())
                if len(first) == 8:
                    self._set_scales(np.mean(first, axis=0))
            else:
                self.lc.adam(self._lr())
                self.samples += 1
                if self.samples % 50 == 0:
                    self.losses.append(float(self.lc.loss[0].item()))
            if self.resync <= 1 or (k + 1) % self.resync == 0 or not self.scaled:
                self.qcn, self.target = self.target, self.qcn
            else:  # the corrected coarse step from the current coarse state
                self.lc.forward(self.qcn, self.dF, self.dG)
                self.lc.apply(self.qcn, self.plain, self.dF, self.dG, self.nu, self.nu, self.tau, self.kappa,
                              self.plain)
                self.qcn.copy_(self.plain)
        fine.close()
        torch.cuda.synchronize()

    def close(self):
        self.coarse.close()


# ---------------------------------------------------------------------------
# Evaluation (errors measured on the host)
# ---------------------------------------------------------------------------
def remap_matrix(n_from, n_to):
    """Conservative 1D remap on [0, 1]: row i averages the n_from cells over
    coarse cell i by overlap length (an exact block average when n_to divides
    n_from)."""
    R = np.zeros((n_to, n_from))
    for i in range(n_to):
        a, b = i / n_to, (i + 1) / n_to
        j0 = int(math.floor(a * n_from))
        j1 = min(int(math.ceil(b * n_from)), n_from)
        for j in range(j0, j1):
            lo, hi = max(a, j / n_from), min(b, (j + 1) / n_from)
            if hi > lo:
                R[i, j] = (hi - lo) * n_to
    return R


def remap(q, n_to):
    n = q.shape[-1]
    if n == n_to:
        return np.asarray(q, dtype=np.float64)
    R = remap_matrix(n, n_to)
    return np.stack([R @ np.asarray(q[f], dtype=np.float64) @ R.T for f in range(q.shape[0])])


def _timed_plain(prob, q0, dt, steps, repeat=2):
    """Final state and best GPU wall time of `steps` plain fixed steps."""
    torch = _torch()
    best, out = float("inf"), None
    for _ in range(repeat):
        q = _dev(q0)
        s = claw.Solver(prob, q)
        s.advance_fixed([dt] * 2, log=False)  # warm the kernels
        q.copy_(_dev(q0))
        s.close()
        s = claw.Solver(prob, q)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance_fixed([dt] * steps, log=False)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
        out = q.cpu().numpy()
        s.close()
    return out, best


def _timed_learned(lc, prob, q0, dt, steps, tau, kappa, repeat=2):
    torch = _torch()
    best, out = float("inf"), None
    for _ in range(repeat):
        q = _dev(q0)
        s = claw.Solver(prob, q)
        lc.advance(s, 2, dt, tau, kappa)
        q.copy_(_dev(q0))
        s.close()
        s = claw.Solver(prob, q)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lc.advance(s, steps, dt, tau, kappa)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
        out = q.cpu().numpy()
        s.close()
    return out, best


def evaluate(lc, seeds, n_coarse=512, steps_coarse=250, grids=(512, 1024), tau=TAU, kappa=KAPPA,
             ref_factor=4):
    """Errors and times of plain runs on `grids` (multiples of n_coarse that
    divide the reference's side, so every remap is an exact block average) and
    of the learned run on n_coarse, against the plain run at ref_factor *
    n_coarse coarse-grained; all runs span the same time T = steps_coarse *
    dt_c and start from the cell averages of the reference's initial state."""
    nr = ref_factor * n_coarse
    if any(n % n_coarse or nr % n for n in grids):
        raise ValueError("plain grids must nest between the coarse grid and the reference")
    dt_c = 2 * fine_dt(2 * n_coarse)
    T = steps_coarse * dt_c
    rows = []
    for seed in seeds:
        pr, qr0, _ = inputs.sw_hump(n=nr, seed=seed, dtype="f32")
        ref_steps = steps_coarse * ref_factor
        qref, _ = _timed_plain(pr, qr0, T / ref_steps, ref_steps, repeat=1)
        qref_c = remap(qref, n_coarse)
        href = qref_c[0]
        row = {"seed": int(seed), "plain": {}}
        for n in grids:
            p, _, _ = inputs.sw_hump(n=n, seed=seed, dtype="f32")
            q0 = remap(qr0, n).astype(np.float32)
            steps = int(math.ceil(steps_coarse * n / n_coarse - 1e-9))
            q, t = _timed_plain(p, q0, T / steps, steps)
            qc = remap(q, n_coarse)
            err = float(np.mean(np.abs(qc[0] - href)))
            row["plain"][int(n)] = {"l1": err, "seconds": t, "steps": steps,
                                    "l1_fields": [float(np.mean(np.abs(qc[f] - qref_c[f]))) for f in range(3)]}
        p, _, _ = inputs.sw_hump(n=n_coarse, seed=seed, dtype="f32")
        q0 = remap(qr0, n_coarse).astype(np.float32)
        q, t = _timed_learned(lc, p, q0, dt_c, steps_coarse, tau, kappa)
        row["learned"] = {"l1": float(np.mean(np.abs(q[0] - href))), "seconds": t, "steps": steps_coarse,
                          "l1_fields": [float(np.mean(np.abs(q[f] - qref_c[f]))) for f in range(3)],
                          "mass_drift": float(abs(q[0].astype(np.float64).sum() - q0[0].astype(np.float64).sum())
                                              / q0[0].astype(np.float64).sum())}
        rows.append(row)
    return summarize(rows)


def one_step_gain(lc, seeds, n_fine=1024, steps_fine=500, every=10, tau=TAU, kappa=KAPPA):
    """Teacher-forced one-step errors on held-out runs: from Q_c = C(Q_f^{2n})
    the plain coarse step and the corrected one, each against C(Q_f^{2n+2});
    mean absolute error per field over the sampled steps, (plain, learned)."""
    torch = _torch()
    nf, nc = int(n_fine), int(n_fine) // 2
    dtf = fine_dt(nf)
    dtc, nu = 2 * dtf, 2 * dtf * nc
    shp = (3, nc, nc)
    plain = torch.empty(shp, dtype=torch.float32, device="cuda")
    qcn, target, out = torch.empty_like(plain), torch.empty_like(plain), torch.empty_like(plain)
    dF = torch.empty((3, nc, nc + 1), dtype=torch.float32, device="cuda")
    dG = torch.empty((3, nc + 1, nc), dtype=torch.float32, device="cuda")
    pc, _, _ = inputs.sw_hump(n=nc, seed=0, dtype="f32")
    coarse = claw.Solver(pc, plain)
    e_plain, e_learned, count = np.zeros(3), np.zeros(3), 0
    for seed in seeds:
        pf, qf0, _ = inputs.sw_hump(n=nf, seed=seed, dtype="f32")
        qf = _dev(qf0)
        fine = claw.Solver(pf, qf)
        claw.claw_lc_coarsen(nc, nc, qf, qcn, _stream())
        for k in range(steps_fine // 2):
            plain.copy_(qcn)
            coarse.advance_fixed([dtc], log=False)
            fine.advance_fixed([dtf, dtf], log=False)
            claw.claw_lc_coarsen(nc, nc, qf, target, _stream())
            if k % every == every // 2:
                lc.forward(qcn, dF, dG)
                lc.apply(qcn, plain, dF, dG, nu, nu, tau, kappa, out)
                torch.cuda.synchronize()
                tg = target.cpu().numpy().astype(np.float64)
                e_plain += np.abs(plain.cpu().numpy() - tg).mean(axis=(1, 2))
                e_learned += np.abs(out.cpu().numpy() - tg).mean(axis=(1, 2))
                count += 1
            qcn, target = target, qcn
        fine.close()
    coarse.close()
    return (e_plain / count).tolist(), (e_learned / count).tolist()


def summarize(rows):
    grids = sorted(rows[0]["plain"])
    l1 = np.array([[r["plain"][n]["l1"] for n in grids] for r in rows]).mean(axis=0)
    tp = np.array([[r["plain"][n]["seconds"] for n in grids] for r in rows]).mean(axis=0)
    l1_learned = float(np.mean([r["learned"]["l1"] for r in rows]))
    t_learned = float(np.mean([r["learned"]["seconds"] for r in rows]))
    out = {"grids": grids, "l1_plain": l1.tolist(), "seconds_plain": tp.tolist(), "l1_learned": l1_learned,
           "seconds_learned": t_learned, "rows": rows,
           "mass_drift_max": max(r["learned"]["mass_drift"] for r in rows)}
    # equal-error resolution by log-log interpolation of the plain curve
    # (a power law between neighbouring plain grids, for error and for time)
    lg, ll, lt = np.log(grids), np.log(l1), np.log(tp)
    if l1_learned >= l1[0]:
        out["n_equal"] = float(grids[0])
        out["speedup_equal_l1"] = float(tp[0] / t_learned)
        out["note"] = "learned error not below the plain coarse run"
    elif l1_learned <= l1[-1]:
        out["n_equal"] = float(grids[-1])
        out["speedup_equal_l1"] = float(tp[-1] / t_learned)
        out["note"] = "learned error at or below the finest plain run: lower bound"
    else:
        k = int(np.searchsorted(-ll, -math.log(l1_learned)))  # ll decreasing
        f = (math.log(l1_learned) - ll[k - 1]) / (ll[k] - ll[k - 1])
        ln = lg[k - 1] + f * (lg[k] - lg[k - 1])
        t_eq = math.exp(lt[k - 1] + f * (lt[k] - lt[k - 1]))
        out["n_equal"] = float(math.exp(ln))
        out["speedup_equal_l1"] = float(t_eq / t_learned)
    out["speedup_vs_plain_finest"] = float(tp[-1] / t_learned)
    return out
