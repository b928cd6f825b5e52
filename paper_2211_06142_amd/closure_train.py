"""Learned closure for the coarse-grained model (an extension; not in
arXiv:2211.06142): the dataset from paired fine and coarse runs, training on
the GPU with the library's own network kernels, and the gain test.

Pairing.  A fine run (grains of the paper's size distribution) and a coarse
run of the same geometry at coarse-graining factor k (section 2.4, SSW or SSP
scaling) are stepped under the same prescribed fluid field.  Both report, per
CFD cell and coupling evaluation, the solid fraction and the drag density
(eq 6-7); both list their bonded contacts.

Targets, per CFD cell c and time window w:
  y_drag = ln( D_fine / D_coarse ),  D = |f_d,c| / eps_s,c, the drag force per
           unit solid volume, averaged over the couplings of the window;
  y_coh  = ln( A_fine / (k A_coarse) ),  A = the pull-off forces 3 pi gamma R*
           of the bonded contacts whose contact point lies in c (the adhesion
           the bonds can hold, Table 1 point C), per unit solid volume, at the
           end of the window; k A_coarse is what the coarse-graining law
           (gamma_g = k gamma, section 2.4) predicts for A_fine, so y_coh is
           the law's residual.
Both are clipped to [-ln 2, ln 2], the range the closure can express (its
factors are exp(clip(y, +-ln 2))).  A cell enters only where both runs hold
solid (eps_s above a floor) and, for y_coh, bonds.  Every coarse parcel that
sits in such a cell at the end of the window gets the cell's targets, with its
closure features of the window's last coupling.

Gain test, on three packings of the same configuration (different seeds, so
that no judged run shares its grains with the training data): the dataset
comes from the training pair; on the judging pair the produced mass M(t) of
the fine run (the truth), of the plain coarse run and of the coarse run with
the trained closure give the error at the horizon |M_cg - M_fine| / M_fine,
and the closure is kept only if its error is not larger than the plain coarse
model's (else the plain model, c = 1, is the fallback); the reporting pair,
seen by neither step, gives the errors that are reported (with the RMSRE of
eq 41 over M(t)).
"""
import math
import time

import numpy as np

from . import dem

LN2 = math.log(2.0)


# ---------------------------------------------------------------------------
# host-side bookkeeping (no physics beyond the pull-off force 3 pi gamma R*)
# ---------------------------------------------------------------------------
def cell_index(x, grid):
    """flat index (x fastest) of the CFD cell holding each point; -1 outside"""
    lo, hi, nn = grid
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    nn = np.asarray(nn, dtype=np.int64)
    q = np.floor((np.asarray(x, dtype=np.float64) - lo) / ((hi - lo) / nn)).astype(np.int64)
    inside = np.all((q >= 0) & (q < nn), axis=1)
    flat = q[:, 0] + nn[0] * (q[:, 1] + nn[1] * q[:, 2])
    return np.where(inside, flat, -1)


def pulloff_density(x, r, pairs, bonded, gamma, grid, eps_s):
    """sum over bonded contacts of 3 pi gamma R*, binned by the cell of the
    contact point (on the centre line, r_a from a's centre in proportion
    r_a : r_c), per unit solid volume of the cell"""
    ncell = int(np.prod(grid[2]))
    out = np.zeros(ncell)
    if len(pairs) == 0:
        return out
    b = bonded.astype(bool)
    a, c = pairs[b, 0], pairs[b, 1]
    ra, rc = r[a], r[c]
    pt = (x[a] * rc[:, None] + x[c] * ra[:, None]) / (ra + rc)[:, None]
    cell = cell_index(pt, grid)
    f = 3.0 * math.pi * gamma * ra * rc / (ra + rc)
    ok = cell >= 0
    np.add.at(out, cell[ok], f[ok])
    lo, hi, nn = grid
    vcell = float(np.prod((np.asarray(hi) - np.asarray(lo)) / np.asarray(nn)))
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(eps_s > 0.0, out / (eps_s * vcell), 0.0)


def log_ratio(fine, coarse, valid):
    """clipped ln(fine / coarse) where valid (and both positive), NaN elsewhere"""
    ok = valid & (fine > 0.0) & (coarse > 0.0)
    y = np.full(fine.shape, np.nan)
    y[ok] = np.clip(np.log(fine[ok] / coarse[ok]), -LN2, LN2)
    return y


def assemble(features, cells, y_drag, y_coh):
    """rows of (features, targets) for parcels whose cell has both targets"""
    ok = cells >= 0
    idx = np.where(ok)[0]
    yd, yc = y_drag[cells[idx]], y_coh[cells[idx]]
    keep = np.isfinite(yd) & np.isfinite(yc)
    idx = idx[keep]
    return features[idx], np.stack([yd[keep], yc[keep]], axis=1)


def normaliser(X):
    """(mean[6], sd[6]) of the training features; a constant feature gets sd 1"""
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 1e-12 * np.maximum(np.abs(mu), 1.0), sd, 1.0)
    return np.concatenate([mu, sd])


# ---------------------------------------------------------------------------
# runs
# ---------------------------------------------------------------------------
def make_sim(w, closure=None, norm=None):
    """a run of workload w; below 50 000 particles 8 lanes per particle
    (timed on the coarse cylinders: the step kernel has too few particles to
    fill the chip with 4)"""
    sim = dem.Simulation(dem.params_from_workload(w), w["x"], w["r"])
    sim.map_fluid(w["u_cell"], w["gradp_cell"])
    sim.set_lanes(8 if len(w["r"]) < 50000 else 4)
    if closure is not None:
        sim.set_closure(closure, norm)
    return sim


def zero_network():
    """a network whose output is exactly 0: factors exactly 1 (the plain model),
    used to read the closure features of a plain run"""
    return dem.Mlp(np.zeros(dem.MLP_NPARAMS))


class Recorder:
    """Steps a run window by window and keeps what the dataset needs."""

    def __init__(self, w, sim, features=False):
        self.w, self.sim, self.features = w, sim, features
        self.ce = int(w["fluid"]["couple_every"])
        self.mass = []        # (step, produced mass)
        self.windows = []     # per window: drag density, solid fraction, pull-off density, features, cells
        self.gamma = float(w["material"]["gamma"]) * float(w.get("k", 1.0))

    def run_window(self, steps, keep=True):
        ncell = int(np.prod(self.w["grid"][2]))
        dsum = np.zeros(ncell)
        esum = np.zeros(ncell)
        nc = 0
        done = 0
        if not keep:
            self.sim.step(steps)
            done = steps
        while done < steps:
            n = min(self.ce, steps - done)
            self.sim.step(n)
            done += n
            if keep:
                eps, fd = self.sim.fluid_out()
                mag = np.linalg.norm(fd, axis=1)
                with np.errstate(divide="ignore", invalid="ignore"):
                    dsum += np.where(eps > 0.0, mag / eps, 0.0)
                esum += eps
                nc += 1
        st = self.sim.state()
        self.mass.append((int(st["step"]), float(st["produced_mass"])))
        if not keep:
            return
        eps_mean = esum / max(nc, 1)
        rec = {"drag": dsum / max(nc, 1), "eps": eps_mean}
        alive = st["alive"].astype(bool)
        pr = self.sim.pairs(sort=False)
        rec["coh"] = pulloff_density(st["x"], self.w["r"], pr["pairs"], pr["bonded"], self.gamma,
                                     self.w["grid"], eps_mean)
        if self.features:
            cl = self.sim.read_closure()
            cells = cell_index(st["x"], self.w["grid"])
            cells[~alive] = -1
            rec["features"] = cl["features"]
            rec["cells"] = cells
        self.windows.append(rec)


def build_dataset(fine, coarse, eps_floor=0.05):
    """(X, Y) over the windows both recorders kept.  The cohesion target is the
    residual of the coarse-graining law: with gamma_g = k gamma and R*_g =
    k R* a parcel bond holds k^2 the pull-off force of a grain bond, over k^3
    fewer bonds per unit volume, so the law itself expects A_coarse = A_fine /
    k; the target is ln(A_fine / (k A_coarse)).  The drag law k^3 f(d / k)
    keeps the drag per unit solid volume, so the drag target needs no such
    factor."""
    kc = float(coarse.w.get("k", 1.0)) / float(fine.w.get("k", 1.0))
    Xs, Ys = [], []
    for wf, wc in zip(fine.windows, coarse.windows):
        valid = (wf["eps"] > eps_floor) & (wc["eps"] > eps_floor)
        yd = log_ratio(wf["drag"], wc["drag"], valid)
        yc = log_ratio(wf["coh"], kc * wc["coh"], valid)
        X, Y = assemble(wc["features"], wc["cells"], yd, yc)
        Xs.append(X)
        Ys.append(Y)
    if not Xs:
        return np.zeros((0, 6)), np.zeros((0, 2))
    return np.concatenate(Xs), np.concatenate(Ys)


def he_params(seed, scale=1.0):
    """He-normal weights, zero biases, packed in the library's order
    (W1 6x64 | b1 | W2 64x64 | b2 | W3 64x64 | b3 | W4 64x2 | b4, W row-major
    with the input index first), rounded to FP32"""
    rng = np.random.default_rng(seed)
    sizes = [6, 64, 64, 64, 2]
    out = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append(rng.normal(0.0, scale * math.sqrt(2.0 / a), size=(a, b)).ravel())
        out.append(np.zeros(b))
    return np.concatenate(out).astype(np.float32).astype(np.float64)


def train_net(X, Y, norm, epochs=30, batch=4096, lr=2e-3, seed=0, init_scale=0.5):
    """Adam on the GPU with the library's BF16 forward/backward kernels over
    shuffled minibatches; returns the network and the loss of every step"""
    net = dem.Mlp(he_params(seed, init_scale))
    Xn = ((X - norm[:6]) / norm[6:]).astype(np.float32)
    Yf = Y.astype(np.float32)
    rng = np.random.default_rng(seed)
    losses = []
    n = len(Xn)
    for _ in range(epochs):
        perm = rng.permutation(n)
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            losses.append(net.train_step(Xn[idx], Yf[idx], lr))
    return net, losses


def _timed_run(w, steps, closure=None, norm=None, log=None, chunk=20000):
    """wall time of `steps` steps (dem_step calls of `chunk` steps,
    synchronised at the end) from the initial packing, and the produced mass
    at the end; log: a line after every call"""
    import torch
    sim = make_sim(w, closure, norm)
    sim.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        sim.step(n)
        done += n
        if log:
            log("%s: timed %d of %d steps" % (w["name"], done, steps))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m = float(sim.state()["produced_mass"])
    sim.close()
    return wall, m


def _mass_series(w, steps, window, closure=None, norm=None, until_mass=None, max_steps=None, log=None,
                 log_every=40):
    """produced mass at the end of every window of a run from the initial
    packing; with until_mass: windows until the produced mass reaches it (at
    most max_steps), the horizon then being the steps taken; log: a progress
    line every log_every windows"""
    rec = Recorder(w, make_sim(w, closure, norm))

    def progress():
        if log and len(rec.mass) % log_every == 0:
            log("%s: %d steps, produced %.4g kg" % (w["name"], len(rec.mass) * window, rec.mass[-1][1]))

    if until_mass is None:
        for _ in range(steps // window):
            rec.run_window(window, keep=False)
            progress()
    else:
        while True:
            rec.run_window(window, keep=False)
            progress()
            done = len(rec.mass) * window
            if rec.mass[-1][1] >= until_mass or done >= max_steps:
                break
    rec.sim.close()
    return np.array([m for _, m in rec.mass])


def _errors(mf, m):
    """error at the horizon and RMSRE over the windows where the fine run has produced mass"""
    e = abs(m[-1] - mf[-1]) / mf[-1] if mf[-1] > 0 else float("nan")
    ok = mf > 0
    r = float(np.sqrt(np.mean(((m[ok] - mf[ok]) / mf[ok]) ** 2))) if ok.any() else float("nan")
    return float(e), r


def gain_test(train, judge, report, horizon=20000, window=500, epochs=40, batch=4096, lr=2e-3, seed=0,
              log=None, report_mass=None, report_max_steps=400000):
    """train, judge, report: (fine workload, coarse workload) pairs of three
    packings.  Paired runs of the training pair give the dataset and the
    network; the judging pair decides keep or fall back; the reporting pair
    gives the reported errors of the plain and the learned coarse model.
    report_mass: the reporting runs last until the fine run has produced that
    mass (at most report_max_steps) instead of `horizon` steps."""
    say = log or (lambda *a: None)
    nwin = horizon // window
    wf, wc = train
    fine = Recorder(wf, make_sim(wf))
    plain = Recorder(wc, make_sim(wc, zero_network(), np.r_[np.zeros(6), np.ones(6)]), features=True)
    for _ in range(nwin):
        fine.run_window(window)
        plain.run_window(window)
    fine.sim.close()
    plain.sim.close()
    X, Y = build_dataset(fine, plain)
    norm = normaliser(X)
    net, losses = train_net(X, Y, norm, epochs=epochs, batch=batch, lr=lr, seed=seed)
    say("trained on %d samples of %d windows, loss %.4g -> %.4g" % (len(X), nwin, losses[0], losses[-1]))
    out = {"n_fine": int(len(wf["r"])), "n_coarse": int(len(wc["r"])), "k": float(wc.get("k", 1.0)),
           "scheme": wc.get("scheme", "ssw"), "horizon_steps": int(horizon), "window_steps": int(window),
           "train_samples": int(len(X)), "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
           "packings": {"train": wf["name"], "judge": judge[0]["name"], "report": report[0]["name"]}}
    for role, (f, c) in (("judge", judge), ("report", report)):
        if role == "report" and report_mass is not None:
            mf = _mass_series(f, 0, window, until_mass=report_mass, max_steps=report_max_steps, log=log)
            out["report_horizon_steps"] = int(len(mf) * window)
        else:
            mf = _mass_series(f, horizon, window, log=log)
        steps = len(mf) * window
        mp = _mass_series(c, steps, window, log=log)
        ml = _mass_series(c, steps, window, net, norm, log=log)
        ep, rp = _errors(mf, mp)
        el, rl = _errors(mf, ml)
        out[role] = {"mass_fine": float(mf[-1]), "mass_plain_cg": float(mp[-1]), "mass_learned_cg": float(ml[-1]),
                     "err_plain_cg": ep, "err_learned_cg": el, "rmsre_plain_cg": rp, "rmsre_learned_cg": rl,
                     "mass_series": {"fine": mf, "plain": mp, "learned": ml}}
        say("%s packing: error plain %.4f learned %.4f, RMSRE plain %.4f learned %.4f" % (role, ep, el, rp, rl))
    accepted = bool(out["judge"]["err_learned_cg"] <= out["judge"]["err_plain_cg"])
    out["closure_accepted"] = accepted
    rf, rc = report
    rsteps = out.get("report_horizon_steps", horizon)
    say("timing the fine and the kept coarse model over %d steps" % rsteps)
    wall_fine, _ = _timed_run(rf, rsteps, log=log)
    wall_cg, _ = _timed_run(rc, rsteps, net if accepted else None, norm if accepted else None, log=log)
    out.update(wall_fine_s=wall_fine, wall_cg_s=wall_cg, speedup_vs_fine=wall_fine / wall_cg, net=net, norm=norm)
    # the model the rule keeps, on the reporting packing
    r = out["report"]
    out["err_kept_cg"] = r["err_learned_cg"] if accepted else r["err_plain_cg"]
    out["rmsre_kept_cg"] = r["rmsre_learned_cg"] if accepted else r["rmsre_plain_cg"]
    return out
