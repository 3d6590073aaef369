"""Training and evaluation of the learned coarse-grid correction, driven through the C ABI.

A fine D3Q27 x D3Q19 run (n_f = 4 n_c) is the teacher: at snapshot times its state a is
restricted to the coarse grid, the fine run advances 4 steps (one coarse step at the same
Mach number) and is restricted again (b), and the coarse step of a gives c.  Each coarse
node yields one training pair: its 47 features in a and the non-conserved moments of
b - c returned to the node each population streamed from.  The network is trained on
those pairs with the library's gradient and Adam kernels, then attached to a coarse run
(the fused learned step) and compared with the fine run's energy and dissipation
histories, next to the plain coarse run.

Every numerical step runs in the library's kernels; this module allocates device
buffers, draws the random numbers the training consumes (initial weights, minibatch
rows) and sequences the calls.  The error metrics at the end are host-side analysis of
a few hundred diagnostic records.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import stgv

IN, HID, OUT, NPARAM, NNORM = (stgv.MLP_IN, stgv.MLP_HIDDEN, stgv.MLP_OUT, stgv.MLP_PARAMS,
                               stgv.MLP_NORM)
RATIO = 4                      # fine n / coarse n; one coarse step = RATIO fine steps


def steps_per_unit_time(n, u0=0.05):
    """Lattice steps per convective time L/U (L = n / 2 pi lattice units)."""
    return n / (2.0 * math.pi) / u0


def physics(fr, seed=0, re=1600.0, sc=0.7, u0=0.05, g_over_n=0.02, forcing="shift", noise_amp=1e-6):
    """Keyword set of one stratified Taylor-Green run (grid size added by the caller)."""
    return dict(forcing=forcing, u0=u0, re=re, fr=fr, sc=sc, g_over_n=g_over_n,
                noise_amp=noise_amp, seed=seed)


def init_params(seed):
    """Glorot-uniform hidden layers, zero biases and a zero output layer: the untrained
    network is the plain method."""
    rng = np.random.default_rng(seed)

    def glorot(rows, cols):
        a = math.sqrt(6.0 / (rows + cols))
        return rng.uniform(-a, a, (rows, cols))

    parts = [glorot(HID, IN), np.zeros(HID), glorot(HID, HID), np.zeros(HID),
             np.zeros((OUT, HID)), np.zeros(OUT)]
    theta = np.concatenate([p.ravel() for p in parts]).astype(np.float32)
    assert theta.size == NPARAM
    return theta


class PairBuffer:
    """Device rows of features [capacity][47] and targets [capacity][41]."""

    def __init__(self, capacity, device="cuda:0"):
        self.x = torch.empty((capacity, IN), dtype=torch.float32, device=device)
        self.y = torch.empty((capacity, OUT), dtype=torch.float32, device=device)
        self.rows = 0

    @property
    def capacity(self):
        return self.x.shape[0]


SETTLE = (0, 2, 4, 8, 16, 32)   # plain coarse steps a restricted state evolves before pairing


def teacher_run(nc, phys, t_end, snapshots, pairs=None, diag_every_c=0, settle=SETTLE, device="cuda:0"):
    """Run the fine teacher (n = RATIO nc) to t_end and, at `snapshots` evenly spaced
    times, append one training pair per coarse node to `pairs` (if given).

    At a snapshot the restricted fine state first evolves k plain coarse steps (k cycling
    through `settle`) while the teacher advances RATIO k steps, so the features cover the
    states a coarse run actually visits (a restricted state lacks the grid-scale
    non-equilibrium a coarse run builds up at tau ~ 1/2); the target is the restricted
    teacher one coarse step later minus the coarse step of that state.  Returns the
    teacher's diagnostic records (every RATIO * diag_every_c fine steps, if > 0)."""
    nf = RATIO * nc
    steps = int(round(t_end * steps_per_unit_time(nf, phys["u0"])))
    fine = stgv.Simulation(device=device, n=nf, diag_every=RATIO * diag_every_c, **phys)
    coarse = stgv.Simulation(device=device, n=nc, **phys) if pairs is not None else None
    span = RATIO * (max(settle) + 1)
    marks = [] if pairs is None else sorted({int(s) for s in
                                            np.linspace(0, max(steps - span, 0), snapshots).round()})
    nc3 = nc ** 3
    done = 0
    for j, s in enumerate(marks):
        if s < done:
            continue
        k = settle[j % len(settle)]
        _advance(fine, s - done)
        done = s
        if pairs.rows + nc3 > pairs.capacity:
            raise ValueError("pair buffer full")
        a = fine.restrict_to(coarse)
        if k > 0:
            coarse.load(a, step=0)
            coarse.step(k)
            a = coarse.populations()
            _advance(fine, RATIO * k)
            done += RATIO * k
        fine.step(RATIO)
        done += RATIO
        b = fine.restrict_to(coarse)
        coarse.load(a, step=0)
        coarse.step(1)
        c = coarse.populations()
        stgv.lbm_training_pairs(coarse.ctx, a, b, c, pairs.x[pairs.rows:], pairs.y[pairs.rows:])
        pairs.rows += nc3
    if steps > done:
        _advance(fine, steps - done)
    torch.cuda.synchronize(device)
    recs = fine.diagnostics(raise_unstable=False) if diag_every_c > 0 else []
    fine.close()
    if coarse is not None:
        coarse.close()
    return recs


def _advance(sim, steps, chunk=2048):
    while steps > 0:
        k = min(chunk, steps)
        sim.step(k)
        steps -= k


class Network:
    """FP32 master parameters, Adam moments, normalisation and the packed copy."""

    def __init__(self, theta=None, norm=None, seed=0, device="cuda:0"):
        self.device = device
        self.theta = torch.tensor(init_params(seed) if theta is None else np.asarray(theta, np.float32),
                                  device=device)
        self.norm = torch.tensor(np.concatenate([np.zeros(IN), np.ones(IN), np.ones(OUT)])
                                 if norm is None else np.asarray(norm, np.float64),
                                 dtype=torch.float32, device=device)
        self.m = torch.zeros(NPARAM, device=device)
        self.v = torch.zeros(NPARAM, device=device)
        self.packed = torch.empty(stgv.lbm_mlp_packed_bytes(), dtype=torch.uint8, device=device)
        self.t = 0
        self.pack()

    def stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def pack(self):
        stgv.lbm_mlp_pack(self.theta, self.norm, self.packed, self.stream())

    def normalise_from(self, pairs, rows=None):
        rows = pairs.rows if rows is None else rows
        work = torch.empty(stgv.lbm_mlp_norm_work_bytes(), dtype=torch.uint8, device=self.device)
        stgv.lbm_mlp_norm(pairs.x, pairs.y, rows, self.norm, work, self.stream())
        self.pack()

    def state(self):
        return {"theta": self.theta.cpu().numpy(), "norm": self.norm.cpu().numpy()}


def mean_loss(net, pairs, zero=False, batch=65536):
    """Mean squared error of the network (or of a zero prediction) over all rows of
    `pairs`, in units of the normalised targets, with the gradient kernel's loss."""
    probe = Network(net.theta.cpu().numpy(), net.norm.cpu().numpy(), device=net.device)
    if zero:
        th = probe.theta.clone()
        th[NPARAM - OUT * HID - OUT:] = 0.0        # W3, b3
        probe.theta = th
        probe.pack()
    loss = torch.empty(1, dtype=torch.float64, device=net.device)
    grad = torch.empty(NPARAM, dtype=torch.float32, device=net.device)
    work = torch.empty(stgv.lbm_mlp_grad_work_bytes(batch), dtype=torch.uint8, device=net.device)
    total, count = 0.0, 0
    for r0 in range(0, pairs.rows, batch):
        nb = min(batch, pairs.rows - r0)
        idx = torch.arange(r0, r0 + nb, dtype=torch.int64, device=net.device)
        stgv.lbm_mlp_grad(probe.packed, pairs.x, pairs.y, idx, nb, grad, loss, work, net.stream())
        total += loss.item() * nb
        count += nb
    return total / max(count, 1)


def train(net, pairs, steps, batch=16384, lr=2e-3, lr_min=2e-5, seed=0, log_every=500, log=None):
    """Adam on minibatches drawn uniformly (with replacement) from the pair rows; cosine
    learning-rate decay from lr to lr_min.  Returns the logged (step, batch loss) pairs."""
    rng = np.random.default_rng(seed)
    loss = torch.empty(1, dtype=torch.float64, device=net.device)
    grad = torch.empty(NPARAM, dtype=torch.float32, device=net.device)
    work = torch.empty(stgv.lbm_mlp_grad_work_bytes(batch), dtype=torch.uint8, device=net.device)
    history = []
    chunk = 64
    for s0 in range(0, steps, chunk):
        ns = min(chunk, steps - s0)
        rows = torch.from_numpy(rng.integers(0, pairs.rows, size=(ns, batch), dtype=np.int64)).to(net.device)
        for k in range(ns):
            s = s0 + k
            stgv.lbm_mlp_grad(net.packed, pairs.x, pairs.y, rows[k], batch, grad, loss, work, net.stream())
            net.t += 1
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * s / max(steps - 1, 1)))
            stgv.lbm_mlp_adam(net.theta, net.m, net.v, grad, net.t, rate, net.stream())
            net.pack()
            if log_every and (s % log_every == 0 or s == steps - 1):
                history.append((s, loss.item()))
                if log:
                    log(f"train step {s}: batch loss {history[-1][1]:.4e} (lr {rate:.2e})")
    return history


def coarse_run(nc, phys, t_end, diag_every, net=None, device="cuda:0"):
    """A coarse run to t_end with (net given) or without the learned correction."""
    steps = int(round(t_end * steps_per_unit_time(nc, phys["u0"])))
    sim = stgv.Simulation(device=device, n=nc, diag_every=diag_every, **phys)
    if net is not None:
        sim.set_mlp(net.packed)
    t0 = time.perf_counter()
    _advance(sim, steps)
    torch.cuda.synchronize(device)
    wall = time.perf_counter() - t0
    recs = sim.diagnostics(raise_unstable=False)
    sim.close()
    return recs, steps, wall


def guarded_run(nc, phys, t_end, diag_every, net, check_every=None, keep=4, device="cuda:0"):
    """A learned coarse run with the plain step as its fallback.

    The state is kept every `check_every` steps (default 10 diagnostic intervals; the
    last `keep` states).  An interval is bad when one of its records is non-finite, has
    max|u| above the lattice speed of sound, or has a total energy E_k + E_p above the
    initial one by more than 1 % (the decaying flow has no energy source).  On the first
    bad interval the run returns to the newest kept state, detaches the network and goes
    on with the plain step; if the plain step fails too, it steps back to older kept
    states.  Returns (records, step of the fallback or None)."""
    steps = int(round(t_end * steps_per_unit_time(nc, phys["u0"])))
    check_every = check_every or 10 * diag_every
    sim = stgv.Simulation(device=device, n=nc, diag_every=diag_every, **phys)
    if net is not None:
        sim.set_mlp(net.packed)
    sim.sample()
    first = sim.diagnostics(raise_unstable=False)[0]
    e0 = first["ek"] + first["ep"]
    kept = [(0, sim.populations().clone(), [])]              # (step, state, records up to it)
    recs, fallback, learned_on, done = [], None, net is not None, 0
    while done < steps:
        k = min(check_every, steps - done)
        sim.step(k)
        new, status = stgv.lbm_diagnostics(sim.ctx, raise_unstable=False)
        bad = (status == stgv.LBM_EUNSTABLE
               or any(r["nonfinite"] or not (r["ek"] + r["ep"] <= 1.01 * e0) for r in new))
        if bad:
            if learned_on:
                sim.set_mlp(None)
                learned_on = False
            elif len(kept) > 1:
                kept.pop()
            else:
                sim.close()
                raise stgv.LbmError(stgv.LBM_EUNSTABLE, "the plain step is unstable from the initial state")
            done, state, recs = kept[-1][0], kept[-1][1], list(kept[-1][2])
            sim.load(state, step=done)
            fallback = done
            continue
        recs.extend(new)
        done += k
        kept.append((done, sim.populations().clone(), list(recs)))
        del kept[:-keep]
    sim.close()
    return recs, fallback


SERIES = ("ek", "ep", "eps_k", "eps_p")


def decay_rate(recs):
    """-dE/dt of the total energy E_k + E_p by central differences over the records
    (times t[1:-1]): the dissipation rate a run actually realises, resolved or not."""
    t = np.array([r["t"] for r in recs])
    e = np.array([r["ek"] + r["ep"] for r in recs])
    return t[1:-1], -(e[2:] - e[:-2]) / (t[2:] - t[:-2])


def _rel(a, b):
    """||a - b|| / ||b||; a zero reference gives 0 for an exact match, else infinity."""
    d, nb = float(np.linalg.norm(a - b)), float(np.linalg.norm(b))
    return d / nb if nb > 0 else (0.0 if d == 0 else math.inf)


def series_errors(recs, ref):
    """Relative L2 errors of the histories against the reference at the common record
    times: E_k, E_p, eps_k, eps_p and eps = eps_k + eps_p from the diagnostics, and the
    decay rate -dE/dt; plus the peak time and height of eps and of -dE/dt."""
    rt = {round(r["t"], 6): r for r in ref}
    common = [(r, rt[round(r["t"], 6)]) for r in recs if round(r["t"], 6) in rt]
    if len(common) < 3:
        raise ValueError("fewer than 3 common record times")
    out = {"records": len(common)}
    finite = all(math.isfinite(r["ek"]) and math.isfinite(r["ep"]) and r["nonfinite"] == 0
                 for r, _ in common)
    out["finite"] = finite
    if not finite:
        for key in SERIES + ("eps", "dEdt"):
            out[key] = math.inf
        return out
    for key in SERIES + ("eps",):
        a = np.array([(r["eps_k"] + r["eps_p"]) if key == "eps" else r[key] for r, _ in common])
        b = np.array([(q["eps_k"] + q["eps_p"]) if key == "eps" else q[key] for _, q in common])
        out[key] = _rel(a, b)
    t = np.array([r["t"] for r, _ in common])
    eps = np.array([r["eps_k"] + r["eps_p"] for r, _ in common])
    eref = np.array([q["eps_k"] + q["eps_p"] for _, q in common])
    out["eps_peak"] = [float(t[eps.argmax()]), float(eps.max())]
    out["eps_peak_ref"] = [float(t[eref.argmax()]), float(eref.max())]
    ta, da = decay_rate([r for r, _ in common])
    _, db = decay_rate([q for _, q in common])
    out["dEdt"] = _rel(da, db)
    out["dEdt_peak"] = [float(ta[da.argmax()]), float(da.max())]
    out["dEdt_peak_ref"] = [float(ta[db.argmax()]), float(db.max())]
    return out


def score(err):
    """Model-selection score of a rollout: E_k, E_p and -dE/dt errors summed."""
    return err["ek"] + err["ep"] + err["dEdt"]


def with_gain(net, gain):
    """A copy of the network whose correction is scaled by `gain` (y_scale * gain)."""
    out = Network(net.theta.cpu().numpy(), net.norm.cpu().numpy(), device=net.device)
    out.norm[IN + IN:] *= gain
    out.pack()
    return out


GAINS = (0.0, 0.05, 0.1, 0.2, 0.35, 0.5, 1.0)

# Raw network file read by the command-line driver (stgv_run --mlp): an 8-byte magic,
# the parameter and normalisation counts (int32), then the FP32 parameters and the FP32
# normalisation (x mean, x inverse scale, y scale x gain), little-endian.
NET_MAGIC = b"STGVMLP1"


def export_network(theta, norm, path, gain=1.0):
    """Write the network (master parameters `theta`, normalisation `norm`) with its
    correction scaled by `gain` in the driver's raw format."""
    theta = np.asarray(theta, dtype=np.float32).ravel()
    norm = np.asarray(norm, dtype=np.float64).ravel().copy()
    if theta.size != NPARAM or norm.size != IN + IN + OUT:
        raise ValueError(f"expected {NPARAM} parameters and {IN + IN + OUT} normalisation values")
    norm[IN + IN:] *= gain
    with open(path, "wb") as fh:
        fh.write(NET_MAGIC)
        fh.write(np.array([theta.size, norm.size], dtype="<i4").tobytes())
        fh.write(theta.astype("<f4").tobytes())
        fh.write(norm.astype("<f4").tobytes())


def pipeline(nc=64, train_fr=(0.3, 1.0, 3.0), seeds=(0,), test_fr=0.6, t_end=30.0, snapshots=64,
             train_steps=6000, batch=16384, lr=2e-3, gains=GAINS, diag_records=100, device="cuda:0",
             log=print, save=None):
    """Teacher runs, training, the choice of the correction gain by rollouts at the
    training Froude numbers (gain 0 is the plain method, so a correction that does not
    help is switched off), held-out one-step losses and the comparison of the plain and
    learned coarse runs against the teacher at the test Froude number.  Returns a
    JSON-ready summary, the deployed network (None when gain 0 wins) and the records."""
    nc3 = nc ** 3
    t_all = time.perf_counter()
    runs = [(fr, seed) for fr in train_fr for seed in seeds]
    train_pairs = PairBuffer(len(runs) * snapshots * nc3, device)
    test_pairs = PairBuffer(snapshots * nc3, device)
    de_c = max(1, int(round(t_end * steps_per_unit_time(nc) / diag_records)))
    t0 = time.perf_counter()
    val_refs = {}
    for fr, seed in runs:
        recs = teacher_run(nc, physics(fr, seed), t_end, snapshots, train_pairs,
                           diag_every_c=de_c if seed == seeds[0] else 0, device=device)
        if seed == seeds[0]:
            val_refs[fr] = recs
        log(f"teacher Fr={fr} seed={seed}: {train_pairs.rows} training rows")
    ref = teacher_run(nc, physics(test_fr, 0), t_end, snapshots, test_pairs, diag_every_c=de_c, device=device)
    t_teach = time.perf_counter() - t0
    log(f"teachers done in {t_teach:.1f} s; test rows {test_pairs.rows}")

    net = Network(seed=0, device=device)
    net.normalise_from(train_pairs)
    t0 = time.perf_counter()
    hist = train(net, train_pairs, train_steps, batch=batch, lr=lr, log=log)
    torch.cuda.synchronize(device)
    t_train = time.perf_counter() - t0
    losses = {"train_zero": mean_loss(net, train_pairs, zero=True),
              "train_net": mean_loss(net, train_pairs),
              "test_zero": mean_loss(net, test_pairs, zero=True),
              "test_net": mean_loss(net, test_pairs)}
    log(f"training {train_steps} steps in {t_train:.1f} s; one-step losses {losses}")
    del train_pairs, test_pairs
    torch.cuda.empty_cache()

    validation = {}
    for gain in gains:
        cand = with_gain(net, gain) if gain > 0 else None
        errs = [series_errors(coarse_run(nc, physics(fr, seeds[0]), t_end, de_c, net=cand, device=device)[0],
                              val_refs[fr]) for fr in train_fr]
        validation[gain] = float(np.mean([score(e) for e in errs]))
        log(f"validation gain {gain}: mean score {validation[gain]:.4f}")
    best = min(validation, key=lambda g: (validation[g], g))
    deployed = with_gain(net, best) if best > 0 else None

    phys = physics(test_fr, 0)
    plain, steps_c, wall_plain = coarse_run(nc, phys, t_end, de_c, device=device)
    _, _, wall_learned = coarse_run(nc, phys, t_end, de_c, net=deployed or with_gain(net, 0.0), device=device)
    # the deployed run, with the plain step as its fallback
    learned, fallback = guarded_run(nc, phys, t_end, de_c, deployed, device=device)
    e_plain, e_learned = series_errors(plain, ref), series_errors(learned, ref)
    summary = {
        "workload": f"learned {nc}^3 vs plain {nc}^3 vs plain {RATIO * nc}^3 teacher, stratified TGV "
                    f"Re 1600 Sc 0.7, velocity shift, G/N 0.02; train Fr {list(train_fr)} seeds "
                    f"{list(seeds)}, test Fr {test_fr}, to t = {t_end}",
        "train_rows": len(runs) * snapshots * nc3, "test_rows": snapshots * nc3,
        "train_steps": train_steps, "batch": batch, "loss_history": hist, "one_step_loss": losses,
        "one_step_ratio_test": losses["test_net"] / losses["test_zero"],
        "validation_score_by_gain": validation, "gain": best,
        "errors_plain": e_plain, "errors_learned": e_learned,
        "score_plain": score(e_plain), "score_learned": score(e_learned), "fallback_step": fallback,
        "coarse_steps": steps_c,
        "mlups_plain": nc3 * steps_c / wall_plain / 1e6,
        "mlups_learned": nc3 * steps_c / wall_learned / 1e6,
        "seconds": {"teachers": t_teach, "training": t_train, "total": time.perf_counter() - t_all},
    }
    if save:
        st = net.state()                      # the trained network, undamped, and the chosen gain
        np.savez(save, theta=st["theta"], norm=st["norm"], gain=best)
    return summary, deployed, (plain, learned, ref)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--nc", type=int, default=64)
    ap.add_argument("--train-fr", type=float, nargs="+", default=[0.3, 1.0, 3.0])
    ap.add_argument("--seeds", type=int, nargs="+", default=[0])
    ap.add_argument("--test-fr", type=float, default=0.6)
    ap.add_argument("--t-end", type=float, default=30.0)
    ap.add_argument("--snapshots", type=int, default=64)
    ap.add_argument("--train-steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=None, help="JSON summary path")
    ap.add_argument("--save", default=None, help="npz path for the trained network")
    ap.add_argument("--export", default=None,
                    help="only write the network of --net (default: the shipped one) in the raw "
                         "format of stgv_run --mlp, at --gain (default: its validated gain)")
    ap.add_argument("--net", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                                                  "learned64.npz"))
    ap.add_argument("--gain", type=float, default=None)
    a = ap.parse_args(argv)
    if a.export:
        z = np.load(a.net, allow_pickle=False)
        gain = float(z["gain"]) if a.gain is None else a.gain
        export_network(z["theta"], z["norm"], a.export, gain)
        print(f"wrote {a.export} (gain {gain})")
        return
    summary, _, _ = pipeline(a.nc, tuple(a.train_fr), tuple(a.seeds), a.test_fr, a.t_end, a.snapshots,
                             a.train_steps, a.batch, a.lr, log=lambda s: print(s, flush=True), save=a.save)
    text = json.dumps(summary, indent=1)
    print(text)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)


if __name__ == "__main__":
    main()
