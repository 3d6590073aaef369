#!/usr/bin/env python
"""Throughput of the stratified Taylor-Green D3Q27 x D3Q19 DDF lattice Boltzmann step on one MI355X.

Workload (default): 256^3 periodic box, D3Q27 momentum x D3Q19 scalar lattice,
Shan-Chen velocity-shift buoyancy, Re 1600, Fr 1, Sc 0.7, U0 0.05, FP32
populations in the AA in-place layout, energy / dissipation diagnostics every
16 steps (~ t_c / 50), synthetic Taylor-Green initial state with 1e-6 seeded
density noise.  One "step" = one fused stream-collide-force launch (plus, on
diagnostic steps, the dissipation stencil and the final reduction).

Prints ONE JSON line: MLUPS (whole job), ms per step, the roofline of the step
kernel (algorithmic bytes 2 (Q_f + Q_g) b per node over its HIP-event-timed
average duration, against the 8 TB/s HBM peak), the streaming-copy ceiling, the
ceiling of the step's own access pattern (free streaming: the same loads, stores,
launch shapes and block order with no collision), the HBM traffic read from the committed rocprofv3 counter summary when it was
taken on the current kernel sources, the FP64 oracle timed on the host cores
(the only part of this script that runs the oracle), and the error of the GPU's
energy and dissipation histories against the oracle's stored 64^3 histories.

"forms" adds the precision and learned forms: step-kernel throughput of FP16 /
BF16 weight-shifted storage, of FP64 arithmetic, of every stencil pair (FP32, and
FP16 for the D3Q7-scalar sweep) and of the learned 64^3 step, and their energy /
dissipation histories (E_k, E_p, eps_k, eps_p, -dE/dt) to t = 30 against the plain
FP32 256^3 run of the same stratified TGV (Fr 0.6); the 512^3 FP16 case with its
counter traffic, and its 2000-step run against the FP32 run of the same flow; the
128^3 Fr 0.5 case beside the oracle's 64^3 histories; and the 256^3 Froude sweep (Fr 0.3, 1, 3: FP16 against FP32 storage; at Fr 0.3 Guo against the
shift, and Guo in FP16 against Guo in FP32).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
PEAK_HBM_GBS = 8000.0
T_START = time.time()


def progress(msg):
    """One progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench {time.time() - T_START:6.1f} s] {msg}", file=sys.stderr, flush=True)
FORCING_NAMES = {"guo": "Guo source-term", "shift": "velocity-shift", "edm": "exact-difference (EDM)",
                 "hcz": "He-Shan-Doolen source-term"}


def read_traffic(workload_key, n3, bytes_per_node):
    """HBM bytes per launch from profiles/<key>_counters.txt if its source hash is current."""
    path = os.path.join(ROOT, "profiles", f"{workload_key}_counters.txt")
    if not os.path.exists(path):
        return None, "no counter summary"
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    from paper_2605_14505_amd.profsummary import kernel_source_hash
    if kv.get("source_hash") != kernel_source_hash():
        return None, "counters predate the current kernel sources"
    try:
        return float(kv["hbm_bytes_per_launch"]), os.path.relpath(path, ROOT)
    except (KeyError, ValueError):
        return None, "malformed counter summary"


def host_cpu_model():
    """The host CPU's model name (Linux), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(n, steps, forcing):
    """The FP64 oracle as it stands, single-threaded BLAS, on a bounded sample of the workload."""
    from threadpoolctl import threadpool_limits

    from oracle import lattice as lat, model
    p = model.Params(n=n, q_f=27, q_g=19, forcing=forcing, u0=0.05, re=1600.0, fr=1.0, sc=0.7,
                     g_over_n=0.02, noise_amp=1e-6, seed=0)
    with threadpool_limits(limits=1):
        U = model.units(p)
        lf, lg = lat.BY_Q[27], lat.BY_Q[19]
        f, g = model.init_tgv(p)
        t0 = time.perf_counter()
        for _ in range(steps):
            fs, gs, _ = model.collide(f, g, lf, lg, U)
            f, g = model.stream(fs, lf), model.stream(gs, lg)
        dt = time.perf_counter() - t0
    del f, g
    return {"value": round(n ** 3 * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} steps of the same stratified-TGV D3Q27x19 {forcing} step on a {n}^3 box "
                      f"(the 256^3 box needs 25 GB and ~4 min per oracle step), NumPy FP64, one "
                      f"thread, {dt:.1f} s"}


def energy_error(stgv):
    """Max error of the GPU's E_k, E_p, eps_k, eps_p histories (relative to each history's
    largest value) against the FP64 oracle's, stored by tests/golden/make_series_64.py (which
    calls only the oracle): 64^3, velocity shift, Re 1600, Fr 0.5, 2500 steps; for FP32 and
    FP16 population storage."""
    import json

    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "series_64_shift.json")))
    ref = gold["fp64"]
    out = {"workload": f"{gold['params']['n']}^3 D3Q27x19 velocity shift, Re {gold['params']['re']:g}, "
                       f"Fr {gold['params']['fr']:g}, Sc {gold['params']['sc']:g}, {gold['steps']} steps, "
                       f"records every {gold['every']}, against the FP64 oracle's histories "
                       f"(tests/golden/series_64_shift.json)"}
    for storage in ("fp32", "fp16"):
        sim = stgv.Simulation(diag_every=gold["every"], storage=storage, **gold["params"])
        sim.step(gold["steps"] + 1)
        recs = sim.diagnostics()
        sim.close()
        assert [r["step"] for r in recs] == [d["step"] for d in ref]
        for key in ("ek", "ep", "eps_k", "eps_p"):
            top = max(abs(d[key]) for d in ref)
            err = max(abs(r[key] - d[key]) for r, d in zip(recs, ref)) / top
            out[key if storage == "fp32" else f"{key}_fp16"] = float(f"{err:.3e}")
    return out


def kernel_time(stgv, stream, kw, steps, warmup, packed=None):
    """Average step-kernel time (ms) over `steps` launches, HIP events on the launch stream."""
    import torch
    sim = stgv.Simulation(diag_every=0, **kw)
    if packed is not None:
        sim.set_mlp(packed)
    sim.step(warmup)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    ev1.synchronize()
    sim.close()
    return ev0.elapsed_time(ev1) / steps


def history(stgv, kw, t_end, diag_every, packed=None, spectrum_at=None):
    """Diagnostic records of one run to t_end (convective times L/U); with spectrum_at,
    also the kinetic-energy spectrum at that time and the time its call took (ms)."""
    import torch
    from paper_2605_14505_amd import learned
    per = learned.steps_per_unit_time(kw["n"], kw["u0"])
    steps = int(round(t_end * per))
    stop = int(round(spectrum_at * per)) if spectrum_at is not None else None
    sim = stgv.Simulation(diag_every=diag_every, **kw)
    if packed is not None:
        sim.set_mlp(packed)
    spec = None
    done = 0
    while done < steps:
        k = min(2048, steps - done, (stop - done) if stop is not None and stop > done else steps)
        sim.step(k)
        done += k
        if stop is not None and done == stop:
            sim.spectrum()                                   # plan and work buffer
            stream = torch.cuda.current_stream()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            e = sim.spectrum()
            ev1.record(stream)
            ev1.synchronize()
            spec = (e.cpu().numpy(), ev0.elapsed_time(ev1))
    torch.cuda.synchronize()
    recs = sim.diagnostics(raise_unstable=False)
    sim.close()
    return (recs, spec) if spectrum_at is not None else recs


def sweep_128(stgv, stream, steps, warmup):
    """The 128^3 velocity-shift case at Fr 0.5 (Re 1600, Sc 0.7, FP32) over 5000 steps: MLUPS,
    and its E_k, E_p, eps_k, eps_p histories beside the FP64 oracle's 64^3 histories of the
    same flow (tests/golden/series_64_shift.json, 2500 steps: the same physical times), whose
    difference is the resolution's, not an error of either."""
    import torch
    from paper_2605_14505_amd import learned
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "series_64_shift.json")))
    kw = dict(gold["params"], n=128)
    ms = kernel_time(stgv, stream, kw, steps, warmup)
    every = 2 * gold["every"]
    sim = stgv.Simulation(diag_every=every, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(2 * gold["steps"] + 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recs = sim.diagnostics(raise_unstable=False)
    sim.close()
    err = learned.series_errors(recs, gold["fp64"])
    return {"workload": "128^3 D3Q27x19 velocity shift, Re 1600, Fr 0.5, Sc 0.7, G/N 0.02, FP32, 5001 steps "
                        f"(t = {recs[-1]['t']:.2f}), records every {every} steps",
            "kernel_ms": round(ms, 5), "mlups": round(128 ** 3 / (ms * 1e-3) / 1e6, 1),
            "run_mlups": round(128 ** 3 * (2 * gold["steps"] + 1) / wall / 1e6, 1),
            "hbm_frac": round(368 * 128 ** 3 / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "finite": all(r["nonfinite"] == 0 for r in recs),
            "vs_oracle_64": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in err.items()
                             if k in ("records", "ek", "ep", "eps_k", "eps_p", "dEdt")}}


def sweep_256_fr(stgv, steps=10000, every=16):
    """The 256^3 Froude sweep (D3Q27x19, velocity shift, Re 1600, Sc 0.7, G/N 0.02, 10000 steps,
    t = 12.3): relative L2 errors of the FP16-storage histories against the FP32 run at each
    Fr (and, over 5000 steps, for the D3Q27xD3Q7 and D3Q19xD3Q7 pairs), and at Fr 0.3 the
    Guo source-term run against the velocity shift and Guo with FP16 storage against Guo
    with FP32."""
    import torch
    from paper_2605_14505_amd import learned
    out = {"workload": f"256^3 D3Q27x19, Re 1600, Sc 0.7, G/N 0.02, {steps} steps, records every {every}; "
                       "relative L2 errors of the histories"}
    keep = ("finite", "ek", "ep", "eps_k", "eps_p", "dEdt")

    def run(n_steps=steps, **kw):
        kw = dict(dict(q_f=27, q_g=19), **kw)
        sim = stgv.Simulation(diag_every=every, n=256, **kw)
        sim.step(n_steps + 1)
        torch.cuda.synchronize()
        recs = sim.diagnostics(raise_unstable=False)
        sim.close()
        return recs

    for fr in (0.3, 1.0, 3.0):
        phys = learned.physics(fr)
        ref = run(**phys)
        e16 = learned.series_errors(run(storage="fp16", **phys), ref)
        row = {"fp16_vs_fp32": {k: (round(v, 6) if isinstance(v, float) else v) for k, v in e16.items() if k in keep}}
        if fr == 0.3:
            guo = run(**dict(phys, forcing="guo"))
            eg = learned.series_errors(guo, ref)
            row["guo_vs_shift_fp32"] = {k: (round(v, 6) if isinstance(v, float) else v)
                                        for k, v in eg.items() if k in keep}
            eg16 = learned.series_errors(run(storage="fp16", **dict(phys, forcing="guo")), guo)
            row["guo_fp16_vs_guo_fp32"] = {k: (round(v, 6) if isinstance(v, float) else v)
                                           for k, v in eg16.items() if k in keep}
        # the D3Q7-scalar pairs of the sweep, FP16 against FP32 storage, over 5000 steps
        for qf, qg in ((27, 7), (19, 7)):
            ref_p = run(n_steps=steps // 2, q_f=qf, q_g=qg, **phys)
            ep = learned.series_errors(run(n_steps=steps // 2, q_f=qf, q_g=qg, storage="fp16", **phys), ref_p)
            row[f"fp16_vs_fp32_{qf}x{qg}_{steps // 2}_steps"] = {
                k: (round(v, 6) if isinstance(v, float) else v) for k, v in ep.items() if k in keep}
        out[f"fr_{fr:g}"] = row
    return out


def run_512(stgv, steps=2000, every=100):
    """The 512^3 case (D3Q27x19, velocity shift, Re 3200, Fr 0.5, Sc 0.7, G/N 0.02, 2000 steps,
    t = 1.23): FP16 storage in the AA layout (12.35 GB) and the FP32 run of the same flow
    (24.7 GB): whole-run MLUPS with diagnostics every `every` steps, whether both stay
    finite, and the relative L2 errors of the FP16 histories against the FP32 ones."""
    import time
    import torch
    from paper_2605_14505_amd import learned
    phys = learned.physics(0.5, re=3200.0)
    recs, rate = {}, {}
    for storage in ("fp16", "fp32"):
        sim = stgv.Simulation(diag_every=every, n=512, q_f=27, q_g=19, storage=storage, **phys)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps + 1)
        torch.cuda.synchronize()
        rate[storage] = round(512 ** 3 * (steps + 1) / (time.perf_counter() - t0) / 1e6, 1)
        recs[storage] = sim.diagnostics(raise_unstable=False)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    keep = ("finite", "ek", "ep", "eps_k", "eps_p", "dEdt")
    e16 = learned.series_errors(recs["fp16"], recs["fp32"])
    return {"workload": f"512^3 D3Q27x19 velocity shift, Re 3200, Fr 0.5, Sc 0.7, G/N 0.02, {steps} steps "
                        f"(t = 1.23), records every {every}",
            "run_mlups_fp16": rate["fp16"], "run_mlups_fp32": rate["fp32"],
            "finite_fp16": all(r["nonfinite"] == 0 for r in recs["fp16"]),
            "finite_fp32": all(r["nonfinite"] == 0 for r in recs["fp32"]),
            "fp16_vs_fp32": {k: (round(v, 6) if isinstance(v, float) else v) for k, v in e16.items() if k in keep}}


def forms(stgv, stream, t_end, steps, warmup):
    """Precision and learned forms against the plain FP32 256^3 run."""
    import numpy as np
    import torch
    from paper_2605_14505_amd import learned
    n, nc = 256, 64
    phys = learned.physics(0.6)
    base = dict(n=n, q_f=27, q_g=19, **phys)
    out = {"workload": f"stratified TGV, Re 1600, Fr 0.6, Sc 0.7, velocity shift, G/N 0.02, to t = {t_end}; "
                       f"errors are relative L2 over the histories against the plain FP32 {n}^3 run"}
    rates = {}
    for name, extra, bpn in (("fp32", {}, 368), ("fp16", {"storage": "fp16"}, 184),
                             ("bf16", {"storage": "bf16"}, 184), ("fp64_arith", {"compute": "fp64"}, 368)):
        ms = kernel_time(stgv, stream, dict(base, **extra), steps, warmup)
        rates[name] = {"kernel_ms": round(ms, 5), "mlups": round(n ** 3 / (ms * 1e-3) / 1e6, 1),
                       "hbm_frac": round(bpn * n ** 3 / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    pairs = {}
    for qf, qg in ((27, 19), (27, 27), (19, 19), (19, 15), (15, 7), (7, 27), (27, 7), (19, 7)):
        ms = kernel_time(stgv, stream, dict(base, q_f=qf, q_g=qg), steps, warmup)
        bpn = 2 * (qf + qg) * 4
        pairs[f"{qf}x{qg}"] = {"kernel_ms": round(ms, 5), "mlups": round(n ** 3 / (ms * 1e-3) / 1e6, 1),
                               "bytes_per_node": bpn,
                               "hbm_frac": round(bpn * n ** 3 / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    out["stencil_pairs_fp32"] = pairs
    progress("forms: storage, arithmetic and stencil-pair timings done")
    # FP16 weight-shifted storage for the pairs of the D3Q7-scalar sweep
    for qf, qg in ((27, 19), (27, 7), (19, 7)):
        ms = kernel_time(stgv, stream, dict(base, q_f=qf, q_g=qg, storage="fp16"), steps, warmup)
        bpn = 2 * (qf + qg) * 2
        pairs[f"{qf}x{qg}_fp16"] = {"kernel_ms": round(ms, 5), "mlups": round(n ** 3 / (ms * 1e-3) / 1e6, 1),
                                    "bytes_per_node": bpn,
                                    "hbm_frac": round(bpn * n ** 3 / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    # the largest single-GPU case: 512^3, FP16 storage in place (12.35 GB), Re 3200, Fr 0.5
    big = dict(n=512, q_f=27, q_g=19, storage="fp16", **dict(phys, re=3200.0, fr=0.5))
    ms = kernel_time(stgv, stream, big, max(20, steps // 4), warmup)
    traffic, traffic_src = read_traffic("step_512_27x19_fp16_fp32_shift", 512 ** 3, 184)
    out["large_512_fp16"] = {"kernel_ms": round(ms, 4), "mlups": round(512 ** 3 / (ms * 1e-3) / 1e6, 1),
                             "bytes_per_node": 184,
                             "hbm_frac": round(184 * 512 ** 3 / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                             "traffic": traffic, "traffic_source": traffic_src}
    progress("forms: 512^3 FP16 timing done")
    out["run_512"] = run_512(stgv)
    progress("forms: 512^3 2000-step FP16 and FP32 runs done")
    out["sweep_128_fr05"] = sweep_128(stgv, stream, steps, warmup)
    progress("forms: 128^3 Fr 0.5 run done")
    out["sweep_256_fr"] = sweep_256_fr(stgv)
    progress("forms: 256^3 Froude sweep done")
    net_path = os.path.join(ROOT, "paper_2605_14505_amd", "data", "learned64.npz")
    if os.path.exists(net_path):
        z = np.load(net_path, allow_pickle=False)
        gain = float(z["gain"])
        net = learned.with_gain(learned.Network(z["theta"], z["norm"]), gain if gain > 0 else 1.0)
    else:
        net, gain = learned.Network(seed=0), None       # throughput only: weights do not change it
    coarse = dict(base, n=nc)
    for name, packed in (("plain_64", None), ("learned_64", net.packed)):
        ms = kernel_time(stgv, stream, coarse, 20 * steps // 4, warmup, packed)
        rates[name] = {"kernel_ms": round(ms, 5), "mlups": round(nc ** 3 / (ms * 1e-3) / 1e6, 1)}
    out["throughput"] = rates
    progress("forms: learned-step timing done")
    de_c = max(1, int(round(t_end * learned.steps_per_unit_time(nc) / 100)))
    ref, (spec, spec_ms) = history(stgv, base, t_end, 4 * de_c, spectrum_at=min(15.0, t_end))
    _, _, post = stgv.lbm_postprocess(ref, 1600.0, 0.6, 30.0)
    k = np.arange(1, spec.size)
    sel = (k >= 4) & (k <= 24)
    slope = float(np.polyfit(np.log(k[sel]), np.log(spec[1:][sel]), 1)[0])
    out["postprocess_fp32_256"] = {
        "gamma_b": round(post["gamma_b"], 5), "fr_t": round(post["fr_t"], 5),
        "r_max": round(post["r_max"], 4), "t_r_max": round(post["t_r_max"], 3),
        "spectrum_t": min(15.0, t_end), "spectrum_ms": round(spec_ms, 3),
        "spectrum_slope_k4_24": round(slope, 3),
        "spectrum_head": [float(f"{v:.4e}") for v in spec[:12]]}
    progress("forms: FP32 256^3 reference history to t = 30 done")
    errs = {}
    for name, extra in (("fp16", {"storage": "fp16"}), ("bf16", {"storage": "bf16"})):
        errs[name] = learned.series_errors(history(stgv, dict(base, **extra), t_end, 4 * de_c), ref)
    errs["plain_64"] = learned.series_errors(history(stgv, coarse, t_end, de_c), ref)
    if gain is not None:
        errs["learned_64"] = learned.series_errors(
            history(stgv, coarse, t_end, de_c, net.packed if gain > 0 else None), ref)
        errs["learned_64"]["gain"] = gain
        out["learned_training"] = {
            "train_fr": [0.3, 1.0, 3.0], "train_seeds": [0], "test_fr": 0.6, "test_seed": 0,
            "seeds": "seed 0 only: the seed sets only the 1e-6 initial density noise, so further "
                     "seeds repeat the same teacher flows"}
    keep = ("finite", "ek", "ep", "eps_k", "eps_p", "eps", "dEdt", "dEdt_peak", "dEdt_peak_ref")
    out["errors"] = {k: {q: (round(v[q], 6) if isinstance(v[q], float) else v[q]) for q in keep + ("gain",)
                         if q in v} for k, v in errs.items()}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--q-f", type=int, default=27)
    ap.add_argument("--q-g", type=int, default=19)
    ap.add_argument("--forcing", default="shift", choices=["guo", "shift", "edm", "hcz"])
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--compute", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--diag-every", type=int, default=16)
    ap.add_argument("--cpu-sample-n", type=int, default=128)
    ap.add_argument("--cpu-sample-steps", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-energy-error", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--forms-t", type=float, default=30.0,
                    help="convective time of the precision / learned form histories")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs the single-GPU step only: the library has no halo exchange across "
              "GPUs (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    sys.path.insert(0, ROOT)
    from paper_2605_14505_amd import stgv

    n, K, W = args.n, args.steps, args.warmup
    n3 = n ** 3
    bpe = 4 if args.storage == "fp32" else 2
    bytes_per_node = 2 * (args.q_f + args.q_g) * bpe
    common = dict(n=n, q_f=args.q_f, q_g=args.q_g, forcing=args.forcing, storage=args.storage,
                  compute=args.compute, u0=0.05, re=1600.0, fr=1.0, sc=0.7, g_over_n=0.02,
                  noise_amp=1e-6, seed=0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    # ---- whole-job throughput: K steps with diagnostics at the production cadence
    sim = stgv.Simulation(diag_every=args.diag_every, **common)
    sim.step(W)
    torch.cuda.synchronize()
    sim.diagnostics(raise_unstable=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recs = sim.diagnostics(raise_unstable=False)
    finite = all(r["nonfinite"] == 0 for r in recs)
    sim.close()
    del sim
    mlups = n3 * K / wall / 1e6
    progress(f"timed region: {K} steps, {wall * 1e3 / K:.4f} ms per step")

    # ---- the step kernel alone, HIP events on the launch stream
    sim = stgv.Simulation(diag_every=0, **common)
    sim.step(W)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sim.step(K)
    ev1.record(stream)
    ev1.synchronize()
    kernel_ms = ev0.elapsed_time(ev1) / K
    sim.close()
    del sim
    achieved = bytes_per_node * n3 / (kernel_ms * 1e-3) / 1e9

    # ---- streaming-copy ceiling on buffers of the same size as the state
    nbytes = min(2 << 30, (args.q_f + args.q_g) * n3 * bpe)
    nbytes -= nbytes % 16
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    for _ in range(3):
        stgv.lbm_bw_probe(0, b, a, nbytes, stream.cuda_stream)
    ev0.record(stream)
    reps = 20
    for _ in range(reps):
        stgv.lbm_bw_probe(0, b, a, nbytes, stream.cuda_stream)
    ev1.record(stream)
    ev1.synchronize()
    copy_gbs = 2 * nbytes * reps / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del a, b

    # ---- the step's own access pattern: free streaming (same loads, stores, launch
    # shapes and block order, identity collision) on a state of the same configuration
    sim = stgv.Simulation(diag_every=0, **common)
    sim.free_stream(W + W % 2)
    ev0.record(stream)
    sim.free_stream(K + K % 2)
    ev1.record(stream)
    ev1.synchronize()
    pattern_gbs = bytes_per_node * n3 * (K + K % 2) / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    sim.close()
    del sim

    key = f"step_{n}_{args.q_f}x{args.q_g}_{args.storage}_{args.compute}_{args.forcing}"
    traffic, traffic_src = read_traffic(key, n3, bytes_per_node)

    out = {
        "metric": "MLUPS + % HBM roofline per D3Q27x19 step at 256^3; energy error vs FP64 oracle",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(wall / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.compute == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"stratified Taylor-Green vortex, {n}^3 periodic box, D3Q{args.q_f}xD3Q{args.q_g}, "
                        f"{FORCING_NAMES[args.forcing]} buoyancy, "
                        f"{args.storage} populations (AA in place), {args.compute} arithmetic, "
                        f"diagnostics every {args.diag_every} steps",
            "n": n, "q_f": args.q_f, "q_g": args.q_g, "re": 1600, "fr": 1.0, "sc": 0.7, "u0": 0.05, "g_over_n": 0.02,
            "storage": args.storage, "compute": args.compute, "diag_every": args.diag_every,
            "finite": finite,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "kernel": "lbm_step_kernel",
            "kernel_ms": round(kernel_ms, 5),
            "bytes_per_node": bytes_per_node,
            "step_mlups": round(n3 / (kernel_ms * 1e-3) / 1e6, 1),
            "copy_ceiling_gbs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4),
            "pattern_ceiling_gbs": round(pattern_gbs, 1),
            "frac_of_pattern": round(achieved / pattern_gbs, 4),
            "traffic_source": traffic_src,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_n, args.cpu_sample_steps, args.forcing)
        out["cpu_baseline"]["host_threads_available"] = os.cpu_count()
        out["cpu_baseline"]["host_cpu"] = host_cpu_model()
        progress("CPU oracle baseline done")
    if not args.no_energy_error:
        out["energy_error"] = energy_error(stgv)
        progress("energy error against the oracle's 64^3 histories done")
    if not args.no_forms:
        out["forms"] = forms(stgv, stream, args.forms_t, K, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
