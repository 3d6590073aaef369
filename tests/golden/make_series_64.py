"""Write tests/golden/series_64_shift.json: the FP64 oracle's energy and dissipation
history of the 64^3 stratified Taylor-Green run (D3Q27 x D3Q19, velocity shift, Re 1600,
Fr 0.5, Sc 0.7, U0 0.05, G/N 0.02, noise 1e-6 seed 0) over 2500 steps, records every 50
steps, and the same history with the populations rounded to FP32 after every step (the
floor any FP32-storage implementation reaches).  Calls only the oracle.

    python tests/golden/make_series_64.py [OUT.json]   (two processes, ~5-10 minutes on a fast host)
"""
import json
import multiprocessing as mp
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import model  # noqa: E402

PARAMS = dict(n=64, q_f=27, q_g=19, forcing="shift", u0=0.05, re=1600.0, fr=0.5, sc=0.7,
              g_over_n=0.02, noise_amp=1e-6, seed=0)
STEPS, EVERY = 2501, 50
KEYS = ("step", "t", "ek", "ep", "eps_k", "eps_p")


def _series(job):
    """The run in chunks of 10 records (a progress line after each), the records
    renumbered to the run's own step count."""
    storage, steps, every = job
    p = model.Params(**PARAMS)
    U = model.units(p)
    t0 = time.time()
    state, out, done = None, [], 0
    chunk = 10 * every
    while done < steps:
        k = min(chunk, steps - done)
        state, ser = model.run(p, k, diag_every=every, state=state, U=U, storage=storage)
        for d in ser:
            rec = {key: float(getattr(d, key)) for key in KEYS if key not in ("step", "t")}
            rec["step"] = done + int(d.step)
            rec["t"] = rec["step"] * U.u0 / U.L
            out.append(rec)
        done += k
        print(f"{storage or 'fp64'}: {done}/{steps} steps, {time.time() - t0:.0f} s", flush=True)
    return out


def main(steps=STEPS, every=EVERY):
    out = {"params": PARAMS, "steps": steps - 1, "every": every}
    with mp.get_context("spawn").Pool(2) as pool:
        fp64, fp32 = pool.map(_series, [(None, steps, every), ("fp32", steps, every)])
    out["fp64"], out["fp32_storage"] = fp64, fp32
    path = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                               "series_64_shift.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main()
