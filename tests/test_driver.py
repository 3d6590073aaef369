"""The command-line driver stgv_run (C ABI only, no Python in the loop): its argument and
parameter errors on the CPU, and on the GPU the same diagnostic records as a run through
the Python binding with the same parameters."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RUNNER = os.path.join(ROOT, "paper_2605_14505_amd", "bin", "stgv_run")

pytestmark = pytest.mark.skipif(not os.path.exists(RUNNER), reason="stgv_run not built")


def run(*args, timeout=60):
    return subprocess.run([RUNNER, *map(str, args)], capture_output=True, text=True, timeout=timeout)


def test_help_and_bad_options():
    r = run("--help")
    assert r.returncode == 0 and "usage" in r.stderr
    for bad in (["--forcing", "foo"], ["--storage", "fp8"], ["--bogus", "1"], ["--n"], ["--steps", "-1"]):
        r = run(*bad)
        assert r.returncode == 2, bad
        assert "usage" in r.stderr


@pytest.mark.parametrize("args,msg", [
    (["--n", "3"], "n = 3"),
    (["--qf", "27", "--qg", "5"], "stencil pair"),
    (["--storage", "fp16", "--compute", "fp64"], "LBM_EINVAL"),
    (["--u0", "0.5"], "LBM_EINVAL"),
])
def test_parameter_errors_stop_before_the_gpu(args, msg):
    # lbm_query_sizes validates on the CPU, so these never allocate device memory
    r = run(*args)
    assert r.returncode == 1
    assert "parameters" in r.stderr and msg in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("forcing,storage", [("shift", "fp32"), ("guo", "fp16")])
def test_driver_records_match_the_binding(forcing, storage, tmp_path):
    import torch

    from paper_2605_14505_amd import stgv

    kw = dict(n=32, q_f=27, q_g=19, forcing=forcing, storage=storage, u0=0.05, re=400.0, fr=1.0, sc=0.7,
              g_over_n=0.02, noise_amp=1e-6, seed=5, diag_every=25)
    r = run("--n", 32, "--qf", 27, "--qg", 19, "--forcing", forcing, "--storage", storage, "--re", 400, "--fr", 1,
            "--sc", 0.7, "--u0", 0.05, "--gn", 0.02, "--noise", 1e-6, "--seed", 5, "--steps", 200, "--diag", 25,
            "--spectrum", tmp_path / "spectrum.txt", timeout=120)
    assert r.returncode == 0, r.stderr
    assert "MLUPS" in r.stderr
    lines = r.stdout.strip().splitlines()
    assert lines[0] == "step,t,ek,ep,eps_k,eps_p,mass,umax"
    rows = [list(map(float, ln.split(","))) for ln in lines[1:]]
    sim = stgv.Simulation(device="cuda:0", **kw)
    sim.step(200)
    recs = sim.diagnostics()
    spec = sim.spectrum().cpu().numpy()
    sim.close()
    torch.cuda.synchronize()
    assert len(rows) == len(recs) == 8
    for row, rec in zip(rows, recs):
        assert int(row[0]) == rec["step"]
        # same library, same kernels: equal up to the 11 significant digits printed
        for j, key in enumerate(("ek", "ep", "eps_k", "eps_p", "mass"), start=2):
            assert row[j] == pytest.approx(rec[key], rel=1e-10, abs=1e-300), (rec["step"], key)
    # the post-processing line: the binding's lbm_postprocess over the same records
    _, _, post = stgv.lbm_postprocess(recs, re=400.0, fr=1.0, t_end=recs[-1]["t"])
    line = [ln for ln in r.stderr.splitlines() if "Gamma_b" in ln][0].split()
    got = {k: float(line[line.index(k) + 1]) for k in ("Gamma_b", "Fr_t", "R_max")}
    assert got["Gamma_b"] == pytest.approx(post["gamma_b"], rel=1e-5)
    assert got["Fr_t"] == pytest.approx(post["fr_t"], rel=1e-5)
    assert got["R_max"] == pytest.approx(post["r_max"], rel=1e-5)
    # the spectrum file: the binding's spectrum of the same final state
    table = [ln.split() for ln in (tmp_path / "spectrum.txt").read_text().splitlines()]
    assert [int(t[0]) for t in table] == list(range(stgv.lbm_spectrum_shells(32)))
    # the transforms are single precision and the two processes' results differ in the
    # last bits (measured ~2e-9 of a shell), so the bar is relative to the total energy
    total = float(spec.sum())
    for (k, e), ref in zip(table, spec):
        assert abs(float(e) - ref) <= 1e-7 * total, k


def _header(n, q_f=27, q_g=19, storage=0, step=0, fr=1.0, forcing=1):
    # the lbm_params of include/stgv.h, as the driver's defaults set them, then the step
    import struct
    params = struct.pack("<10i6dQ", n, q_f, q_g, forcing, storage, 0, 0, 50, -1, 0,
                         0.05, 1600.0, fr, 0.7, 0.02, 1e-6, 0)
    return b"STGVCKP2" + params + struct.pack("<q", step)


@pytest.mark.parametrize("content", [None, b"junk", "wrong_n", "truncated", "wrong_storage", "wrong_fr",
                                     "wrong_forcing", "old_format"])
def test_resume_rejects_what_is_not_a_checkpoint_of_the_run(content, tmp_path):
    # the file is read and checked before any GPU work: exit status 2
    path = tmp_path / "state.bin"
    body = bytes(46 * 32 ** 3 * 4)
    if content == "wrong_n":
        path.write_bytes(_header(16) + bytes(46 * 16 ** 3 * 4))
    elif content == "truncated":
        path.write_bytes(_header(32) + bytes(100))
    elif content == "wrong_storage":
        path.write_bytes(_header(32, storage=1) + body)
    elif content == "wrong_fr":
        path.write_bytes(_header(32, fr=0.5) + body)
    elif content == "wrong_forcing":
        path.write_bytes(_header(32, forcing=0) + body)
    elif content == "old_format":
        import struct
        path.write_bytes(b"STGVCKP1" + struct.pack("<iiiiq", 32, 27, 19, 0, 0) + body)
    elif content is not None:
        path.write_bytes(content)
    r = run("--n", 32, "--resume", path)
    assert r.returncode == 2
    assert str(path) in r.stderr
    if content in ("wrong_storage", "wrong_fr", "wrong_forcing"):
        assert {"wrong_storage": "storage", "wrong_fr": "Fr", "wrong_forcing": "forcing"}[content] in r.stderr
    # the header that matches is accepted up to the body (a full one is the GPU test's)
    if content == "truncated":
        assert "not a checkpoint" in r.stderr


@pytest.mark.gpu
@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_checkpoint_and_resume_reproduce_the_uninterrupted_run(storage, tmp_path):
    common = ["--n", 32, "--storage", storage, "--fr", 0.5, "--re", 400, "--diag", 25, "--seed", 3]
    whole = run(*common, "--steps", 120, "--checkpoint", tmp_path / "whole.bin", timeout=120)
    assert whole.returncode == 0, whole.stderr
    # stop after an odd number of steps, so the run resumes in the other AA parity
    first = run(*common, "--steps", 71, "--checkpoint", tmp_path / "part.bin", timeout=120)
    assert first.returncode == 0, first.stderr
    rest = run(*common, "--steps", 49, "--resume", tmp_path / "part.bin", "--checkpoint", tmp_path / "end.bin",
               timeout=120)
    assert rest.returncode == 0, rest.stderr
    rows = {ln.split(",")[0]: ln for ln in whole.stdout.strip().splitlines()[1:]}
    resumed = rest.stdout.strip().splitlines()[1:]
    assert [ln.split(",")[0] for ln in resumed] == ["75", "100"]
    for ln in resumed:
        assert ln == rows[ln.split(",")[0]]
    # the final states, header (step 120) included, are the same bytes
    assert (tmp_path / "end.bin").read_bytes() == (tmp_path / "whole.bin").read_bytes()


def test_network_export_round_trip_and_rejection(tmp_path):
    import numpy as np

    from paper_2605_14505_amd import learned

    rng = np.random.default_rng(0)
    theta = rng.standard_normal(learned.NPARAM).astype(np.float32)
    norm = np.concatenate([rng.standard_normal(47), rng.random(47), rng.random(41) + 0.5])
    path = tmp_path / "net.bin"
    learned.export_network(theta, norm, path, gain=0.25)
    raw = path.read_bytes()
    assert raw[:8] == learned.NET_MAGIC
    counts = np.frombuffer(raw[8:16], dtype="<i4")
    assert list(counts) == [learned.NPARAM, 135]
    body = np.frombuffer(raw[16:], dtype="<f4")
    np.testing.assert_array_equal(body[:learned.NPARAM], theta)
    np.testing.assert_array_equal(body[learned.NPARAM:learned.NPARAM + 94], norm[:94].astype(np.float32))
    np.testing.assert_array_equal(body[learned.NPARAM + 94:], (norm[94:] * 0.25).astype(np.float32))
    # the driver checks a network file before any GPU work
    bad = tmp_path / "bad.bin"
    bad.write_bytes(raw[:100])
    r = run("--n", 64, "--mlp", bad)
    assert r.returncode == 2 and "not a network file" in r.stderr


@pytest.mark.gpu
def test_driver_runs_the_learned_step_like_the_binding(tmp_path):
    import numpy as np
    import torch

    from paper_2605_14505_amd import learned, stgv

    z = np.load(os.path.join(ROOT, "paper_2605_14505_amd", "data", "learned64.npz"), allow_pickle=False)
    learned.export_network(z["theta"], z["norm"], tmp_path / "net.bin", gain=1.0)
    r = run("--n", 64, "--fr", 0.6, "--re", 1600, "--sc", 0.7, "--steps", 100, "--diag", 25, "--mlp",
            tmp_path / "net.bin", timeout=120)
    assert r.returncode == 0, r.stderr
    rows = [list(map(float, ln.split(","))) for ln in r.stdout.strip().splitlines()[1:]]
    kw = dict(n=64, q_f=27, q_g=19, forcing="shift", u0=0.05, re=1600.0, fr=0.6, sc=0.7, g_over_n=0.02,
              noise_amp=1e-6, seed=0, diag_every=25)
    net = learned.with_gain(learned.Network(z["theta"], z["norm"]), 1.0)
    sim = stgv.Simulation(device="cuda:0", **kw)
    sim.set_mlp(net.packed)
    sim.step(100)
    recs = sim.diagnostics()
    plain = stgv.Simulation(device="cuda:0", **kw)
    plain.step(100)
    recs_plain = plain.diagnostics()
    sim.close()
    plain.close()
    torch.cuda.synchronize()
    assert [int(row[0]) for row in rows] == [rec["step"] for rec in recs] == [0, 25, 50, 75]
    for row, rec in zip(rows, recs):
        for j, key in enumerate(("ek", "ep", "eps_k", "eps_p", "mass"), start=2):
            assert row[j] == pytest.approx(rec[key], rel=1e-10, abs=1e-300), (rec["step"], key)
    # the network did act: the histories leave the plain step's
    assert rows[-1][4] != pytest.approx(recs_plain[-1]["eps_k"], rel=1e-9)


def test_learned_driver_exports_the_shipped_network(tmp_path, capsys):
    import numpy as np

    from paper_2605_14505_amd import learned

    out = tmp_path / "net.bin"
    learned.main(["--export", str(out), "--gain", "0.5"])
    assert "gain 0.5" in capsys.readouterr().out
    z = np.load(os.path.join(ROOT, "paper_2605_14505_amd", "data", "learned64.npz"), allow_pickle=False)
    body = np.frombuffer(out.read_bytes()[16:], dtype="<f4")
    np.testing.assert_array_equal(body[:learned.NPARAM], z["theta"].astype(np.float32))
    np.testing.assert_allclose(body[learned.NPARAM + 94:], (z["norm"][94:] * 0.5).astype(np.float32))
