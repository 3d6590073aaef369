"""GPU parity of the learned-correction kernels (through the C ABI) against the FP64 oracle.

The network runs on BF16 MFMA with FP32 accumulation: weights, activations and
back-propagated deltas are rounded to BF16 (8 significand bits), products are exact and
sums are FP32.  Every output and every gradient entry is held to its own tolerance: the
rounding errors are propagated element by element through the oracle's FP64 forward and
backward pass as independent errors (first order, see `bf16_bounds`), and an entry off by
more than 6 standard deviations of that model, plus a worst-case bound on the FP32 sums,
fails; everything else (packing, normalisation, Adam,
restriction, training pairs) is FP32 arithmetic on the same inputs and is compared at
FP32 rounding level.
"""
import numpy as np
import pytest

from inputs import sample_nodes, uniform_deviations
from oracle import lattice as lat, learned as L, model

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
stgv = pytest.importorskip("paper_2605_14505_amd.stgv")

DEV = "cuda:0"


def stream():
    return torch.cuda.current_stream().cuda_stream


def t32(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device=DEV)


def packed_net(theta, norm):
    params = t32(theta)
    nrm = t32(np.concatenate([np.asarray(v, dtype=np.float64) for v in norm]))
    packed = torch.empty(stgv.lbm_mlp_packed_bytes(), dtype=torch.uint8, device=DEV)
    stgv.lbm_mlp_pack(params, nrm, packed, stream())
    return packed


def rel_norm(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


U_F32 = 2.0 ** -24
K_SIGMA = 6.0            # outputs / gradient entries beyond 6 sigma of the rounding model fail


def bf16_ulp2(v):
    """Square of the BF16 spacing at |v| (8 significand bits): a rounding to nearest is off
    by at most half of it, and by sqrt(1/12) of it in the root-mean-square sense."""
    e = np.floor(np.log2(np.maximum(np.abs(v), 1e-300)))
    return np.where(np.abs(v) > 0, (2.0 ** (e - 7)) ** 2, 0.0)


def _layer(W, b, a, va):
    """z = W a + b with W and a rounded to BF16 (a carrying errors of variance va before
    its rounding), exact products and FP32 sums: z, the variance of its error, and the
    bound on the FP32 sum's own error."""
    ra = va + bf16_ulp2(a) / 12.0
    z = a @ W.T + b
    vz = ra @ (W * W).T + (a * a) @ (bf16_ulp2(W) / 12.0).T
    acc = (W.shape[1] + 2) * U_F32 * (np.abs(a) @ np.abs(W).T + np.abs(b))
    return z, vz, acc


def _tanh(z, vz, acc):
    """BF16(tanhf(z)): the error passes through tanh' = 1 - h^2 (libm's FP32 tanh adds a
    few ulps, folded into the sum's bound)."""
    h = np.tanh(z)
    t = 1.0 - h * h
    return h, t * t * vz, t * acc + 4 * U_F32


def bf16_bounds(theta, x, norm, y=None):
    """Oracle outputs (and, with targets y, the gradient) of the network on FP32 rows x,
    with the element-wise tolerance of BF16 operands and FP32 accumulation: K_SIGMA times
    the standard deviation of the rounding error, first order, every BF16 rounding an
    independent error uniform over half a BF16 spacing of the value it rounds, plus a
    worst-case bound on the FP32 sums.  Returns (y_out, tol) or (grad, tol, loss)."""
    p = L.unpack(theta)
    mean, iscale, ys = (np.asarray(v, np.float64) for v in norm)
    xn = (x - mean) * iscale
    # FP32 normalisation with FP32 mean / iscale (worst case), then the BF16 rounding
    ax = 4 * U_F32 * (np.abs(x) + np.abs(mean)) * np.abs(iscale)
    z1, v1, a1 = _layer(p["W1"], p["b1"], xn, 0.0)
    a1 = a1 + ax @ np.abs(p["W1"]).T
    h1, vh1, ah1 = _tanh(z1, v1, a1)
    z2, v2, a2 = _layer(p["W2"], p["b2"], h1, vh1)
    a2 = a2 + ah1 @ np.abs(p["W2"]).T
    h2, vh2, ah2 = _tanh(z2, v2, a2)
    o, vo, ao = _layer(p["W3"], p["b3"], h2, vh2)
    ao = ao + ah2 @ np.abs(p["W3"]).T
    if y is None:
        out = o * ys
        return out, (K_SIGMA * np.sqrt(vo) + ao) * ys + 2 * U_F32 * np.abs(out)
    B = x.shape[0]
    c = 2.0 / (B * L.N_OUT)
    res = o - y / ys
    d0 = c * res
    vd0, ad0 = c * c * vo, c * (ao + 3 * U_F32 * np.abs(y / ys) + U_F32 * np.abs(res))

    def back(W, d, vd, ad, h, vh, ah):
        v, vv, av = _layer(W.T, np.zeros(W.shape[1]), d, vd)
        av = av + ad @ np.abs(W)
        t = 1.0 - h * h
        r = v * t
        return r, t * t * vv + 4 * v * v * h * h * vh, np.abs(t) * av + 2 * np.abs(v * h) * ah + 2 * U_F32 * np.abs(r)

    d1, vd1, ad1 = back(p["W3"], d0, vd0, ad0, h2, vh2, ah2)
    d2, vd2, ad2 = back(p["W2"], d1, vd1, ad1, h1, vh1, ah1)

    def outer(d, vd, ad, a, va, aa):
        rd, ra = vd + bf16_ulp2(d) / 12.0, va + bf16_ulp2(a) / 12.0
        g = d.T @ a
        vg = rd.T @ (a * a) + (d * d).T @ ra
        ag = ad.T @ np.abs(a) + np.abs(d).T @ aa + (B + 2) * U_F32 * (np.abs(d).T @ np.abs(a))
        return g, K_SIGMA * np.sqrt(vg) + ag + U_F32 * np.abs(g)

    gW1, tW1 = outer(d2, vd2, ad2, xn, 0.0, ax)
    gW2, tW2 = outer(d1, vd1, ad1, h1, vh1, ah1)
    gW3, tW3 = outer(d0, vd0, ad0, h2, vh2, ah2)
    gb = []
    for d, vd, ad in ((d2, vd2, ad2), (d1, vd1, ad1), (d0, vd0, ad0)):
        rd = vd + bf16_ulp2(d) / 12.0
        gsum = d.sum(0)
        gb.append((gsum, K_SIGMA * np.sqrt(rd.sum(0)) + ad.sum(0) + (B + 2) * U_F32 * np.abs(d).sum(0)))
    grad = L.pack({"W1": gW1, "b1": gb[0][0], "W2": gW2, "b2": gb[1][0], "W3": gW3, "b3": gb[2][0]})
    tol = L.pack({"W1": tW1, "b1": gb[0][1], "W2": tW2, "b2": gb[1][1], "W3": tW3, "b3": gb[2][1]})
    return grad, tol, float(np.mean(res * res))


def random_norm(rng):
    return (0.1 * rng.standard_normal(47), 1.0 + 0.2 * rng.uniform(-1, 1, 47),
            1e-3 * (1.0 + rng.uniform(0, 1, 41)))


@pytest.mark.parametrize("rows", [1, 64, 150])
def test_forward_matches_oracle(rows):
    rng = np.random.default_rng(rows)
    theta = L.init_params(1) + 0.01 * rng.standard_normal(L.N_PARAMS)
    norm = random_norm(rng)
    x = rng.standard_normal((rows, 47)) * 0.5 + norm[0]
    packed = packed_net(theta, norm)
    y = torch.empty((rows, 41), dtype=torch.float32, device=DEV)
    stgv.lbm_mlp_forward(packed, t32(x), rows, y, stream())
    xf = x.astype(np.float32).astype(np.float64)
    o, _ = L.forward(theta, (xf - norm[0]) * norm[1])
    ref = o * norm[2]
    # the same FP32 network parameters the GPU was given (t32 rounds them)
    th32 = theta.astype(np.float32).astype(np.float64)
    nrm32 = tuple(np.asarray(v, np.float64).astype(np.float32).astype(np.float64) for v in norm)
    bref, bound = bf16_bounds(th32, xf, nrm32)
    got = y.cpu().numpy().astype(np.float64)
    err = np.abs(got - bref)          # the network the GPU was given: FP32 parameters
    print(f"\nforward rows={rows}: relative L2 error {rel_norm(got, ref):.3e}; error / bound: "
          f"max {np.max(err / bound):.3f}, median {np.median(err / bound):.3f}; "
          f"median bound / |y| {np.median(bound / np.abs(bref)):.3e}")
    assert np.all(err <= bound), np.unravel_index(np.argmax(err / bound), err.shape)


def test_gradient_and_loss_match_oracle():
    rng = np.random.default_rng(5)
    theta = L.init_params(2) + 0.01 * rng.standard_normal(L.N_PARAMS)
    norm = random_norm(rng)
    n = 300
    x = rng.standard_normal((n, 47)) * 0.7 + norm[0]
    y = rng.standard_normal((n, 41)) * norm[2]
    idx = rng.permutation(n)[:200]                       # ragged: 200 = 3 blocks + 8
    packed = packed_net(theta, norm)
    grad = torch.empty(L.N_PARAMS, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float64, device=DEV)
    work = torch.empty(stgv.lbm_mlp_grad_work_bytes(200), dtype=torch.uint8, device=DEV)
    stgv.lbm_mlp_grad(packed, t32(x), t32(y), torch.tensor(idx, dtype=torch.int64, device=DEV), 200,
                      grad, loss, work, stream())
    xf = x.astype(np.float32).astype(np.float64)[idx]
    yf = y.astype(np.float32).astype(np.float64)[idx]
    ref_loss, ref_g = L.loss_and_grad(theta, (xf - norm[0]) * norm[1], yf / norm[2])
    th32 = theta.astype(np.float32).astype(np.float64)
    nrm32 = tuple(np.asarray(v, np.float64).astype(np.float32).astype(np.float64) for v in norm)
    bgrad, bound, bloss = bf16_bounds(th32, xf, nrm32, yf)
    g = grad.cpu().numpy().astype(np.float64)
    err = np.abs(g - bgrad)
    parts, got, bnd = L.unpack(ref_g), L.unpack(g), L.unpack(bound)
    for name in parts:
        ratio = np.abs(got[name] - L.unpack(bgrad)[name]) / bnd[name]
        print(f"grad {name}: relative L2 error {rel_norm(got[name], parts[name]):.3e}; error / bound "
              f"max {ratio.max():.3f}, median {np.median(ratio):.3f}")
    assert np.all(err <= bound), (int(np.argmax(err / bound)), float(np.max(err / bound)))
    # the loss: a mean of 200 x 41 squared residuals, each off by its BF16-level output error
    assert abs(loss.item() - bloss) < 0.02 * bloss
    assert bloss == pytest.approx(ref_loss, rel=1e-3)      # FP32 against FP64 parameters


def test_adam_matches_oracle():
    rng = np.random.default_rng(7)
    theta = rng.standard_normal(L.N_PARAMS) * 0.1
    th = t32(theta)
    m = torch.zeros(L.N_PARAMS, device=DEV)
    v = torch.zeros(L.N_PARAMS, device=DEV)
    rt, rm, rv = theta.astype(np.float32).astype(np.float64), np.zeros(L.N_PARAMS), np.zeros(L.N_PARAMS)
    for t in (1, 2, 3):
        gr = rng.standard_normal(L.N_PARAMS) * 1e-3
        stgv.lbm_mlp_adam(th, m, v, t32(gr), t, 1e-3, stream())
        rt, rm, rv = L.adam_step(rt, gr.astype(np.float32).astype(np.float64), rm, rv, t, 1e-3)
    np.testing.assert_allclose(th.cpu().numpy(), rt, rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(m.cpu().numpy(), rm, rtol=1e-5, atol=1e-10)   # FP32 ulps of |m| ~ 1e-4


def test_normalisation_matches_oracle():
    rng = np.random.default_rng(8)
    n = 5000
    x = rng.standard_normal((n, 47)) * rng.uniform(0.1, 3, 47) + rng.uniform(-1, 1, 47)
    x[:, 0] = 0.25                                        # a constant column
    y = rng.standard_normal((n, 41)) * 1e-4
    norm = torch.empty(135, dtype=torch.float32, device=DEV)
    work = torch.empty(stgv.lbm_mlp_norm_work_bytes(), dtype=torch.uint8, device=DEV)
    stgv.lbm_mlp_norm(t32(x), t32(y), n, norm, work, stream())
    ref = L.norm_from_data(x.astype(np.float32), y.astype(np.float32))
    got = norm.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got[:47], ref[0], rtol=1e-6, atol=1e-7)
    assert got[47] == 0.0
    np.testing.assert_allclose(got[48:94], ref[1][1:], rtol=1e-4)
    np.testing.assert_allclose(got[94:], ref[2], rtol=1e-6)


@pytest.mark.parametrize("forcing", ["guo", "shift"])
def test_restriction_matches_oracle(forcing):
    kwf = dict(n=32, forcing=forcing, u0=0.05, re=200.0, fr=0.5, sc=0.7, g_over_n=0.5,
               noise_amp=1e-4, seed=1)
    kwc = dict(kwf, n=8)
    fine = stgv.Simulation(**kwf)
    coarse = stgv.Simulation(**kwc)
    fine.step(3)                                          # odd parity: exercises the AA decode
    got = fine.restrict_to(coarse).cpu().numpy().astype(np.float64)
    pops = fine.populations().cpu().numpy().astype(np.float64)
    lf, lg = lat.D3Q27, lat.D3Q19
    f = pops[:27] + lf.w[:, None, None, None]
    g = pops[27:] + lg.w[:, None, None, None]
    pf, pc = model.Params(**kwf), model.Params(**kwc)
    fc, gc = L.restrict(f, g, pf, pc)
    ref = np.concatenate([fc - lf.w[:, None, None, None], gc - lg.w[:, None, None, None]])
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"\nrestriction {forcing}: relative L-inf {err:.3e}")
    assert err < 2e-6


@pytest.mark.parametrize("forcing", ["guo", "shift"])
def test_training_pairs_match_oracle(forcing):
    kw = dict(n=12, forcing=forcing, u0=0.05, re=100.0, fr=0.5, sc=0.7, g_over_n=0.5)
    sim = stgv.Simulation(**kw)
    rng_dev = [uniform_deviations(46, 12, 1e-3, seed=s) for s in (11, 12, 13)]
    a, b, c = (torch.from_numpy(d).to(DEV) for d in rng_dev)
    x = torch.empty((12 ** 3, 47), dtype=torch.float32, device=DEV)
    y = torch.empty((12 ** 3, 41), dtype=torch.float32, device=DEV)
    stgv.lbm_training_pairs(sim.ctx, a, b, c, x, y)
    torch.cuda.synchronize()
    lf, lg = lat.D3Q27, lat.D3Q19
    w = np.concatenate([lf.w, lg.w])[:, None, None, None]
    A, B, C = (d.astype(np.float64) + w for d in rng_dev)
    rx, ry = L.pairs_from((A[:27], A[27:]), (B[:27], B[27:]), (C[:27], C[27:]), model.Params(**kw))
    gx = x.cpu().numpy().T.reshape(47, 12, 12, 12)
    gy = y.cpu().numpy().T.reshape(41, 12, 12, 12)
    ex = np.abs(gx - rx).max(axis=(1, 2, 3)) / (np.abs(rx).max(axis=(1, 2, 3)) + 1e-30)
    ey = np.abs(gy - ry).max() / np.abs(ry).max()
    print(f"\npairs {forcing}: features max rel {ex.max():.3e}, targets {ey:.3e}")
    assert ex.max() < 1e-4 and ey < 1e-5


def _learned_kw(**over):
    kw = dict(n=64, forcing="shift", u0=0.05, re=1600.0, fr=0.6, sc=0.7, g_over_n=0.02,
              noise_amp=1e-6, seed=0)
    kw.update(over)
    return kw


@pytest.mark.parametrize("forcing", ["guo", "shift"])
def test_zero_output_layer_reproduces_the_plain_step(forcing):
    # The fused learned step splits a node over two lanes and evaluates the collision in
    # plain FP32 (the plain step keeps its velocity-linear terms exact, see lbm_device.hpp).
    # With a zero output layer it must be the plain step to FP32 arithmetic: within a few
    # FP32 roundings of the largest population deviation of the FP64 oracle (run from the
    # same FP32 state), at both AA parities, and never worse than twice the plain step.
    kw = _learned_kw(forcing=forcing, noise_amp=1e-3)
    theta = L.unpack(L.init_params(3))
    theta["W3"][:] = 0.0
    theta["b3"][:] = 0.0
    packed = packed_net(L.pack(theta), (np.zeros(47), np.ones(47), np.ones(41)))
    plain = stgv.Simulation(**kw)
    learned = stgv.Simulation(**kw)
    learned.set_mlp(packed)
    lf, lg = lat.D3Q27, lat.D3Q19
    w = np.concatenate([lf.w, lg.w])[:, None, None, None]
    pops = plain.populations().cpu().numpy().astype(np.float64) + w
    f, g = pops[:27], pops[27:]
    U = model.units(model.Params(**kw))
    for n in (1, 2):                                       # ends on an odd, then an even step
        plain.step(n)
        learned.step(n)
        for _ in range(n):
            fs, gs, _ = model.collide(f, g, lf, lg, U)
            f, g = model.stream(fs, lf), model.stream(gs, lg)
        ref = np.concatenate([f, g]) - w
        a = plain.populations().cpu().numpy().astype(np.float64)
        b = learned.populations().cpu().numpy().astype(np.float64)
        e_plain, e_learned = np.abs(a - ref).max(), np.abs(b - ref).max()
        print(f"\n{forcing} step {plain.step_count}: |plain - oracle| {e_plain:.2e}, "
              f"|learned - oracle| {e_learned:.2e}, |plain - learned| {np.abs(a - b).max():.2e}")
        # sixteen roundings of the largest value per step the learned run has taken (only the
        # oracle restarts from the plain kernel's state)
        fp32_bound = 16 * 2.0 ** -24 * np.abs(ref).max() * plain.step_count
        assert e_plain <= fp32_bound
        assert e_learned <= max(2.0 * e_plain, fp32_bound)
        # the oracle ran from the plain kernel's rounding; restart it from the FP32 state
        f, g = (a + w)[:27], (a + w)[27:]


@pytest.mark.parametrize("n,layout", [(64, "aa"), (128, "aa"), (128, "ab")])
def test_learned_diagnostics_match_the_plain_step(n, layout):
    # The learned step's diagnostic instance writes the fields and the FP64 partials of its
    # own blocks.  With a zero output layer it is the plain step to FP32 rounding, so every
    # record must be the plain run's to ~1e-7; a block whose partials were missed or
    # counted twice moves the energies by percents.
    kw = _learned_kw(n=n, forcing="shift", noise_amp=1e-3)
    theta = L.unpack(L.init_params(3))
    theta["W3"][:] = 0.0
    theta["b3"][:] = 0.0
    packed = packed_net(L.pack(theta), (np.zeros(47), np.ones(47), np.ones(41)))
    plain = stgv.Simulation(layout=layout, diag_every=2, **kw)
    learned = stgv.Simulation(layout=layout, diag_every=2, **kw)
    learned.set_mlp(packed)
    plain.step(7)
    learned.step(7)
    rp, rl = plain.diagnostics(), learned.diagnostics()
    assert len(rp) == len(rl) >= 4
    worst = 0.0
    for a, b in zip(rp, rl):
        assert a["step"] == b["step"] and b["nonfinite"] == 0
        for k in ("ek", "ep", "eps_k", "eps_p", "umax"):
            worst = max(worst, abs(a[k] - b[k]) / abs(a[k]))
    print(f"\nlearned vs plain diagnostics, n={n} {layout}: {len(rp)} records, worst rel {worst:.2e}")
    assert worst < 1e-5                                  # measured: 2e-7
    plain.close()
    learned.close()


@pytest.mark.parametrize("layout,before", [("aa", 2), ("aa", 3), ("ab", 2)])
def test_learned_step_matches_oracle(layout, before):
    kw = _learned_kw(n=64, forcing="guo", re=800.0)
    rng = np.random.default_rng(4)
    theta = L.init_params(4) + 0.01 * rng.standard_normal(L.N_PARAMS)
    sim = stgv.Simulation(layout=layout, **kw)
    sim.step(before)                                      # even (2) or odd (3) AA parity next
    pops = sim.populations().cpu().numpy().astype(np.float64)
    # normalisation from the state's own features, outputs scaled to ~1e-6 corrections
    lf, lg = lat.D3Q27, lat.D3Q19
    f0 = pops[:27] + lf.w[:, None, None, None]
    g0 = pops[27:] + lg.w[:, None, None, None]
    p = model.Params(**kw)
    U = model.units(p)
    xs = L.features(f0, g0, U).reshape(47, -1).T
    mean, iscale, _ = L.norm_from_data(xs, np.ones((1, 41)))
    norm = (mean, iscale, np.full(41, 1e-6))
    packed = packed_net(theta, norm)
    sim.set_mlp(packed)
    sim.step(1)
    got = sim.populations().cpu().numpy().astype(np.float64)
    fs, gs, _ = L.learned_collide(f0, g0, U, theta, norm)
    f1, g1 = model.stream(fs, lf), model.stream(gs, lg)
    ref = np.concatenate([f1 - lf.w[:, None, None, None], g1 - lg.w[:, None, None, None]])
    fp, gp, _ = model.collide(f0, g0, lf, lg, U)
    plain = np.concatenate([model.stream(fp, lf) - lf.w[:, None, None, None],
                            model.stream(gp, lg) - lg.w[:, None, None, None]])
    corr = ref - plain
    err_corr = np.abs((got - plain) - corr).max() / np.abs(corr).max()
    print(f"\nlearned step ({layout}, after {before}): correction magnitude {np.abs(corr).max():.3e}, "
          f"relative error {err_corr:.3e}")
    assert err_corr < 0.05
    # the correction leaves mass, momentum and scalar untouched
    e = lf.e.astype(float)
    dcorr_f = got[:27] - plain[:27]
    assert abs(dcorr_f.sum()) < 1e-9 * dcorr_f.size


@pytest.mark.parametrize("n,layout,before,forcing", [(128, "aa", 2, "shift"), (128, "aa", 3, "shift"),
                                                     (192, "aa", 3, "guo"), (192, "ab", 2, "shift"),
                                                     (256, "aa", 3, "shift")])
def test_learned_step_sampled_parity_wider_boxes(n, layout, before, forcing):
    # n = 128 and 192 put two and three blocks along each row (64^3 has one); 256 is the
    # largest box the learned form takes (3.1 GB of state behind one base).  A node's
    # value after the step is the collision at x - e_i, so the oracle runs on the 3 x 3 x 3
    # patch of pre-step populations around each sampled node, the samples including the
    # edges of the blocks' 32-node runs and of their row pairs.
    torch.cuda.empty_cache()
    kw = _learned_kw(n=n, forcing=forcing, re=800.0)
    rng = np.random.default_rng(5)
    theta = L.init_params(5) + 0.01 * rng.standard_normal(L.N_PARAMS)
    sim = stgv.Simulation(layout=layout, **kw)
    sim.step(before)                                      # even (2) or odd (3) AA parity next
    xs_edge = sorted({0, 31, 32, 63, 64, 127, 128, n - 65, n - 64, n - 1} & set(range(n)))
    pts = sorted(set(sample_nodes(n, 40, seed=n + before))
                 | {(z, y, x) for z in (0, n - 1) for y in (0, 1, 2, n - 1) for x in xs_edge})
    c = np.array(pts, dtype=np.int64)                                      # (m, 3) as (z, y, x)
    d = np.array([(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])
    patch = torch.from_numpy(((c[:, None, :] + d[None]) % n).reshape(-1, 3)).to(DEV)
    pops = sim.populations()
    pre = pops[:, patch[:, 0], patch[:, 1], patch[:, 2]].cpu().numpy().astype(np.float64)
    del pops
    m = len(pts)
    pre = pre.reshape(46, m, 3, 3, 3)
    lf, lg = lat.D3Q27, lat.D3Q19
    wf, wg = lf.w[:, None, None, None], lg.w[:, None, None, None]
    U = model.units(model.Params(**kw))
    xs = np.concatenate([L.features(pre[:27, k] + wf, pre[27:, k] + wg, U).reshape(47, -1).T
                         for k in range(m)])
    mean, iscale, _ = L.norm_from_data(xs, np.ones((1, 41)))
    norm = (mean, iscale, np.full(41, 1e-6))
    sim.set_mlp(packed_net(theta, norm))
    sim.step(1)
    idx = torch.from_numpy(c).to(DEV)
    pops = sim.populations()
    got = pops[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().astype(np.float64)   # (46, m)
    del pops
    ref, plain = np.empty_like(got), np.empty_like(got)
    for k in range(m):
        f0, g0 = pre[:27, k] + wf, pre[27:, k] + wg
        fs, gs, _ = L.learned_collide(f0, g0, U, theta, norm)
        fp, gp, _ = model.collide(f0, g0, lf, lg, U)
        ref[:, k] = np.concatenate([model.stream(fs, lf)[:, 1, 1, 1] - lf.w,
                                    model.stream(gs, lg)[:, 1, 1, 1] - lg.w])
        plain[:, k] = np.concatenate([model.stream(fp, lf)[:, 1, 1, 1] - lf.w,
                                      model.stream(gp, lg)[:, 1, 1, 1] - lg.w])
    corr = ref - plain
    err_corr = np.abs((got - plain) - corr).max() / np.abs(corr).max()
    print(f"\nlearned step n={n} ({layout}, after {before}, {forcing}), {m} nodes: correction "
          f"magnitude {np.abs(corr).max():.3e}, relative error {err_corr:.3e}")
    # BF16 operands (2^-9 relative each) put the correction ~4e-3 off; a wrong slot,
    # node or array is off by O(1)
    assert err_corr < 0.02
    sim.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("forcing", ["edm", "hcz"])
def test_learned_form_rejects_other_forcing_schemes(forcing):
    sim = stgv.Simulation(**_learned_kw(forcing=forcing))
    packed = packed_net(L.init_params(0), (np.zeros(47), np.ones(47), np.ones(41)))
    with pytest.raises(stgv.LbmError) as ei:
        sim.set_mlp(packed)
    assert ei.value.status == stgv.LBM_EINVAL
    coarse = torch.empty((46, 64, 64, 64), dtype=torch.float32, device=DEV)
    x = torch.empty((64 ** 3, 47), dtype=torch.float32, device=DEV)
    y = torch.empty((64 ** 3, 41), dtype=torch.float32, device=DEV)
    with pytest.raises(stgv.LbmError):
        stgv.lbm_training_pairs(sim.ctx, coarse, coarse, coarse, x, y)


@pytest.mark.parametrize("n,storage", [(320, "fp32"), (96, "fp32"), (64, "fp16")])
def test_learned_form_rejects_unsupported_boxes(n, storage):
    # the fused learned step addresses a lattice of at most 256^3 nodes with 32-bit byte
    # offsets, runs 128-node blocks (n % 64 == 0) and reads FP32 populations
    sim = stgv.Simulation(**dict(_learned_kw(), n=n, storage=storage))
    packed = packed_net(L.init_params(0), (np.zeros(47), np.ones(47), np.ones(41)))
    with pytest.raises(stgv.LbmError) as ei:
        sim.set_mlp(packed)
    assert ei.value.status == stgv.LBM_EINVAL
    assert "n <= 256" in str(ei.value)
    sim.close()
