"""Free streaming (lbm_stream) against the oracle's streaming, bit for bit.

lbm_stream runs the step's own loads, stores, launch shapes and block order with the
identity in place of the collision, so after k calls every population deviation has
moved k links along its velocity: df_i(x) = df_i(x - k e_i) of the loaded state.  Values
only move, so the comparison is exact in every storage type; the loaded state is first
rounded to the storage type on the oracle side (the load rounds it on the GPU).
"""
import numpy as np
import pytest

from inputs import index_pattern, index_pattern_state, sample_nodes, uniform_deviations
from oracle import lattice as lat, model

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
stgv = pytest.importorskip("paper_2605_14505_amd.stgv")


def make_sim(n, q_f, q_g, storage="fp32", layout="aa"):
    return stgv.Simulation(n=n, q_f=q_f, q_g=q_g, forcing="shift", u0=0.05, re=800.0, fr=1.0, sc=1.0,
                           g_over_n=0.02, storage=storage, layout=layout, diag_every=0)


def oracle_streamed(dev, q_f, q_g, k):
    lf, lg = lat.BY_Q[q_f], lat.BY_Q[q_g]
    f, g = dev[:q_f], dev[q_f:]
    for _ in range(k):
        f, g = model.stream(f, lf), model.stream(g, lg)
    return np.concatenate([f, g])


def check_free_streaming(n, q_f, q_g, storage, layout, seed):
    print(f"\nfree streaming n={n} {q_f}x{q_g} {storage} {layout}", flush=True)
    dev = uniform_deviations(q_f + q_g, n, 1e-2, seed=seed)
    ref0 = model.round_storage(dev.astype(np.float64), storage)
    sim = make_sim(n, q_f, q_g, storage, layout)
    sim.load(torch.from_numpy(dev), step=0)
    done = 0
    for k in (1, 2, 3):
        sim.free_stream(k - done)
        done = k
        got = sim.populations().cpu().numpy().astype(np.float64)
        ref = oracle_streamed(ref0, q_f, q_g, k)
        bad = np.argwhere(got != ref)
        assert bad.size == 0, (k, bad[:5].tolist(), int(bad.shape[0]))
        assert sim.step_count == k
    sim.close()


@pytest.mark.parametrize("layout", ["aa", "ab"])
@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_free_streaming_is_the_oracle_stream(storage, layout):
    check_free_streaming(20, 27, 19, storage, layout, seed=11)


@pytest.mark.parametrize("q_f,q_g", [(27, 7), (19, 7), (27, 27), (19, 19), (19, 15), (15, 7), (7, 27)])
def test_free_streaming_other_pairs_ragged(q_f, q_g):
    check_free_streaming(7, q_f, q_g, "fp32", "aa", seed=q_f * 100 + q_g)


@pytest.mark.parametrize("n", [96, 130])
def test_free_streaming_other_launch_shapes(n):
    # n = 96: 32 x 8 node blocks; n = 130: 192-wide blocks with idle lanes at the row end
    check_free_streaming(n, 27, 19, "fp32", "aa", seed=n)


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_free_streaming_row_aligned_odd_step(storage):
    # 2-byte storage at 128^3: blocks of two whole rows, the odd step row-aligned
    check_free_streaming(128, 27, 19, storage, "aa", seed=128)


@pytest.mark.parametrize("n,storage,q_f,q_g", [(320, "fp32", 27, 19), (256, "fp32", 27, 19), (512, "fp32", 27, 19),
                                               (512, "fp16", 27, 19), (512, "bf16", 27, 19),
                                               (256, "fp32", 19, 19), (256, "fp32", 7, 27), (256, "fp16", 27, 7),
                                               (768, "fp16", 27, 19)])
def test_free_streaming_sampled_large(n, storage, q_f, q_g):
    # 320^3: rows split over 5 blocks, XCD-ordered shifted odd step; 256^3: the row-aligned
    # odd step on whole rows; 512^3: the row-aligned odd step whose seam lanes reach across
    # block edges; 768^3: three blocks per row, the middle one with a seam at both edges.
    # Two calls cover an even and an odd step.
    torch.cuda.empty_cache()
    print(f"\nfree streaming sampled n={n} {storage} {q_f}x{q_g}", flush=True)
    sim = make_sim(n, q_f, q_g, storage)
    sim.load(index_pattern_state(q_f + q_g, n, "cuda:0"), step=0)
    e = np.concatenate([lat.BY_Q[q_f].e, lat.BY_Q[q_g].e])          # (q, 3) as (x, y, z)
    pts = sample_nodes(n, 3000, seed=n)
    edges = sorted({v for v in (0, 1, 63, 64, 255, 256, 511, 512, n - 2, n - 1) if 0 <= v < n})
    pts += [(z, y, x) for z in (0, n // 2, n - 1) for y in (0, n - 1) for x in edges]
    zyx = np.array(pts, dtype=np.int64)
    idx = torch.from_numpy(zyx).to("cuda:0")
    q = np.arange(q_f + q_g)
    for k in (1, 2):
        sim.free_stream(1)
        pops = sim.populations()                                      # (q, n, n, n) FP32
        got = pops[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()  # (q, m)
        del pops
        src_z = (zyx[None, :, 0] - k * e[:, None, 2]) % n
        src_y = (zyx[None, :, 1] - k * e[:, None, 1]) % n
        src_x = (zyx[None, :, 2] - k * e[:, None, 0]) % n
        ref = index_pattern(q[:, None], src_z, src_y, src_x)
        assert np.array_equal(got.astype(np.float64), ref), k
    sim.close()
    torch.cuda.empty_cache()


def test_free_streaming_rejects_a_negative_count():
    sim = make_sim(8, 27, 19)
    with pytest.raises(stgv.LbmError):
        sim.free_stream(-1)
    sim.free_stream(0)
    assert sim.step_count == 0
    sim.close()
