"""The trained surrogate of p_w: accuracy on held-out queries, images against the FP64 oracle
(relative L2 <= 1e-2, the tolerance stated for the learned path), and its cost against the
closed form it replaces."""

import numpy as np
import pytest

import oracle
from workloads import scenes as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    import torch
    assert torch.cuda.is_available()
    from paper_2303_15762_amd import Renderer
    from paper_2303_15762_amd.surrogate import Surrogate
    R = Renderer(0)
    S = Surrogate(R)
    p, hist = S.train()
    print("training history", hist)
    S.install(p)
    yield R, S, p, hist, torch
    R.close()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_training_converges(trained):
    R, S, p, hist, torch = trained
    assert hist["val_loss"][-1] < 2e-3
    assert hist["val_loss"][-1] < 0.01 * hist["val_loss"][0]


def test_surrogate_pw_on_held_out_queries(trained):
    R, S, p, hist, torch = trained
    _, _, q = S.samples(200000, seed=77, with_queries=True)
    got = R.bsdf_eval(q, mode=1).cpu().numpy().astype(np.float64)
    ref = oracle.pw_batch(q.cpu().numpy().astype(np.float64))
    qn = q.cpu().numpy().astype(np.float64)
    k = qn[:, 4]
    ci = np.sqrt(1 - (qn[:, 5] ** 2 + qn[:, 6] ** 2) / k ** 2)
    co = np.sqrt(1 - (qn[:, 7] ** 2 + qn[:, 8] ** 2) / k ** 2)
    g = (k * (ci + co) * qn[:, 1]) ** 2
    peak = qn[:, 2] ** 2 / (4 * np.pi * g)
    big = ref > 1e-2 * peak
    rel = np.abs(got[big] - ref[big]) / ref[big]
    print("surrogate p_w: median rel err", np.median(rel), "p90", np.quantile(rel, 0.9),
          "p99", np.quantile(rel, 0.99), "abs err / peak max", (np.abs(got - ref) / peak).max())
    assert np.median(rel) < 1e-2
    assert np.quantile(rel, 0.9) < 3e-2
    assert (np.abs(got - ref) / peak).max() < 5e-2


def test_surrogate_trace_matches_oracle(trained):
    R, S, p, hist, torch = trained
    wl = W.mid_terrain(width=41, height=29, spp=16, n_lambda=8)
    R.load_workload(wl)
    img, st = R.render_workload(wl, bsdf_mode=1)
    o, _ = oracle.render(wl)
    e = rel_l2(img.cpu().numpy(), o)
    print("surrogate trace: rel L2", e, st)
    assert st["surrogate_evals"] > 0
    assert e <= 1e-2


def test_surrogate_cost_against_closed_form(trained):
    """What the network buys: p_w of rough-surface queries inside its domain (g in [16, 400]),
    closed form (a Poisson series of ~12 sqrt(g) Gaussians, one exponential each) against one
    matrix-core pass per 64 queries.  Measured: the bfloat16 network is 1.15-1.25x faster per
    query (it is bound by the two transcendental instructions of each of its 256 GELUs per
    query); the FP8 network with its two-term activations is slower than the closed form.  On
    a frame the closed form of those queries is under 1 % of the time (the bench reports the
    bound), so the frame cannot gain more than that."""
    R, S, p, hist, torch = trained
    _, _, q = S.samples(1 << 22, seed=78, with_queries=True)
    t = {}
    for mode in (0, 1, 2):
        R.bsdf_eval(q, mode=mode)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(R.stream)
        for _ in range(5):
            R.bsdf_eval(q, mode=mode)
        e1.record(R.stream)
        torch.cuda.synchronize()
        t[mode] = e0.elapsed_time(e1) / 5
    print(f"p_w of {q.shape[0]} in-domain rough queries: closed form {t[0]:.3f} ms, BF16 network "
          f"{t[1]:.3f} ms ({t[0] / t[1]:.2f}x), FP8 network {t[2]:.3f} ms ({t[0] / t[2]:.2f}x)")
    assert t[0] / t[1] >= 1.05
    # on a frame: how many measurements the network answered, and the closed form's share
    wl = W.mid_terrain(width=128, height=96, spp=16, n_lambda=8)
    R.load_workload(wl)
    _, st0 = R.render_workload(wl)
    _, st1 = R.render_workload(wl, bsdf_mode=1)
    n_in = st1["surrogate_evals"]
    share = n_in * (t[0] / q.shape[0]) / st0["ms"]
    print(f"mid crop: {n_in} network queries, {st1['fallbacks']} rough queries outside its domain, "
          f"closed form of the network's queries ~{100 * share:.2f} % of the frame's kernel time")
    assert n_in > 0 and share < 0.05


@pytest.mark.parametrize("mode", [1, 2])
def test_surrogate_trace_deterministic(trained, mode):
    """The queued network evaluations land in per-(path, interaction) slots that are added to
    the path records in a fixed order, and no value depends on the queue order (the FP8
    network scales activations per query): renders are bitwise identical, whatever order the
    queries were queued in."""
    R, S, p, hist, torch = trained
    wl = W.mid_terrain(width=64, height=48, spp=8, n_lambda=8)
    R.load_workload(wl)
    a, sa = R.render_workload(wl, bsdf_mode=mode)
    for _ in range(3):
        b, sb = R.render_workload(wl, bsdf_mode=mode)
        assert sa["surrogate_evals"] > 0 and sa["surrogate_evals"] == sb["surrogate_evals"]
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_surrogate_deep_paths_in_bounded_launches(trained):
    """Up to 64 interactions per path: a launch holds at most 52 GiB of queues and result
    slots (84 B per (path, interaction) slot with the learned p_w: a network query, a shadow
    ray and the value), i.e. 10.4M paths here, so the 18.9M-path frame runs in two launches.
    The image equals the sum of two renders over sample ranges that each fit one launch, and
    matches the oracle on sampled pixels."""
    import dataclasses
    R, S, p, hist, torch = trained
    wl = dataclasses.replace(W.mid_terrain(width=512, height=512, spp=9, n_lambda=8), max_depth=64)
    R.load_workload(wl)
    img, st = R.render_workload(wl, bsdf_mode=1)
    assert st["paths"] == 512 * 512 * 9 * 8 and st["nonfinite"] == 0 and st["surrogate_evals"] > 0
    a, _ = R.render_workload(wl, bsdf_mode=1, spp_begin=0, spp_count=5)
    b, _ = R.render_workload(wl, bsdf_mode=1, spp_begin=5, spp_count=4)
    g = img.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose((a + b).cpu().numpy(), g, rtol=1e-5, atol=1e-9 * np.abs(g).max())
    rng = np.random.default_rng(21)
    lit = np.argwhere(g.sum(0) > 0)
    pix_yx = lit[rng.choice(len(lit), size=min(300, len(lit)), replace=False)]
    pix = np.stack([pix_yx[:, 1], pix_yx[:, 0]], 1)
    o, ost = oracle.render(wl, pixels=pix)
    e = rel_l2(g[:, pix_yx[:, 0], pix_yx[:, 1]], o)
    print("deep surrogate paths: rel L2 on", len(pix), "pixels:", e, st)
    assert e <= 1e-2


def test_fp8_surrogate_against_bf16_and_oracle(trained):
    """The same trained network with E4M3 operands: held-out p_w and the terrain image, both
    against the FP64 closed form / oracle, next to the BF16 operands (the precision comparison
    of the learned path)."""
    R, S, p, hist, torch = trained
    _, _, q = S.samples(200000, seed=79, with_queries=True)
    qn = q.cpu().numpy().astype(np.float64)
    ref = oracle.pw_batch(qn)
    k = qn[:, 4]
    ci = np.sqrt(1 - (qn[:, 5] ** 2 + qn[:, 6] ** 2) / k ** 2)
    co = np.sqrt(1 - (qn[:, 7] ** 2 + qn[:, 8] ** 2) / k ** 2)
    g = (k * (ci + co) * qn[:, 1]) ** 2
    peak = qn[:, 2] ** 2 / (4 * np.pi * g)
    big = ref > 1e-2 * peak
    stats = {}
    for mode in (1, 2):
        got = R.bsdf_eval(q, mode=mode).cpu().numpy().astype(np.float64)
        rel = np.abs(got[big] - ref[big]) / ref[big]
        stats[mode] = (np.median(rel), np.quantile(rel, 0.9), (np.abs(got - ref) / peak).max())
        print("p_w mode", mode, "median rel", stats[mode][0], "p90", stats[mode][1], "abs/peak max", stats[mode][2])
    assert stats[2][0] < 5e-2 and stats[2][2] < 0.2
    wl = W.mid_terrain(width=41, height=29, spp=16, n_lambda=8)
    R.load_workload(wl)
    o, _ = oracle.render(wl)
    errs = {}
    for mode in (1, 2):
        img, st = R.render_workload(wl, bsdf_mode=mode)
        errs[mode] = rel_l2(img.cpu().numpy(), o)
        print("image mode", mode, "rel L2", errs[mode], "surrogate evals", st["surrogate_evals"])
        assert st["surrogate_evals"] > 0
    assert errs[2] <= 1e-2


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("view", ["window", "low_resolution"])
def test_surrogate_with_composite_interactions(trained, mode, view):
    """Composite interactions with the learned p_w: measurements at a material boundary keep the
    closed-form composite p_w, the other in-domain rough ones go to the network.  A
    full-resolution window of the mid terrain over tile boundaries, and the whole terrain on a
    41 x 29 sensor (wide footprints: many boundary hits), against the
    FP64 oracle's composite render (surrogate bar 1e-2); the paths are those of the
    closed-form composite render (the network changes measurement values only)."""
    R, S, p, hist, torch = trained
    if view == "window":
        wl = W.as_float32_inputs(W.mid_terrain(window=(230, 230, 48, 40), spp=16))
    else:
        wl = W.as_float32_inputs(W.mid_terrain(width=41, height=29, spp=16, n_lambda=8))
    R.load_workload(wl)
    R.boundaries(2e-3)
    img_c, st_c = R.render_workload(wl, composite=True)
    img_s, st_s = R.render_workload(wl, composite=True, bsdf_mode=mode)
    o, ost = oracle.render(wl, composite=True, reach_m=2e-3)
    e = rel_l2(img_s.cpu().numpy(), o)
    e_c = rel_l2(img_c.cpu().numpy(), o)
    print("composite with learned p_w, mode", mode, ": rel L2", e, "(closed form", e_c, ") surrogate evals",
          st_s["surrogate_evals"], "composite", st_s["composite"], st_c["composite"])
    # (the wide footprints of the low-resolution view put most rough hits within reach of a
    # boundary, so few queries are left for the network there too)
    assert st_s["surrogate_evals"] > (200 if view == "low_resolution" else 50)
    assert st_s["composite"] == st_c["composite"] > 1000
    assert st_s["segments"] == st_c["segments"]
    assert e <= 1e-2
