"""GPU parity of the learned-proposal kernels against the FP64 oracle, and what
the trained network gains over the method without it."""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import run_gpu, say, select
from oracle import proposal as P

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1109_3186_amd", "proposal_weights.npz")


def _plan(cfg, in_dtype="ci8", max_block=1 << 15):
    from paper_1109_3186_amd import Plan
    p = Plan(cfg["volts"].shape[1], cfg["chan_freqs"], cfg["f_s"], cfg["dump_len"], max_block_samples=max_block,
             in_dtype=in_dtype)
    p.set_dm_trials(cfg["dm_lists"][0])
    return p


def test_tile_kernel_matches_oracle(gpu):
    import torch
    cfg = synth.make_small(seed=41, m_ant=3, n_chan=4, s=1 << 14, f_lo=1.2e9, f_s=1e6, n_dm=32, dm_max=500.0,
                           dump_len=100, ci8=True, n_pulses=2)
    with _plan(cfg) as plan:
        tile = plan.power_tile(torch.from_numpy(cfg["volts"]).to(gpu), 256, 64).cpu().numpy()
        lay = plan.layout()
        shift = lay["shift"].reshape(4, 32)
        # fine-bin form: [2, C, U] power at 8-sample resolution
        rng = np.random.Generator(np.random.PCG64(42))
        pw = rng.random((2, 4, 2048)).astype(np.float32) * 100
        tiles = plan.tiles_from_power(torch.from_numpy(pw).to(gpu), 8, 256, 64).cpu().numpy()
    ref = P.tile_from_prefix(P.power_prefix(cfg["volts"]), shift, 256, 64)
    assert np.max(np.abs(tile - ref) / np.abs(ref).max()) <= 1e-6
    for t in range(2):
        pre = np.concatenate([np.zeros((4, 1)), np.cumsum(pw[t].astype(np.float64), axis=1)], axis=1)
        ref2 = P.tile_from_prefix(pre, shift, 256, 64, fine=8)
        assert np.max(np.abs(tiles[t] - ref2) / np.abs(ref2).max()) <= 1e-6


def _flat(params):
    from paper_1109_3186_amd.proposal import flatten
    return flatten(params)


def test_cnn_forward_backward_adam_match_oracle(gpu):
    import torch

    from paper_1109_3186_amd import Cnn
    from paper_1109_3186_amd.proposal import unflatten
    rng = np.random.Generator(np.random.PCG64(43))
    d, L, nt = 16, 128, 2
    tiles = rng.standard_normal((nt, d, L)) * 3 + 10
    tiles[0, 5, 40:44] += 30  # a bump so that some channels have a clear maximum
    params = P.init_params(44)
    params["b1"] = rng.standard_normal(32) * 0.1
    params["b5"] = np.array([0.3])
    labels = (rng.random(nt * d) < 0.3).astype(np.float64)
    net = Cnn(d, L, nt)
    net.set_weights(_flat(params))
    t_dev = torch.from_numpy(tiles.astype(np.float32)).to(gpu)
    scores = net.forward(t_dev).cpu().numpy()
    x = np.concatenate([P.rows3(P.standardise(tiles[i])) for i in range(nt)])
    ref, cache = P.forward(params, x)
    assert np.max(np.abs(scores - ref)) <= 1e-4 * max(1.0, np.abs(ref).max())
    loss_rows = net.loss(torch.from_numpy(labels.astype(np.float32)).to(gpu)).cpu().numpy()
    lref, ds = P.loss_and_grad(ref, labels)
    assert abs(loss_rows.mean() - lref) <= 1e-5 * max(1.0, abs(lref))
    net.backward()
    g = unflatten(net.get_grads())
    gref = P.backward(params, cache, ds)
    for k in gref:
        rel = np.linalg.norm(g[k] - gref[k]) / max(np.linalg.norm(gref[k]), 1e-12)
        say("grad %s rel %.2e" % (k, rel))
        assert rel <= 1e-3, k
    # one Adam step from zero state on the GPU's own gradients
    before = net.get_weights()
    net.adam(lr=1e-3)
    after = net.get_weights()
    gflat = net.get_grads().astype(np.float64)
    expect = before - 1e-3 * gflat / (np.abs(gflat) + 1e-8)
    assert np.max(np.abs(after - expect)) <= 1e-6
    net.close()


@pytest.mark.parametrize("level", [1.0, 2.0 ** -6])
def test_cnn_fp16_forward_backward_match_oracle(gpu, level):
    """FP16 matrix-core form (binary16 operands, FP32 accumulation) against the FP64
    oracle: scores within 1e-2 of the largest |score|, the mean loss within 1e-2, and
    every gradient tensor within 1e-2 (relative, norm) of the analytic backward taken
    through the same ReLU gates and pooling maxima as the kernels' forward pass (a
    unit whose pre-activation is within binary16 rounding of zero can pass on one
    side and not the other, and that decision, not the arithmetic, would then decide
    the difference; the kernels' decisions are read from their activations).  At
    level 2^-6 each layer's W and b are scaled so that its activations are level^l
    times the unscaled ones (W_l by level, b_l by level^l) and w5 by level^-4, so the
    scores are those of the unscaled network while h4 ~ 2^-24 and its gradients sit
    far below binary16's normal range: only the per-tile power-of-two scales keep
    the products exact to binary16 precision there."""
    import torch

    from paper_1109_3186_amd import Cnn
    from paper_1109_3186_amd.proposal import unflatten
    rng = np.random.Generator(np.random.PCG64(43))
    d, L, nt = 16, 128, 2
    tiles = rng.standard_normal((nt, d, L)) * 3 + 10
    tiles[0, 5, 40:44] += 30
    params = P.init_params(44)
    params["b1"] = rng.standard_normal(32) * 0.1
    params["b5"] = np.array([0.3])
    for l in range(1, 5):
        params["W%d" % l] = params["W%d" % l] * level
        params["b%d" % l] = params["b%d" % l] * level ** l
    params["w5"] = params["w5"] * level ** -4
    labels = (rng.random(nt * d) < 0.3).astype(np.float64)
    net = Cnn(d, L, nt, precision="fp16")
    net.set_weights(_flat(params))
    t_dev = torch.from_numpy(tiles.astype(np.float32)).to(gpu)
    scores = net.forward(t_dev).cpu().numpy()
    x = np.concatenate([P.rows3(P.standardise(tiles[i])) for i in range(nt)])
    ref, cache = P.forward(params, x)
    serr = np.max(np.abs(scores - ref)) / max(1.0, np.abs(ref).max())
    loss_rows = net.loss(torch.from_numpy(labels.astype(np.float32)).to(gpu)).cpu().numpy()
    lref, ds = P.loss_and_grad(ref, labels)
    say("FP16 level %g: scores max error %.2e of max |score|, loss %.6f vs %.6f" % (level, serr, loss_rows.mean(), lref))
    assert serr <= 1e-2
    assert abs(loss_rows.mean() - lref) <= 1e-2 * max(1.0, abs(lref))
    net.backward()
    g = unflatten(net.get_grads())
    acts = [net.get_activations(l, nt * d).astype(np.float64) for l in range(1, 5)]
    dec = {"gates": [a > 0 for a in acts], "arg": np.argmax(acts[3], axis=2)}
    flips = sum(int(np.sum(a != (b > 0))) for a, b in zip(dec["gates"], cache["acts"][1:]))
    say("FP16 level %g: %d ReLU gates and %d maxima taken the other way than in FP64" %
        (level, flips, int(np.sum(dec["arg"] != cache["arg"]))))
    gref = P.backward(params, cache, ds, decisions=dec)
    gown = P.backward(params, cache, ds)
    worst = 0.0
    for k in gref:
        rel = np.linalg.norm(g[k] - gref[k]) / max(np.linalg.norm(gref[k]), 1e-300)
        own = np.linalg.norm(g[k] - gown[k]) / max(np.linalg.norm(gown[k]), 1e-300)
        worst = max(worst, rel)
        say("FP16 level %g grad %s rel %.2e (oracle's own decisions %.2e; |g| %.2e)" %
            (level, k, rel, own, np.linalg.norm(gref[k])))
        assert rel <= 1e-2, k
    assert worst > 1e-7  # binary16 operands: not the FP32 form by mistake
    net.close()


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
@pytest.mark.parametrize("d, L", [(5, 192), (3, 64)])
def test_cnn_ragged_shape_matches_oracle(gpu, precision, d, L):
    """192 bins (layers of 192, 96, 48, 24 steps: every layer ends in a partial
    64-step tile, and the last is shorter than one) with 5 DM rows, and the smallest
    shape, 64 bins (64, 32, 16, 8 steps) with 3 rows (edge rows repeated on both
    sides of every tile); 3 tiles of different levels: scores, and the gradients
    through the kernels' own gates and maxima, against the FP64 oracle."""
    import torch

    from paper_1109_3186_amd import Cnn
    from paper_1109_3186_amd.proposal import unflatten
    rng = np.random.Generator(np.random.PCG64(50 + L))
    nt = 3
    tiles = rng.standard_normal((nt, d, L)) * np.array([1.0, 30.0, 0.01])[:, None, None] + 7
    tiles[1, 0, L - 12:L - 2] += 200.0  # a bump near the end of an edge row
    params = P.init_params(51)
    for l in range(1, 5):
        params["b%d" % l] = rng.standard_normal(32) * 0.05
    labels = (rng.random(nt * d) < 0.4).astype(np.float64)
    net = Cnn(d, L, nt, precision=precision)
    net.set_weights(_flat(params))
    scores = net.forward(torch.from_numpy(tiles.astype(np.float32)).to(gpu)).cpu().numpy()
    x = np.concatenate([P.rows3(P.standardise(tiles[i])) for i in range(nt)])
    ref, cache = P.forward(params, x)
    tol = 1e-4 if precision == "fp32" else 1e-2
    serr = np.max(np.abs(scores - ref)) / max(1.0, np.abs(ref).max())
    net.loss(torch.from_numpy(labels.astype(np.float32)).to(gpu))
    net.backward()
    g = unflatten(net.get_grads())
    acts = [net.get_activations(l, nt * d).astype(np.float64) for l in range(1, 5)]
    assert [a.shape[-1] for a in acts] == [L, L // 2, L // 4, L // 8]
    dec = {"gates": [a > 0 for a in acts], "arg": np.argmax(acts[3], axis=2)}
    _, ds = P.loss_and_grad(ref, labels)
    gref = P.backward(params, cache, ds, decisions=dec)
    worst = max(np.linalg.norm(g[k] - gref[k]) / max(np.linalg.norm(gref[k]), 1e-300) for k in gref)
    say("%s %d x %d: scores %.2e, worst gradient %.2e" % (precision, d, L, serr, worst))
    assert serr <= tol
    assert worst <= (1e-3 if precision == "fp32" else 1e-2)
    net.close()


def test_cnn_precision_switch(gpu):
    """Changing the precision discards the last forward pass; both forms score the
    same tiles alike (within binary16 rounding), and an unknown value is refused."""
    import torch

    from paper_1109_3186_amd import Cnn
    from paper_1109_3186_amd.binding import DdxError
    rng = np.random.Generator(np.random.PCG64(46))
    d, L = 32, 256
    tiles = torch.from_numpy((rng.standard_normal((1, d, L)) * 2 + 5).astype(np.float32)).to(gpu)
    net = Cnn(d, L, 1)
    net.set_weights(_flat(P.init_params(46)))
    s32 = net.forward(tiles).cpu().numpy()
    net.set_precision("fp16")
    with pytest.raises(DdxError):
        net.loss(torch.zeros(d, device=gpu))
    s16 = net.forward(tiles).cpu().numpy()
    err = np.max(np.abs(s16 - s32)) / max(1.0, np.abs(s32).max())
    say("FP16 vs FP32 scores: max %.2e of max |score|" % err)
    assert 0 < err <= 1e-2
    with pytest.raises(ValueError):
        net.set_precision("bf16")
    from paper_1109_3186_amd.binding import lib
    assert lib().ddx_cnn_set_precision(net._h, 7) != 0
    net.close()


def test_cnn_adam_several_steps_match_oracle(gpu):
    """Adam past its first step: (1) with the gradients held fixed, k steps move every
    weight by exactly k lr g / (|g| + eps) (the bias-corrected moments are g and g^2 at
    every step); (2) four steps of forward, backward and Adam from the same start on
    the GPU and in the oracle, each side with its own gradients, stay together."""
    import torch

    from paper_1109_3186_amd import Cnn
    from paper_1109_3186_amd.proposal import unflatten
    rng = np.random.Generator(np.random.PCG64(47))
    d, L, nt = 16, 128, 2
    tiles = rng.standard_normal((nt, d, L)) * 3 + 10
    tiles[1, 9, 70:75] += 25
    params = P.init_params(48)
    labels = (rng.random(nt * d) < 0.3).astype(np.float64)
    t_dev = torch.from_numpy(tiles.astype(np.float32)).to(gpu)
    lab_dev = torch.from_numpy(labels.astype(np.float32)).to(gpu)
    # (1) fixed gradients
    net = Cnn(d, L, nt)
    net.set_weights(_flat(params))
    net.forward(t_dev)
    net.loss(lab_dev)
    net.backward()
    w0 = net.get_weights().astype(np.float64)
    g = net.get_grads().astype(np.float64)
    lr, eps = 1e-3, 1e-8
    for k in range(1, 5):
        net.adam(lr=lr, eps=eps)
        expect = w0 - k * lr * g / (np.abs(g) + eps)
        err = np.max(np.abs(net.get_weights() - expect))
        say("fixed-gradient Adam step %d: max |w - closed form| %.2e" % (k, err))
        assert err <= 2e-6
    net.close()
    # (2) trajectories; eps large enough that gradient rounding moves a step by < lr 1e-2
    lr, eps = 1e-3, 1e-2
    net = Cnn(d, L, nt)
    net.set_weights(_flat(params))
    x = np.concatenate([P.rows3(P.standardise(tiles[i])) for i in range(nt)])
    ref = {k: v.copy() for k, v in params.items()}
    state = {}
    for step in range(4):
        net.forward(t_dev)
        net.loss(lab_dev)
        net.backward()
        net.adam(lr=lr, eps=eps)
        score, cache = P.forward(ref, x)
        _, ds = P.loss_and_grad(score, labels)
        P.adam_step(ref, P.backward(ref, cache, ds), state, lr=lr, eps=eps)
        got = unflatten(net.get_weights())
        err = max(float(np.max(np.abs(got[k] - ref[k]))) for k in ref)
        say("Adam trajectory step %d: max |w_gpu - w_oracle| %.2e" % (step + 1, err))
        assert err <= 1e-4
    net.close()


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_overfit_32_tiles(gpu, precision):
    """Training on 32 fixed tiles (one pulse each, S/N 30-40) drives the mean loss
    to near zero and ranks every tile's labelled rows first."""
    import torch

    from paper_1109_3186_amd import Cnn
    from paper_1109_3186_amd.train_proposal import he_init, make_plan
    p = synth.c1_params()
    plan = make_plan(p)
    rng = np.random.Generator(np.random.PCG64(45))
    gen = torch.Generator(device=gpu)
    gen.manual_seed(45)
    nt = 32
    power, labels, pulses = synth.power_batch(p, nt, 32, rng, gen, gpu, pulse_frac=1.0, snr_range=(30.0, 40.0),
                                              max_pulses=1)
    tiles = plan.tiles_from_power(power, 32, 1024, 1024)
    del power
    net = Cnn(p["n_dm"], 1024, nt, precision=precision)
    net.set_weights(he_init(1))
    first = None
    for it in range(400):
        scores = net.forward(tiles)
        loss = float(net.loss(labels.reshape(-1)).mean())
        first = loss if first is None else first
        net.backward()
        net.adam(lr=3e-3)
    scores = net.forward(tiles)
    loss = float(net.loss(labels.reshape(-1)).mean())
    say("%s overfit on %d tiles: loss %.4f -> %.5f" % (precision, nt, first, loss))
    assert loss <= 0.01 * first
    s = scores.cpu().numpy().reshape(nt, -1)
    y = labels.cpu().numpy().reshape(nt, -1)
    for t in range(nt):
        top = set(np.argsort(-s[t])[:int(y[t].sum())])
        assert top == set(np.nonzero(y[t])[0]), t
    net.close()
    plan.close()


def _recall(scores, pulses, k, dstep):
    hit = tot = 0
    for t, pl in enumerate(pulses):
        top = set(np.argsort(-scores[t], kind="stable")[:k].tolist())
        for q in pl:
            d0 = q["dm"] / dstep
            tot += 1
            hit += int(math.floor(d0) in top or math.ceil(d0) in top)
    return hit / max(tot, 1), tot


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights (run python -m paper_1109_3186_amd.train_proposal)")
@pytest.mark.parametrize("snr", [(5.0, 50.0), (5.0, 10.0)])
def test_trained_network_recall_and_gain(gpu, snr):
    """Recall at the top 10% of DM rows on held-out tiles: the trained network against
    the untrained one and against the method without a network (rank rows by their
    maximum standardised tile value), over the training S/N range and at S/N 5-10,
    where the row maximum is weakest."""
    import torch

    from paper_1109_3186_amd import Cnn
    from paper_1109_3186_amd.proposal import load_weights
    from paper_1109_3186_amd.train_proposal import he_init, make_plan
    p = synth.c1_params()
    plan = make_plan(p)
    rng = np.random.Generator(np.random.PCG64(9001 if snr[1] > 10 else 9002))
    gen = torch.Generator(device=gpu)
    gen.manual_seed(9001 if snr[1] > 10 else 9002)
    nets = {"trained": load_weights(WEIGHTS), "trained_fp16": load_weights(WEIGHTS), "untrained": he_init(1114)}
    k = int(math.ceil(0.1 * p["n_dm"]))
    res = {n: [] for n in list(nets) + ["rowmax"]}
    allpulses = []
    cnns = {}
    for name, w in nets.items():
        cnns[name] = Cnn(p["n_dm"], 1024, 8, precision="fp16" if name.endswith("fp16") else "fp32")
        cnns[name].set_weights(w)
    for b in range(50):
        power, labels, pulses = synth.power_batch(p, 8, 32, rng, gen, gpu, pulse_frac=1.0, max_pulses=1,
                                                  snr_range=snr)
        tiles = plan.tiles_from_power(power, 32, 1024, 1024)
        for name, net in cnns.items():
            res[name].append(net.forward(tiles).cpu().numpy().reshape(8, -1))
        tn = tiles.cpu().numpy()
        res["rowmax"].append(np.stack([P.standardise(tn[i]).max(axis=1) for i in range(8)]))
        allpulses += pulses
    out = {}
    for name in res:
        sc = np.concatenate(res[name])
        out[name] = _recall(sc, allpulses, k, p["dm_max"] / p["n_dm"])
    say("S/N %s: recall at top %d of %d rows over %d pulses: %s" % (snr, k, p["n_dm"], out["trained"][1],
                                                                    {n: round(v[0], 4) for n, v in out.items()}))
    for name in ("trained", "trained_fp16"):
        if snr[1] > 10:
            assert out[name][0] >= 0.99
            assert out[name][0] >= out["untrained"][0] + 0.2
        assert out[name][0] >= out["rowmax"][0]
    for n in cnns.values():
        n.close()
    plan.close()


def test_device_topk_selection(gpu):
    """ddx_select_active_dms: the k best logits (ties to the lower DM, NaN last) become
    the plan's active DMs, as a stable descending sort of the same FP32 values gives;
    more than k logits above the threshold switch every DM on (fallback)."""
    import torch

    from paper_1109_3186_amd import Plan
    fc = synth.chan_freqs(1.2e9, 2, 1e6)
    rng = np.random.Generator(np.random.PCG64(49))
    n = 256
    with Plan(2, fc, 1e6, 1000, max_block_samples=1 << 15, compact_records=True, max_record_pairs=2 * n) as p:
        p.set_dm_trials(synth.dm_grid(n, 2000.0))
        for trial in range(3):
            s = rng.standard_normal(n).astype(np.float32) - 3.0
            s[rng.integers(0, n, 20)] = np.float32(-1.25)      # ties
            s[rng.integers(0, n, 3)] = np.nan
            k = int(rng.integers(1, 40))
            mask, fb = p.select_active_dms(torch.from_numpy(s).to(gpu), k, logit_threshold=0.0)
            key = np.where(np.isnan(s), -np.inf, s)
            ref = np.zeros(n, np.uint8)
            ref[np.argsort(-key, kind="stable")[:k]] = 1
            assert not fb and np.array_equal(mask.cpu().numpy(), ref), trial
            lay = p.layout()
            for c in range(2):
                active = lay["record_pos"][lay["dm_offset"][c]:lay["dm_offset"][c + 1]] >= 0
                assert np.array_equal(active, ref.astype(bool))
        s = np.full(n, -5.0, np.float32)
        s[:30] = 1.0                                            # 30 above the threshold
        mask, fb = p.select_active_dms(torch.from_numpy(s).to(gpu), 26, logit_threshold=0.0)
        assert fb and mask.cpu().numpy().all()
        mask, fb = p.select_active_dms(torch.from_numpy(s).to(gpu), 30, logit_threshold=0.0)
        assert not fb and mask.cpu().numpy().sum() == 30
