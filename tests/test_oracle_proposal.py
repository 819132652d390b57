"""Pins of the proposal oracle (tiles, CNN forward/backward, Adam) on the CPU."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import proposal as P


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def test_conv_matches_direct_loops():
    rng = _rng(1)
    x = rng.standard_normal((2, 3, 11))
    w = rng.standard_normal((4, 3, P.KERNEL))
    for stride in (1, 2):
        out = P.conv(x, w, stride)
        lout = (11 + stride - 1) // stride
        ref = np.zeros((2, 4, lout))
        for b in range(2):
            for o in range(4):
                for t in range(lout):
                    for i in range(3):
                        for k in range(P.KERNEL):
                            j = stride * t + k - P.PAD
                            if 0 <= j < 11:
                                ref[b, o, t] += w[o, i, k] * x[b, i, j]
        np.testing.assert_allclose(out, ref, atol=1e-12)


def test_gradients_match_central_differences():
    rng = _rng(2)
    params = P.init_params(3)
    x = rng.standard_normal((3, 3, 24))
    labels = np.array([1.0, 0.0, 1.0])

    def loss_of(pr):
        s, _ = P.forward(pr, x)
        return P.loss_and_grad(s, labels)[0]

    s, cache = P.forward(params, x)
    _, ds = P.loss_and_grad(s, labels)
    grads = P.backward(params, cache, ds)
    h = 1e-6
    for name in ["W1", "b1", "W2", "W3", "W4", "b4", "w5", "b5"]:
        flat = params[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = loss_of(params)
            flat[idx] = old - h
            lm = loss_of(params)
            flat[idx] = old
            num = (lp - lm) / (2 * h)
            ana = grads[name].reshape(-1)[idx]
            assert abs(num - ana) <= 1e-7 + 1e-5 * abs(num), (name, idx, num, ana)


def test_backward_with_given_decisions():
    """backward(..., decisions=...): with the ReLU gates and the pooling's argmax held
    fixed the score is a polynomial in the parameters, the gated network
    h_l = gate_l * (W_l * h_{l-1} + b_l), score = w5 . h4[arg] + b5, written out
    here; the gradients given another network's decisions match its central
    differences, and given this network's own decisions agree with the plain backward
    (to the last bits: the same values, in another memory order)."""
    rng = _rng(21)
    params = P.init_params(22)
    for l in range(1, 5):
        params["b%d" % l] = rng.standard_normal(P.WIDTH) * 0.2
    x = rng.standard_normal((3, 3, 32))
    ds = rng.standard_normal(3)
    s, cache = P.forward(params, x)
    own = {"gates": [a > 0 for a in cache["acts"][1:]], "arg": cache["arg"]}
    g0, g1 = P.backward(params, cache, ds), P.backward(params, cache, ds, decisions=own)
    for k in g0:
        np.testing.assert_allclose(g1[k], g0[k], rtol=1e-13, atol=0, err_msg=k)
    # decisions of a perturbed network: some gates and maxima differ from this one's
    other = {k: v + 0.3 * rng.standard_normal(v.shape) for k, v in params.items()}
    _, c2 = P.forward(other, x)
    dec = {"gates": [a > 0 for a in c2["acts"][1:]], "arg": c2["arg"]}
    flips = sum(int(np.sum(a != b)) for a, b in zip(own["gates"], dec["gates"])) + int(np.sum(own["arg"] != dec["arg"]))
    assert flips > 0
    grads = P.backward(params, cache, ds, decisions=dec)

    def gated(pr):
        h = x
        for li, st in enumerate(P.STRIDES):
            h = (P.conv(h, pr["W%d" % (li + 1)], st) + pr["b%d" % (li + 1)][None, :, None]) * dec["gates"][li]
        bi, ci = np.meshgrid(np.arange(h.shape[0]), np.arange(h.shape[1]), indexing="ij")
        return float(ds @ (h[bi, ci, dec["arg"]] @ pr["w5"] + pr["b5"][0]))

    h = 1e-5
    for name in ["W1", "b1", "W2", "b2", "W3", "W4", "b4", "w5", "b5"]:
        flat = params[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(5, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            fp = gated(params)
            flat[idx] = old - h
            fm = gated(params)
            flat[idx] = old
            num = (fp - fm) / (2 * h)
            ana = grads[name].reshape(-1)[idx]
            assert abs(num - ana) <= 1e-8 + 1e-6 * abs(num), (name, idx, num, ana)


def test_adam_first_step_moves_by_lr_times_sign():
    params = {"a": np.array([1.0, -2.0, 3.0])}
    grads = {"a": np.array([0.5, -4.0, 1e-3])}
    state = {}
    P.adam_step(params, grads, state, lr=0.01)
    # first step: m_hat = g, v_hat = g^2, update = lr g / (|g| + eps) ~ lr sign(g)
    np.testing.assert_allclose(params["a"], [0.99, -1.99, 2.99], atol=1e-7)


def test_tile_matches_brute_force():
    rng = _rng(4)
    x = synth.noise_complex(rng, (3, 2, 700))
    prefix = P.power_prefix(x)
    shift = np.array([[0, 5, 17], [3, 0, 40], [0, 0, 1]])
    tile = P.tile_from_prefix(prefix, shift, 50, 14)
    p = (np.abs(x) ** 2).sum(axis=1)
    for d in range(3):
        for t in range(14):
            tot, cnt = 0.0, 0
            for c in range(3):
                for n in range(t * 50 + shift[c, d], (t + 1) * 50 + shift[c, d]):
                    if 0 <= n < 700:
                        tot += p[c, n]
                        cnt += 1
            ref = tot * 3 * 50 / cnt if cnt else 0.0
            assert abs(tile[d, t] - ref) < 1e-9 * max(1.0, ref)
    # the fine-bin form equals the per-sample one when shifts are multiples of the fine bin
    fine = 10
    pf = np.concatenate([np.zeros((3, 1)), np.cumsum(p.reshape(3, -1, fine).sum(axis=2), axis=1)], axis=1)
    sh10 = shift // 10 * 10
    np.testing.assert_allclose(P.tile_from_prefix(pf, sh10, 50, 14, fine=fine),
                               P.tile_from_prefix(prefix, sh10, 50, 14), rtol=1e-12)


def test_tile_peaks_at_the_injected_dm():
    """Incoherent dedispersion (Sec. 2.3.1) of a strong noise-free pulse across 16 channels."""
    fc = synth.chan_freqs(1.2e9, 16, 1e6)
    dms = synth.dm_grid(32, 2000.0)
    rng = _rng(5)
    s = 1 << 17
    x = np.zeros((16, 2, s), dtype=np.complex128)
    n0, dm = 20000, 1000.0
    for c in range(16):
        synth.inject_pulse(x[c], fc[c], 1e6, dm, n0, synth.pulse_wave(rng, 100, 50.0, 1.0), f_ref=fc[-1],
                           phases=np.zeros(2))
    _, shift = oracle.channel_delays(fc, dms, 1e6)
    tile = P.tile_from_prefix(P.power_prefix(x), shift, 1024, s // 1024)
    d, t = np.unravel_index(np.argmax(tile), tile.shape)
    assert d == 16 and abs(t - n0 // 1024) <= 10


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2 at every step,
    so t steps move each weight by exactly t lr g / (|g| + eps)."""
    g = np.array([0.5, -4.0, 1e-3, 2.0])
    params = {"a": np.array([1.0, -2.0, 3.0, 0.25])}
    state = {}
    lr, eps = 0.01, 1e-8
    for t in range(1, 7):
        P.adam_step(params, {"a": g.copy()}, state, lr=lr, eps=eps)
        expect = np.array([1.0, -2.0, 3.0, 0.25]) - t * lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(params["a"], expect, rtol=0, atol=1e-12)


def test_adam_matches_library_over_several_steps():
    """Six steps with changing gradients from a nonzero start against torch.optim.Adam
    (an independent implementation of the same Kingma & Ba recurrence)."""
    import torch
    rng = _rng(46)
    w0 = rng.standard_normal(7)
    grads = [rng.standard_normal(7) * (k + 1) for k in range(6)]
    params = {"w": w0.copy()}
    state = {}
    tw = torch.tensor(w0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tw], lr=0.05, betas=(0.8, 0.95), eps=1e-6)
    for g in grads:
        P.adam_step(params, {"w": g}, state, lr=0.05, beta1=0.8, beta2=0.95, eps=1e-6)
        tw.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        np.testing.assert_allclose(params["w"], tw.detach().numpy(), rtol=0, atol=1e-13)


def test_standardise_and_row_triples_brute_force():
    """standardise: zero mean, unit (population) deviation over the whole tile, checked
    on a hand example; rows3: row d's input is rows d-1, d, d+1 with the edge rows
    repeated, checked element by element."""
    t = np.array([[1.0, 3.0], [5.0, 7.0]])      # mean 4, population sd sqrt(5)
    np.testing.assert_allclose(P.standardise(t), (t - 4.0) / math.sqrt(5.0), rtol=0, atol=1e-15)
    z = np.arange(12.0).reshape(4, 3)
    r = P.rows3(z)
    for d in range(4):
        for j, dd in enumerate((max(d - 1, 0), d, min(d + 1, 3))):
            assert np.array_equal(r[d, j], z[dd])


def test_pack_upper_brute_force():
    import oracle
    m = 5
    v = np.arange(m * m).reshape(m, m) + 1j
    got = oracle.pack_upper(v)
    want = [v[i, j] for i in range(m) for j in range(i, m)]
    assert np.array_equal(got, want)
    assert all(oracle.packed_index(i, j, m) == k for k, (i, j) in
               enumerate((i, j) for i in range(m) for j in range(i, m)))
