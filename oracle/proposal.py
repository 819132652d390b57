"""FP64 oracle of the learned DM proposal: DM-time power tiles and the 1-D CNN.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Tiles are the paper's incoherent dedispersion (Sec. 2.3.1: detect, integrate,
delay each channel by the trial DM's delay, sum over channels) of power beams
(Sec. 2.4.1: detected power summed over antennas).  The network that ranks DM
trials from a tile is this project's (the paper has none); its definition here
is the reference for the GPU kernels' forward and backward passes.

Tile (per trial d, time bin t of B samples; channel delays shift[c, d] samples
behind the highest channel, from Eq. dmdelay):
    T[d, t] = C B * sum_c sum_{n in W(c,d,t)} p_c[n] / #W,
    W(c, d, t) = [t B + shift[c, d], (t + 1) B + shift[c, d]) within the stream,
    p_c[n] = sum_p |x_{c,p}[n]|^2,
i.e. the mean power over the samples that exist, scaled to a full bin.  With
fine-resolution power P_c[u] = sum of p_c over samples [u F, (u+1) F) the same
definition is applied with shifts rounded to whole fine bins (rint(shift / F)).

Network (per DM row d; input channels = tile rows d-1, d, d+1 after the tile is
standardised, edge rows repeated):
    h1 = relu(conv(x, W1, stride 1) + b1)     3 -> 32 channels, kernel 9, pad 4
    h2 = relu(conv(h1, W2, stride 2) + b2)    32 -> 32
    h3 = relu(conv(h2, W3, stride 2) + b3)    32 -> 32
    h4 = relu(conv(h3, W4, stride 2) + b4)    32 -> 32
    g  = max over time of h4                  32
    s  = w5 . g + b5                          score (logit)
conv(x, W, stride)[o, t] = sum_{i, k} W[o, i, k] x[i, stride t + k - 4] (zero outside).
Loss: mean over rows of the logistic loss softplus(s) - y s.
"""

import numpy as np

KERNEL = 9
PAD = 4
WIDTH = 32
STRIDES = (1, 2, 2, 2)


def power_prefix(volts):
    """p_c[n] = sum over antennas of |x|^2 and its prefix sums, for [C, M, S] complex
    or [C, M, 2S] interleaved int8 voltages.  Returns S_c with S_c[0] = 0."""
    v = np.asarray(volts)
    if v.dtype == np.int8:
        re = v[..., 0::2].astype(np.float64)
        im = v[..., 1::2].astype(np.float64)
        p = (re * re + im * im).sum(axis=1)
    else:
        p = (np.abs(v.astype(np.complex128)) ** 2).sum(axis=1)
    return np.concatenate([np.zeros((p.shape[0], 1)), np.cumsum(p, axis=1)], axis=1)


def tile_from_prefix(prefix, shift, bin_len, n_bins, fine=1):
    """T[d, t] from per-channel prefix sums of power at resolution `fine` samples.

    prefix: [C, U + 1] prefix sums over U fine bins; shift: [C, D] samples.
    Shifts are rounded to whole fine bins; bin_len must be a multiple of fine."""
    prefix = np.asarray(prefix, dtype=np.float64)
    n_chan, u1 = prefix.shape
    units = u1 - 1
    b = bin_len // fine
    sh = np.rint(np.asarray(shift, dtype=np.float64) / fine).astype(np.int64)  # [C, D]
    d_count = sh.shape[1]
    t = np.arange(n_bins)
    tile = np.zeros((d_count, n_bins))
    count = np.zeros((d_count, n_bins))
    for c in range(n_chan):
        a0 = np.clip(t[None, :] * b + sh[c][:, None], 0, units)
        a1 = np.clip(t[None, :] * b + b + sh[c][:, None], 0, units)
        tile += prefix[c][a1] - prefix[c][a0]
        count += a1 - a0
    return np.where(count > 0, tile * (n_chan * b) / np.maximum(count, 1), 0.0)


def standardise(tile):
    """(T - mean) / std over the whole tile."""
    m = tile.mean()
    s = tile.std()
    return (tile - m) / (s if s > 0 else 1.0)


def rows3(z):
    """Network input for every DM row: rows d-1, d, d+1 (edges repeated) -> [D, 3, T]."""
    up = np.concatenate([z[:1], z[:-1]], axis=0)
    dn = np.concatenate([z[1:], z[-1:]], axis=0)
    return np.stack([up, z, dn], axis=1)


def init_params(seed=0):
    """He-style initial weights (the GPU network can be given these exactly)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = {}
    cin = 3
    for li in range(4):
        fan = cin * KERNEL
        params["W%d" % (li + 1)] = rng.standard_normal((WIDTH, cin, KERNEL)) * np.sqrt(2.0 / fan)
        params["b%d" % (li + 1)] = np.zeros(WIDTH)
        cin = WIDTH
    params["w5"] = rng.standard_normal(WIDTH) * np.sqrt(1.0 / WIDTH)
    params["b5"] = np.zeros(1)
    return params


def conv(x, w, stride):
    """x [B, I, L] -> [B, O, L_out], L_out = ceil(L / stride), zero padding PAD."""
    bsz, cin, length = x.shape
    lout = (length + stride - 1) // stride
    xp = np.zeros((bsz, cin, length + 2 * PAD + stride))
    xp[:, :, PAD:PAD + length] = x
    # gather windows: [B, I, L_out, K]
    idx = stride * np.arange(lout)[:, None] + np.arange(KERNEL)[None, :]
    win = xp[:, :, idx]
    return np.einsum("oik,bitk->bot", w, win)


def conv_backward(x, w, stride, gout):
    """Gradients of conv wrt x and w, by the transposed gather."""
    bsz, cin, length = x.shape
    lout = gout.shape[-1]
    xp = np.zeros((bsz, cin, length + 2 * PAD + stride))
    xp[:, :, PAD:PAD + length] = x
    idx = stride * np.arange(lout)[:, None] + np.arange(KERNEL)[None, :]
    win = xp[:, :, idx]
    gw = np.einsum("bot,bitk->oik", gout, win)
    gwin = np.einsum("oik,bot->bitk", w, gout)
    gxp = np.zeros_like(xp)
    for k in range(KERNEL):
        np.add.at(gxp, (slice(None), slice(None), idx[:, k]), gwin[..., k])
    return gxp[:, :, PAD:PAD + length], gw


def forward(params, x):
    """x [B, 3, L] -> scores [B], plus the activations the backward pass needs."""
    acts = [x]
    h = x
    for li, s in enumerate(STRIDES):
        h = np.maximum(conv(h, params["W%d" % (li + 1)], s) + params["b%d" % (li + 1)][None, :, None], 0.0)
        acts.append(h)
    g = h.max(axis=2)
    arg = h.argmax(axis=2)
    score = g @ params["w5"] + params["b5"][0]
    return score, {"acts": acts, "g": g, "arg": arg}


def loss_and_grad(score, labels):
    """Mean logistic loss and its gradient wrt the scores."""
    s = np.asarray(score, dtype=np.float64)
    y = np.asarray(labels, dtype=np.float64)
    loss = np.mean(np.logaddexp(0.0, s) - y * s)
    dscore = (1.0 / (1.0 + np.exp(-s)) - y) / s.shape[0]
    return loss, dscore


def backward(params, cache, dscore, decisions=None):
    """Analytic gradients of the score-weighted sum sum_b dscore[b] score[b].

    decisions: optional {"gates": [4 boolean arrays shaped like the layers'
    activations], "arg": [B, 32] time indices}: the ReLU gates (which units
    passed) and the pooling's argmax to take in place of the ones this forward
    pass took.  Both are discrete decisions made in floating point; a network
    evaluated in another precision can take a few of them the other way.  With
    them held fixed the score is the gated network h_l = gate_l (W_l * h_{l-1} +
    b_l), score = w5 . h4[arg] + b5, whose activations are recomputed here from
    the cache's input and whose gradients are returned."""
    grads = {}
    acts = cache["acts"]
    if decisions is None:
        g, arg = cache["g"], cache["arg"]
        gates = [a > 0 for a in acts[1:]]
    else:
        arg = np.asarray(decisions["arg"])
        gates = [np.asarray(m, dtype=bool) for m in decisions["gates"]]
        acts = [acts[0]]
        for li, s in enumerate(STRIDES):
            acts.append((conv(acts[-1], params["W%d" % (li + 1)], s) + params["b%d" % (li + 1)][None, :, None])
                        * gates[li])
    h4 = acts[-1]
    bi, ci = np.meshgrid(np.arange(h4.shape[0]), np.arange(h4.shape[1]), indexing="ij")
    if decisions is not None:
        g = h4[bi, ci, arg]
    grads["w5"] = g.T @ dscore
    grads["b5"] = np.array([dscore.sum()])
    gg = dscore[:, None] * params["w5"][None, :]
    gh = np.zeros_like(h4)
    gh[bi, ci, arg] = gg
    for li in range(3, -1, -1):
        gpre = gh * gates[li]
        grads["b%d" % (li + 1)] = gpre.sum(axis=(0, 2))
        gx, gw = conv_backward(acts[li], params["W%d" % (li + 1)], STRIDES[li], gpre)
        grads["W%d" % (li + 1)] = gw
        gh = gx
    return grads


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = beta1 * m + (1 - beta1) * grads[k]
        v[...] = beta2 * v + (1 - beta2) * grads[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params
