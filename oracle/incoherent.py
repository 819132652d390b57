"""FP64 oracle of classical incoherent dedispersion of power beams.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

What it computes (Bannister & Cornwell 2011, Sec. 2.3.1 and 2.4.1):

* a power beam: the detected power |x|^2 of every antenna summed over antennas
  and integrated over a sampling interval (Sec. 2.4.1);
* brute-force incoherent dedispersion: for every trial DM, each channel of the
  power spectrogram delayed by its dispersion delay (Eq. dmdelay, relative to
  the highest channel, rounded to whole samples) and the channels summed
  (Sec. 2.3.1);
* the tree method the paper cites (Sec. 2.3.1, after Taylor 1974), which assumes
  linear dispersion: for n = 2^k channels it forms, in k merging stages, every
  sweep j = 0 .. n - 1 whose delay grows from 0 at the first channel to j at the
  last.  Merging two adjacent groups of n/2 channels into a group of n, sweep j
  adds sweep floor(j/2) of the first group to sweep floor(j/2) of the second
  group advanced by j - floor(j/2) samples, so the delay of channel c in sweep j
  is D_n(j, c) = D_{n/2}(floor(j/2), c) for c < n/2 and j - floor(j/2) +
  D_{n/2}(floor(j/2), c - n/2) otherwise, with D_1 = 0.

Channel 0 is the least delayed (highest frequency) channel; samples past the end
of the spectrogram count as zero.
"""
import numpy as np


def power_beam(volts, n_int):
    """p[c][t] = sum_antennas sum_{n in [t n_int, (t + 1) n_int)} |x_{c,p}[n]|^2 for
    volts [C][M][S] complex; complete intervals only."""
    v = np.asarray(volts, dtype=np.complex128)
    n_t = v.shape[2] // n_int
    p = np.abs(v[:, :, :n_t * n_int]) ** 2
    return p.sum(axis=1).reshape(v.shape[0], n_t, n_int).sum(axis=2)


def dm_delays(freqs_hz, t_samp_s, dms, k_dm=4.148808e15):
    """delay[c][d] = rint(K DM_d (f_c^-2 - f_top^-2) / t_samp) (Eq. dmdelay), f_top the
    highest channel frequency, in whole samples (ties to even)."""
    f = np.asarray(freqs_hz, dtype=np.float64)
    top = f.max()
    dm = np.asarray(dms, dtype=np.float64)
    sec = k_dm * dm[None, :] * (1.0 / (f[:, None] ** 2) - 1.0 / (top * top))
    return np.rint(sec / t_samp_s).astype(np.int64)


def brute_force(power, delays, n_out):
    """out[d][t] = sum_c power[c][t + delays[c][d]], t < n_out (samples before the
    first or past the last count as zero)."""
    p = np.asarray(power, dtype=np.float64)
    dl = np.asarray(delays, dtype=np.int64)
    C, n_t = p.shape
    out = np.zeros((dl.shape[1], n_out))
    for d in range(dl.shape[1]):
        for c in range(C):
            lo = int(dl[c, d])
            t0 = max(0, -lo)                        # outputs before t0 read before sample 0
            s0, s1 = t0 + lo, min(n_t, lo + n_out)  # the samples that exist
            if s1 > s0:
                out[d, t0:t0 + s1 - s0] += p[c, s0:s1]
    return out


def tree_delays(n, j):
    """D_n(j, c) for c = 0 .. n - 1 (the tree's implied per-channel delays)."""
    if n == 1:
        return [0]
    h = j // 2
    first = tree_delays(n // 2, h)
    return first + [j - h + x for x in first]


def tree(power):
    """The tree method: k = log2(C) merging stages over the power spectrogram [C][T];
    returns [C][T], row j = sweep j over all channels."""
    p = np.asarray(power, dtype=np.float64)
    C, n_t = p.shape
    if C & (C - 1):
        raise ValueError("the tree needs a power-of-two channel count")
    rows = p.copy()   # groups of size 1: row c = channel c, its only sweep
    n = 1
    while n < C:
        n *= 2
        out = np.zeros_like(rows)
        for g in range(C // n):
            for j in range(n):
                h = j // 2
                a = rows[g * n + h]                 # first half: group 2g of size n/2
                b = rows[g * n + n // 2 + h]        # second half: group 2g + 1
                s = j - h
                out[g * n + j] = a
                if s < n_t:                         # advanced past the end: adds nothing
                    out[g * n + j, :n_t - s] += b[s:]
        rows = out
    return rows
