"""FP64 oracle of the Chirpolator pre-integrator.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

What it computes, in the paper's order (Bannister & Cornwell 2011):

* mixing (Sec. 3.2, Eq. xpq): x_pq[n] = s_p[n] s_q[n]^*, for antenna pairs p < q;
* block partial DFTs (App. A.3, the block-based sliding DFT):
    V_k[m] = sum_{n=0}^{L-1} exp(-2 pi i (n + m L) k / N) x[n + m L],
  for the bins -kmax <= k <= kmax (Sec. "compute only DFTs required");
* the moving sum over N / L blocks (App. A.3, Eq. block_cic):
    S_k[m] = S_k[m-1] + V_k[m] - V_k[m - N/L],
  started from S_k[-1] = 0 with V_k[m] = 0 for m < 0, so that S_k[m] is bin k of
  the DFT of the N samples ending with block m, phase-referenced to sample 0;
* the closed form of the DFT of a mixed linear chirp (Sec. 3.2, Eqs. dft, phidn,
  dn, phipq1): Phi_pq(k - k0) D_N(k - k0), k0 = fdot tau N / f_s (Eq. f0);
* DFT factorisation across the bank of lengths N = N0 d (App. A.3,
  "Factorizing the DFTs");
* the shared multiplications of a positive and a negative bin (App. A.3,
  Eqs. fpos, fneg).

numpy in float64 / complex128, loops where they keep the definition readable.
"""
import math

import numpy as np


def pairs(m_ant):
    """Antenna pairs (p, q), p < q, in row-major order."""
    return [(p, q) for p in range(m_ant) for q in range(p + 1, m_ant)]


def mix(s, p, q):
    """x_pq[n] = s_p[n] s_q[n]^* (Sec. 3.2, Eq. xpq)."""
    s = np.asarray(s, dtype=np.complex128)
    return s[p] * np.conj(s[q])


def bins(kmax):
    """The bins -kmax .. kmax, in increasing order."""
    return np.arange(-kmax, kmax + 1)


def block_partial_dft(x, n_win, L, ks):
    """V[m, j] = sum_{n<L} exp(-2 pi i (n + m L) ks[j] / N) x[n + m L] for every
    complete block m of x (App. A.3).  The exponent's integer (n + m L) k is reduced
    modulo N before the angle is formed, so the phase is exact for any stream length."""
    x = np.asarray(x, dtype=np.complex128)
    nb = x.size // L
    ks = np.asarray(ks, dtype=np.int64)
    out = np.zeros((nb, ks.size), dtype=np.complex128)
    n = np.arange(L, dtype=np.int64)
    for m in range(nb):
        idx = n + m * L
        for j, k in enumerate(ks):
            w = np.exp(-2j * np.pi * (((idx * k) % n_win) / n_win))
            out[m, j] = np.sum(w * x[m * L:(m + 1) * L])
    return out


def block_cic(v, n_win, L):
    """S[m] = S[m-1] + V[m] - V[m - N/L] (Eq. block_cic), S[-1] = 0, V[m < 0] = 0."""
    if n_win % L:
        raise ValueError("N must be a multiple of L")
    r = n_win // L
    s = np.zeros_like(v)
    acc = np.zeros(v.shape[1:], dtype=v.dtype)
    for m in range(v.shape[0]):
        acc = acc + v[m] - (v[m - r] if m >= r else 0)
        s[m] = acc
    return s


def sliding_dft(x, n_win, L, ks):
    """Definition of the block-sampled sliding DFT: bin k of the N samples that end
    with block m, x[n] = 0 for n < 0, phase referenced to sample 0:
        S[m, j] = sum_{n = (m+1) L - N}^{(m+1) L - 1} x[n] exp(-2 pi i n ks[j] / N)."""
    x = np.asarray(x, dtype=np.complex128)
    nb = x.size // L
    ks = np.asarray(ks, dtype=np.int64)
    out = np.zeros((nb, ks.size), dtype=np.complex128)
    for m in range(nb):
        end = (m + 1) * L
        lo = max(0, end - n_win)
        n = np.arange(lo, end, dtype=np.int64)
        for j, k in enumerate(ks):
            out[m, j] = np.sum(x[lo:end] * np.exp(-2j * np.pi * (((n * k) % n_win) / n_win)))
    return out


def preintegrate(s, n_win, L, kmax, pair_kmax=None):
    """The pre-integrator on a stream: S[m, pair, k] for every pair p < q, every bin
    -kmax..kmax and every block m whose window is complete (m >= N/L - 1).  With
    per-pair budgets (App. A.3, "compute only DFTs required on a baseline basis")
    the bins |k| > pair_kmax[pair] are left at zero."""
    ks = bins(kmax)
    prs = pairs(np.asarray(s).shape[0])
    first = n_win // L - 1
    out = []
    for i, (p, q) in enumerate(prs):
        v = block_partial_dft(mix(s, p, q), n_win, L, ks)
        sp = block_cic(v, n_win, L)[first:]
        if pair_kmax is not None:
            sp[:, np.abs(ks) > pair_kmax[i]] = 0
        out.append(sp)
    return np.stack(out, axis=1)


def pair_bin_budgets(positions, kmax):
    """Bin budget per pair p < q proportional to the baseline length (the tone of a
    pair sits at k0 = B tau with tau <= b_pq / c, Eq. f0): ceil(kmax b_pq / b_max)."""
    pos = np.asarray(positions, dtype=np.float64)
    b = np.array([np.hypot(*(pos[p] - pos[q])) for p, q in pairs(pos.shape[0])])
    return np.minimum(kmax, np.ceil(kmax * b / b.max())).astype(np.int32)


def dirichlet(x, n):
    """D_N(x) of Eq. dn: N at x = 0, sin(pi x) / sin(pi x / N) otherwise (-N < x < N)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    z = np.abs(x) < 1e-300
    out[z] = n
    out[~z] = np.sin(np.pi * x[~z]) / np.sin(np.pi * x[~z] / n)
    return out


def linear_chirp(n_samp, fdot, f_s, tau=0.0):
    """s[n] = exp(pi i fdot (n / f_s - tau)^2): the unit chirp of Sec. 3.2 (Eq. chirp),
    sampled at f_s and delayed by tau seconds."""
    t = np.arange(n_samp, dtype=np.float64) / f_s - tau
    return np.exp(1j * np.pi * fdot * t * t)


def mixed_chirp_dft(ks, n_win, fdot, tau, f_s):
    """Eqs. phidn, dn, phipq1: X[k] = Phi(k - k0) D_N(k - k0), k0 = fdot tau N / f_s,
    Phi(x) = exp(-pi i fdot tau^2) exp(-pi i x (N - 1) / N), for the DFT over
    n = 0..N-1 of x[n] = s[n] s^*[n - tau f_s] with s the chirp of Eq. chirp."""
    x = np.asarray(ks, dtype=np.float64) - fdot * tau * n_win / f_s
    phi = np.exp(-1j * np.pi * fdot * tau * tau) * np.exp(-1j * np.pi * x * (n_win - 1) / n_win)
    return phi * dirichlet(x, n_win)


def factorised_bin(x, end, n0, d, k, D):
    """App. A.3, "Factorizing the DFTs": bin k of the length-N0 d DFT of the samples
    ending at `end` (exclusive) as the sum of D adjacent bins k / D of length
    N0 d / D, when D divides both k and d.  With the phase referenced to sample 0,
    the j-th shorter window ends at end - j N0 d / D.  (The printed shift, d' N0,
    is this for d = D, the case of the paper's example.)"""
    if k % D or d % D:
        raise ValueError("D must divide k and d")
    n_short = n0 * d // D
    total = 0j
    for j in range(D):
        total += window_dft(x, end - j * n_short, n_short, k // D)
    return total


def window_dft(x, end, n_win, k):
    """sum_{n = end - N}^{end - 1} x[n] exp(-2 pi i n k / N), x[n] = 0 outside x."""
    x = np.asarray(x, dtype=np.complex128)
    lo, hi = max(0, end - n_win), min(end, x.size)
    n = np.arange(lo, hi, dtype=np.int64)
    return complex(np.sum(x[lo:hi] * np.exp(-2j * np.pi * (((n * k) % n_win) / n_win))))


def factorisable_fraction(k_max, d_max):
    """Fraction of (k, d), 1 <= k <= k_max, 1 <= d <= d_max, whose bin can be
    factorised (k and d share a factor > 1)."""
    hits = sum(1 for k in range(1, k_max + 1) for d in range(1, d_max + 1) if math.gcd(k, d) > 1)
    return hits / (k_max * d_max)


def pos_neg_products(a, b, c, d):
    """Eqs. fpos, fneg: (a + ib)(c - id) and (a + ib)(c + id) from the four shared
    products ac, bd, ad, bc.  Returns (r_k, r_-k, multiplications, additions)."""
    ac, bd, ad, bc = a * c, b * d, a * d, b * c
    return complex(ac + bd, bc - ad), complex(ac - bd, ad + bc), 4, 4


def bank_direct(s, n0, n_len, L, kmax):
    """The pre-integrator for every window length n0 d, d = 1 .. n_len (a DFT length
    per DM trial, App. A.3), each from its definition."""
    return [preintegrate(s, n0 * d, L, kmax) for d in range(1, n_len + 1)]


def _smallest_prime(x):
    p = 2
    while p * p <= x:
        if x % p == 0:
            return p
        p += 1
    return x


def bank_factorised(s, n0, n_len, L, kmax):
    """The same bank with App. A.3's factorisation at block resolution: a bin k of
    length n0 d with p = the smallest prime factor of gcd(|k|, d) > 1 is the sum of
    the p windows of bin k / p of length n0 d / p that tile its window; with each
    length's output starting at its first complete window, window w of length d
    takes windows w + (p - 1 - j) n0 (d / p) / L, j < p, of length d / p."""
    ks = bins(kmax)
    out = []
    for d in range(1, n_len + 1):
        full = preintegrate(s, n0 * d, L, kmax)
        for j, k in enumerate(ks):
            g = math.gcd(abs(int(k)), d)
            if g == 1:
                continue
            p = _smallest_prime(g)
            short, rs = out[d // p - 1], n0 * (d // p) // L
            for w in range(full.shape[0]):
                full[w, :, j] = sum(short[w + (p - 1 - i) * rs, :, kmax + int(k) // p] for i in range(p))
        out.append(full)
    return out


def gauss_sum(a, L):
    """G(a, L) = sum_{n=0}^{L-1} exp(2 pi i a n^2) (App. A.2, Eq. gaussum): the sum of a
    chirp over L samples that starts at the centre of a DFT bin; the coherence loss
    is eta = |G(a, L)| / L."""
    n = np.arange(L, dtype=np.float64)
    return complex(np.sum(np.exp(2j * np.pi * a * n * n)))


def coherence_loss(a, L):
    """eta = |G(a, L)| / L."""
    return abs(gauss_sum(a, L)) / L
