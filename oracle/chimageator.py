"""FP64 oracle of the Chimageator on a uniform linear array (Sec. 4, "Formulation for
a uniform linear array"; the pre- and post-integrator split of Sec. 5.1).

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

Antennas p = 0 .. M - 1 on a line with equal spacing; a chirp from angle theta
reaches antenna p a time p tau_1 late (tau_1 = spacing sin(theta) / c).  What is
computed, in the paper's order:

* mixing x_{p,p+l}[n] = s_p[n] s_{p+l}[n]^* (Eq. xpq_chimg), whose tone (dropping
  the tau^2 term, Eq. chimg_xpq) is exp(2 pi i fdot tau_1 l t), t from the chirp's
  start;
* gridding of the redundant spacings l = 1 .. M - 1, x'_l[n] = sum_p w_l
  x_{p,p+l}[n], with natural weights w_l = 1 / (M - l) (uniform: w_l = 1);
* integration to the shortest sampling interval: the average over blocks of L
  samples (the Chimageator's pre-integrator output, Sec. 5.1), G_l[m];
* the spatial DFT over l (zero padded to N_s bins), Y_k[m] = sum_l G_l[m]
  exp(-2 pi i k l / N_s): a tone in l of u cycles per spacing peaks at k0 = N_s u;
* the trajectory sum (Eq. chimg_pth): a chirp that sweeps the band in T (T_b
  blocks of L samples) and starts at block m0 puts its peak at k0 = k_end (n -
  m0 L) / (T_b L) at sample n, k_end = N_s tau_1 f_s the end bin (Eq. chimgf0 at n
  = f_s T); a block average is taken at its mean sample, n = m L + (L - 1) / 2;
  P = sum_{m=m0}^{m0+T_b-1} conj(Phi(x_m)) Y_{k_m}[m] with
  k_m = rint(k0(m)) mod N_s, x_m = k0(m) - rint(k0(m)), and Phi(x) = exp(pi i M x
  / N_s), the phase of the geometric sum sum_{l=1}^{M-1} exp(2 pi i l x / N_s)
  (= Phi(x) sin(pi (M - 1) x / N_s) / sin(pi x / N_s)).
"""
import numpy as np


def grid_blocks(s, L, weights="natural"):
    """G[m][l - 1] = w_l / L sum_{p < M - l} sum_{n in block m} s_p[n] s_{p+l}[n]^*,
    l = 1 .. M - 1, for every complete block m of L samples."""
    s = np.asarray(s, dtype=np.complex128)
    M = s.shape[0]
    nb = s.shape[1] // L
    G = np.zeros((nb, M - 1), dtype=np.complex128)
    for l in range(1, M):
        w = 1.0 / (M - l) if weights == "natural" else 1.0
        for p in range(M - l):
            x = s[p, :nb * L] * np.conj(s[p + l, :nb * L])
            G[:, l - 1] += w * x.reshape(nb, L).sum(axis=1) / L
    return G


def spatial_dft(G, n_s):
    """Y[m][k] = sum_{l=1}^{M-1} G[m][l - 1] exp(-2 pi i k l / N_s), k < N_s."""
    G = np.asarray(G, dtype=np.complex128)
    l = np.arange(1, G.shape[1] + 1)
    k = np.arange(n_s)
    w = np.exp(-2j * np.pi * ((np.outer(k, l) % n_s) / n_s))
    return G @ w.T


def phase(x, M, n_s):
    """Phi(x) = exp(pi i M x / N_s)."""
    return np.exp(1j * np.pi * M * np.asarray(x, dtype=np.float64) / n_s)


def trajectory(Y, M, n_s, k_end, t_blocks, m0, L):
    """P for one trial (end bin k_end, duration t_blocks blocks of L samples, start
    block m0)."""
    Y = np.asarray(Y)
    total = 0j
    for m in range(m0, m0 + t_blocks):
        k0 = k_end * ((m - m0) * L + (L - 1) / 2.0) / (t_blocks * L)
        kr = np.rint(k0)
        total += np.conj(phase(k0 - kr, M, n_s)) * Y[m, int(kr) % n_s]
    return total


def trajectories(Y, M, n_s, trials, L):
    """P[i][m0] for trials [(k_end, t_blocks)], every start m0 with the trajectory
    inside the blocks (zero elsewhere)."""
    Y = np.asarray(Y)
    nb = Y.shape[0]
    P = np.zeros((len(trials), nb), dtype=np.complex128)
    for i, (k_end, tb) in enumerate(trials):
        for m0 in range(0, nb - tb + 1):
            P[i, m0] = trajectory(Y, M, n_s, k_end, tb, m0, L)
    return P


def gradient_sums(Y, M, n_s, grads, lengths, L):
    """App. B, optimising the imaging step: trajectories with the same gradient g
    (bins per block) share their path, so every duration is a partial sum of the
    longest.  P[i][j][m0] = sum_{q < lengths[j]} conj(Phi(x_q)) Y_{k_q}[m0 + q] with
    k0(q) = g_i (q L + (L - 1) / 2) / L (the block average at its mean sample),
    zero where m0 + lengths[j] > blocks.  Written as separate sums, one per length."""
    Y = np.asarray(Y)
    nb = Y.shape[0]
    P = np.zeros((len(grads), len(lengths), nb), dtype=np.complex128)
    for i, g in enumerate(grads):
        for j, T in enumerate(lengths):
            for m0 in range(0, nb - T + 1):
                total = 0j
                for q in range(T):
                    k0 = g * (q * L + (L - 1) / 2.0) / L
                    kr = np.rint(k0)
                    total += np.conj(phase(k0 - kr, M, n_s)) * Y[m0 + q, int(kr) % n_s]
                P[i, j, m0] = total
    return P


def nearest_cells(x, spacing):
    """Gridding of a line of antennas at ascending positions x (Sec. 4: an arbitrary
    array interpolated onto the regular grid of spacings): pair p < q goes to cell
    l = rint((x_q - x_p) / spacing) (ties to even); cells l >= 1 are kept.  Returns
    {l: [(p, q), ...]} with the pairs in row-major order."""
    x = np.asarray(x, dtype=np.float64)
    cells = {}
    for p in range(x.size):
        for q in range(p + 1, x.size):
            l = int(np.rint((x[q] - x[p]) / spacing))
            if l >= 1:
                cells.setdefault(l, []).append((p, q))
    return cells


def grid_blocks_cells(s, L, cells, n_cells):
    """G[m][l - 1] = 1 / (count_l L) sum_{(p, q) in cell l} sum_{n in block m}
    s_p[n] s_q[n]^* for l = 1 .. n_cells (zero for empty cells): natural weights
    over the pairs that fall in a cell.  The spatial DFT and trajectories then
    treat the cells as a line of n_cells + 1 elements (M = n_cells + 1 in Phi)."""
    s = np.asarray(s, dtype=np.complex128)
    nb = s.shape[1] // L
    G = np.zeros((nb, n_cells), dtype=np.complex128)
    for l, prs in cells.items():
        if l > n_cells:
            continue
        for p, q in prs:
            x = s[p, :nb * L] * np.conj(s[q, :nb * L])
            G[:, l - 1] += x.reshape(nb, L).sum(axis=1) / (len(prs) * L)
    return G


# ---- App. B "Spectral smearing": the trajectory widened by 2F bins -------------------


def tone_amplitude(x, M, n_s):
    """S(x) = sin(pi (M - 1) x / N_s) / sin(pi x / N_s) (S(0) = M - 1): with Phi(x) the
    response Y_k = Phi(x) S(x) of the spacings l = 1 .. M - 1 to a spatial tone at
    k0 = k + x (the geometric sum written out)."""
    x = np.asarray(x, dtype=np.float64)
    num = np.sin(np.pi * (M - 1) * x / n_s)
    den = np.sin(np.pi * x / n_s)
    safe = np.where(np.abs(den) < 1e-300, 1.0, den)
    return np.where(np.abs(den) < 1e-300, float(M - 1), num / safe)


def trajectory_widened(Y, M, n_s, k_end, t_blocks, m0, L, F, a=1):
    """App. B, spectral smearing: at every step the 2F + 1 bins around the trajectory,
    k_m + t (t = -F .. F, k_m = rint(k0)), each weighted by the matched filter of the
    spatial tone, conj(Phi(x_t)) S(x_t) / (M - 1) with x_t = k0 - (k_m + t) (the
    reading of the Chirpolator's 2F + 1 taps, Sec. 3.4, on the spatial DFT).  At an
    integer k0 the F = 0 weight is 1, as in Eq. chimg_pth.  a > 1: the steps are the
    integrated samples of App. B's sampling, as in `trajectory_sampled`."""
    Y = np.asarray(Y)
    total = 0j
    for j in range(t_blocks // a):
        k0 = k_end * (j * a * L + (a * L - 1) / 2.0) / (t_blocks * L)
        kr = np.rint(k0)
        for t in range(-F, F + 1):
            x = k0 - (kr + t)
            w = np.conj(phase(x, M, n_s)) * tone_amplitude(x, M, n_s) / (M - 1)
            total += w * sum(Y[m0 + j * a + r, int(kr + t) % n_s] for r in range(a))
    return total


# ---- App. B "Sampling": per-trajectory integration ------------------------------------


def sampling_blocks(k_end, t_blocks, kappa_t0):
    """Blocks per integrated sample of a trajectory: it is sampled kappa_t =
    max(1, |k_end| kappa_t0) times over its duration (the oversampling proportional to
    the end bin, App. B; at least once), i.e. every t_blocks / kappa_t blocks, taken as
    max(1, floor(t_blocks / kappa_t)) whole blocks."""
    kappa_t = max(1.0, abs(k_end) * kappa_t0)
    return max(1, int(np.floor(t_blocks / kappa_t)))


def trajectory_sampled(Y, M, n_s, k_end, t_blocks, m0, L, a):
    """App. B, sampling: the spatial spectra integrated over a blocks (Y'_k[j] =
    sum_{r < a} Y_k[m0 + j a + r], the integrate-and-dump of Eq. Yk), then the
    phase-corrected trajectory over the floor(t_blocks / a) integrated samples, each
    at the mean time of its a L samples.  a = 1 is `trajectory`."""
    Y = np.asarray(Y)
    total = 0j
    for j in range(t_blocks // a):
        k0 = k_end * (j * a * L + (a * L - 1) / 2.0) / (t_blocks * L)
        kr = np.rint(k0)
        k = int(kr) % n_s
        ysum = sum(Y[m0 + j * a + r, k] for r in range(a))
        total += np.conj(phase(k0 - kr, M, n_s)) * ysum
    return total


# ---- Sec. 4 step 4 and App. B gridding: a two-dimensional array ------------------------


def nearest_cells_2d(pos, spacing):
    """Gridding of a planar array (Sec. 4: an arbitrary array interpolated onto a
    regular grid): pair p < q goes to cell c = rint((r_q - r_p) / spacing) per axis
    (ties to even).  Only one half plane is kept, cu > 0 or (cu = 0 and cv > 0) (the
    other half holds the conjugate products); a pair whose cell falls in the other
    half is stored the other way round, (q, p), in cell -c.  Cells (0, 0) are dropped.
    Returns {(cu, cv): [(p, q), ...]} with the pairs in row-major order of p < q."""
    pos = np.asarray(pos, dtype=np.float64)
    cells = {}
    for p in range(pos.shape[0]):
        for q in range(p + 1, pos.shape[0]):
            cu, cv = (int(v) for v in np.rint((pos[q] - pos[p]) / spacing))
            a, b = p, q
            if cu < 0 or (cu == 0 and cv < 0):
                cu, cv, a, b = -cu, -cv, q, p
            if (cu, cv) != (0, 0):
                cells.setdefault((cu, cv), []).append((a, b))
    return cells


def grid_blocks_2d(s, L, cells, n_s):
    """G[m][cu][cv mod N_s] = 1 / (count_c L) sum_{(a, b) in cell c} sum_{n in block m}
    s_a[n] s_b[n]^* (natural weights over the pairs in a cell) on an N_s x N_s grid, the
    cells' coordinates taken modulo N_s (as the spatial DFT sees them)."""
    s = np.asarray(s, dtype=np.complex128)
    nb = s.shape[1] // L
    G = np.zeros((nb, n_s, n_s), dtype=np.complex128)
    for (cu, cv), prs in cells.items():
        for a, b in prs:
            x = s[a, :nb * L] * np.conj(s[b, :nb * L])
            G[:, cu % n_s, cv % n_s] += x.reshape(nb, L).sum(axis=1) / (len(prs) * L)
    return G


def spatial_dft_2d(G, n_s):
    """Y[m][ku][kv] = sum_{cu, cv} G[m][cu][cv] exp(-2 pi i (ku cu + kv cv) / N_s),
    as two one-dimensional DFT matrices."""
    G = np.asarray(G, dtype=np.complex128)
    k = np.arange(n_s)
    W = np.exp(-2j * np.pi * ((np.outer(k, k) % n_s) / n_s))
    return np.einsum("uc,mcd,vd->muv", W, G, W)


def response_2d(cells, xu, xv, n_s):
    """R(x) = sum over the occupied cells c of exp(2 pi i (xu cu + xv cv) / N_s): the
    spatial DFT of a unit tone of one cycle per N_s / k0 cells, read at bin k0 - x."""
    return sum(np.exp(2j * np.pi * (xu * cu + xv * cv) / n_s) for (cu, cv) in cells)


def trajectory_2d(Y, cells, n_s, k_end, t_blocks, m0, L):
    """Eq. chimg_pth on the planar grid: at step m the trajectory's bin is k0 = k_end
    (m - m0 + ...) / T per axis (k_end = (ku, kv) the end bins), the image bin is
    rint(k0) mod N_s per axis, and the phase correction is that of the occupied cells'
    tone response, conj(R(x)) / |R(x)| (for a uniform line, conj(Phi(x)))."""
    Y = np.asarray(Y)
    total = 0j
    for m in range(m0, m0 + t_blocks):
        f = ((m - m0) * L + (L - 1) / 2.0) / (t_blocks * L)
        k0u, k0v = k_end[0] * f, k_end[1] * f
        ru, rv = np.rint(k0u), np.rint(k0v)
        R = response_2d(cells, k0u - ru, k0v - rv, n_s)
        w = np.conj(R) / abs(R) if abs(R) > 0 else 0.0
        total += w * Y[m, int(ru) % n_s, int(rv) % n_s]
    return total
