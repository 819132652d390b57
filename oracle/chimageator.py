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
