"""FP64 oracle of the Chirpolator post-integrator: the detection image P(theta) and
E(theta) = |P|^2 formed from the pre-integrator's DFT bins.

TEST INFRASTRUCTURE ONLY: the product path never imports this module.

What it computes (Bannister & Cornwell 2011):

* the geometric delay of a baseline for the direction cosines (l, m) (App. A.1, Eq.
  tau3D), with the baseline vector (u, v, w) = r_p - r_q in metres, so that antenna
  q receives the signal tau_pq later than antenna p;
* the tone of the mixed pair at k0 = fdot tau N / f_s bins (Eq. f0), k0' = round(k0)
  (Eq. f0dash, ties to even);
* the phase term Phi_pq(x) of Eq. phipq1 and the amplitude D_N(x) of Eq. dn;
* the matched filter over 2F + 1 bins around k0' (Sec. 3.4, "Compensating for the
  smearing"), summed as a vector over all pairs p < q (Eq. pth), and E = |P|^2
  (Eq. eth).

Readings where the paper leaves a choice (each stated where it is used):

* Array phase: for one baseline the paper puts antenna p at the phase centre, so the
  constant phase of the mixed tone is -pi fdot tau^2.  In an array every antenna is
  delayed by a_p = -r_p . (l, m, n - 1) / c (n = sqrt(1 - l^2 - m^2)) relative to the
  phase centre, and the same mixing gives -pi fdot tau_pq (a_p + a_q), which is the
  paper's term when a_p = 0.
* Window: the pre-integrator's bins are phase-referenced to sample 0 of the stream;
  the window that starts at sample w L is re-referenced to its own first sample
  (X[k] = S[k] exp(2 pi i w L k / N)), the DFT of Eq. dft, and the chirp's own time
  origin is taken at that first sample (the window aligned with the chirp).
* Filter weights: conj(Phi_pq(x)) D_N(x) / N with the same offset x = k0' + t - k0 in
  both factors, t = -F .. F.  The 1 / N makes F = 0 at an integer k0 reduce to Eq.
  pth, whose ideal sum is N M (M - 1) / 2; the printed generalisation writes the
  amplitude's argument without the k0' shift, which we read as a slip.
* Bins outside the computed range -kmax .. kmax contribute zero.
"""
import numpy as np

C_LIGHT = 299792458.0   # m / s


def antenna_delays(ant_xyz, l, m):
    """a_p = -r_p . (l, m, n - 1) / c, the arrival time at antenna p relative to the
    phase centre for the direction (l, m); n - 1 = -(l^2 + m^2) / (1 + n)."""
    r = np.asarray(ant_xyz, dtype=np.float64)
    nm1 = -(l * l + m * m) / (1.0 + np.sqrt(1.0 - l * l - m * m))
    return -(r[:, 0] * l + r[:, 1] * m + r[:, 2] * nm1) / C_LIGHT


def baseline_delay(ant_xyz, p, q, l, m):
    """Eq. tau3D with (u, v, w) = r_p - r_q: tau_pq = a_q - a_p."""
    r = np.asarray(ant_xyz, dtype=np.float64)
    u, v, w = r[p] - r[q]
    nm1 = -(l * l + m * m) / (1.0 + np.sqrt(1.0 - l * l - m * m))
    return (u * l + v * m + w * nm1) / C_LIGHT


def dirichlet(x, n):
    """D_N(x) of Eq. dn (N at x = 0)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.full(x.shape, float(n))
    nz = x != 0
    out[nz] = np.sin(np.pi * x[nz]) / np.sin(np.pi * x[nz] / n)
    return out


def phase_term(x, fdot, tau, a_sum, n):
    """Phi_pq(x) of Eq. phipq1 with the array reading of the constant phase:
    exp(-pi i fdot tau (a_p + a_q)) exp(-pi i x (N - 1) / N)."""
    x = np.asarray(x, dtype=np.float64)
    return np.exp(-1j * np.pi * fdot * tau * a_sum) * np.exp(-1j * np.pi * x * (n - 1) / n)


def window_reference(S, n_win, L, kmax, first_window=0, w_step=1):
    """Rows i of S (window first_window + i w_step, bins -kmax .. kmax, phase from
    sample 0) re-referenced to each window's first sample w L."""
    S = np.asarray(S, dtype=np.complex128)
    ks = np.arange(-kmax, kmax + 1, dtype=np.int64)
    out = np.empty_like(S)
    for i in range(S.shape[0]):
        w = first_window + i * w_step
        out[i] = S[i] * np.exp(2j * np.pi * (((w * L * ks) % n_win) / n_win))
    return out


def image(S, ant_xyz, pix_lm, fdot, f_s, n_win, L, kmax, F, first_window=0, w_step=1):
    """P[i, j] = sum_{p<q} sum_{t=-F}^{F} conj(Phi_pq(x)) D_N(x) / N X_pq[k0' + t],
    x = k0' + t - k0, for every row i of S (window first_window + i w_step) and
    every direction pix_lm[j] = (l, m).  S is [rows][pairs][2 kmax + 1], pairs p < q
    in row-major order, as the pre-integrator writes it."""
    X = window_reference(S, n_win, L, kmax, first_window, w_step)
    ant = np.asarray(ant_xyz, dtype=np.float64)
    M = ant.shape[0]
    pix = np.asarray(pix_lm, dtype=np.float64).reshape(-1, 2)
    P = np.zeros((X.shape[0], pix.shape[0]), dtype=np.complex128)
    for j, (l, m) in enumerate(pix):
        a = antenna_delays(ant, l, m)
        b = 0
        for p in range(M):
            for q in range(p + 1, M):
                tau = baseline_delay(ant, p, q, l, m)
                k0 = fdot * tau * n_win / f_s
                k0r = int(np.rint(k0))
                for t in range(-F, F + 1):
                    k = k0r + t
                    if abs(k) > kmax:
                        continue
                    x = k - k0
                    g = np.conj(phase_term(x, fdot, tau, a[p] + a[q], n_win)) * dirichlet(x, n_win) / n_win
                    P[:, j] += g * X[:, b, k + kmax]
                b += 1
    return P


def energy(P):
    """E = |P|^2 (Eq. eth)."""
    return np.abs(np.asarray(P)) ** 2

