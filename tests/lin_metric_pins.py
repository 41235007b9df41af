"""Pins of the oracle's plain linear-convolution reference (``oracle.lin``) and
of its metrics (``oracle.metrics``) against what the mathematics fixes.

Each pin takes the module under test as an argument (so the mutation test can
run the same pins on deliberately broken copies) and returns a relative error
(or an absolute error in dB for the leakage pins); the tests require FP64
rounding level.

Linear reference (Sec. I-II: FC approximates a linear convolution with the
prototype filter whose frequency samples are the real weights D):
 * lin_tx_cont_i1    I = 1, c = 0, D the DFT of a short Hermitian FIR h:
                     tx_cont_lin is np.convolve(x, h) placed at the first input
                     sample (textbook linear convolution).
 * lin_tx_cont_tone  I > 1, c != 0: a low-rate tone at bin kappa gives, where
                     the whole prototype lies inside the burst, the high-rate
                     tone at c + kappa with amplitude D[kappa + L/2] / sqrt(I)
                     (the prototype's frequency response at the tone is
                     D / I on the interpolated grid; only one image lies in the
                     band).
 * lin_tx_sync_i1    I = 1, c = 0: every symbol (CP included) convolved with h
                     by np.convolve and placed at its own grid position
                     sigma_n + S_L,n; the symbols add.
 * lin_tx_sync_split I > 1, c != 0: the synchronised reference is the sum over
                     symbols of the continuous reference of that symbol alone,
                     shifted to the symbol's grid and rotated by the carrier
                     phase of the shift.
 * lin_rx_cont_adj   <tx_cont_lin x, y> = <x, rx_cont_lin y>: the receiver is
                     the transmitter's adjoint (exact when the finite
                     prototype is Hermitian, i.e. its lone sample at d = -N/2
                     is zero: D with a zero alternating sum).
 * lin_rx_sync_adj   <tx_sync_lin x, y> = <x_u, rx_sync_lin y> for inputs x
                     that are zero on the CPs (x_u the useful parts): the
                     receiver samples each symbol's useful-part grid.
Metrics:
 * bh_closed_form    Blackman-Harris window: centre value a0 + a1 + a2 + a3 = 1,
                     end value a0 - a1 + a2 - a3, and the periodic window of
                     scipy.signal.windows.blackmanharris (sym=False).
 * welch_vs_scipy    Welch PSD shape equal to scipy.signal.welch with the same
                     window, segment N, overlap N/2, no detrending, two-sided.
 * oob_tone_edges    A tone on an integer bin k0 has, under this window, a PSD
                     of exactly seven lines: a0^2 at k0 and a_m^2/4 at k0 +- m
                     (the window's DFT has those seven taps). The out-of-band
                     ratio of tones just outside and just inside the in-band
                     region's edges is therefore a closed form in a0..a3.
 * oob_two_tones     One tone deep in band (power a^2) and one far out of band
                     (power b^2): 10 log10(b^2 / (a^2 + b^2)).
 * complexity_cases  The Sec. V formula evaluated by hand (literal integers) for
                     three configurations with N_tb > 0 (alpha = 2 and 3,
                     beta = 1 and 1/2, L_OFDM equal to and below L_m).
"""
from fractions import Fraction

import numpy as np
from scipy import signal as sps

from oracle import numerology as nu

BH = (0.35875, 0.48829, 0.14128, 0.01168)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _cvec(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _hermitian_fir(rng, L, T):
    """h[-T..T] with h[-d] = conj(h[d]) and its DFT on L bins in fftshifted
    order (real)."""
    h = _cvec(rng, T + 1)
    h[0] = h[0].real
    full = np.r_[np.conj(h[1:][::-1]), h]
    kap = np.arange(L) - L // 2
    D = np.real(np.exp(-2j * np.pi * np.outer(kap, np.arange(-T, T + 1)) / L) @ full)
    return full, D


def _zero_alternating_sum(rng, L):
    """Real weights with sum_p (-1)^p D[p] = 0: the prototype's sample at
    d = -N/2 vanishes, so the finite prototype is exactly Hermitian."""
    D = rng.uniform(0.2, 1.0, L)
    alt = np.sum(D * (-1.0) ** np.arange(L))
    D[1] += alt            # (-1)^1 D[1] absorbs the alternating sum
    return D


# ------------------------------------------------------- linear reference --
def lin_tx_cont_i1(lin, L=32, n=150, T=3, seed=21, lam=Fraction(1, 2)):
    rng = np.random.default_rng(seed)
    h, D = _hermitian_fir(rng, L, T)
    ov = nu.Overlap(L, L, lam)
    x = _cvec(rng, n)
    y = lin.tx_cont_lin(x, L, L, 0, D, lam=lam)
    ref = np.zeros(len(y), dtype=complex)
    conv = np.convolve(x, h)                 # conv[k] = sum_l x[l] h[k - l - T]
    ref[ov.L_O - T:ov.L_O - T + len(conv)] = conv
    return rel(y, ref)


def lin_tx_cont_tone(lin, L=32, N=128, c=-9, seed=22):
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N)
    D = rng.uniform(0.1, 1.0, L)
    n = 16 * L
    worst = 0.0
    for kap in (-L // 2, -7, 0, 5, L // 2 - 1):
        x = np.exp(2j * np.pi * kap * np.arange(n) / L)
        y = lin.tx_cont_lin(x, L, N, c, D)
        t = np.arange(len(y))
        t0 = I * ov.L_O                       # high-rate instant of x[0]
        ref = (D[kap + L // 2] / np.sqrt(I) * np.exp(2j * np.pi * c * t / N)
               * np.exp(2j * np.pi * kap * (t - t0) / N))
        lo, hi = t0 + N // 2, t0 + I * (n - 1) - N // 2
        worst = max(worst, rel(y[lo:hi], ref[lo:hi]))
    return worst


def lin_tx_sync_i1(lin, L=32, T=2, seed=23, ncp=(4, 3, 3, 4, 3)):
    rng = np.random.default_rng(seed)
    h, D = _hermitian_fir(rng, L, T)
    ov = nu.Overlap(L, L)
    x = _cvec(rng, sum(L + c for c in ncp))
    y = lin.tx_sync_lin(x, L, L, 0, D, list(ncp))
    sig = nu.sync_sigma(list(ncp), L)
    ref = np.zeros(len(y) + 4 * L, dtype=complex)
    pos = 0
    for k, lc in enumerate(ncp):
        conv = np.convolve(x[pos:pos + L + lc], h)
        start = sig[k] + (ov.L_L - lc) - T     # symbol sample 0 at sigma_n + S_L,n
        ref[start:start + len(conv)] += conv
        pos += L + lc
    return rel(y, ref[:len(y)])


def lin_tx_sync_split(lin, L=16, N=64, c=7, ncp=(9, 5, 6, 7), seed=24):
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N)
    D = rng.uniform(0.1, 1.0, L)
    lcp = [v // I for v in ncp]
    x = _cvec(rng, sum(L + lc for lc in lcp))
    y = lin.tx_sync_lin(x, L, N, c, D, list(ncp))
    sig = nu.sync_sigma(list(ncp), N)
    ref = np.zeros(len(y) + 8 * N, dtype=complex)
    pos = 0
    for k, lc in enumerate(lcp):
        xs = x[pos:pos + L + lc]
        pos += L + lc
        # trailing zeros lengthen the continuous output (its length is the
        # FC block grid's) so that it holds the symbol's whole filtered tail
        yc = lin.tx_cont_lin(np.r_[xs, np.zeros(L)], L, N, c, D)
        # the continuous reference puts sample 0 at I L_O; this symbol's grid
        # puts it at sigma_n + I S_L,n
        shift = sig[k] + I * (ov.L_L - lc) - I * ov.L_O
        lo = max(0, -shift)
        ref[shift + lo:shift + len(yc)] += np.exp(2j * np.pi * ((c * shift) % N) / N) * yc[lo:]
    return rel(y, ref[:len(y)])


def lin_rx_cont_adj(lin, L=16, N=64, c=5, n=60, seed=25):
    rng = np.random.default_rng(seed)
    D = _zero_alternating_sum(rng, L)
    x = _cvec(rng, n)
    yx = lin.tx_cont_lin(x, L, N, c, D)
    y = _cvec(rng, len(yx))
    lhs = np.vdot(yx, y)
    rhs = np.vdot(x, lin.rx_cont_lin(y, L, N, c, D, n))
    return float(abs(lhs - rhs) / abs(lhs))


def lin_rx_sync_adj(lin, L=16, N=64, c=-6, ncp=(9, 5, 6, 7), seed=26):
    rng = np.random.default_rng(seed)
    I = N // L
    D = _zero_alternating_sum(rng, L)
    lcp = [v // I for v in ncp]
    xu = _cvec(rng, (len(ncp), L))
    x = np.concatenate([np.r_[np.zeros(lc, dtype=complex), xu[k]] for k, lc in enumerate(lcp)])
    yx = lin.tx_sync_lin(x, L, N, c, D, list(ncp))
    y = _cvec(rng, len(yx))
    lhs = np.vdot(yx, y)
    rhs = np.vdot(xu.ravel(), lin.rx_sync_lin(y, L, N, c, D, list(ncp)).ravel())
    return float(abs(lhs - rhs) / abs(lhs))


LIN_PINS = {
    "lin_tx_cont_i1": lin_tx_cont_i1,
    "lin_tx_cont_i1_ola_quarter": lambda lin: lin_tx_cont_i1(lin, L=64, T=5, lam=Fraction(1, 4)),
    "lin_tx_cont_tone": lin_tx_cont_tone,
    "lin_tx_sync_i1": lin_tx_sync_i1,
    "lin_tx_sync_split": lin_tx_sync_split,
    "lin_rx_cont_adj": lin_rx_cont_adj,
    "lin_rx_cont_adj_quarter": lambda lin: lin_rx_cont_adj(lin, L=32, N=128, c=-11, n=90),
    "lin_rx_sync_adj": lin_rx_sync_adj,
}


# ---------------------------------------------------------------- metrics --
def bh_closed_form(metrics, n=64):
    w = metrics.blackman_harris(n)
    a0, a1, a2, a3 = BH
    e = max(abs(w[n // 2] - (a0 + a1 + a2 + a3)), abs(w[0] - (a0 - a1 + a2 - a3)), abs(w[n // 2] - 1.0))
    return max(e, rel(w, sps.windows.blackmanharris(n, sym=False)))


def welch_vs_scipy(metrics, N=64, seed=27):
    rng = np.random.default_rng(seed)
    y = _cvec(rng, 7 * N + 5)
    got = metrics.welch_psd(y, N)
    _, ref = sps.welch(y, window=sps.windows.blackmanharris(N, sym=False), nperseg=N, noverlap=N // 2,
                       detrend=False, return_onesided=False, scaling="spectrum")
    return rel(got / np.sum(got), ref / np.sum(ref))


def _tone(N, k0, n_frames=9, amp=1.0, phase=0.0):
    t = np.arange((n_frames + 1) * N // 2)
    return amp * np.exp(1j * phase) * np.exp(2j * np.pi * ((k0 * t) % N) / N)


def oob_tone_edges(metrics, N=128, c=-20, K=24, n_tb=3, guard=5):
    a0, a1, a2, a3 = BH
    side = (a1 ** 2 + a2 ** 2 + a3 ** 2) / 4      # one side's three lines
    total = a0 ** 2 + 2 * side
    lo, hi = c - K // 2 - n_tb - guard, c + K // 2 + n_tb + guard
    band = [(c, K, n_tb)]
    out_edge = 10 * np.log10((a0 ** 2 + side) / total)     # centre and one side outside
    in_edge = 10 * np.log10(side / total)                  # one side outside
    cases = [(hi, out_edge), (lo - 1, out_edge), (hi - 1, in_edge), (lo, in_edge),
             (hi + 3, 0.0), (c, -np.inf)]
    worst = 0.0
    for k0, ref in cases:
        with np.errstate(divide="ignore"):
            got = metrics.oob_ratio_db(_tone(N, k0 % N), N, band, guard=guard)
        if np.isinf(ref):
            worst = max(worst, 0.0 if got < -250 else abs(got + 300))
        else:
            worst = max(worst, abs(got - ref))
    return worst


def oob_two_tones(metrics, N=256, seed=28):
    rng = np.random.default_rng(seed)
    a, b = 1.0, 0.05
    y = _tone(N, 10, amp=a, phase=rng.uniform(0, 6.28)) + _tone(N, 100, amp=b, phase=rng.uniform(0, 6.28))
    got = metrics.oob_ratio_db(y, N, [(12, 16, 4)], guard=8)
    return abs(got - 10 * np.log10(b ** 2 / (a ** 2 + b ** 2)))


def complexity_cases(metrics):
    # N = 1024, one subband L_m = L_OFDM = 64, N_tb = 8, 48 active: mu(1024) =
    # 10240 - 3072 + 4 = 7172, mu(64) = 384 - 192 + 4 = 196
    c1 = metrics.complexity_per_symbol(1024, [(64, 64, 8, 48)], alpha=2, beta=1)
    r1 = (2 * 7172 + 2 * 196 + 6 * 2 * 8 + 196) / 48
    # N = 256, beta = 1/2: (16, 16, N_tb 4, 12 active) and (128, 128, 6, 96):
    # mu(256) = 1284, mu(16) = 20, mu(128) = 516
    c2 = metrics.complexity_per_symbol(256, [(16, 16, 4, 12), (128, 128, 6, 96)], alpha=2, beta=0.5)
    r2 = (2 * 1284 + (20 + 48 + 20) + (516 + 72 + 516)) / 108
    # alpha = 3 (blocks per symbol of a continuous scheme), one subband
    # L_m = 128 with L_OFDM = 16 taken apart: N = 128, N_tb = 2, 12 active
    c3 = metrics.complexity_per_symbol(128, [(128, 16, 2, 12)], alpha=3, beta=1)
    r3 = (3 * 516 + 3 * 516 + 6 * 3 * 2 + 20) / 12
    return max(abs(c1 - r1) / r1, abs(c2 - r2) / r2, abs(c3 - r3) / r3)


METRIC_PINS = {
    "bh_closed_form": bh_closed_form,
    "welch_vs_scipy": welch_vs_scipy,
    "oob_tone_edges": oob_tone_edges,
    "oob_two_tones": oob_two_tones,
    "complexity_cases": complexity_cases,
}
TOL = 1e-9
