"""OFDM demodulation, error and leakage metrics, complexity formula (oracle).

Test infrastructure only (see ``oracle/__init__``).

Pinned (tests/lin_metric_pins.py): the window by its closed-form values and
scipy's periodic Blackman-Harris window, the PSD by scipy's Welch estimate,
the out-of-band ratio by tones whose seven-line spectra give closed forms at
the in-band region's edges, the complexity formula by hand-evaluated cases.
"""
import numpy as np

from .fc import dft_matrix
from .numerology import split_radix_mults


def ofdm_demod(symbols):
    """x_hat = (1/sqrt(L)) W_L x_hat_OFDM per symbol (Sec. IV), rows = symbols."""
    symbols = np.atleast_2d(np.asarray(symbols, dtype=complex))
    L = symbols.shape[1]
    return symbols @ dft_matrix(L).T / np.sqrt(L)


def active_bins(L, K):
    """FFT indices kappa mod L of the K active subcarriers kappa in [-K/2, K/2)."""
    return (np.arange(-K // 2, K // 2)) % L


def err_db(y, ref):
    """10 log10(sum |y - ref|^2 / sum |ref|^2): waveform or symbol EVM in dB."""
    y = np.asarray(y, dtype=complex).ravel()
    ref = np.asarray(ref, dtype=complex).ravel()
    den = np.sum(np.abs(ref) ** 2)
    num = np.sum(np.abs(y - ref) ** 2)
    if den == 0:
        return -np.inf if num == 0 else np.inf
    if num == 0:
        return -np.inf
    return 10.0 * np.log10(num / den)


def blackman_harris(n):
    k = np.arange(n)
    a = (0.35875, 0.48829, 0.14128, 0.01168)
    return (a[0] - a[1] * np.cos(2 * np.pi * k / n) + a[2] * np.cos(4 * np.pi * k / n)
            - a[3] * np.cos(6 * np.pi * k / n))


def welch_psd(y, N):
    """Welch PSD over N bins: Blackman-Harris window of length N, hop N/2."""
    y = np.asarray(y, dtype=complex)
    w = blackman_harris(N)
    frames = [y[s:s + N] * w for s in range(0, len(y) - N + 1, N // 2)]
    if not frames:
        raise ValueError("signal shorter than one PSD frame")
    F = np.stack(frames, axis=1)
    return np.sum(np.abs(dft_matrix(N) @ F) ** 2, axis=1)


def oob_ratio_db(y, N, bands, guard=8):
    """Out-of-band power over total power in dB.

    bands = [(c, K, n_tb), ...] in the bins of this N; the in-band region is the
    union of [c - K/2 - n_tb - guard, c + K/2 + n_tb + guard).
    """
    psd = welch_psd(y, N)
    inband = np.zeros(N, dtype=bool)
    for c, K, n_tb in bands:
        lo = c - K // 2 - n_tb - guard
        inband[np.arange(lo, c + K // 2 + n_tb + guard) % N] = True
    tot = np.sum(psd)
    return 10.0 * np.log10(np.sum(psd[~inband]) / tot)


def complexity_per_symbol(n_long, subbands, alpha=2.0, beta=1.0):
    """Real multiplications per data symbol, Sec. V:
    C = (alpha mu(N) + sum_m [alpha beta mu(L_m) + 6 alpha N_tb,m + mu(L_OFDM,m)])
        / sum_m L_act,m, with subbands = [(L_m, L_OFDM_m, N_tb_m, L_act_m), ...].
    """
    hi = alpha * split_radix_mults(n_long)
    lo = sum(alpha * beta * split_radix_mults(Lm) + 6 * alpha * ntb + split_radix_mults(Lo)
             for Lm, Lo, ntb, _ in subbands)
    return (hi + lo) / sum(k for *_, k in subbands)
