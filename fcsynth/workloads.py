"""Benchmark and test workloads as plain subband parameter lists.

Each subband is a dict with the fields of the C-ABI subband descriptor:
scs_khz, first_symbol, n_symbols, n_active (K), n_tb, n_short (L), n_long (N),
center_bin (c), overlap (num, den), mode, stream, taper. Modes are the strings
'cont_ola', 'cont_ols', 'sync_ola', 'sync_ols'.
"""
import numpy as np


def subband(scs_khz, n_symbols, n_active, n_tb, n_short, n_long, center_bin, mode,
            stream=0, first_symbol=0, overlap=(1, 2), taper=0):
    return dict(scs_khz=scs_khz, first_symbol=first_symbol, n_symbols=n_symbols,
                n_active=n_active, n_tb=n_tb, n_short=n_short, n_long=n_long,
                center_bin=center_bin, overlap=tuple(overlap), mode=mode, stream=stream,
                taper=taper)


def next_pow2(v):
    return 1 << int(np.ceil(np.log2(v)))


def plain_tx_slot():
    """One 15 kHz subband, 24 PRB (K = 288), L = 512, N = 2048 (I = 4), one
    14-symbol slot, continuous overlap-save, 50 % overlap, QPSK, c = 0."""
    return [subband(15, 14, 288, 8, 512, 2048, 0, 'cont_ols')], dict(qam=4, seed=1, io='c64')


def mixed_numerology(mode_tx='sync_ola'):
    """20 MHz carrier at 30.72 MS/s, one 1 ms subframe: subband A 15 kHz
    48 PRB (L = 1024, N = 2048, c = -312, 14 symbols) and subband B 30 kHz
    24 PRB (L = 512, N = 1024, c = +156, 28 symbols); 16-QAM; N_tb = 8."""
    return [subband(15, 14, 576, 8, 1024, 2048, -312, mode_tx),
            subband(30, 28, 288, 8, 512, 1024, 156, mode_tx)], dict(qam=16, seed=2, io='c64')


def batched_carriers(n_carriers=256, seed=3, n_tb=8, n_symbols=14):
    """Independent carriers, one stream each, one slot each: width W ~ U{1..106}
    PRB, mu ~ U{0,1,2}, N ~ U{1024, 2048, 4096}, L = max(64, next_pow2(12W + 16)),
    N raised to at least 2L, centre c uniform in the range that keeps
    [c - L/2, c + L/2) inside [-3N/8, 3N/8); 64-QAM; symbol-synchronised OLA."""
    rng = np.random.default_rng(seed)
    sbs = []
    for k in range(n_carriers):
        W = int(rng.integers(1, 107))
        mu = int(rng.integers(0, 3))
        N = int(rng.choice([1024, 2048, 4096]))
        L = max(64, next_pow2(12 * W + 16))
        N = max(N, 2 * L)
        lo, hi = -3 * N // 8 + L // 2, 3 * N // 8 - L // 2
        c = int(rng.integers(lo, hi + 1))
        ntb = n_tb if np.isscalar(n_tb) else int(rng.integers(n_tb[0], n_tb[1] + 1))
        sbs.append(subband(15 << mu, n_symbols, 12 * W, ntb, L, N, c, 'sync_ola', stream=k))
    return sbs, dict(qam=64, seed=seed, io='f16')


def weight_opt_carriers(n_carriers=256, n_slots=64, seed=5):
    """The batched carriers (widths, numerologies, long transforms and centres
    of batched_carriers) for transition-weight optimisation: N_tb ~ U{4..16}
    per carrier, L = max(64, next_pow2(12 W + 2 N_tb)) (N raised to at least
    2 L and c clamped into its range where the wider transition bands need a
    longer short transform), n_slots slots of 16-QAM per carrier, FP32."""
    base, _ = batched_carriers(n_carriers)
    rng = np.random.default_rng(seed)
    sbs = []
    for k, s in enumerate(base):
        ntb = int(rng.integers(4, 17))
        K = s["n_active"]
        L = max(64, next_pow2(K + 2 * ntb))
        N = max(s["n_long"], 2 * L)
        lo, hi = -3 * N // 8 + L // 2, 3 * N // 8 - L // 2
        c = min(max(s["center_bin"], lo), hi)
        sbs.append(subband(s["scs_khz"], 14 * n_slots, K, ntb, L, N, c, 'sync_ola', stream=k))
    return sbs, dict(qam=16, seed=seed, io='c64', mu_oob=1.0)


RX_WIDTHS = (4, 12, 24, 33, 51, 66, 11, 72)
RX_SHORT = (64, 256, 512, 512, 1024, 1024, 256, 1024)


def rx_filterbank(n_symbols=280):
    """100 MHz carrier, 30 kHz, N = 4096 at 122.88 MS/s, eight contiguous
    subbands of the listed widths starting at bin -1638, 256-QAM, 30 dB SNR,
    symbol-synchronised OLS analysis, one 10 ms frame (280 symbols)."""
    sbs, s = [], -1638
    for W, L in zip(RX_WIDTHS, RX_SHORT):
        sbs.append(subband(30, n_symbols, 12 * W, 8, L, 4096, s + 6 * W, 'sync_ols'))
        s += 12 * W
    return sbs, dict(qam=256, seed=4, io='bf16', snr_db=30.0)


def wideband_slot(mode, n=1024):
    """10 MHz uplink at 15 kHz: one subband of 52 PRB (624 active
    subcarriers) centred at bin 0, an 8-bin transition band on each side,
    L = N = n (I = 1, the channel-filter case: 1024, or the 768 = 3 x 256 of
    the paper's complexity discussion), one 14-symbol slot of 64-QAM; mode
    'cont_ols' or 'sync_ola'."""
    return [subband(15, 14, 624, 8, n, n, 0, mode)], dict(qam=64, seed=6, io='c64')
