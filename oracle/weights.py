"""Frequency-domain window weights D (oracle side).

Test infrastructure only (see ``oracle/__init__``).

Sec. III-B defines D as a real diagonal of subband weights with passband,
transition-band and stop-band values; the paper takes optimised transition
weights from earlier work and does not print them. Reading used here: a
raised-cosine transition of n_tb bins per side,
w_i = (1 + cos(pi i / (n_tb + 1))) / 2 for i = 1..n_tb counted outward from
the passband, unit weight on the K active bins kappa in [-K/2, K/2), zero
elsewhere. Output is in fftshifted order: index p = kappa + L/2.
"""
import numpy as np


def rc_transition(n_tb):
    i = np.arange(1, n_tb + 1)
    return 0.5 * (1.0 + np.cos(np.pi * i / (n_tb + 1)))


def rc_weights(L, K, n_tb):
    if K % 2 or K + 2 * n_tb > L:
        raise ValueError("need even K and K + 2 n_tb <= L")
    D = np.zeros(L)
    half = L // 2
    D[half - K // 2:half + K // 2] = 1.0
    w = rc_transition(n_tb)
    for i in range(1, n_tb + 1):
        D[half + K // 2 - 1 + i] = w[i - 1]     # kappa = K/2 - 1 + i
        D[half - K // 2 - i] = w[i - 1]         # kappa = -K/2 - i
    return D
