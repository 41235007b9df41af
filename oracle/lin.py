"""Plain reference: direct linear convolution with one centred period of the
FC kernel, i.e. what the block-wise FC approximates (Sec. I and II: FC
approximates linear convolution through block-wise circular convolutions).

Test infrastructure only (see ``oracle/__init__``).

Pinned (tests/lin_metric_pins.py): textbook convolution at I = 1 (continuous
and per symbol), the steady-state tone response at I > 1, the synchronised
form as a sum of shifted single-symbol continuous forms, and both receivers
as exact adjoints of their transmitters.

The FC block with real weights D, centre bin c and interpolation I applies, in
its own time axis, y[tau] = sqrt(I) exp(j2pi c tau/N) sum_i s[i] g0[(tau - I i) mod N]
with the N-periodic kernel g0[d] = (1/N) sum_p D[p] exp(j2pi (p - L/2) d / N).
The plain reference uses one centred period d in [-N/2, N/2) of g0 as an FIR
filter on the I-fold zero-stuffed input, with the carrier in global time.
"""
from fractions import Fraction

import numpy as np

from .numerology import Overlap, cont_output_len, lowrate_cp, sync_sigma, sync_output_len


def prototype(L, N, D):
    """g0[d] for d = -N/2 .. N/2-1 (array index d + N/2)."""
    D = np.asarray(D, dtype=float)
    d = np.arange(-N // 2, N // 2)
    kappa = np.arange(L) - (-(-L // 2))
    return (np.exp(2j * np.pi * np.outer(d, kappa) / N) @ D) / N


def _carrier(c, N, t):
    return np.exp(2j * np.pi * ((c * t) % N) / N)


def _filter_stuffed(v, g0, N, length):
    """(v * g0)[t] for t in [0, length), g0 centred at array index N/2."""
    full = np.convolve(v, g0)
    out = np.zeros(length, dtype=complex)
    seg = full[N // 2:N // 2 + length]
    out[:len(seg)] = seg
    return out


def tx_cont_lin(x, L, N, c, D, lam=Fraction(1, 2)):
    """x[l] sits at t_l = I (l + L_O); output length as the continuous FC."""
    ov = Overlap(L, N, lam)
    Q = cont_output_len(len(x), ov)
    v = np.zeros(Q, dtype=complex)
    v[ov.I * (ov.L_O + np.arange(len(x)))] = x
    t = np.arange(Q)
    return np.sqrt(ov.I) * _carrier(c, N, t) * _filter_stuffed(v, prototype(L, N, D), N, Q)


def _sync_positions(L, ov, ncp):
    lcp = lowrate_cp(ncp, ov.I, exact=False)
    sigma = sync_sigma(ncp, ov.N)
    pos = []
    for n, lc in enumerate(lcp):
        S_L = ov.L_L - lc
        pos.append(sigma[n] + ov.I * (S_L + np.arange(L + lc)))
    return pos, sigma


def tx_sync_lin(x, L, N, c, D, ncp):
    """Symbol n's sample l sits at sigma_n + I (S_L,n + l) (its own grid)."""
    ov = Overlap(L, N, Fraction(1, 2))
    Q = sync_output_len(ncp, ov)
    pos, _ = _sync_positions(L, ov, ncp)
    v = np.zeros(Q, dtype=complex)
    v[np.concatenate(pos)] = x
    t = np.arange(Q)
    return np.sqrt(ov.I) * _carrier(c, N, t) * _filter_stuffed(v, prototype(L, N, D), N, Q)


def rx_cont_lin(yh, L, N, c, D, n_x, lam=Fraction(1, 2)):
    """Adjoint of ``tx_cont_lin``: demodulate, filter, sample at t_l."""
    ov = Overlap(L, N, lam)
    t = np.arange(len(yh))
    f = _filter_stuffed(np.conj(_carrier(c, N, t)) * yh, prototype(L, N, D), N, len(yh))
    return np.sqrt(ov.I) * f[ov.I * (ov.L_O + np.arange(n_x))]


def rx_sync_lin(yh, L, N, c, D, ncp):
    """Filtered, demodulated input sampled on each symbol's useful-part grid
    sigma_n + N_L + I l, l in [0, L): the CP-free symbols, shape (B, L)."""
    ov = Overlap(L, N, Fraction(1, 2))
    t = np.arange(len(yh))
    f = _filter_stuffed(np.conj(_carrier(c, N, t)) * yh, prototype(L, N, D), N, len(yh))
    sigma = sync_sigma(ncp, N)
    return np.stack([np.sqrt(ov.I) * f[s + ov.N_L + ov.I * np.arange(L)] for s in sigma])
