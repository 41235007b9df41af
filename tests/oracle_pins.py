"""Pins of the FC oracle against what the paper and the mathematics fix.

Each pin takes the oracle module ``fc`` as an argument (so the mutation test can
run the same pins on deliberately broken copies) and returns a relative error;
the tests require it to be at FP64 rounding level.

Pins (none of them re-types the oracle's formulas):
 * pr1_*   perfect reconstruction with unit weights on all L bins: the output
           sampled on each symbol's low-rate grid, demodulated and scaled by
           sqrt(I), is the input (FC with an all-pass D is ideal periodic
           interpolation; the windows tile the input). Pins phi, theta, Xi,
           sqrt(I), windows and placement.
 * tone_*  a low-rate complex tone at bin kappa yields, in steady state, a
           high-rate tone at c + kappa with amplitude D[kappa + L/2]/sqrt(I)
           (TX) and the reverse with sqrt(I) D (RX). Pins D indexing and shift.
 * lin_i1_* with I = 1 and c = 0, FC with D = DFT of a short Hermitian FIR h is
           textbook overlap-add / overlap-save: exactly np.convolve(x, h).
 * brute_* a tiny case evaluated by explicit loops of the time-domain circular
           convolution form, independent of the DFT matrices.
 * adjoint_* <TX x, y> = <x, RX y> for the three model pairs.
"""
from fractions import Fraction

import numpy as np

from oracle import numerology as nu


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _cvec(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


# ------------------------------------------------------------------ PR-1 --
def pr1_sync(fc, L=16, N=64, c=7, ncp=(8, 4, 4, 8, 4), seed=0):
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N)
    lcp = nu.lowrate_cp(ncp, I, exact=True)
    x = _cvec(rng, sum(L + l for l in lcp))
    y = fc.tx_sync(x, L, N, c, np.ones(L), list(ncp))
    sig = nu.sync_sigma(ncp, N)
    got, pos = [], 0
    for n in range(len(ncp)):
        t = sig[n] + I * (ov.L_L - lcp[n] + np.arange(L + lcp[n]))
        got.append(y[t] * np.exp(-2j * np.pi * c * t / N) * np.sqrt(I))
    return rel(np.concatenate(got), x)


def pr1_cont(fc, ola, L=16, N=64, c=-5, n=75, seed=1, lam=Fraction(1, 2)):
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N, lam)
    x = _cvec(rng, n)
    y = fc.tx_cont(x, L, N, c, np.ones(L), lam=lam, ola=ola)
    t = I * (ov.L_O + np.arange(n))
    return rel(y[t] * np.exp(-2j * np.pi * c * t / N) * np.sqrt(I), x)


# ------------------------------------------------------------------ tones --
def tone_tx(fc, ola=False, L=32, N=128, c=9, seed=2, lam=Fraction(1, 2)):
    """Continuous OLS (exact in steady state for any real D)."""
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N, lam)
    D = rng.uniform(0.1, 1.0, L)
    worst = 0.0
    n = 12 * L
    for kap in (-L // 2, -5, 0, 3, L // 2 - 1):
        x = np.exp(2j * np.pi * kap * np.arange(n) / L)
        y = fc.tx_cont(x, L, N, c, D, lam=lam, ola=ola)
        t = np.arange(len(y))
        ref = (D[kap + L // 2] / np.sqrt(I) * np.exp(2j * np.pi * c * t / N)
               * np.exp(2j * np.pi * kap * (t - I * ov.L_O) / N))
        lo, hi = I * ov.L_O + N, I * (ov.L_O + n) - N
        worst = max(worst, rel(y[lo:hi], ref[lo:hi]))
    return worst


def tone_rx(fc, L=32, N=128, c=-11, seed=3, lam=Fraction(1, 2)):
    """Continuous RX-OLS of a high-rate tone at c + kappa."""
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N, lam)
    D = rng.uniform(0.1, 1.0, L)
    n_x = 12 * L
    Q = nu.cont_output_len(n_x, ov)
    t = np.arange(Q)
    worst = 0.0
    for kap in (-L // 2, -3, 0, 7, L // 2 - 1):
        yh = np.exp(2j * np.pi * (c + kap) * t / N)
        xh = fc.rx_cont(yh, L, N, c, D, n_x, lam=lam, ola=False)
        l = np.arange(n_x)
        ref = np.sqrt(I) * D[kap + L // 2] * np.exp(2j * np.pi * kap * I * (ov.L_O + l) / N)
        sl = slice(L, n_x - L)
        worst = max(worst, rel(xh[sl], ref[sl]))
    return worst


def tone_rx_sync(fc, L=32, N=128, c=5, seed=4):
    """Symbol-synchronised RX of a tone: every useful sample sees the tone."""
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N)
    D = rng.uniform(0.1, 1.0, L)
    ncp = [9, 7, 7, 9]
    Q = nu.sync_output_len(ncp, ov)
    t = np.arange(Q)
    sig = nu.sync_sigma(ncp, N)
    worst = 0.0
    for kap in (-L // 2, -2, 0, 6, L // 2 - 1):
        yh = np.exp(2j * np.pi * (c + kap) * t / N)
        z = fc.rx_sync(yh, L, N, c, D, ncp)
        for n, s in enumerate(sig):
            tt = s + ov.N_L + I * np.arange(L)
            ref = np.sqrt(I) * D[kap + L // 2] * np.exp(2j * np.pi * kap * tt / N)
            worst = max(worst, rel(z[n], ref))
    return worst


# ------------------------------------------------------------- I = 1 ----
def short_fir(rng, L, T):
    """Hermitian FIR h[-T..T] (so its DFT is real) and D in fftshifted order."""
    h = _cvec(rng, T + 1)
    h[0] = h[0].real
    full = np.zeros(2 * T + 1, dtype=complex)
    full[T:] = h
    full[:T] = np.conj(h[1:][::-1])
    kap = np.arange(L) - L // 2
    d = np.arange(-T, T + 1)
    D = np.real(np.exp(-2j * np.pi * np.outer(kap, d) / L) @ full)
    return full, D


def lin_i1_cont(fc, ola, L=32, n=150, T=3, seed=5, lam=Fraction(1, 2)):
    rng = np.random.default_rng(seed)
    h, D = short_fir(rng, L, T)
    ov = nu.Overlap(L, L, lam)
    x = _cvec(rng, n)
    y = fc.tx_cont(x, L, L, 0, D, lam=lam, ola=ola)
    ref = np.zeros(len(y), dtype=complex)
    conv = np.convolve(x, h)            # conv[k] = sum x[l] h[k - l - ... ] with h at -T
    ref[ov.L_O - T:ov.L_O - T + len(conv)] = conv
    # OLS only produces output inside the keep windows; compare where defined
    if ola:
        return rel(y, ref)
    lo, hi = ov.N_L, len(y) - ov.N_T
    return rel(y[lo:hi], ref[lo:hi])


def lin_i1_sync(fc, L=32, T=2, seed=6):
    rng = np.random.default_rng(seed)
    h, D = short_fir(rng, L, T)
    ncp = [4, 3, 3, 4, 3]                 # I = 1: N_CP = L_CP, and L_CP <= L/4 - T
    ov = nu.Overlap(L, L)
    x = _cvec(rng, sum(L + c for c in ncp))
    y = fc.tx_sync(x, L, L, 0, D, ncp)
    conv = np.convolve(x, h)
    ref = np.zeros(len(y), dtype=complex)
    start = ov.N_L - ncp[0] - T          # first CP sample at N_L - N_CP,0
    ref[start:start + len(conv)] = conv
    return rel(y, ref)


# ---------------------------------------------------------- brute force --
def brute_cont(fc, ola, L=8, N=32, c=3, n=21, seed=7):
    """y_blk[tau] = sqrt(I) phi_r exp(j2pi c tau/N) sum_i s[i] g0[(tau - I i) mod N],
    g0[d] = (1/N) sum_p D[p] exp(j2pi (p - L/2) d / N); explicit loops."""
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N)
    D = rng.uniform(-1.0, 1.0, L)
    x = _cvec(rng, n)
    R = nu.cont_block_count(n, ov)
    u = np.zeros((R - 1) * ov.L_S + L, dtype=complex)
    u[ov.L_O:ov.L_O + n] = x
    g0 = np.zeros(N, dtype=complex)
    for d in range(N):
        for p in range(L):
            g0[d] += D[p] * np.exp(2j * np.pi * (p - L // 2) * d / N) / N
    y = np.zeros(nu.cont_output_len(n, ov), dtype=complex)
    for r in range(R):
        s = u[r * ov.L_S:r * ov.L_S + L].copy()
        if ola:
            s[:ov.L_L] = 0
            s[L - ov.L_T:] = 0
        phi = np.exp(2j * np.pi * r * c * ov.L_S / L)
        for tau in range(N):
            if not ola and not (ov.N_L <= tau < ov.N_L + ov.N_S):
                continue
            acc = 0j
            for i in range(L):
                acc += s[i] * g0[(tau - I * i) % N]
            y[r * ov.N_S + tau] += np.sqrt(I) * phi * np.exp(2j * np.pi * c * tau / N) * acc
    return rel(fc.tx_cont(x, L, N, c, D, ola=ola), y)


def brute_sync(fc, L=8, N=32, c=-3, ncp=(6, 5, 5), seed=8):
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N)
    D = rng.uniform(-1.0, 1.0, L)
    lcp = [v // I for v in ncp]
    x = _cvec(rng, sum(L + v for v in lcp))
    g0 = np.zeros(N, dtype=complex)
    for d in range(N):
        for p in range(L):
            g0[d] += D[p] * np.exp(2j * np.pi * (p - L // 2) * d / N) / N
    sig = [0]
    for v in ncp[1:]:
        sig.append(sig[-1] + N + v)
    y = np.zeros(sig[-1] + 3 * N // 2, dtype=complex)
    pos = 0
    for n in range(len(ncp)):
        S_L = L // 4 - lcp[n]
        z = np.zeros(3 * L // 2, dtype=complex)
        z[S_L:S_L + L + lcp[n]] = x[pos:pos + L + lcp[n]]
        pos += L + lcp[n]
        for r in (0, 1):
            s = z[r * L // 2:r * L // 2 + L].copy()
            if r == 0:
                s[L - L // 4:] = 0          # tail zeros; leading S_L already zero
            else:
                s[:L // 4] = 0
                s[L - L // 4:] = 0
            for tau in range(N):
                acc = 0j
                for i in range(L):
                    acc += s[i] * g0[(tau - I * i) % N]
                t = sig[n] + r * N // 2 + tau
                y[t] += np.sqrt(I) * np.exp(2j * np.pi * c * t / N) * acc
    return rel(fc.tx_sync(x, L, N, c, D, list(ncp)), y)


def pr1_sync_ols(fc, L=16, N=64, c=7, ncp=(8, 4, 4, 8, 4), seed=10):
    """Synchronised OLS TX with unit weights on all L bins: every kept output
    sample on the symbol's low-rate grid is the input sample (each block is
    an ideal periodic interpolator; the kept windows tile the symbols)."""
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N)
    lcp = nu.lowrate_cp(ncp, I, exact=True)
    x = _cvec(rng, sum(L + l for l in lcp))
    y = fc.tx_sync_ols(x, L, N, c, np.ones(L), list(ncp))
    sig = nu.sync_sigma(ncp, N)
    got = []
    for n in range(len(ncp)):
        t = sig[n] + I * (ov.L_L - lcp[n] + np.arange(L + lcp[n]))
        got.append(y[t] * np.exp(-2j * np.pi * c * t / N) * np.sqrt(I))
    return rel(np.concatenate(got), x)


def brute_sync_ols(fc, L=8, N=32, c=5, ncp=(6, 5, 5), seed=11, taper=0):
    """Explicit loops of the time-domain circular convolution per block, the
    output windows applied sample by sample. With a taper of T samples the
    first block's output before its kept range and the second block's after
    it are kept too, T/2 samples each side of the edge, weighted by the
    cross-fade weight w(k) = sin^2(pi (k + 1/2) / (2T)) (k counted along the
    edge in time), its mirror 1 - w(k) on the falling edge."""
    rng = np.random.default_rng(seed)
    h = taper // 2
    I = N // L
    D = rng.uniform(-1.0, 1.0, L)
    lcp = [v // I for v in ncp]
    x = _cvec(rng, sum(L + v for v in lcp))
    g0 = np.zeros(N, dtype=complex)
    for d in range(N):
        for p in range(L):
            g0[d] += D[p] * np.exp(2j * np.pi * (p - L // 2) * d / N) / N
    sig = [0]
    for v in ncp[1:]:
        sig.append(sig[-1] + N + v)
    y = np.zeros(sig[-1] + 3 * N // 2, dtype=complex)
    pos = 0
    for n in range(len(ncp)):
        z = np.zeros(3 * L // 2, dtype=complex)
        z[L // 4 - lcp[n]:L // 4 - lcp[n] + L + lcp[n]] = x[pos:pos + L + lcp[n]]
        pos += L + lcp[n]
        for r in (0, 1):
            s = z[r * L // 2:r * L // 2 + L]
            lo = N // 4 - (ncp[n] if r == 0 else 0)
            start, stop = (lo - h, 3 * N // 4) if r == 0 else (lo, 3 * N // 4 + h)
            for tau in range(start, stop):
                acc = 0j
                for i in range(L):
                    acc += s[i] * g0[(tau - I * i) % N]
                wgt = 1.0
                if r == 0 and tau < lo + h:
                    wgt = np.sin(np.pi * (tau - (lo - h) + 0.5) / (2 * taper)) ** 2
                if r == 1 and tau >= 3 * N // 4 - h:
                    wgt = 1.0 - np.sin(np.pi * (tau - (3 * N // 4 - h) + 0.5) / (2 * taper)) ** 2
                t = sig[n] + r * N // 2 + tau
                y[t] += wgt * np.sqrt(I) * np.exp(2j * np.pi * c * t / N) * acc
    return rel(fc.tx_sync_ols(x, L, N, c, D, list(ncp), taper=taper) if taper else
               fc.tx_sync_ols(x, L, N, c, D, list(ncp)), y)


def taper_interior(fc, L=16, N=64, c=-5, ncp=(9, 5, 6, 7), T=6, seed=12):
    """Tapering changes nothing outside the T-sample edges around the symbol
    boundaries, and the falling and rising edges of neighbouring symbols
    cross-fade to one (rising + mirrored rising = 1)."""
    rng = np.random.default_rng(seed)
    I = N // L
    D = rng.uniform(-1.0, 1.0, L)
    lcp = nu.lowrate_cp(list(ncp), I, exact=False)
    x = _cvec(rng, sum(L + v for v in lcp))
    y0 = fc.tx_sync_ols(x, L, N, c, D, list(ncp))
    y1 = fc.tx_sync_ols(x, L, N, c, D, list(ncp), taper=T)
    sig = nu.sync_sigma(list(ncp), N)
    edge = np.zeros(len(y0), dtype=bool)
    for n in range(len(ncp)):
        for e in (sig[n] + N // 4 - ncp[n], sig[n] + N // 2 + 3 * N // 4):
            edge[e - T // 2:e + T // 2] = True
    w = fc.taper_ramp(T)
    return rel(y1[~edge], y0[~edge]) + float(np.max(np.abs(w + w[::-1] - 1.0)))


# -------------------------------------------------------------- adjoints --
def adjoint_cont(fc, tx_ola, L=16, N=64, c=6, n=70, seed=9, lam=Fraction(1, 2)):
    rng = np.random.default_rng(seed)
    D = rng.uniform(-1.0, 1.0, L)
    x = _cvec(rng, n)
    y = fc.tx_cont(x, L, N, c, D, lam=lam, ola=tx_ola)
    w = _cvec(rng, len(y))
    xa = fc.rx_cont(w, L, N, c, D, n, lam=lam, ola=not tx_ola)
    lhs, rhs = np.vdot(w, y), np.vdot(xa, x)
    return abs(lhs - rhs) / abs(lhs)


def adjoint_sync(fc, L=16, N=64, c=-6, ncp=(9, 5, 6, 7), seed=10):
    rng = np.random.default_rng(seed)
    D = rng.uniform(-1.0, 1.0, L)
    lcp = nu.lowrate_cp(ncp, N // L, exact=False)
    x = _cvec(rng, sum(L + v for v in lcp))
    y = fc.tx_sync(x, L, N, c, D, list(ncp))
    w = _cvec(rng, len(y))
    xa = fc.rx_sync(w, L, N, c, D, list(ncp), keep_cp=True)
    lhs, rhs = np.vdot(w, y), np.vdot(xa, x)
    return abs(lhs - rhs) / abs(lhs)


def concat_sync_vs_keepcp(fc, L=16, N=64, c=4, ncp=(9, 5, 6), seed=11):
    """The CP-free RX output is the useful part of the adjoint (keep-CP) output."""
    rng = np.random.default_rng(seed)
    D = rng.uniform(-1.0, 1.0, L)
    lcp = nu.lowrate_cp(ncp, N // L, exact=False)
    ov = nu.Overlap(L, N)
    Q = nu.sync_output_len(ncp, ov)
    w = _cvec(rng, Q)
    a = fc.rx_sync(w, L, N, c, D, list(ncp))
    b = fc.rx_sync(w, L, N, c, D, list(ncp), keep_cp=True)
    parts, pos = [], 0
    for v in lcp:
        parts.append(b[pos + v:pos + v + L])
        pos += L + v
    return rel(a, np.stack(parts))


# ------------------------------------------- RX with OFDM demodulation ----
def tone_rx_subcarriers(fc, L=32, N=128, c=5, seed=6):
    """A tone at long bin c + kappa, demodulated per symbol (Sec. IV): one
    nonzero subcarrier, kappa mod L, of value sqrt(L I) D[kappa + L/2] times
    the tone's phase at the symbol's first useful high-rate sample."""
    rng = np.random.default_rng(seed)
    I = N // L
    ov = nu.Overlap(L, N)
    D = rng.uniform(0.1, 1.0, L)
    ncp = [9, 7, 7, 9]
    Q = nu.sync_output_len(ncp, ov)
    t = np.arange(Q)
    sig = nu.sync_sigma(ncp, N)
    worst = 0.0
    for kap in (-L // 2, -3, 0, 5, L // 2 - 1):
        yh = np.exp(2j * np.pi * (c + kap) * t / N)
        X = fc.rx_sync_subcarriers(yh, L, N, c, D, ncp)
        for n, s in enumerate(sig):
            ref = np.zeros(L, dtype=complex)
            ref[kap % L] = np.sqrt(L * I) * D[kap + L // 2] * np.exp(2j * np.pi * kap * (s + ov.N_L) / N)
            worst = max(worst, rel(X[n], ref))
    return worst


def reduced_vs_direct(fc, seed=7):
    """Sec. V-A: the simplified processing (one IFFT and one FFT per symbol)
    equals the direct one (two IFFTs, concatenation, FFT) on arbitrary input."""
    rng = np.random.default_rng(seed)
    worst = 0.0
    for L, N, c, ncp in ((16, 64, 7, [9, 5, 6]), (32, 128, -11, [20, 18, 18]), (64, 256, 40, [36, 20, 20])):
        ov = nu.Overlap(L, N)
        Q = nu.sync_output_len(ncp, ov)
        yh = _cvec(rng, Q)
        D = rng.uniform(-1.0, 1.0, L)
        worst = max(worst, rel(fc.rx_sync_subcarriers_reduced(yh, L, N, c, D, ncp),
                               fc.rx_sync_subcarriers(yh, L, N, c, D, ncp)))
    return worst


# ----------------------------------------------------- OFDM modulation ----
def ofdm_round_trip(fc, seed=8):
    """Demodulating each modulated symbol (CP dropped) with the forward DFT
    returns the grid on its subcarriers and zeros elsewhere."""
    rng = np.random.default_rng(seed)
    worst = 0.0
    for L, K, lcp in ((16, 12, [2, 1, 1]), (64, 40, [5, 4, 4]), (128, 96, [10, 9])):
        grid = rng.standard_normal((len(lcp), K)) + 1j * rng.standard_normal((len(lcp), K))
        x = fc.ofdm_modulate(grid, L, lcp)
        pos = 0
        for n, l in enumerate(lcp):
            sym = x[pos + l:pos + l + L]
            assert np.allclose(x[pos:pos + l], sym[L - l:])            # cyclic prefix
            X = np.exp(-2j * np.pi * np.outer(np.arange(L), np.arange(L)) / L) @ sym / np.sqrt(L)
            ref = np.zeros(L, dtype=complex)
            ref[np.arange(-K // 2, K // 2) % L] = grid[n]
            worst = max(worst, rel(X, ref))
            pos += l + L
    return worst


def ofdm_vs_numpy_fft(fc, seed=9):
    """Cross-check of the dense-matrix modulator against numpy's FFT."""
    rng = np.random.default_rng(seed)
    L, K, lcp = 32, 24, [3, 2]
    grid = rng.standard_normal((2, K)) + 1j * rng.standard_normal((2, K))
    X = np.zeros((2, L), dtype=complex)
    X[:, np.arange(-K // 2, K // 2) % L] = grid
    xs = np.fft.ifft(X, axis=1) * np.sqrt(L)
    ref = np.concatenate([np.r_[xs[n][L - lcp[n]:], xs[n]] for n in range(2)])
    return rel(fc.ofdm_modulate(grid, L, lcp), ref)


ALL_PINS = {
    "pr1_sync": lambda fc: pr1_sync(fc),
    "pr1_cont_ols": lambda fc: pr1_cont(fc, False),
    "pr1_cont_ola": lambda fc: pr1_cont(fc, True),
    "pr1_cont_ola_quarter": lambda fc: pr1_cont(fc, True, L=32, N=128, lam=Fraction(1, 4)),
    "tone_tx": lambda fc: tone_tx(fc),
    "tone_rx": lambda fc: tone_rx(fc),
    "tone_rx_quarter": lambda fc: tone_rx(fc, lam=Fraction(1, 4)),
    "tone_tx_quarter": lambda fc: tone_tx(fc, L=32, N=128, c=-7, lam=Fraction(1, 4)),
    "tone_rx_sync": lambda fc: tone_rx_sync(fc),
    "lin_i1_ola": lambda fc: lin_i1_cont(fc, True),
    "lin_i1_ols": lambda fc: lin_i1_cont(fc, False),
    "lin_i1_sync": lambda fc: lin_i1_sync(fc),
    "brute_ola": lambda fc: brute_cont(fc, True),
    "brute_ols": lambda fc: brute_cont(fc, False),
    "brute_sync": lambda fc: brute_sync(fc),
    "adjoint_txola_rxols": lambda fc: adjoint_cont(fc, True),
    "adjoint_txols_rxola": lambda fc: adjoint_cont(fc, False),
    "adjoint_quarter_ola": lambda fc: adjoint_cont(fc, True, L=32, N=128, c=5, lam=Fraction(1, 4)),
    "adjoint_quarter_ols": lambda fc: adjoint_cont(fc, False, L=32, N=128, c=-9, lam=Fraction(1, 4)),
    "adjoint_sync": lambda fc: adjoint_sync(fc),
    "concat_vs_keepcp": lambda fc: concat_sync_vs_keepcp(fc),
    "tone_rx_subcarriers": lambda fc: tone_rx_subcarriers(fc),
    "reduced_vs_direct": lambda fc: reduced_vs_direct(fc),
    "ofdm_round_trip": lambda fc: ofdm_round_trip(fc),
    "ofdm_vs_numpy_fft": lambda fc: ofdm_vs_numpy_fft(fc),
    "pr1_sync_ols": lambda fc: pr1_sync_ols(fc),
    "brute_sync_ols": lambda fc: brute_sync_ols(fc),
    "brute_sync_ols_taper": lambda fc: brute_sync_ols(fc, taper=4),
    "taper_interior": lambda fc: taper_interior(fc),
    # transform lengths that are not powers of two (3 x 2^k, as the paper's
    # 768 = 3 x 256 short transform, Sec. VI-C): the same pins at L = 24
    # (N = 96) and, for the brute-force loops, L = 12 (N = 48)
    "pr1_sync_l24": lambda fc: pr1_sync(fc, L=24, N=96, c=7, ncp=(20, 16, 16, 20, 16)),
    "pr1_cont_ols_l24": lambda fc: pr1_cont(fc, False, L=24, N=96),
    "pr1_cont_ola_l24": lambda fc: pr1_cont(fc, True, L=24, N=96),
    "tone_tx_l24": lambda fc: tone_tx(fc, L=24, N=96, c=9),
    "tone_rx_l24": lambda fc: tone_rx(fc, L=24, N=96, c=-11),
    "tone_rx_sync_l24": lambda fc: tone_rx_sync(fc, L=24, N=96),
    "lin_i1_ols_l24": lambda fc: lin_i1_cont(fc, False, L=24),
    "lin_i1_ola_l24": lambda fc: lin_i1_cont(fc, True, L=24),
    "lin_i1_sync_l24": lambda fc: lin_i1_sync(fc, L=24),
    "brute_ola_l12": lambda fc: brute_cont(fc, True, L=12, N=48),
    "brute_ols_l12": lambda fc: brute_cont(fc, False, L=12, N=48),
    "brute_sync_l12": lambda fc: brute_sync(fc, L=12, N=48),
    "adjoint_sync_l24": lambda fc: adjoint_sync(fc, L=24, N=96),
    "adjoint_cont_l24": lambda fc: adjoint_cont(fc, True, L=24, N=96),
    "tone_rx_subcarriers_l24": lambda fc: tone_rx_subcarriers(fc, L=24, N=96),
}
TOL = 1e-10
