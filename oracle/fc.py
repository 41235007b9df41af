"""Exact fast-convolution (FC) method in FP64: literal evaluation of the
paper's block matrices. This is the parity reference for the GPU path.

Test infrastructure only (see ``oracle/__init__``). No FFTs: every DFT is a
dense matrix with integer-reduced exponents, W_n[k, l] = exp(-j2pi((k*l) mod n)/n),
and W_n^{-1} = conj(W_n)/n (Sec. III-B).

Conventions fixed by this oracle (readings of the paper where it is silent):
 * bins are 0-based: Xi(p) = (c - ceil(L/2) + p) mod N; c may be negative;
 * the weights D are real and indexed in fftshifted order (p = kappa + L/2);
 * TX scale sqrt(I) (Sec. III-B, first equation of the continuous SFB);
 * RX uses conj(phi_r*theta_n) and scale 1/sqrt(I), which makes every RX
   model the exact Hermitian adjoint of the matching TX model (Sec. IV states
   G = conj(F)^T; the factor I that W^{-1} = conj(W)/n introduces is absorbed
   by the scale);
 * theta_n = exp(j2pi c sigma_n / N) (Sec. III-C writes it for N_OFDM = N);
 * each subband's output lives in its own local time axis; ``place`` puts
   several of them on a common stream.
"""
from fractions import Fraction
from functools import lru_cache

import numpy as np

from .numerology import (Overlap, cont_block_count, cont_output_len, lowrate_cp,
                         sync_sigma, sync_output_len)


# ---------------------------------------------------------------- matrices --
@lru_cache(maxsize=16)
def dft_matrix(n):
    """W_n with W_n[k, l] = exp(-j 2 pi ((k l) mod n) / n)."""
    k = np.arange(n, dtype=np.int64)
    e = np.outer(k, k) % n
    w = np.exp(-2j * np.pi * e / n)
    w.setflags(write=False)
    return w


@lru_cache(maxsize=16)
def idft_matrix(n):
    """W_n^{-1} = conj(W_n) / n."""
    w = np.conj(dft_matrix(n)) / n
    w.setflags(write=False)
    return w


def unit_phase(num, den):
    """exp(j 2 pi num/den) with the integer argument reduced mod den first."""
    return np.exp(2j * np.pi * (num % den) / den)


def shift_matrix(L):
    """DFT shift P^(L/2), the circulant permutation of Sec. III-B:
    [[0_{floor(L/2) x ceil(L/2)}, I_floor(L/2)], [I_ceil(L/2), 0]]."""
    fl, cl = L // 2, -(-L // 2)
    P = np.zeros((L, L))
    P[:fl, cl:] = np.eye(fl)
    P[fl:, :cl] = np.eye(cl)
    return P


def xi(L, N, c):
    """0-based bin map Xi(p) = (c - ceil(L/2) + p) mod N (Sec. III-B)."""
    return (c - (-(-L // 2)) + np.arange(L)) % N


def mapping_matrix(L, N, c, phi=1.0):
    """M(phi) in C^{N x L}: [M]_{q,p} = phi if Xi(p) = q (Sec. III-B)."""
    M = np.zeros((N, L), dtype=complex)
    M[xi(L, N, c), np.arange(L)] = phi
    return M


def block_core(L, N, c, D):
    """T = W_N^{-1} M(1) D P^(L/2) W_L, an N x L matrix.

    M(1) has exactly one unit entry per column, in row Xi(p), so W_N^{-1} M(1)
    equals the columns Xi(p) of W_N^{-1}; tests check this against the dense
    mapping matrix at small sizes.
    """
    D = np.asarray(D, dtype=float)
    inner = D[:, None] * (shift_matrix(L) @ dft_matrix(L))
    return idft_matrix(N)[:, xi(L, N, c)] @ inner


def block_core_rx(L, N, c, D):
    """W_L^{-1} P^(-L/2) D M(1)^T W_N, an L x N matrix (Sec. IV)."""
    D = np.asarray(D, dtype=float)
    Pinv = shift_matrix(L).T                      # P^(-L/2) = (P^(L/2))^-1
    left = idft_matrix(L) @ Pinv * D[None, :]
    return left @ dft_matrix(N)[xi(L, N, c), :]


# ---------------------------------------------------------------- windows --
def window_low(ov):
    """a = [0_{L_L}; 1_{L_S}; 0_{L_T}] (OLA analysis, and RX-OLS synthesis)."""
    return np.r_[np.zeros(ov.L_L), np.ones(ov.L_S), np.zeros(ov.L_T)]


def window_high(ov):
    """s = [0_{N_L}; 1_{N_S}; 0_{N_T}] (OLS synthesis, and RX-OLA analysis)."""
    return np.r_[np.zeros(ov.N_L), np.ones(ov.N_S), np.zeros(ov.N_T)]


# ------------------------------------------------------------- continuous --
def tx_cont(x, L, N, c, D, lam=Fraction(1, 2), ola=False):
    """Continuous FC synthesis of one subband (Sec. III-B).

    w = sqrt(I) F [0_{L_O}; x; 0_{L_O}] with F block diagonal over R
    overlapping blocks: block r reads u[r L_S : r L_S + L] and its output is
    placed at r N_S. OLA: F_r = W_N^{-1} M(phi_r) D P W_L A. OLS:
    F_r = S W_N^{-1} M(phi_r) D P W_L. phi_r = exp(j 2 pi r c L_S / L).
    Returns the high-rate output of length (R-1) N_S + N.
    """
    ov = Overlap(L, N, lam)
    x = np.asarray(x, dtype=complex)
    R = cont_block_count(len(x), ov)
    # zero padding by L_O at both ends (extra zeros at the end only make room
    # for the last block)
    u = np.zeros((R - 1) * ov.L_S + L, dtype=complex)
    u[ov.L_O:ov.L_O + len(x)] = x
    T = block_core(L, N, c, D)
    a, s = window_low(ov), window_high(ov)
    y = np.zeros(cont_output_len(len(x), ov), dtype=complex)
    segs = np.stack([u[r * ov.L_S:r * ov.L_S + L] for r in range(R)], axis=1)
    if ola:
        segs = segs * a[:, None]
    blocks = T @ segs
    for r in range(R):
        phi = unit_phase(r * c * ov.L_S, L)
        yb = np.sqrt(ov.I) * phi * blocks[:, r]
        if not ola:
            yb = s * yb
        y[r * ov.N_S:r * ov.N_S + N] += yb
    return y


def rx_cont(yh, L, N, c, D, n_x, lam=Fraction(1, 2), ola=False):
    """Continuous FC analysis of one subband (Sec. IV), the adjoint of
    ``tx_cont`` with the other combining model.

    Block r takes yh[r N_S : r N_S + N]. RX-OLS: z_r = S G_r(phi_r) w_r with the
    low-rate window S = [0_{L_L}; 1_{L_S}; 0_{L_T}]. RX-OLA: z_r = G_r A w_r
    with the high-rate window A = [0_{N_L}; 1_{N_S}; 0_{N_T}]. Blocks add at
    r L_S in the padded low-rate axis; returns the n_x samples after the L_O
    leading padding.
    """
    ov = Overlap(L, N, lam)
    yh = np.asarray(yh, dtype=complex)
    R = cont_block_count(n_x, ov)
    Q = cont_output_len(n_x, ov)
    if len(yh) != Q:
        raise ValueError("high-rate input must have length (R-1) N_S + N")
    G = block_core_rx(L, N, c, D)
    a, s = window_low(ov), window_high(ov)
    blks = np.stack([yh[r * ov.N_S:r * ov.N_S + N] for r in range(R)], axis=1)
    if ola:
        blks = blks * s[:, None]
    z = G @ blks
    u = np.zeros((R - 1) * ov.L_S + L, dtype=complex)
    for r in range(R):
        phi = np.conj(unit_phase(r * c * ov.L_S, L))
        zr = phi * z[:, r] / np.sqrt(ov.I)
        if not ola:
            zr = a * zr
        u[r * ov.L_S:r * ov.L_S + L] += zr
    return u[ov.L_O:ov.L_O + n_x]


# ----------------------------------------------------------- synchronised --
def split_symbols(x, L, lcp):
    """Cut a concatenated CP-OFDM stream into its symbols."""
    out, pos = [], 0
    for lc in lcp:
        out.append(np.asarray(x[pos:pos + L + lc], dtype=complex))
        pos += L + lc
    if pos != len(x):
        raise ValueError("input length does not match the CP schedule")
    return out


def tx_sync(x, L, N, c, D, ncp):
    """Symbol-synchronised OLA FC synthesis (Sec. III-C to III-E).

    Per symbol n: truncated low-rate CP L_CP,n = floor(N_CP,n / I); zero padding
    z = [0_{S_L,n}; x_CP,n; 0_{L_T}] with S_L,n = L_L - L_CP,n (length 3L/2);
    two segments z^(r) = R_L^(r)T z with analysis windows
    a_0 = [0_{S_L,n}; 1_{L_S + L_CP,n}; 0_{L_T}] and a_1 = [0_{L_L}; 1_{L_S}; 0_{L_T}];
    w^(r) = sqrt(I) F^(OLA)_r(phi_r theta_n) z^(r) with
    theta_n = exp(j 2 pi c sigma_n / N); w_n = sum_r R_N^(r) w^(r) (length 3N/2);
    then the symbol-wise OLA w = sum_n Gamma_{sigma_n} w_n over Q samples.
    """
    ov = Overlap(L, N, Fraction(1, 2))
    lcp = lowrate_cp(ncp, ov.I, exact=False)
    if any(lc > ov.L_L for lc in lcp):
        raise ValueError("low-rate CP longer than the leading overlap L_L")
    syms = split_symbols(x, L, lcp)
    sigma = sync_sigma(ncp, N)            # N_OFDM = I * L_OFDM = N
    y = np.zeros(sync_output_len(ncp, ov), dtype=complex)
    T = block_core(L, N, c, D)
    for n, xs in enumerate(syms):
        S_L = ov.L_L - lcp[n]
        z = np.r_[np.zeros(S_L), xs, np.zeros(ov.L_T)]
        a = [np.r_[np.zeros(S_L), np.ones(ov.L_S + lcp[n]), np.zeros(ov.L_T)],
             window_low(ov)]
        theta = unit_phase(c * sigma[n], N)
        wn = np.zeros(3 * N // 2, dtype=complex)
        for r in (0, 1):
            seg = z[r * L // 2:r * L // 2 + L] * a[r]
            phi = unit_phase(r * c * ov.L_S, L)
            wn[r * N // 2:r * N // 2 + N] += np.sqrt(ov.I) * phi * theta * (T @ seg)
        y[sigma[n]:sigma[n] + 3 * N // 2] += wn
    return y


def taper_ramp(T):
    """Rising edge of T samples, w_i = sin^2(pi (i + 1/2) / (2T)), i = 0..T-1.
    Sec. III-D asks for a smooth edge without giving its shape; this raised
    cosine is symmetric about its midpoint, so the falling edge w_{T-1-i}
    equals 1 - w_i and the two edges of neighbouring symbols cross-fade.
    The shape itself is a reading: pinned only through that cross-fade
    property and the leakage it removes (parity unpinned beyond them)."""
    i = np.arange(T)
    return np.sin(np.pi * (i + 0.5) / (2 * T)) ** 2


def tx_sync_ols(x, L, N, c, D, ncp, taper=0):
    """Symbol-synchronised OLS FC synthesis (Sec. III-D, the alternative to
    the OLA scheme): the two blocks of each symbol are not windowed on the
    input side; instead each filtered block is windowed after the
    convolution so that only one block is non-zero in the overlap:
    s_0 = [0_{N_L - N_CP,n}; 1_{N_S + N_CP,n}; 0_{N_T}] and
    s_1 = [0_{N_L}; 1_{N_S}; 0_{N_T}]. The filtered symbols are then combined
    symbol-wise at sigma_n as in the OLA scheme; their kept ranges tile the
    output.

    taper = T > 0 (even) smooths the symbol's outer edges, the rising edge of
    s_0 and the falling edge of s_1 (Sec. III-D): each becomes the ramp of
    ``taper_ramp`` over the T samples centred on the hard edge, so the
    falling edge of one symbol and the rising edge of the next overlap and
    add. Needs T/2 <= N_L - N_CP,n and T/2 <= N_T."""
    ov = Overlap(L, N, Fraction(1, 2))
    lcp = lowrate_cp(ncp, ov.I, exact=False)
    if any(lc > ov.L_L for lc in lcp):
        raise ValueError("low-rate CP longer than the leading overlap L_L")
    if taper % 2 or taper < 0 or taper // 2 > ov.N_T or any(taper // 2 > ov.N_L - v for v in ncp):
        raise ValueError("taper must be even and fit the leading and trailing overlaps")
    syms = split_symbols(x, L, lcp)
    sig = sync_sigma(ncp, N)
    out = np.zeros(sync_output_len(ncp, ov), dtype=complex)
    T = block_core(L, N, c, D)
    ramp, h = taper_ramp(taper), taper // 2
    for n, xs in enumerate(syms):
        zpad = np.r_[np.zeros(ov.L_L - lcp[n]), xs, np.zeros(ov.L_T)]
        s_win = [np.r_[np.zeros(ov.N_L - ncp[n]), np.ones(ov.N_S + ncp[n]), np.zeros(ov.N_T)],
                 np.r_[np.zeros(ov.N_L), np.ones(ov.N_S), np.zeros(ov.N_T)]]
        if taper:
            e0, e1 = ov.N_L - ncp[n], ov.N_L + ov.N_S      # the hard edges being smoothed
            s_win[0][e0 - h:e0 + h] = ramp
            s_win[1][e1 - h:e1 + h] = ramp[::-1]
        th = unit_phase(c * sig[n], N)
        for r in (0, 1):
            blk = T @ zpad[r * L // 2:r * L // 2 + L]
            ph_r = unit_phase(r * c * ov.L_S, L)
            out[sig[n] + r * N // 2:sig[n] + r * N // 2 + N] += s_win[r] * np.sqrt(ov.I) * ph_r * th * blk
    return out


def perm_quarter(L, sign):
    """The selection matrices P_L^(+L/4) and P_L^(-L/4) of the RX
    concatenation (Sec. IV): they move the middle half [L/4, 3L/4) of a block
    into the first (+) or second (-) half of the output."""
    P = np.zeros((L, L))
    rows = np.arange(L // 2) + (0 if sign > 0 else L // 2)
    P[rows, L // 4 + np.arange(L // 2)] = 1.0
    return P


def rx_sync(yh, L, N, c, D, ncp, keep_cp=False):
    """Symbol-synchronised OLS FC analysis (Sec. IV).

    w_n = Gamma_{sigma_n}^T yh (length 3N/2), w_n^(r) = R_N^(r)T w_n,
    z^(r) = G_r(phi_r theta_n) w_n^(r), and the symbol without CP is
    P^(L/4) z^(0) + P^(-L/4) z^(1). Returns an array (B, L).

    keep_cp=True returns instead the exact adjoint of ``tx_sync``: each symbol
    of length L + L_CP,n is [z^(0)[S_L,n : 3L/4]; z^(1)[L/4 : 3L/4]] (the two TX
    analysis windows tile the padded symbol, so the adjoint concatenates the
    window supports); the result is the concatenated CP-OFDM-shaped stream.
    """
    ov = Overlap(L, N, Fraction(1, 2))
    lcp = lowrate_cp(ncp, ov.I, exact=False)
    sigma = sync_sigma(ncp, N)
    yh = np.asarray(yh, dtype=complex)
    if len(yh) != sync_output_len(ncp, ov):
        raise ValueError("high-rate input must have length Q")
    G = block_core_rx(L, N, c, D)
    P0, P1 = perm_quarter(L, +1), perm_quarter(L, -1)
    out = []
    for n in range(len(ncp)):
        wn = yh[sigma[n]:sigma[n] + 3 * N // 2]
        theta = np.conj(unit_phase(c * sigma[n], N))
        z = []
        for r in (0, 1):
            phi = np.conj(unit_phase(r * c * ov.L_S, L))
            z.append(phi * theta * (G @ wn[r * N // 2:r * N // 2 + N]) / np.sqrt(ov.I))
        if keep_cp:
            S_L = ov.L_L - lcp[n]
            out.append(np.r_[z[0][S_L:3 * L // 4], z[1][L // 4:3 * L // 4]])
        else:
            out.append(P0 @ z[0] + P1 @ z[1])
    if keep_cp:
        return np.concatenate(out)
    return np.stack(out)


def ofdm_modulate(grid, L, lcp):
    """CP-OFDM modulation of Sec. III-A with L_OFDM = L: per symbol
    x_n = sqrt(L) W_L^{-1} X_n, where X_n carries the symbol's K values on
    subcarriers kappa in [-K/2, K/2) at index kappa mod L, then the last
    L_CP,n samples prepended (truncated low-rate CP in the synchronised
    model). grid is (B, K); returns the concatenated low-rate stream."""
    grid = np.atleast_2d(np.asarray(grid, dtype=complex))
    B, K = grid.shape
    Winv = idft_matrix(L)
    out = []
    for n in range(B):
        X = np.zeros(L, dtype=complex)
        X[np.arange(-K // 2, K // 2) % L] = grid[n]
        x = np.sqrt(L) * (Winv @ X)
        out.append(np.r_[x[L - lcp[n]:], x])
    return np.concatenate(out)


def tx_sync_grid(grid, L, N, c, D, ncp):
    """Synchronised FC TX of a QAM grid: CP-OFDM modulation with the
    truncated low-rate CP L_CP,n = floor(N_CP,n / I) (Sec. III-E), then
    tx_sync."""
    ov = Overlap(L, N, Fraction(1, 2))
    return tx_sync(ofdm_modulate(grid, L, lowrate_cp(ncp, ov.I, exact=False)), L, N, c, D, ncp)


def rx_sync_subcarriers(yh, L, N, c, D, ncp):
    """Symbol-synchronised RX followed by the OFDM demodulation of Sec. IV
    (L_OFDM = L): x_hat_n = (1/sqrt(L)) W_L x_hat_OFDM,n for every symbol, the
    direct approach (two short IFFTs and one FFT per symbol). Returns (B, L);
    subcarrier kappa is column kappa mod L."""
    return rx_sync(yh, L, N, c, D, ncp) @ dft_matrix(L) / np.sqrt(L)


def rx_sync_blocks_freq(yh, L, N, c, D, ncp):
    """The two frequency-domain FC block outputs of every symbol before the
    short IFFT, g^(r) with z^(r) = W_L^{-1} g^(r) (Sec. IV blocks, Sec. V-A
    notation): P^(-L/2) D M(1)^T W_N w_n^(r), times the conj phase and
    1/sqrt(I). Returns an array (B, 2, L)."""
    ov = Overlap(L, N, Fraction(1, 2))
    sigma = sync_sigma(ncp, N)
    yh = np.asarray(yh, dtype=complex)
    if len(yh) != sync_output_len(ncp, ov):
        raise ValueError("high-rate input must have length Q")
    Dv = np.asarray(D, dtype=float)
    Gf = (shift_matrix(L).T * Dv[None, :]) @ dft_matrix(N)[xi(L, N, c), :]
    out = []
    for n in range(len(ncp)):
        wn = yh[sigma[n]:sigma[n] + 3 * N // 2]
        th_n = np.conj(unit_phase(c * sigma[n], N))
        g = []
        for r in (0, 1):
            phi_r = np.conj(unit_phase(r * c * ov.L_S, L))
            g.append(phi_r * th_n * (Gf @ wn[r * N // 2:r * N // 2 + N]) / np.sqrt(ov.I))
        out.append(g)
    return np.array(out)


def omega(L, phi):
    """Omega_phi = diag(W_L^(phi k)), k = 0..L-1, W_L = exp(-j 2 pi / L) (Sec. V-A)."""
    return np.exp(-2j * np.pi * ((phi * np.arange(L)) % L) / L)


def rx_sync_subcarriers_reduced(yh, L, N, c, D, ncp):
    """Sec. V-A simplified joint processing of the FC short IFFTs and the OFDM
    FFT: per symbol x = Omega_{-L/4} [F (g0 - Omega_{L/2} g1) + Omega_{L/2} g1]
    with F = Omega_{L/4} C Omega_{-L/4} and the half-band matrix
    C = W_L S_hat W_L^{-1}, S_hat the synthesis window shifted by L/4, read as
    diag([1_{L/2}; 0_{L/2}]); times the demodulation's 1/sqrt(L). One short
    IFFT and one FFT per symbol. Returns (B, L) like rx_sync_subcarriers."""
    g = rx_sync_blocks_freq(yh, L, N, c, D, ncp)
    S_hat = np.diag(np.r_[np.ones(L // 2), np.zeros(L // 2)])
    C = dft_matrix(L) @ S_hat @ idft_matrix(L)
    F = omega(L, L // 4)[:, None] * C * omega(L, -L // 4)[None, :]
    out = []
    for g0, g1 in g:
        h1 = omega(L, L // 2) * g1
        out.append(omega(L, -L // 4) * (F @ (g0 - h1) + h1) / np.sqrt(L))
    return np.stack(out)


# ----------------------------------------------------------------- stream --
def place(parts, length=None):
    """Sum local outputs onto one stream: parts = [(offset, array), ...]."""
    if length is None:
        length = max(o + len(a) for o, a in parts)
    y = np.zeros(length, dtype=complex)
    for o, a in parts:
        y[o:o + len(a)] += a
    return y
