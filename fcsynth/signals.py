"""Random QAM, CP-OFDM modulation and AWGN (seeded, numpy only)."""
import numpy as np

_QAM_NORM = {4: np.sqrt(2.0), 16: np.sqrt(10.0), 64: np.sqrt(42.0), 256: np.sqrt(170.0)}


def qam(rng, order, shape):
    """Uniform square-QAM symbols with unit average power."""
    if order not in _QAM_NORM:
        raise ValueError("QAM order must be 4, 16, 64 or 256")
    m = int(round(np.sqrt(order)))
    levels = 2 * np.arange(m) - (m - 1)
    re = levels[rng.integers(0, m, size=shape)]
    im = levels[rng.integers(0, m, size=shape)]
    return (re + 1j * im) / _QAM_NORM[order]


def qam_grid(rng, order, n_symbols, n_active):
    """(n_symbols, n_active) grid of QAM symbols on subcarriers -K/2 .. K/2-1."""
    return qam(rng, order, (n_symbols, n_active))


def cp_ofdm(grid, L, lcp):
    """Low-rate CP-OFDM: per symbol x = sqrt(L) IDFT_L(X) with the active
    subcarriers kappa in [-K/2, K/2) at index kappa mod L, then the last
    lcp[n] samples prepended. Returns the concatenated complex128 stream."""
    grid = np.asarray(grid)
    B, K = grid.shape
    kap = np.arange(-K // 2, K // 2) % L
    out = []
    for n in range(B):
        X = np.zeros(L, dtype=complex)
        X[kap] = grid[n]
        x = np.fft.ifft(X) * np.sqrt(L)
        out.append(np.r_[x[L - lcp[n]:], x] if lcp[n] else x)
    return np.concatenate(out)


def cp_ofdm_highrate(grids, centers, N, ncp):
    """High-rate CP-OFDM carrying several subbands in one N-point IDFT per
    symbol: grids[m] is (B, K_m) placed at bins c_m + kappa mod N."""
    B = grids[0].shape[0]
    out = []
    for n in range(B):
        X = np.zeros(N, dtype=complex)
        for g, c in zip(grids, centers):
            K = g.shape[1]
            X[(c + np.arange(-K // 2, K // 2)) % N] = g[n]
        x = np.fft.ifft(X) * np.sqrt(N)
        out.append(np.r_[x[N - ncp[n]:], x])
    return np.concatenate(out)


def awgn(rng, n, var):
    """Circular complex Gaussian noise of total variance ``var`` per sample."""
    s = np.sqrt(var / 2.0)
    return s * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
