"""Numerology and block-schedule arithmetic (oracle side, integer, exact).

Test infrastructure only (see ``oracle/__init__``).

Paper references are to Yli-Kaakinen et al., "Frequency-Domain Signal
Processing for Spectrally-Enhanced CP-OFDM Waveforms in 5G New Radio"
(arXiv 2008.00672).
"""
from fractions import Fraction
import math


def nr_normal_cp(n_long, mu, l):
    """High-rate normal-CP length of the symbol with index ``l`` in its subframe.

    Sec. III-A: NR/LTE normal CP uses two lengths; the first symbol of each half
    subframe (0.5 ms) is longer. Expressed at the rate n_long * SCS, the 3GPP
    normal CP is 144/2048 of the useful symbol, plus 16*2^mu/2048 of it for the
    symbols l = 0 and l = 7*2^mu of a subframe of 14*2^mu symbols. Sec. III-E
    gives the check values 80 / 72 samples at n_long = 1024, 15 kHz.
    """
    if (n_long * 144) % 2048 or (n_long * (1 << mu) * 16) % 2048:
        raise ValueError("NR normal CP is not an integer number of samples at this n_long")
    ncp = n_long * 144 // 2048
    if l % (7 * (1 << mu)) == 0:
        ncp += n_long * (1 << mu) * 16 // 2048
    return ncp


def nr_cp_list(n_long, mu, first_symbol, n_symbols):
    """N_CP for ``n_symbols`` consecutive symbols starting at ``first_symbol``."""
    per_subframe = 14 * (1 << mu)
    return [nr_normal_cp(n_long, mu, (first_symbol + n) % per_subframe)
            for n in range(n_symbols)]


def lowrate_cp(ncp_high, interp, exact):
    """Low-rate CP lengths L_CP,n from high-rate N_CP,n.

    Sec. III-B: N_CP = I * L_CP with integer L_CP in the continuous model.
    Sec. III-E: in the symbol-synchronised model the low-rate CP is truncated,
    L_CP = floor(N_CP / I), and the FC extrapolates the fractional remainder.
    """
    out = []
    for n in ncp_high:
        if exact and n % interp:
            raise ValueError("continuous FC needs an integer low-rate CP (N_CP %% I != 0)")
        out.append(n // interp)
    return out


class Overlap:
    """Overlap split of Sec. III-B for one subband.

    L_O = lambda*L overlapping input samples, L_S = L - L_O, leading part
    L_L = ceil(L_O/2), tailing part L_T = floor(L_O/2); on the output side
    N_O = lambda*N, N_S = N - N_O. The paper calls the output leading/tailing
    split "similar"; this reading takes N_L = I*L_L and N_T = I*L_T, which needs
    L_O even so that both halves are equal.
    """

    def __init__(self, L, N, lam=Fraction(1, 2)):
        lam = Fraction(lam)
        if N % L:
            raise ValueError("N must be a multiple of L")
        if (lam * L).denominator != 1:
            raise ValueError("lambda*L must be an integer")
        self.L, self.N, self.lam = L, N, lam
        self.I = N // L
        self.L_O = int(lam * L)
        self.L_S = L - self.L_O
        self.L_L = -(-self.L_O // 2)
        self.L_T = self.L_O // 2
        self.N_O = self.I * self.L_O
        self.N_S = N - self.N_O
        self.N_L = self.I * self.L_L
        self.N_T = self.I * self.L_T


def cont_block_count(n_in, ov):
    """Number of continuous FC blocks R for n_in low-rate input samples.

    Sec. III-B: the input is zero padded by L_O samples at both ends; the
    paper leaves R "typical". This reading takes the smallest R whose OLS
    keep-windows reach the end of the input: R*L_S >= n_in + L_T.
    It gives 5 blocks for two symbols at 50 % overlap (Fig. 3 caption).
    """
    return -(-(n_in + ov.L_T) // ov.L_S)


def cont_output_len(n_in, ov):
    """High-rate length (R-1)*N_S + N of a continuous FC burst."""
    R = cont_block_count(n_in, ov)
    return (R - 1) * ov.N_S + ov.N


def sync_sigma(ncp_high, n_ofdm):
    """Start index sigma_n of each filtered symbol (Sec. III-D).

    sigma_n = n*N_OFDM + sum_{q=1..n} N_CP,q.
    """
    out, acc = [], 0
    for n in range(len(ncp_high)):
        if n > 0:
            acc += ncp_high[n]
        out.append(n * n_ofdm + acc)
    return out


def sync_output_len(ncp_high, ov):
    """Q = N_L + N_T + B*N_OFDM + sum_{n=1..B-1} N_CP,n (Sec. III-D)."""
    return ov.N_L + ov.N_T + len(ncp_high) * ov.N + sum(ncp_high[1:])


def first_cp_start(mode_sync, ov, ncp0):
    """High-rate position of the start of the first symbol's CP in the local
    coordinates of one subband's output.

    Continuous: x[0] sits at low-rate index L_O of the padded input, i.e. at
    high-rate I*L_O = N_O. Synchronised: the useful part of symbol 0 starts at
    N_L, so its (high-rate) CP starts at N_L - N_CP,0.
    """
    return (ov.N_L - ncp0) if mode_sync else ov.N_O


def mu_of_scs(scs_khz):
    mu = int(round(math.log2(scs_khz / 15)))
    if 15 * (1 << mu) != scs_khz:
        raise ValueError("SCS must be 15*2^mu kHz")
    return mu


def split_radix_mults(L):
    """mu(L) = L log2 L - 3L + 4 real multiplications (Sec. V)."""
    return L * int(round(math.log2(L))) - 3 * L + 4
