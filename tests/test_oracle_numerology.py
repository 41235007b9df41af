"""Pins of the oracle's integer arithmetic against values the paper prints."""
import json
import os
from fractions import Fraction

import pytest

from oracle import numerology as nu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_nr_cp_10mhz():
    g = GOLD["nr_cp_10mhz_15khz"]
    cps = nu.nr_cp_list(g["n_long"], g["mu"], 0, 14)
    assert cps[0] == g["first"] and cps[7] == g["first"]
    assert all(c == g["other"] for i, c in enumerate(cps) if i % 7)


def test_lowrate_cp_l128():
    g = GOLD["lowrate_cp_l128"]
    I = 1024 // g["n_short"]
    lcp = nu.lowrate_cp(nu.nr_cp_list(1024, 0, 0, 14), I, exact=True)
    assert lcp[0] == g["first"] and lcp[1] == g["other"]


def test_lowrate_cp_fractional_and_truncation():
    g = GOLD["lowrate_cp_fractional"]
    cps = nu.nr_cp_list(1024, 0, 0, 2)
    for L, f, o in zip(g["n_short"], g["first"], g["other"]):
        I = 1024 // L
        assert Fraction(cps[0], I) == Fraction(f).limit_denominator(1000)
        assert Fraction(cps[1], I) == Fraction(o).limit_denominator(1000)
        # the continuous model rejects them, the synchronised one truncates
        with pytest.raises(ValueError):
            nu.lowrate_cp(cps, I, exact=True)
        assert nu.lowrate_cp(cps, I, exact=False) == [int(f), int(o)]


def test_fig5_extrapolation():
    g = GOLD["extrapolation_fig5"]
    lcp = nu.lowrate_cp([g["ncp_high"]], g["interp"], exact=False)[0]
    assert lcp == g["lcp_low"]
    assert g["ncp_high"] - g["interp"] * lcp == g["extrapolated_high"]


def test_block_counts_two_symbols():
    g = GOLD["blocks_two_symbols"]
    L = g["n_short"]
    ov = nu.Overlap(L, 8 * L, Fraction(1, 2))
    assert nu.cont_block_count(2 * L + sum(g["lcp"]), ov) == g["continuous"]
    assert 2 * 2 == g["synchronised"]      # two blocks per symbol by construction


def test_dynamic_overlap_first_block():
    # first block: a_0 = [0_{S_L}; 1_{L_S + L_CP}; 0_{L_T}] has S_L + L_T zeros,
    # so its overlap factor is (L_O - L_CP)/L = 0.5 - L_CP/L
    L = 128
    ov = nu.Overlap(L, 1024)
    for lcp in (9, 10):
        S_L = ov.L_L - lcp
        lead_zeros = S_L
        tail_zeros = ov.L_T
        assert Fraction(lead_zeros + tail_zeros, L) == Fraction(1, 2) - Fraction(lcp, L)


def test_split_radix():
    for k, v in GOLD["split_radix_mults"]["mu"].items():
        assert nu.split_radix_mults(int(k)) == v


def test_overlap_split():
    ov = nu.Overlap(512, 2048, Fraction(1, 2))
    assert (ov.L_O, ov.L_S, ov.L_L, ov.L_T) == (256, 256, 128, 128)
    assert (ov.N_O, ov.N_S, ov.N_L, ov.N_T, ov.I) == (1024, 1024, 512, 512, 4)
    ov = nu.Overlap(128, 1024, Fraction(1, 4))
    assert (ov.L_O, ov.L_S, ov.L_L, ov.L_T) == (32, 96, 16, 16)
    with pytest.raises(ValueError):
        nu.Overlap(100, 1024)


def test_sigma_and_span():
    # every filtered symbol lies inside [0, Q) and the last one ends at Q
    for N, mu in ((2048, 0), (1024, 1), (4096, 1)):
        ncp = nu.nr_cp_list(N, mu, 0, 28)
        ov = nu.Overlap(N // 4, N)
        sig = nu.sync_sigma(ncp, N)
        Q = nu.sync_output_len(ncp, ov)
        assert sig[0] == 0 and sig[-1] + 3 * N // 2 == Q
        for n in range(1, len(sig)):
            assert sig[n] - sig[n - 1] == N + ncp[n]
            # adjacent symbols overlap by N/2 - N_CP,n (Fig. 4 caption)
            assert sig[n - 1] + 3 * N // 2 - sig[n] == N // 2 - ncp[n]


def test_subframe_duration():
    # one 1 ms subframe at 30.72 MS/s: 14 symbols at 15 kHz or 28 at 30 kHz
    assert sum(nu.nr_cp_list(2048, 0, 0, 14)) + 14 * 2048 == 30720
    assert sum(nu.nr_cp_list(1024, 1, 0, 28)) + 28 * 1024 == 30720
    assert sum(nu.nr_cp_list(4096, 1, 0, 28)) + 28 * 4096 == 2 * 61440
