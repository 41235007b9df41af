"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Gate (waveform error against the oracle on the unquantised FP64 input):
FP32 I/O <= -100 dB, FP16 <= -60 dB, BF16 <= -50 dB. The FP32 gate follows
from FP32 storage and arithmetic (unit roundoff 6e-8 over ~2 log2 N butterfly
stages gives about -125 dB); the FP16/BF16 gates are the storage floors
(binary16 / bfloat16 round-to-nearest-even of input and output) with margin.
Every sample is also bounded (fc_cases.assert_gate): its error beyond the
output's own rounding stays within a few roundoffs of the output's rms.
"""
import numpy as np
import pytest

from fc_cases import (assert_gate, from_device, make_inputs, oracle_adj, oracle_rx, oracle_rxd, oracle_tx,
                      oracle_tx_grid, stream_offsets, to_device)
from fcsynth import workloads as W

pytestmark = pytest.mark.gpu


def _plan(subbands, io, Ds):
    from paper_2008_00672_amd import Plan
    p = Plan(subbands, io=io, device=0)
    for i, D in enumerate(Ds):
        p.set_weights(i, D)
    return p


def _cat(xs):
    return np.concatenate(xs)


def _split(v, offs):
    return [v[offs[i]:offs[i + 1]] for i in range(len(offs) - 1)]


def run_tx(subbands, io, seed=0, qam=16, weights="rc"):
    import torch
    from paper_2008_00672_amd import OP_TX
    xs, Ds, _ = make_inputs(subbands, qam, seed, weights)
    p = _plan(subbands, io, Ds)
    lo, hi = p.layout(OP_TX)
    assert [len(x) for x in xs] == list(np.diff(lo))
    y = p.tx(to_device(_cat(xs), io))
    torch.cuda.synchronize()
    got = _split(from_device(y, io), hi)
    ref = oracle_tx(subbands, xs, Ds)
    return got, ref


def run_rx(subbands, io, seed=0, weights="rc", adjoint=False, demod=False):
    import torch
    from paper_2008_00672_amd import OP_ADJ, OP_RX, OP_RXD
    rng = np.random.default_rng(seed)
    _, lens, _ = stream_offsets(subbands)
    streams = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in lens]
    _, Ds, _ = make_inputs(subbands, 4, seed + 1, weights)
    p = _plan(subbands, io, Ds)
    op = OP_ADJ if adjoint else (OP_RXD if demod else OP_RX)
    lo, hi = p.layout(op)
    assert list(np.diff(hi)) == lens
    dev_in = to_device(_cat(streams), io)
    z = p.adjoint(dev_in) if adjoint else (p.rx_demod(dev_in) if demod else p.rx(dev_in))
    torch.cuda.synchronize()
    got = _split(from_device(z, io), lo)
    ref = (oracle_adj if adjoint else (oracle_rxd if demod else oracle_rx))(subbands, streams, Ds)
    return got, ref


def tiny(mode, L=16, N=64, c=5, n_sym=5, lam=(1, 2), ncp=None, K=8, n_tb=2, taper=0):
    s = W.subband(15, n_sym, K, n_tb, L, N, c, mode, overlap=lam, taper=taper)
    s["ncp_high"] = ncp
    return s


CP_INT = [8, 4, 4, 8, 4]        # I = 4: integer low-rate CP
CP_FRAC = [9, 5, 6, 7, 5]       # fractional at I = 4 (synchronised only)

TINY_TX = {
    "cont_ols_16_64": [tiny("cont_ols", ncp=CP_INT)],
    "cont_ola_16_64": [tiny("cont_ola", ncp=CP_INT)],
    "cont_ola_quarter": [tiny("cont_ola", L=32, N=128, c=-9, lam=(1, 4), ncp=[8, 8, 4, 4, 8], K=16, n_tb=4)],
    "sync_ola_frac": [tiny("sync_ola", ncp=CP_FRAC)],
    "sync_ola_64_256": [tiny("sync_ola", L=64, N=256, c=-40, ncp=[20, 18, 18, 18, 20], K=40, n_tb=8)],
    "i1_cont_ols": [tiny("cont_ols", L=32, N=32, c=0, ncp=[4, 3, 3, 3, 4], K=16, n_tb=2)],
    "two_sb_one_group": [tiny("sync_ola", L=16, N=128, c=-20, ncp=CP_FRAC[:3] + [9, 9], n_sym=5),
                         tiny("sync_ola", L=32, N=128, c=25, ncp=CP_FRAC[:3] + [9, 9], n_sym=5, K=16, n_tb=4)],
    "sync_ols_frac": [tiny("sync_ols", ncp=CP_FRAC)],
    "sync_ols_64_256": [tiny("sync_ols", L=64, N=256, c=-40, ncp=[20, 18, 18, 18, 20], K=40, n_tb=8)],
    "sync_ols_two_sb": [tiny("sync_ols", L=16, N=128, c=-20, ncp=CP_FRAC[:3] + [9, 9], n_sym=5),
                        tiny("sync_ols", L=32, N=128, c=25, ncp=CP_FRAC[:3] + [9, 9], n_sym=5, K=16, n_tb=4)],
    # smooth outer window edges: short, and the longest the CP schedule allows
    "sync_ols_taper_6": [tiny("sync_ols", ncp=CP_FRAC, taper=6)],
    "sync_ols_taper_max": [tiny("sync_ols", ncp=CP_FRAC, taper=14)],
    "sync_ols_taper_64_256": [tiny("sync_ols", L=64, N=256, c=-40, ncp=[20, 18, 18, 18, 20], K=40, n_tb=8,
                                   taper=32)],
    "sync_ols_taper_two_sb": [tiny("sync_ols", L=16, N=128, c=-20, ncp=CP_FRAC[:3] + [9, 9], taper=10),
                              tiny("sync_ols", L=32, N=128, c=25, ncp=CP_FRAC[:3] + [9, 9], K=16, n_tb=4,
                                   taper=10)],
}


@pytest.mark.parametrize("name", sorted(TINY_TX))
@pytest.mark.parametrize("weights", ["rc", "random"])
def test_tx_tiny(name, weights):
    got, ref = run_tx(TINY_TX[name], "c64", seed=11, weights=weights)
    assert_gate(got, ref, "c64", name)


TINY_RX = {
    "cont_ols_16_64": [tiny("cont_ols", ncp=CP_INT)],
    "cont_ola_16_64": [tiny("cont_ola", ncp=CP_INT)],
    "sync_16_64": [tiny("sync_ols", ncp=CP_FRAC)],
    "sync_two_sb": [tiny("sync_ols", L=16, N=128, c=-20, ncp=CP_FRAC[:3] + [9, 9]),
                    tiny("sync_ols", L=32, N=128, c=25, ncp=CP_FRAC[:3] + [9, 9], K=16, n_tb=4)],
}


# groups that RX splits into parts (bins feeding more than four subbands;
# subband regions beyond one workgroup's LDS)
RX_SPLIT = {
    "six_overlapping": [W.subband(15, 2, 24, 4, 64, 256, c, "sync_ola") for c in (-12, -6, 0, 6, 12, 18)],
    "four_long": [W.subband(15, 2, 1000, 16, 2048, 4096, c, "sync_ola") for c in (-1000, -300, 300, 1000)],
}


@pytest.mark.parametrize("name", sorted(RX_SPLIT))
@pytest.mark.parametrize("adjoint", [False, True])
def test_rx_split_groups(name, adjoint):
    got, ref = run_rx(RX_SPLIT[name], "c64", seed=9, weights="random", adjoint=adjoint)
    assert_gate(got, ref, "c64", name)


@pytest.mark.parametrize("name", sorted(TINY_RX))
def test_rx_tiny(name):
    got, ref = run_rx(TINY_RX[name], "c64", seed=3, weights="random")
    assert_gate(got, ref, "c64", name)


DEMOD = {
    "sync_16_64": [tiny("sync_ols", ncp=CP_FRAC)],
    "sync_ola_64_256": [tiny("sync_ola", L=64, N=256, c=-40, ncp=[20, 18, 18, 18, 20], K=40, n_tb=8)],
    "sync_two_sb": TINY_RX["sync_two_sb"],
    "six_overlapping": [W.subband(15, 2, 24, 4, 64, 256, c, "sync_ols") for c in (-12, -6, 0, 6, 12, 18)],
    "four_long": [W.subband(15, 2, 1000, 16, 2048, 4096, c, "sync_ols") for c in (-1000, -300, 300, 1000)],
}


@pytest.mark.parametrize("name", sorted(DEMOD))
def test_rx_demod_tiny(name):
    """Sec. V-A simplified RX + demodulation against the direct definition."""
    got, ref = run_rx(DEMOD[name], "c64", seed=13, weights="random", demod=True)
    assert_gate(got, ref, "c64", name)


@pytest.mark.parametrize("io", ["c64", "bf16"])
def test_rx_demod_filterbank(io):
    """The 100 MHz 8-subband filter bank, 28 symbols."""
    sbs, meta = W.rx_filterbank(n_symbols=28)
    got, ref = run_rx(sbs, io, seed=meta["seed"], demod=True)
    assert_gate(got, ref, io, "filterbank demod")


# The demodulating RX keeps the second block's terms in a second LDS region
# set, or in per-task device scratch where two sets would cost workgroups per
# CU. Groups of 4224 region entries take two 33.8 KB sets: kept in LDS for
# FP32 I/O (two workgroups per CU either way), in scratch for FP16 / BF16
# (three with one set); the 2048-point subbands run on the workgroup, the
# 1024-point ones on one wave each. four_long: three 2048-point subbands in
# one group (two 50.7 KB sets: scratch for every I/O type) and one alone
# (two 25.3 KB sets: LDS for every I/O type). tri_768 / tri_1536: the same
# choices for mixed-radix sizes.
TERMS = {
    "wg_and_wave": [W.subband(30, 4, 1600, 8, 2048, 4096, -900, "sync_ols"),
                    W.subband(30, 4, 800, 8, 1024, 4096, 700, "sync_ols"),
                    W.subband(30, 4, 700, 8, 1024, 4096, 1500, "sync_ols")],
    "four_long": DEMOD["four_long"],
    # mixed-radix subbands: five 768-point ones on the waves (two 31.7 KB
    # sets: LDS for FP32, scratch for FP16 / BF16) and four 1536-point ones
    # on the workgroup (two 50.7 KB sets: scratch for every storage type)
    "tri_768": [W.subband(15, 2, 600, 8, 768, 3072, c, "sync_ols") for c in (-1000, -500, 0, 500, 1000)],
    "tri_1536": [W.subband(15, 2, 1200, 8, 1536, 3072, c, "sync_ols") for c in (-700, -200, 200, 700)],
}


@pytest.mark.parametrize("io", ["c64", "f16", "bf16"])
@pytest.mark.parametrize("name", sorted(TERMS))
def test_rx_demod_terms(name, io):
    print("case: demodulating RX %s %s" % (name, io), flush=True)
    got, ref = run_rx(TERMS[name], io, seed=29, weights="random", demod=True)
    assert_gate(got, ref, io, name)


@pytest.mark.parametrize("name", ["cont_ols_16_64", "cont_ola_16_64", "sync_ola_frac"])
def test_adjoint_tiny(name):
    got, ref = run_rx(TINY_TX[name], "c64", seed=5, weights="random", adjoint=True)
    assert_gate(got, ref, "c64", name)


# Edge cases: one symbol, a band filling the short transform (K + 2 N_tb = L),
# the centre bin at either end of its range (|c| + L/2 = N/2), I = 1 at
# L = N = 2048.
EDGE = {
    "one_symbol_sync": [tiny("sync_ola", n_sym=1, ncp=[9])],
    "one_symbol_cont": [tiny("cont_ols", n_sym=1, ncp=[8])],
    "full_band": [tiny("sync_ola", L=64, N=256, c=0, K=48, n_tb=8, ncp=[20, 18, 18, 18, 20])],
    "edge_center_pos": [tiny("sync_ola", L=64, N=256, c=96, K=40, n_tb=8, ncp=[20, 18, 18, 18, 20])],
    "edge_center_neg": [tiny("sync_ola", L=64, N=256, c=-96, K=40, n_tb=8, ncp=[20, 18, 18, 18, 20])],
    "i1_2048": [W.subband(15, 1, 1200, 8, 2048, 2048, 0, "cont_ols")],
    # largest transforms: the whole 4096-bin band as one subband (I = 1), and
    # the narrowest subband at the largest interpolation (L = 16, I = 256)
    "max_4096": [W.subband(30, 1, 3276, 8, 4096, 4096, 0, "sync_ola")],
    "narrow_4096": [W.subband(15, 2, 12, 2, 16, 4096, -1500, "sync_ola")],
    # no active subcarriers: only the transition bins carry weight
    "no_active": [tiny("sync_ola", K=0, n_tb=4, ncp=[9, 5, 6, 7, 5])],
    # short FFTs on the whole workgroup in the long IFFT buffer (L >= 256 at
    # N >= 2048), synchronised and continuous
    "wg_short_256_2048": [W.subband(15, 3, 200, 8, 256, 2048, -500, "sync_ola")],
    "wg_short_512_4096": [W.subband(30, 2, 456, 8, 512, 4096, 900, "sync_ola")],
    "wg_short_1024_4096_cont": [dict(W.subband(15, 2, 900, 8, 1024, 4096, -1000, "cont_ols"),
                                     ncp_high=[320, 288])],
}


@pytest.mark.parametrize("name", sorted(EDGE))
def test_tx_edge(name):
    got, ref = run_tx(EDGE[name], "c64", seed=17, weights="random")
    assert_gate(got, ref, "c64", name)


@pytest.mark.parametrize("name", sorted(EDGE))
def test_rx_edge(name):
    sbs = [dict(s, mode="sync_ols") if s["mode"].startswith("sync") else s for s in EDGE[name]]
    got, ref = run_rx(sbs, "c64", seed=19, weights="random")
    assert_gate(got, ref, "c64", name)


@pytest.mark.parametrize("name", [k for k in sorted(EDGE) if EDGE[k][0]["mode"].startswith("sync")])
def test_rx_demod_edge(name):
    got, ref = run_rx(EDGE[name], "c64", seed=23, weights="random", demod=True)
    assert_gate(got, ref, "c64", name)


def run_tx_grid(subbands, io, seed=0, qam=16, weights="rc"):
    import torch
    from paper_2008_00672_amd import OP_TXG
    _, Ds, grids = make_inputs(subbands, qam, seed, weights)
    p = _plan(subbands, io, Ds)
    lo, hi = p.layout(OP_TXG)
    assert list(np.diff(lo)) == [g.size for g in grids]
    y = p.tx_grid(to_device(_cat([g.ravel() for g in grids]), io))
    torch.cuda.synchronize()
    return _split(from_device(y, io), hi), oracle_tx_grid(subbands, grids, Ds)


GRID = {
    "sync_ola_frac": TINY_TX["sync_ola_frac"],
    "sync_ols_64_256": TINY_TX["sync_ols_64_256"],
    "sync_ols_taper_64_256": TINY_TX["sync_ols_taper_64_256"],
    "sync_ola_64_256": TINY_TX["sync_ola_64_256"],
    "two_sb_one_group": TINY_TX["two_sb_one_group"],
    "one_symbol": EDGE["one_symbol_sync"],
    "full_band": EDGE["full_band"],
}


@pytest.mark.parametrize("name", sorted(GRID))
def test_tx_grid_tiny(name):
    """QAM grid -> OFDM IFFT + truncated CP -> FC, in the kernels."""
    got, ref = run_tx_grid(GRID[name], "c64", seed=29, weights="random")
    assert_gate(got, ref, "c64", name)


@pytest.mark.parametrize("io", ["c64", "f16"])
def test_tx_grid_mixed_numerology(io):
    sbs, meta = W.mixed_numerology("sync_ola")
    got, ref = run_tx_grid(sbs, io, seed=meta["seed"], qam=meta["qam"])
    assert_gate(got, ref, io, "mixed numerology grid TX")


def test_tx_grid_shared_long_transform():
    """Eight subbands on one stream and N: the full long IFFT path."""
    sbs, _ = W.rx_filterbank(n_symbols=4)
    sbs = [dict(s, mode="sync_ola") for s in sbs]
    got, ref = run_tx_grid(sbs, "c64", seed=31, qam=256)
    assert_gate(got, ref, "c64", "filterbank grid TX")


def test_plain_slot_fp32():
    """One 14-symbol slot, continuous OLS, L = 512, N = 2048 (the plain form)."""
    sbs, meta = W.plain_tx_slot()
    got, ref = run_tx(sbs, "c64", seed=meta["seed"], qam=meta["qam"])
    assert_gate(got, ref, "c64", "plain slot")


@pytest.mark.parametrize("io", ["c64", "f16", "bf16"])
def test_mixed_numerology_tx(io):
    sbs, meta = W.mixed_numerology("sync_ola")
    got, ref = run_tx(sbs, io, seed=meta["seed"], qam=meta["qam"])
    assert_gate(got, ref, io, "mixed numerology TX")


@pytest.mark.parametrize("taper", [0, 64])
def test_mixed_numerology_tx_sync_ols(taper):
    """Synchronised OLS TX of the two-numerology subframe (accumulating groups
    on one stream), with hard and with smooth outer window edges."""
    sbs, meta = W.mixed_numerology("sync_ols")
    sbs = [dict(s, taper=taper) for s in sbs]
    got, ref = run_tx(sbs, "c64", seed=meta["seed"], qam=meta["qam"])
    assert_gate(got, ref, "c64", "mixed numerology sync OLS TX, taper %d" % taper)


def test_mixed_numerology_rx():
    sbs, meta = W.mixed_numerology("sync_ols")
    got, ref = run_rx(sbs, "c64", seed=meta["seed"])
    assert_gate(got, ref, "c64", "mixed numerology RX")
