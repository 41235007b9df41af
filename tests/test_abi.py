"""CPU-side checks of the C ABI: the library loads and exports every function
include/fc.h declares; host-only plans reproduce the oracle's schedules and
reject invalid descriptions with the documented status codes (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from fc_cases import stream_offsets, sub_params
from fcsynth import workloads as W
from oracle import weights as ow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fc.h")


def _lib():
    from paper_2008_00672_amd import fc
    if not os.path.exists(fc.LIB_PATH):
        pytest.skip("libfc.so not built")
    return fc


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fc_[a-z_0-9]+)\s*\(", src)))


def test_exports_match_header():
    fc = _lib()
    names = header_functions()
    assert "fc_tx_synthesize" in names and "fc_rx_analyze" in names and "fc_set_weights" in names
    raw = ctypes.CDLL(fc.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), "missing export " + n
    assert set(names) == set(fc.EXPORTS), "binding and header disagree"


def test_status_strings():
    fc = _lib()
    for code in range(0, -8, -1):
        assert fc.lib().fc_status_str(code)
    assert b"gfx950" in fc.lib().fc_version()


def _plan(sbs, io="c64"):
    fc = _lib()
    return fc.Plan(sbs, io=io, device=-1)


@pytest.mark.parametrize("wl", ["plain", "mixed", "rx8", "batched"])
def test_layouts_match_oracle(wl):
    fc = _lib()
    sbs = {"plain": W.plain_tx_slot, "mixed": W.mixed_numerology, "rx8": lambda: W.rx_filterbank(28),
           "batched": lambda: W.batched_carriers(24)}[wl]()[0]
    p = _plan(sbs)
    off, lens, P = stream_offsets(sbs)
    op = fc.OP_RX if wl == "rx8" else fc.OP_TX
    lo, hi = p.layout(op)
    assert list(np.diff(hi)) == lens
    for i, s in enumerate(sbs):
        ncp, lcp, o = p.symbols(i)
        assert ncp == P[i]["ncp"] and lcp == P[i]["lcp"] and o == off[i]
        n_lo = s["n_symbols"] * s["n_short"] if (op == fc.OP_RX and P[i]["sync"]) else P[i]["n_in"]
        assert lo[i + 1] - lo[i] == n_lo


def test_default_weights_are_rc():
    sbs, _ = W.mixed_numerology()
    p = _plan(sbs)
    for i, s in enumerate(sbs):
        assert np.allclose(p.get_weights(i), ow.rc_weights(s["n_short"], s["n_active"], s["n_tb"]), atol=1e-7)


def test_block_counts():
    fc = _lib()
    sbs, _ = W.plain_tx_slot()
    assert _plan(sbs).stats(fc.OP_TX)["blocks"] == 31           # R = ceil((7680 + 128)/256)
    sbs, _ = W.mixed_numerology()
    assert _plan(sbs).stats(fc.OP_TX)["blocks"] == 2 * 14 + 2 * 28
    # synchronised: two blocks per symbol; continuous: five for two symbols (L = 128)
    s = W.subband(15, 2, 96, 8, 128, 1024, 0, "cont_ola")
    assert _plan([s]).stats(fc.OP_TX)["blocks"] == 5
    s = W.subband(15, 2, 96, 8, 128, 1024, 0, "sync_ola")
    assert _plan([s]).stats(fc.OP_TX)["blocks"] == 4


# Subbands of one group whose RX work cannot share one workgroup: six windows
# over the same long bins (each bin feeds at most four subbands in one pass),
# and four L = 2048 subbands (their LDS regions exceed 8192 entries).
RX_SPLIT = {
    "six_overlapping": [W.subband(15, 2, 24, 4, 64, 256, c, "sync_ola") for c in (-12, -6, 0, 6, 12, 18)],
    "four_long": [W.subband(15, 2, 1000, 16, 2048, 4096, c, "sync_ola") for c in (-1000, -300, 300, 1000)],
}


@pytest.mark.parametrize("name", sorted(RX_SPLIT))
def test_rx_group_split(name):
    """TX keeps one group (one long transform per block); RX and the adjoint
    repeat the long transform in a second part."""
    fc = _lib()
    p = _plan(RX_SPLIT[name])
    assert p.stats(fc.OP_TX)["blocks"] == 4
    assert p.stats(fc.OP_RX)["blocks"] == 8
    assert p.stats(fc.OP_ADJ)["blocks"] == 8


BAD = {
    "short_not_pow2": (dict(n_short=96), "FC_E_UNSUPPORTED"),
    "short_3x128": (dict(n_short=384), "FC_E_UNSUPPORTED"),     # mixed radix from 768 only
    "short_5x256": (dict(n_short=1280, n_long=2560), "FC_E_UNSUPPORTED"),
    "interp_not_pow2": (dict(n_short=768, n_long=1024, n_active=288), "FC_E_SHAPE"),
    "interp_three": (dict(n_short=512, n_long=1536, n_active=288), "FC_E_SHAPE"),
    "long_too_big": (dict(n_long=8192), "FC_E_UNSUPPORTED"),
    "short_gt_long": (dict(n_short=4096, n_long=2048), "FC_E_SHAPE"),
    "band_too_wide": (dict(n_active=500, n_tb=8), "FC_E_SHAPE"),
    "center_out_of_range": (dict(center_bin=900), "FC_E_SHAPE"),
    "odd_active": (dict(n_active=287), "FC_E_ARG"),
    "bad_scs": (dict(scs_khz=20), "FC_E_ARG"),
    "bad_mode": (dict(mode=7), "FC_E_ARG"),
    "sync_quarter_overlap": (dict(mode="sync_ola", overlap=(1, 4)), "FC_E_UNSUPPORTED"),
    "overlap_above_half": (dict(overlap=(3, 4)), "FC_E_UNSUPPORTED"),
    "cont_fractional_cp": (dict(mode="cont_ols", n_short=64, n_active=40, n_tb=8), "FC_E_SHAPE"),
    "sync_cp_too_long": (dict(mode="sync_ola", ncp_high=[600] * 14), "FC_E_SHAPE"),
    "zero_symbols": (dict(n_symbols=0), "FC_E_ARG"),
    "taper_not_sync_ols": (dict(taper=16), "FC_E_ARG"),
    "taper_odd": (dict(mode="sync_ols", taper=15), "FC_E_ARG"),
    "taper_negative": (dict(mode="sync_ols", taper=-2), "FC_E_ARG"),
    "taper_past_leading_overlap": (dict(mode="sync_ols", taper=706), "FC_E_SHAPE"),
}
CODES = {"FC_E_ARG": -1, "FC_E_SHAPE": -2, "FC_E_UNSUPPORTED": -3}


@pytest.mark.parametrize("n_short,n_long", [(768, 768), (768, 1536), (768, 3072), (1536, 3072), (3072, 3072)])
def test_mixed_radix_sizes_accepted(n_short, n_long):
    """3 x 2^k transform lengths (768 = 3 x 256, Sec. VI-C) with a power-of-two
    interpolation factor: the plan's layout and CP schedule follow the oracle's."""
    fc = _lib()
    s = W.subband(15, 14, 600, 8, n_short, n_long, 0, "sync_ola")
    p = fc.Plan([s], device=-1)
    _, lens, P = stream_offsets([s])
    lo, hi = p.layout(fc.OP_TX)
    assert hi[-1] == lens[0] and lo[-1] == P[0]["n_in"]
    assert list(p.symbols(0)[0]) == P[0]["ncp"]
    assert p.stats(fc.OP_TX)["blocks"] == 28


@pytest.mark.parametrize("case", sorted(BAD))
def test_validation(case):
    fc = _lib()
    patch, code = BAD[case]
    s = dict(W.plain_tx_slot()[0][0])
    s.update(patch)
    with pytest.raises(fc.FcError) as ei:
        fc.Plan([s], device=-1)
    assert ei.value.status == CODES[code]


def test_nonfinite_weights_rejected():
    fc = _lib()
    p = _plan(W.plain_tx_slot()[0])
    w = np.ones(512, dtype=np.float32)
    w[7] = np.nan
    with pytest.raises(fc.FcError) as ei:
        p.set_weights(0, w)
    assert ei.value.status == -1
    with pytest.raises(ValueError):
        p.set_weights(0, np.ones(10))


def test_compute_on_host_plan_is_state_error():
    fc = _lib()
    p = _plan(W.plain_tx_slot()[0])
    st = fc.lib().fc_tx_synthesize(p._h, ctypes.c_void_p(1), ctypes.c_void_p(1), None)
    assert st == -6


def test_sync_ols_tx_and_no_adjoint():
    """Synchronised OLS has a TX (output windows after the convolution, same
    blocks and layout as synchronised OLA) but no adjoint."""
    fc = _lib()
    s = dict(W.rx_filterbank(14)[0][0])
    p = _plan([s])
    q = _plan([dict(s, mode="sync_ola")])
    assert list(p.layout(fc.OP_TX)[0]) == list(q.layout(fc.OP_TX)[0])
    assert list(p.layout(fc.OP_TX)[1]) == list(q.layout(fc.OP_TX)[1])
    assert p.stats(fc.OP_TX)["blocks"] == q.stats(fc.OP_TX)["blocks"]
    with pytest.raises(fc.FcError):
        p.layout(fc.OP_ADJ)
    p.layout(fc.OP_RX)


def test_tuning_host_plan():
    """Run lengths change the task split, never the blocks; bad values are rejected."""
    fc = _lib()
    sbs, _ = W.mixed_numerology()
    p = _plan(sbs)
    base = p.stats(fc.OP_TX)
    assert p.get_tuning(fc.OP_TX) == dict(run_len=0, conc=4)
    p.set_tuning(fc.OP_TX, run_len=2, conc=1)
    assert p.get_tuning(fc.OP_TX) == dict(run_len=2, conc=1)
    st = p.stats(fc.OP_TX)
    assert st["blocks"] == base["blocks"] and st["tasks"] == base["blocks"] // 2
    p.set_tuning(fc.OP_RX, run_len=4, conc=2)
    assert p.stats(fc.OP_RX)["blocks"] == base["blocks"]
    for bad in (dict(run_len=-1), dict(conc=0), dict(conc=5), dict(run_len=257)):
        with pytest.raises(fc.FcError, match="FC_E_ARG|invalid argument"):
            p.set_tuning(fc.OP_TX, **dict(dict(run_len=0, conc=4), **bad))


def test_transform_plan_host_plan():
    """Transform plans 0/1 per op: set, read back (op and per-class counts),
    the blocks unchanged; out-of-range values rejected."""
    fc = _lib()
    sbs, _ = W.batched_carriers(n_carriers=8)
    p = _plan(sbs, io="f16")
    base = p.stats(fc.OP_TX)
    for op in (fc.OP_TX, fc.OP_RX, fc.OP_ADJ, fc.OP_RXD, fc.OP_TXG):
        assert p.get_transform_plan(op) == 0
        n, n1 = p.get_class_plans(op)
        assert 0 <= n and n1 == 0
        p.set_transform_plan(op, 1)
        assert p.get_transform_plan(op) == 1
        assert p.get_class_plans(op) == (n, n)      # every class with two plans now runs plan 1
    # the 8 carriers' pruned TX classes with n_short <= 1024 have two plans
    assert p.get_class_plans(fc.OP_TX)[0] > 0
    assert p.stats(fc.OP_TX)["blocks"] == base["blocks"]
    for bad in (-1, 2):
        with pytest.raises(fc.FcError, match="invalid argument"):
            p.set_transform_plan(fc.OP_TX, bad)
    with pytest.raises(fc.FcError, match="invalid argument"):
        p.set_transform_plan(7, 0)


def test_autotune_host_plan_rejected():
    """The autotuner needs a device plan: a host-only plan gets FC_E_STATE and
    missing buffers or an unknown op FC_E_ARG, before any device call; the
    result pointers and the tuning are left alone."""
    import ctypes
    fc = _lib()
    E_ARG, E_STATE = -1, -6                    # fc_status values of include/fc.h
    sbs, _ = W.mixed_numerology()
    p = _plan(sbs)
    L = fc.lib()
    r, c, ms = ctypes.c_int32(-7), ctypes.c_int32(-7), ctypes.c_float(-1.0)
    dummy = ctypes.c_void_p(16)                # never dereferenced: the calls fail first
    out = (ctypes.byref(r), ctypes.byref(c), ctypes.byref(ms))
    assert L.fc_plan_autotune(p._h, fc.OP_TX, dummy, dummy, None, *out) == E_STATE
    assert L.fc_plan_autotune(p._h, fc.OP_TX, None, dummy, None, *out) == E_ARG
    assert L.fc_plan_autotune(p._h, fc.OP_TX, dummy, None, None, *out) == E_ARG
    assert L.fc_plan_autotune(p._h, 7, dummy, dummy, None, *out) == E_ARG
    assert L.fc_plan_autotune(None, fc.OP_TX, dummy, dummy, None, *out) == E_ARG
    assert (r.value, c.value, ms.value) == (-7, -7, -1.0)
    assert p.get_tuning(fc.OP_TX) == dict(run_len=0, conc=4)


def test_rx_demod_layout_and_validity():
    """The demodulating RX has the synchronised RX layout (L values per symbol)
    and needs synchronised subbands."""
    fc = _lib()
    sbs, _ = W.mixed_numerology("sync_ols")
    p = _plan(sbs)
    assert list(p.layout(fc.OP_RXD)[0]) == list(p.layout(fc.OP_RX)[0])
    st = p.stats(fc.OP_RXD)
    assert st["blocks"] == p.stats(fc.OP_RX)["blocks"]
    s = W.subband(15, 2, 96, 8, 128, 1024, 0, "cont_ols")
    with pytest.raises(fc.FcError):
        _plan([s]).layout(fc.OP_RXD)


def test_rx_demod_tasks_hold_whole_symbols():
    fc = _lib()
    sbs, _ = W.rx_filterbank(n_symbols=10)
    p = _plan(sbs)
    for run_len in (1, 3, 5):
        p.set_tuning(fc.OP_RXD, run_len, 1)
        # 20 blocks in runs of run_len rounded up to even
        k = run_len + (run_len & 1)
        assert p.stats(fc.OP_RXD)["tasks"] == -(-20 // k)


def test_tx_grid_layout_and_validity():
    """The grid-input TX reads n_symbols * n_active values per subband and
    needs synchronised subbands; its blocks are the TX blocks."""
    fc = _lib()
    sbs, _ = W.mixed_numerology("sync_ola")
    p = _plan(sbs)
    lo, hi = p.layout(fc.OP_TXG)
    assert list(np.diff(lo)) == [s["n_symbols"] * s["n_active"] for s in sbs]
    assert list(hi) == list(p.layout(fc.OP_TX)[1])
    assert p.stats(fc.OP_TXG) == p.stats(fc.OP_TX)
    s = W.subband(15, 2, 96, 8, 128, 1024, 0, "cont_ols")
    with pytest.raises(fc.FcError):
        _plan([s]).layout(fc.OP_TXG)


def test_tuning_rejects_missing_op():
    fc = _lib()
    s = W.subband(15, 2, 96, 8, 128, 1024, 0, "sync_ols")
    with pytest.raises(fc.FcError):
        _plan([s]).set_tuning(fc.OP_ADJ, 8, 1)


def test_graph_calls_reject_bad_arguments():
    fc = _lib()
    L = fc.lib()
    assert L.fc_graph_begin(None) == -1
    assert L.fc_graph_end(None, None) == -1
    assert L.fc_graph_launch(None, None) == -1
    L.fc_graph_destroy(None)


def test_sync_ols_taper_plan():
    """A taper changes neither the layout nor the receiver; the longest taper
    the CP schedule allows (T/2 = N_L - max N_CP,n = 512 - 160) is accepted."""
    fc = _lib()
    s = dict(W.plain_tx_slot()[0][0], mode="sync_ols")
    p0 = fc.Plan([s], device=-1)
    p1 = fc.Plan([dict(s, taper=704)], device=-1)
    for op in (fc.OP_TX, fc.OP_RX, fc.OP_RXD, fc.OP_TXG):
        assert [list(a) for a in p0.layout(op)] == [list(a) for a in p1.layout(op)]
    assert p1.stats(fc.OP_TX)["blocks"] == p0.stats(fc.OP_TX)["blocks"]
    assert p1.stats(fc.OP_RX) == p0.stats(fc.OP_RX)

