"""Mixed-radix transform lengths on the GPU: short transforms of 768 = 3 x 256
points (the paper's example of a non-power-of-two length for the full-band
channel filter, Sec. VI-C) and long transforms of 768, 1536 and 3072 points,
against the FP64 oracle (whose dense DFTs take any length) at the FP32 gate.

TX continuous (OLS, OLA) and synchronised (OLA, OLS), RX, the adjoint, the
demodulating RX, the grid-input TX, two 768-point subbands sharing a long
transform, the weight gradient, and the four chains of the 52-PRB wide-band
case at I = 1 (L = N = 768) against the oracle's.
"""
import numpy as np
import pytest

from fc_cases import assert_gate, make_inputs, oracle_tx_grid, oracle_wgrad, stream_offsets, to_device
from fcsynth import workloads as W
from test_gpu_parity import _cat, _plan, _split, run_rx, run_tx

pytestmark = pytest.mark.gpu


def sb(mode, L, N, K, c, n_sym=14, n_tb=8, stream=0, taper=0):
    return W.subband(15, n_sym, K, n_tb, L, N, c, mode, stream=stream, taper=taper)


CASES = {
    "cont_ols_768_1536": [sb("cont_ols", 768, 1536, 600, 100)],
    "cont_ola_768_3072": [sb("cont_ola", 768, 3072, 480, -700)],
    "cont_ols_768_768": [sb("cont_ols", 768, 768, 624, 0)],
    "sync_ola_768_768": [sb("sync_ola", 768, 768, 624, 0)],
    "sync_ola_768_1536": [sb("sync_ola", 768, 1536, 612, -200, n_sym=7)],
    "sync_ols_768_1536": [sb("sync_ols", 768, 1536, 612, 150, n_sym=7)],
    "sync_ola_1536_3072": [sb("sync_ola", 1536, 3072, 1200, 300, n_sym=5)],
    "sync_ola_3072_3072": [sb("sync_ola", 3072, 3072, 2400, 0, n_sym=4)],
    "two_768_in_3072": [sb("sync_ola", 768, 3072, 600, -500, n_sym=7),
                        sb("sync_ola", 768, 3072, 360, 600, n_sym=7, n_tb=12)],
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_tx(name):
    print("case: mixed-radix TX %s" % name, flush=True)
    got, ref = run_tx(CASES[name], "c64", seed=31)
    assert_gate(got, ref, "c64", name)


@pytest.mark.parametrize("name", sorted(CASES))
def test_rx(name):
    print("case: mixed-radix RX %s" % name, flush=True)
    got, ref = run_rx(CASES[name], "c64", seed=32)
    assert_gate(got, ref, "c64", name)


@pytest.mark.parametrize("name", [n for n in sorted(CASES) if "ols_" not in n or n.startswith("cont")])
def test_adjoint(name):
    print("case: mixed-radix adjoint %s" % name, flush=True)
    got, ref = run_rx(CASES[name], "c64", seed=33, adjoint=True)
    assert_gate(got, ref, "c64", name)


@pytest.mark.parametrize("name", [n for n in sorted(CASES) if n.startswith("sync") or n.startswith("two")])
def test_rx_demod(name):
    print("case: mixed-radix demodulating RX %s" % name, flush=True)
    got, ref = run_rx(CASES[name], "c64", seed=34, demod=True)
    assert_gate(got, ref, "c64", name)


@pytest.mark.parametrize("name", ["sync_ola_768_768", "sync_ols_768_1536", "two_768_in_3072"])
def test_tx_grid(name):
    import torch
    from paper_2008_00672_amd import OP_TXG
    subbands = CASES[name]
    print("case: mixed-radix grid-input TX %s" % name, flush=True)
    _, Ds, grids = make_inputs(subbands, 16, 35, "rc")
    p = _plan(subbands, "c64", Ds)
    lo, hi = p.layout(OP_TXG)
    y = p.tx_grid(to_device(np.concatenate([g.ravel() for g in grids]), "c64"))
    torch.cuda.synchronize()
    got = _split(y.cpu().numpy().astype(np.complex128), hi)
    assert_gate(got, oracle_tx_grid(subbands, grids, Ds), "c64", name)


@pytest.mark.parametrize("name", ["cont_ols_768_1536", "sync_ola_768_768", "sync_ola_1536_3072", "two_768_in_3072"])
def test_weight_grad(name):
    import torch
    from oracle import metrics
    subbands = CASES[name]
    print("case: mixed-radix weight gradient %s" % name, flush=True)
    xs, Ds, _ = make_inputs(subbands, 16, 36, "random")
    p = _plan(subbands, "c64", Ds)
    _, lens, _ = stream_offsets(subbands)
    rng = np.random.default_rng(37)
    gs = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in lens]
    gw = p.weight_grad(to_device(_cat(xs), "c64"), to_device(_cat(gs), "c64"))
    torch.cuda.synchronize()
    offs = np.concatenate([[0], np.cumsum([s["n_short"] for s in subbands])])
    got = _split(gw.cpu().numpy().astype(np.float64), offs)
    bins = [sorted(rng.choice(s["n_short"], size=12, replace=False).tolist()) for s in subbands]
    ref = oracle_wgrad(subbands, xs, gs, bins)
    for k, (g, r, b) in enumerate(zip(got, ref, bins)):
        e = metrics.err_db(g[b], r[b])
        print("subband %d: weight-gradient err %.1f dB" % (k, e), flush=True)
        assert e <= -90.0


def test_wideband_768_chains():
    """The four chains of the 52-PRB wide-band case with L = N = 768 (I = 1)."""
    from wideband import Setup, gpu_chains, oracle_chains
    print("case: wide-band 52 PRB, L = N = 768, four chains", flush=True)
    S = Setup(768)
    y_ref, ref = oracle_chains(S)
    y_gpu, got = gpu_chains(S)
    for k in ("cont", "sync"):
        print("%s TX: OOB %.2f dB (oracle %.2f)" % (k, got["oob_db"][k], ref["oob_db"][k]), flush=True)
        assert_gate([y_gpu[k]], [y_ref[k]], "c64", "%s TX" % k)
        assert abs(got["oob_db"][k] - ref["oob_db"][k]) < 0.1
    for k, v in ref["evm_db"].items():
        print("%s: EVM %.3f dB (oracle %.3f)" % (k, got["evm_db"][k], v), flush=True)
        assert abs(got["evm_db"][k] - v) < 0.05
