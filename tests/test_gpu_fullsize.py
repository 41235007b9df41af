"""Parity at the benchmark's full sizes, in the launch configuration that
bench.py times (autotuned work split), on outputs the oracle can compute one
piece at a time.

TX: 256 uneven carriers x 32 slot-batches (8192 streams), FP16 I/Q; sampled
carriers of sampled batches against the oracle (FP16 gate -60 dB); the same
carriers x 8 batches in FP32 storage (gate -100 dB).
RX: 8 subbands of a 100 MHz carrier x 100 frames, BF16 I/Q; the first 14
symbols of sampled frames against the oracle (BF16 gate -50 dB), for the
time-domain analysis and for the demodulating receiver; 20 frames of the
time-domain analysis in FP32 storage (gate -100 dB).
"""
import numpy as np
import pytest

from fc_cases import (GATE_DB, from_device, make_inputs, oracle_rx, oracle_rxd, oracle_tx, rx_frame_input,
                      stream_offsets, to_device)
from fcsynth import workloads as W
from oracle import metrics
from oracle import weights as ow

pytestmark = pytest.mark.gpu

TX_BATCHES = 32
RX_FRAMES = 100


@pytest.mark.parametrize("io,batches", [("f16", TX_BATCHES), ("c64", 8)], ids=["f16", "fp32"])
def test_batched_tx_full_size(io, batches):
    # FP32 storage: the same carrier set, 8 slot-batches (the FP32 kernel
    # instances at their real shapes; 2048 streams still fill the chip)
    import torch
    from paper_2008_00672_amd import OP_TX, Plan
    sbs, meta = W.batched_carriers()
    allsb = [dict(s, stream=b * len(sbs) + k) for b in range(batches) for k, s in enumerate(sbs)]
    p = Plan(allsb, io=io, device=0)
    xs, _, _ = make_inputs(sbs, meta["qam"], meta["seed"], "rc")
    x1 = to_device(np.concatenate(xs), io)
    x = (x1.repeat(batches) if x1.dim() == 1 else x1.repeat(batches, 1)).contiguous()
    lo, hi = p.layout(OP_TX)
    assert x.shape[0] == lo[-1]
    y = p.empty(int(hi[-1]))
    tune = p.autotune(OP_TX, x, y)
    print("TX autotune:", tune, flush=True)
    y = p.tx(x, y)
    torch.cuda.synchronize()
    for b in (0, batches // 2 - 3, batches - 1):
        for k in (0, 1, 2, 77, 128, 200, 255):
            j = b * len(sbs) + k
            got = from_device(y[int(hi[j]):int(hi[j + 1])], io)
            s = dict(sbs[k], stream=0)
            ref = oracle_tx([s], [xs[k]], [ow.rc_weights(s["n_short"], s["n_active"], s["n_tb"])])[0]
            e = metrics.err_db(got, ref)
            print("batch %d carrier %d (L %d N %d): err %.1f dB" % (b, k, s["n_short"], s["n_long"], e), flush=True)
            assert e <= GATE_DB[io]


@pytest.mark.parametrize("demod,io,frames", [(False, "bf16", RX_FRAMES), (True, "bf16", RX_FRAMES),
                                              (False, "c64", 20)], ids=["rx", "rx_demod", "rx_fp32"])
def test_rx_filterbank_full_size(demod, io, frames):
    # FP32 storage runs its own kernel instance (three waves per SIMD); 20
    # frames are enough workgroups to fill the chip several times over
    import torch
    from paper_2008_00672_amd import OP_RX, OP_RXD, Plan
    sbs, meta = W.rx_filterbank()
    op = OP_RXD if demod else OP_RX
    allsb = [dict(s, stream=f) for f in range(frames) for s in sbs]
    p = Plan(allsb, io=io, device=0)
    y1 = rx_frame_input(sbs, meta["qam"], meta["seed"], meta["snr_db"])
    lo, hi = p.layout(op)
    assert len(y1) == hi[1] - hi[0]
    t = to_device(y1, io)
    r = (t.repeat(frames) if t.dim() == 1 else t.repeat(frames, 1)).contiguous()
    z = p.empty(int(lo[-1]))
    tune = p.autotune(op, r, z)
    print("autotune:", tune, flush=True)
    z = p.rx_demod(r, z) if demod else p.rx(r, z)
    torch.cuda.synchronize()
    B = 14
    sub = [dict(s, n_symbols=B) for s in sbs]
    _, lens, _ = stream_offsets(sub)
    Ds = [ow.rc_weights(s["n_short"], s["n_active"], s["n_tb"]) for s in sbs]
    refs = (oracle_rxd if demod else oracle_rx)(sub, [y1[:lens[0]]], Ds)
    for f in (0, frames // 2 - 9, frames - 1):
        for m, ref in enumerate(refs):
            j = f * len(sbs) + m
            got = from_device(z[int(lo[j]):int(lo[j]) + len(ref)], io)
            e = metrics.err_db(got, ref)
            print("frame %d subband %d (L %d): err %.1f dB" % (f, m, sbs[m]["n_short"], e), flush=True)
            assert e <= GATE_DB[io]
