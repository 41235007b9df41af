"""Parity at the benchmark's full sizes, in the launch configuration that
bench.py times (autotuned work split).

The slot-batches (TX) and frames (RX) of these workloads repeat one input,
so every batch's or frame's output must equal the first one's bit for bit
(the planner gives every stream the same blocks and task boundaries): that
check covers the whole output at no oracle cost. The first batch / frame is
then checked against the oracle in full:

TX: 256 uneven carriers x 32 slot-batches (8192 streams), FP16 I/Q; all 256
carriers of the first batch against the oracle (in four chunks, each within
the per-test time limit); the same carriers x 8 batches in FP32 storage, with
sampled carriers against the oracle.
RX: 8 subbands of a 100 MHz carrier x 100 frames, BF16 I/Q; all 280 symbols
of all 8 subbands of the first frame against the oracle, for the time-domain
analysis and for the demodulating receiver; 20 frames of the time-domain
analysis in FP32 storage, likewise.
Each comparison takes the L2 gate and the per-sample bound of
fc_cases.assert_gate.
"""
import numpy as np
import pytest

from fc_cases import assert_gate, from_device, make_inputs, oracle_rx, oracle_rxd, oracle_tx, rx_frame_input, to_device
from fcsynth import workloads as W
from oracle import weights as ow

pytestmark = pytest.mark.gpu

TX_BATCHES = 32
RX_FRAMES = 100
TX_CHUNKS = 4


def _bits(t):
    """Integer view of a device output (bitwise comparisons)."""
    import torch
    if t.is_complex():
        return torch.view_as_real(t).view(torch.int32)
    return t.view(torch.int16)


@pytest.fixture(scope="module", params=[("f16", TX_BATCHES), ("c64", 8)], ids=["f16", "fp32"])
def tx_full(request):
    # FP32 storage: the same carrier set, 8 slot-batches (the FP32 kernel
    # instances at their real shapes; 2048 streams still fill the chip)
    import torch
    from paper_2008_00672_amd import OP_TX, Plan
    io, batches = request.param
    print("case: batched TX full size, %s, %d batches" % (io, batches), flush=True)
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
    n1 = int(hi[len(sbs)])
    y0 = from_device(y[:n1], io)
    yield dict(io=io, batches=batches, sbs=sbs, xs=xs, y=y, hi=hi, n1=n1, y0=y0)
    del y, x


def test_tx_batches_bit_identical(tx_full):
    import torch
    y, n1, B = tx_full["y"], tx_full["n1"], tx_full["batches"]
    assert y.shape[0] == n1 * B
    first = _bits(y[:n1])
    for b in range(1, B):
        assert torch.equal(_bits(y[b * n1:(b + 1) * n1]), first), "batch %d differs from batch 0" % b


def _check_carriers(tx_full, carriers):
    io, sbs, xs, hi, y0 = tx_full["io"], tx_full["sbs"], tx_full["xs"], tx_full["hi"], tx_full["y0"]
    got, ref = [], []
    for k in carriers:
        s = dict(sbs[k], stream=0)
        ref.append(oracle_tx([s], [xs[k]], [ow.rc_weights(s["n_short"], s["n_active"], s["n_tb"])])[0])
        got.append(y0[int(hi[k]):int(hi[k + 1])])
    assert_gate(got, ref, io, "carriers %s" % list(carriers))


@pytest.mark.parametrize("chunk", range(TX_CHUNKS))
def test_tx_first_batch_against_oracle(tx_full, chunk):
    n = len(tx_full["sbs"])
    if tx_full["io"] == "f16":
        carriers = range(chunk, n, TX_CHUNKS)          # every carrier of the first batch
    else:
        carriers = [k for k in (0, 1, 2, 77, 128, 200, 255) if k % TX_CHUNKS == chunk]
    _check_carriers(tx_full, carriers)


@pytest.fixture(scope="module", params=[(False, "bf16", RX_FRAMES), (True, "bf16", RX_FRAMES), (False, "c64", 20)],
                ids=["rx", "rx_demod", "rx_fp32"])
def rx_full(request):
    # FP32 storage runs its own kernel instance (three waves per SIMD); 20
    # frames are enough workgroups to fill the chip several times over
    import torch
    from paper_2008_00672_amd import OP_RX, OP_RXD, Plan
    demod, io, frames = request.param
    print("case: RX filter bank full size, %s, demod %s, %d frames" % (io, demod, frames), flush=True)
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
    n1 = int(lo[len(sbs)])
    yield dict(io=io, demod=demod, frames=frames, sbs=sbs, y1=y1, z=z, lo=lo, n1=n1, z0=from_device(z[:n1], io))
    del z, r


def test_rx_frames_bit_identical(rx_full):
    import torch
    z, n1, F = rx_full["z"], rx_full["n1"], rx_full["frames"]
    assert z.shape[0] == n1 * F
    first = _bits(z[:n1])
    for f in range(1, F):
        assert torch.equal(_bits(z[f * n1:(f + 1) * n1]), first), "frame %d differs from frame 0" % f


def test_rx_first_frame_against_oracle(rx_full):
    sbs, lo, z0 = rx_full["sbs"], rx_full["lo"], rx_full["z0"]
    Ds = [ow.rc_weights(s["n_short"], s["n_active"], s["n_tb"]) for s in sbs]
    refs = (oracle_rxd if rx_full["demod"] else oracle_rx)(sbs, [rx_full["y1"]], Ds)
    got = [z0[int(lo[m]):int(lo[m + 1])] for m in range(len(sbs))]
    assert_gate(got, refs, rx_full["io"], "all 280 symbols of frame 0")
