"""GPU runtime features through the C ABI: tuning invariance (outputs and
the weight gradient), HIP graph capture and replay, the autotuner.

The work split (blocks per task, concurrent launches) does not change the
arithmetic of any block, so outputs must be bit-identical across tunings;
graph replays must reproduce the eager call exactly, replay after replay,
with eager work and synchronisations in between.
"""
import numpy as np
import pytest

from fc_cases import make_inputs, oracle_tx, stream_offsets, to_device
from fcsynth import workloads as W
from oracle import metrics
from test_gpu_parity import _cat, _plan, _split

pytestmark = pytest.mark.gpu


def _mixed(io="c64"):
    sbs, meta = W.mixed_numerology("sync_ola")
    xs, Ds, _ = make_inputs(sbs, meta["qam"], meta["seed"], "rc")
    p = _plan(sbs, io, Ds)
    return sbs, xs, Ds, p


def _batched(n=24, io="f16"):
    sbs, meta = W.batched_carriers(n_carriers=n)
    xs, Ds, _ = make_inputs(sbs, meta["qam"], meta["seed"], "rc")
    return sbs, xs, Ds, _plan(sbs, io, Ds)


@pytest.mark.parametrize("op", ["tx", "rx", "adjoint"])
def test_tuning_is_bit_exact(op):
    import torch
    from paper_2008_00672_amd import OP_RX, OP_TX
    sbs, xs, Ds, p = _batched()
    if op == "tx":
        inp = to_device(_cat(xs), "f16")
        call, code = p.tx, OP_TX
    elif op == "adjoint":
        _, lens, _ = stream_offsets(sbs)
        rng = np.random.default_rng(5)
        inp = to_device(rng.standard_normal(sum(lens)) + 1j * rng.standard_normal(sum(lens)), "f16")
        call, code = p.adjoint, 2
    else:
        _, lens, _ = stream_offsets(sbs)
        rng = np.random.default_rng(3)
        inp = to_device(rng.standard_normal(sum(lens)) + 1j * rng.standard_normal(sum(lens)), "f16")
        call, code = p.rx, OP_RX
    ref = call(inp).clone()
    torch.cuda.synchronize()
    for run_len, conc in [(2, 1), (8, 4), (16, 2), (64, 4), (0, 1)]:
        p.set_tuning(code, run_len, conc)
        out = call(inp)
        torch.cuda.synchronize()
        print("%s run_len %d conc %d: equal %s" % (op, run_len, conc, torch.equal(out, ref)), flush=True)
        assert torch.equal(out, ref)


@pytest.mark.parametrize("shape", ["carriers", "shared_long"])
def test_weight_grad_is_deterministic(shape):
    """The weight gradient stores per-task partial sums and reduces them in
    block order: bitwise the same for every tuning and on repeated calls.
    carriers: one-subband groups (sums in registers); shared_long: eight
    subbands sharing one long transform (sums in LDS)."""
    import torch
    if shape == "carriers":
        sbs, xs, Ds, p = _batched()
        io = "f16"
    else:
        fb, meta = W.rx_filterbank()
        sbs = [dict(s, mode="sync_ola", n_symbols=14) for s in fb]
        xs, Ds, _ = make_inputs(sbs, meta["qam"], meta["seed"], "rc")
        io = "bf16"
        p = _plan(sbs, io, Ds)
    print("case: weight gradient determinism, %s, %s" % (shape, io), flush=True)
    _, lens, _ = stream_offsets(sbs)
    rng = np.random.default_rng(8)
    g = to_device(rng.standard_normal(sum(lens)) + 1j * rng.standard_normal(sum(lens)), io)
    x = to_device(_cat(xs), io)
    ref = p.weight_grad(x, g).clone()
    torch.cuda.synchronize()
    assert torch.isfinite(ref).all() and ref.abs().max() > 0
    for run_len, conc in [(1, 1), (2, 4), (4, 2), (16, 4), (0, 1)]:
        p.set_tuning(2, run_len, conc)
        for rep in range(2):
            out = p.weight_grad(x, g)
            torch.cuda.synchronize()
            same = torch.equal(out.view(torch.int32), ref.view(torch.int32))
            print("run_len %d conc %d call %d: bitwise equal %s" % (run_len, conc, rep, same), flush=True)
            assert same


@pytest.mark.parametrize("op", ["tx", "tx_grid", "rx", "rx_demod", "adjoint"])
def test_transform_plan_1_parity(op):
    """Transform plan 1 (the other short-FFT placement of the pruned TX, the
    lower-radix long FFT of the RX family) against the oracle: the TX on 12
    batched carriers (FP16), the RX family on the 100 MHz filter bank (14
    symbols, FP32)."""
    import torch
    from fc_cases import assert_gate, oracle_adj, oracle_rx, oracle_rxd, oracle_tx, oracle_tx_grid
    from paper_2008_00672_amd import OP_ADJ, OP_RX, OP_RXD, OP_TX, OP_TXG
    print("case: transform plan 1, %s" % op, flush=True)
    if op in ("tx", "tx_grid"):
        sbs, meta = W.batched_carriers(n_carriers=12)
        xs, Ds, grids = make_inputs(sbs, meta["qam"], meta["seed"], "rc")
        p = _plan(sbs, "f16", Ds)
        code = OP_TX if op == "tx" else OP_TXG
        p.set_transform_plan(code, 1)
        _, hi = p.layout(code)
        if op == "tx":
            y, ref = p.tx(to_device(_cat(xs), "f16")), oracle_tx(sbs, xs, Ds)
        else:
            y = p.tx_grid(to_device(np.concatenate([g.ravel() for g in grids]), "f16"))
            ref = oracle_tx_grid(sbs, grids, Ds)
        torch.cuda.synchronize()
        f = y.to(torch.float32).cpu().numpy()
        assert_gate(_split(f[:, 0] + 1j * f[:, 1], hi), ref, "f16", op)
        return
    fb, meta = W.rx_filterbank(14)
    sbs = [dict(s, mode="sync_ola") for s in fb]
    _, Ds, _ = make_inputs(sbs, 4, 5, "rc")
    p = _plan(sbs, "c64", Ds)
    code = {"rx": OP_RX, "rx_demod": OP_RXD, "adjoint": OP_ADJ}[op]
    p.set_transform_plan(code, 1)
    _, lens, _ = stream_offsets(sbs)
    rng = np.random.default_rng(6)
    st = rng.standard_normal(lens[0]) + 1j * rng.standard_normal(lens[0])
    lo, _ = p.layout(code)
    call = {"rx": p.rx, "rx_demod": p.rx_demod, "adjoint": p.adjoint}[op]
    z = call(to_device(st, "c64"))
    torch.cuda.synchronize()
    ref = {"rx": oracle_rx, "rx_demod": oracle_rxd, "adjoint": oracle_adj}[op](sbs, [st], Ds)
    assert_gate(_split(z.cpu().numpy().astype(np.complex128), lo), ref, "c64", op)


def test_autotune_chooses_transform_plan():
    """The autotuner sweeps both transform plans where they differ and keeps a
    choice whose output still meets the gate."""
    import torch
    from fc_cases import assert_gate
    from paper_2008_00672_amd import OP_RX
    fb, meta = W.rx_filterbank(28)
    sbs = [dict(s, mode="sync_ola", stream=f) for f in range(8) for s in fb]
    _, Ds, _ = make_inputs(sbs, 4, 5, "rc")
    p = _plan(sbs, "c64", Ds)
    _, lens, _ = stream_offsets(sbs)
    rng = np.random.default_rng(7)
    st = to_device(rng.standard_normal(sum(lens)) + 1j * rng.standard_normal(sum(lens)), "c64")
    z = p.empty(int(p.layout(OP_RX)[0][-1]))
    best = p.autotune(OP_RX, st, z, stream=torch.cuda.Stream())
    print("autotune RX with transform plans:", best, flush=True)
    assert best["plan"] in (0, 1) and p.get_transform_plan(OP_RX) == best["plan"]
    ref = p.rx(st).clone()
    p.set_transform_plan(OP_RX, 1 - best["plan"])
    other = p.rx(st)
    torch.cuda.synchronize()
    lo, _ = p.layout(OP_RX)
    a = _split(ref.cpu().numpy().astype(np.complex128), lo)
    b = _split(other.cpu().numpy().astype(np.complex128), lo)
    assert_gate(a, b, "c64", "plan 0 against plan 1")


def test_graph_replay_matches_eager():
    """TX and RX of two plans captured in one graph; three replays, each
    after eager work that clobbers the outputs, each equal to the eager call."""
    import torch
    from paper_2008_00672_amd import Graph, OP_RX
    sbs, xs, Ds, p = _mixed()
    x = to_device(_cat(xs), "c64")
    sbs_r, _, Ds_r, pr = _batched(8, "c64")
    _, lens, _ = stream_offsets(sbs_r)
    rng = np.random.default_rng(4)
    yr = to_device(rng.standard_normal(sum(lens)) + 1j * rng.standard_normal(sum(lens)), "c64")
    y = p.tx(x)
    z = pr.rx(yr)
    torch.cuda.synchronize()
    y_ref, z_ref = y.clone(), z.clone()
    s = torch.cuda.Stream()
    with Graph(s) as g:
        p.tx(x, y, stream=s)
        pr.rx(yr, z, stream=s)
    for rep in range(3):
        y.fill_(float("nan"))
        z.zero_()
        torch.cuda.synchronize()
        g.launch()
        s.synchronize()
        ok = torch.equal(y, y_ref) and torch.equal(z, z_ref)
        print("replay %d equal %s" % (rep, ok), flush=True)
        assert ok
        # eager work on the default stream in between
        (y_ref * 2).sum().item()
    g.close()


def test_graph_sees_new_weights():
    """Weights are read when the kernels run: a replay after fc_set_weights
    gives the new weights' output (checked against the oracle)."""
    import torch
    from paper_2008_00672_amd import Graph
    sbs, xs, Ds, p = _mixed()
    x = to_device(_cat(xs), "c64")
    y = p.tx(x)
    s = torch.cuda.Stream()
    with Graph(s) as g:
        p.tx(x, y, stream=s)
    rng = np.random.default_rng(9)
    D2 = [rng.uniform(-1, 1, len(D)) for D in Ds]
    for i, D in enumerate(D2):
        p.set_weights(i, D)
    g.launch()
    s.synchronize()
    _, lens, _ = stream_offsets(sbs)
    got = _split(y.cpu().numpy().astype(np.complex128), np.cumsum([0] + lens))
    ref = oracle_tx(sbs, xs, [D.astype(np.float32).astype(np.float64) for D in D2])
    for a, b in zip(got, ref):
        e = metrics.err_db(a, b)
        print("graph with new weights: err %.1f dB" % e, flush=True)
        assert e <= -100.0
    g.close()


def test_graph_weight_grad_and_demod():
    """The weight gradient's scratch is allocated by its first call, which a
    capture refuses (FC_E_STATE, nothing recorded); after one eager call the
    gradient and the demodulating RX (whose scratch comes with the plan) are
    captured together and every replay equals the eager calls bit for bit."""
    import torch
    from paper_2008_00672_amd import Graph, OP_RXD
    from paper_2008_00672_amd.fc import FcError
    sbs, xs, Ds, p = _mixed()
    x = to_device(_cat(xs), "c64")
    _, lens, _ = stream_offsets(sbs)
    rng = np.random.default_rng(6)
    gy = to_device(rng.standard_normal(sum(lens)) + 1j * rng.standard_normal(sum(lens)), "c64")
    gw = torch.empty(sum(sb["n_short"] for sb in sbs), dtype=torch.float32, device="cuda:0")
    z = p.empty(int(p.layout(OP_RXD)[0][-1]))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with pytest.raises(FcError) as e:
        with Graph(s):
            p.weight_grad(x, gy, gw, stream=s)
    print("first weight gradient under capture:", e.value, flush=True)
    assert e.value.status == -6
    gw_ref = p.weight_grad(x, gy).clone()
    z_ref = p.rx_demod(gy).clone()
    torch.cuda.synchronize()
    with Graph(s) as g:
        p.weight_grad(x, gy, gw, stream=s)
        p.rx_demod(gy, z, stream=s)
    for rep in range(3):
        gw.fill_(float("nan"))
        z.zero_()
        torch.cuda.synchronize()
        g.launch()
        s.synchronize()
        ok = torch.equal(gw, gw_ref) and torch.equal(z, z_ref)
        print("replay %d equal %s" % (rep, ok), flush=True)
        assert ok
        (gw_ref * 2).sum().item()
    g.close()


def test_graph_demod_with_scratch():
    """The demodulating RX whose second-block terms go to device scratch (the
    100 MHz filter bank in BF16, four frames): graph replays equal the eager
    call bit for bit, with eager work in between."""
    import torch
    from paper_2008_00672_amd import Graph, OP_RXD
    fb, meta = W.rx_filterbank(28)
    sbs = [dict(s, stream=f) for f in range(4) for s in fb]
    _, Ds, _ = make_inputs(sbs, 4, 5, "rc")
    p = _plan(sbs, "bf16", Ds)
    _, lens, _ = stream_offsets(sbs)
    rng = np.random.default_rng(8)
    y = to_device(rng.standard_normal(sum(lens)) + 1j * rng.standard_normal(sum(lens)), "bf16")
    z = p.empty(int(p.layout(OP_RXD)[0][-1]))
    ref = p.rx_demod(y).clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with Graph(s) as g:
        p.rx_demod(y, z, stream=s)
    for rep in range(3):
        z.zero_()
        torch.cuda.synchronize()
        g.launch()
        s.synchronize()
        ok = torch.equal(z, ref)
        print("replay %d equal %s" % (rep, ok), flush=True)
        assert ok
        (ref.float() * 2).sum().item()
    g.close()


@pytest.mark.parametrize("side_stream", [False, True], ids=["null_stream", "side_stream"])
def test_autotune_keeps_results(side_stream):
    # On the null stream the candidates run eagerly; on another stream each is
    # captured as a graph and replayed. Either way the stream is left usable.
    import torch
    from paper_2008_00672_amd import OP_TX
    sbs, xs, Ds, p = _batched(48)
    x = to_device(_cat(xs), "f16")
    ref = p.tx(x).clone()
    out = p.empty(ref.shape[0])
    s = torch.cuda.Stream() if side_stream else None
    torch.cuda.synchronize()
    best = p.autotune(OP_TX, x, out, stream=s)
    print("autotune TX (%s):" % ("side stream" if side_stream else "null stream"), best, flush=True)
    assert best["run_len"] in (0, 8, 16, 32, 64) and best["conc"] in (1, 4) and best["plan"] in (0, 1)
    assert best["ms"] > 0
    assert p.get_tuning(OP_TX) == dict(run_len=best["run_len"], conc=best["conc"])
    assert (best["classes_two_plans"], best["classes_plan1"]) == p.get_class_plans(OP_TX)
    y = p.tx(x, stream=s)
    torch.cuda.synchronize()
    if best["classes_plan1"] == 0:
        assert torch.equal(y, ref)           # every class on plan 0: the same bits
    else:                                    # the other plan rounds differently
        from fc_cases import assert_gate
        f, g = y.to(torch.float32).cpu().numpy(), ref.to(torch.float32).cpu().numpy()
        assert_gate([f[:, 0] + 1j * f[:, 1]], [g[:, 0] + 1j * g[:, 1]], "f16", "plan 1 against plan 0")
