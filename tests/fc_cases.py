"""Test helpers: seeded inputs and oracle references for whole plans.

The oracle side computes stream alignment, CP schedules and outputs from
``oracle`` only; nothing here reads anything from the HIP path except the
outputs being checked.
"""
from fractions import Fraction

import numpy as np

import fcsynth
from oracle import fc as ofc
from oracle import grad as ogr
from oracle import lin as olin
from oracle import numerology as nu
from oracle import weights as ow


def sub_params(s):
    mu = nu.mu_of_scs(s["scs_khz"])
    L, N = s["n_short"], s["n_long"]
    lam = Fraction(*s.get("overlap", (1, 2)))
    ncp = s.get("ncp_high") or nu.nr_cp_list(N, mu, s.get("first_symbol", 0), s["n_symbols"])
    sync = s["mode"].startswith("sync")
    lcp = nu.lowrate_cp(ncp, N // L, exact=not sync)
    ov = nu.Overlap(L, N, lam)
    n_in = sum(L + c for c in lcp)
    Q = nu.sync_output_len(ncp, ov) if sync else nu.cont_output_len(n_in, ov)
    return dict(L=L, N=N, lam=lam, ncp=list(ncp), lcp=lcp, ov=ov, sync=sync, n_in=n_in, Q=Q,
                ola=s["mode"] in ("cont_ola", "sync_ola"), c=s["center_bin"], K=s["n_active"])


def stream_offsets(subbands):
    """Local-axis offset of every subband in its stream (first CPs aligned)
    and the stream lengths."""
    P = [sub_params(s) for s in subbands]
    T = [nu.first_cp_start(p["sync"], p["ov"], p["ncp"][0]) for p in P]
    n_st = max(s["stream"] for s in subbands) + 1
    tmax = [max(T[i] for i, s in enumerate(subbands) if s["stream"] == k) for k in range(n_st)]
    off = [tmax[s["stream"]] - T[i] for i, s in enumerate(subbands)]
    lens = [max(off[i] + P[i]["Q"] for i, s in enumerate(subbands) if s["stream"] == k) for k in range(n_st)]
    return off, lens, P


def make_inputs(subbands, qam_order, seed, weights="rc"):
    """Low-rate CP-OFDM input per subband (complex128) and weights per subband."""
    rng = np.random.default_rng(seed)
    xs, Ds, grids = [], [], []
    for s in subbands:
        p = sub_params(s)
        g = fcsynth.qam_grid(rng, qam_order, s["n_symbols"], p["K"])
        grids.append(g)
        xs.append(fcsynth.cp_ofdm(g, p["L"], p["lcp"]))
        if weights == "rc":
            Ds.append(ow.rc_weights(p["L"], p["K"], s["n_tb"]))
        else:
            Ds.append(rng.uniform(-1.0, 1.0, p["L"]))
    return xs, Ds, grids


def oracle_tx(subbands, xs, Ds, reference="fc"):
    off, lens, P = stream_offsets(subbands)
    streams = [np.zeros(n, dtype=complex) for n in lens]
    for i, s in enumerate(subbands):
        p = P[i]
        if reference == "fc":
            if p["sync"] and not p["ola"]:
                y = ofc.tx_sync_ols(xs[i], p["L"], p["N"], p["c"], Ds[i], p["ncp"], taper=s.get("taper", 0))
            elif p["sync"]:
                y = ofc.tx_sync(xs[i], p["L"], p["N"], p["c"], Ds[i], p["ncp"])
            else:
                y = ofc.tx_cont(xs[i], p["L"], p["N"], p["c"], Ds[i], lam=p["lam"], ola=p["ola"])
        else:
            if p["sync"]:
                y = olin.tx_sync_lin(xs[i], p["L"], p["N"], p["c"], Ds[i], p["ncp"])
            else:
                y = olin.tx_cont_lin(xs[i], p["L"], p["N"], p["c"], Ds[i], lam=p["lam"])
        streams[s["stream"]][off[i]:off[i] + len(y)] += y
    return streams


def oracle_tx_grid(subbands, grids, Ds):
    """Streams from QAM grids: CP-OFDM modulation with the truncated CP, then
    the synchronised FC TX (oracle), summed per stream."""
    off, lens, P = stream_offsets(subbands)
    streams = [np.zeros(n, dtype=complex) for n in lens]
    for i, s in enumerate(subbands):
        p = P[i]
        x = ofc.ofdm_modulate(grids[i], p["L"], p["lcp"])
        if p["ola"]:
            y = ofc.tx_sync(x, p["L"], p["N"], p["c"], Ds[i], p["ncp"])
        else:
            y = ofc.tx_sync_ols(x, p["L"], p["N"], p["c"], Ds[i], p["ncp"], taper=s.get("taper", 0))
        streams[s["stream"]][off[i]:off[i] + len(y)] += y
    return streams


def oracle_rx(subbands, streams, Ds):
    off, lens, P = stream_offsets(subbands)
    outs = []
    for i, s in enumerate(subbands):
        p = P[i]
        seg = streams[s["stream"]][off[i]:off[i] + p["Q"]]
        if p["sync"]:
            outs.append(ofc.rx_sync(seg, p["L"], p["N"], p["c"], Ds[i], p["ncp"]).ravel())
        else:
            outs.append(ofc.rx_cont(seg, p["L"], p["N"], p["c"], Ds[i], p["n_in"], lam=p["lam"], ola=p["ola"]))
    return outs


def oracle_rxd(subbands, streams, Ds):
    """Per subband (B, L) subcarrier values of the synchronised RX followed by
    OFDM demodulation (the direct definition), flattened symbol by symbol."""
    off, lens, P = stream_offsets(subbands)
    outs = []
    for i, s in enumerate(subbands):
        p = P[i]
        seg = streams[s["stream"]][off[i]:off[i] + p["Q"]]
        outs.append(ofc.rx_sync_subcarriers(seg, p["L"], p["N"], p["c"], Ds[i], p["ncp"]).ravel())
    return outs


def oracle_adj(subbands, streams, Ds):
    off, lens, P = stream_offsets(subbands)
    outs = []
    for i, s in enumerate(subbands):
        p = P[i]
        seg = streams[s["stream"]][off[i]:off[i] + p["Q"]]
        if p["sync"]:
            outs.append(ofc.rx_sync(seg, p["L"], p["N"], p["c"], Ds[i], p["ncp"], keep_cp=True))
        else:
            outs.append(ofc.rx_cont(seg, p["L"], p["N"], p["c"], Ds[i], p["n_in"], lam=p["lam"],
                                    ola=not p["ola"]))
    return outs


def rx_frame_input(subbands, qam_order, seed, snr_db):
    """One received frame for subbands sharing one stream and N: the
    subbands' QAM CP-OFDM from one N-point IDFT per symbol (NR CP from the
    oracle's numerology), placed so that the first symbol's useful part starts
    N/4 into the stream (the synchronised receiver's first block), plus AWGN
    at the given SNR over the signal power."""
    rng = np.random.default_rng(seed)
    P = [sub_params(s) for s in subbands]
    ncp = P[0]["ncp"]
    grids = [fcsynth.qam_grid(rng, qam_order, s["n_symbols"], s["n_active"]) for s in subbands]
    N = subbands[0]["n_long"]
    sig = fcsynth.cp_ofdm_highrate(grids, [s["center_bin"] for s in subbands], N, ncp)
    _, lens, _ = stream_offsets(subbands)
    y = np.zeros(lens[0], dtype=complex)
    lead = N // 4 - ncp[0]
    y[lead:lead + len(sig)] = sig
    y += fcsynth.awgn(rng, lens[0], np.mean(np.abs(sig) ** 2) * 10 ** (-snr_db / 10))
    return y


def subband_forward(subband, x):
    """D -> this subband's FC output (oracle), with its input x fixed."""
    p = sub_params(subband)
    if p["sync"]:
        return lambda D: ofc.tx_sync(x, p["L"], p["N"], p["c"], D, p["ncp"])
    return lambda D: ofc.tx_cont(x, p["L"], p["N"], p["c"], D, lam=p["lam"], ola=p["ola"])


def oracle_wgrad(subbands, xs, g_streams, bins=None):
    """Per subband: dJ/dD_p = Re <g, b_p> against the part of the gradient
    stream that the subband's output occupies (``bins``: per-subband lists of
    the bins to evaluate, default all)."""
    off, _, P = stream_offsets(subbands)
    out = []
    for i, s in enumerate(subbands):
        g = g_streams[s["stream"]][off[i]:off[i] + P[i]["Q"]]
        out.append(ogr.weight_grad(subband_forward(s, xs[i]), g, P[i]["L"],
                                   None if bins is None else bins[i]))
    return out


# -------------------------------------------------- storage conversions --
def to_device(a, io, device=0):
    """complex128 numpy -> CUDA tensor of the plan's I/O type (RNE rounding)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).astype(np.complex128))
    if io == "c64":
        return t.to(torch.complex64).to(f"cuda:{device}")
    dt = torch.float16 if io == "f16" else torch.bfloat16
    return torch.view_as_real(t).to(torch.float32).to(dt).contiguous().to(f"cuda:{device}")


def from_device(t, io):
    import torch
    if io == "c64":
        return t.cpu().numpy().astype(np.complex128)
    f = t.to(torch.float32).cpu().numpy()
    return (f[:, 0] + 1j * f[:, 1]).astype(np.complex128)


def quantize(a, io):
    """The rounding to_device applies, on the CPU (for storage/compute splits)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).astype(np.complex128))
    if io == "c64":
        return t.to(torch.complex64).numpy().astype(np.complex128)
    dt = torch.float16 if io == "f16" else torch.bfloat16
    f = torch.view_as_real(t).to(torch.float32).to(dt).to(torch.float32).numpy()
    return (f[:, 0] + 1j * f[:, 1]).astype(np.complex128)


GATE_DB = {"c64": -100.0, "f16": -60.0, "bf16": -50.0}

# Per-sample bound. The L2 gate above averages the error over a whole output;
# an error confined to a few blocks of a long output can pass it. Each sample
# is therefore also checked: |g - r| <= u |r| + PEAK_K u rms(r), where u is the
# unit roundoff of the storage type. The u |r| term is the rounding of the
# stored output itself (round-to-nearest-even: at most u relative per
# component). The PEAK_K u rms(r) term covers the rest: the input's rounding
# carried through the filter (a sum of many independent roundings, about
# 0.45 u rms relative, whose largest value over 10^7 samples is about
# 4.3 standard deviations, i.e. about 2 u) and the FP32 arithmetic. With FP16
# or BF16 storage the former dominates: rounding the oracle's own input and
# output in FP64 gives at most 1.6 u on the batched carriers, so PEAK_K = 4
# leaves a factor 2.5. With FP32 storage the arithmetic dominates (about
# 2 log2 N rounded butterfly stages, measured rms 2-4 u): PEAK_K = 128.
U_IO = {"c64": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}
PEAK_K = {"c64": 128.0, "f16": 4.0, "bf16": 4.0}


def peak_residual(got, ref, io):
    """max_i (|g_i - r_i| - u |r_i|) / (u rms(r)): the per-sample error beyond
    the output's own rounding, in units of the storage type's roundoff."""
    g = np.asarray(got, dtype=complex).ravel()
    r = np.asarray(ref, dtype=complex).ravel()
    rms = np.sqrt(np.mean(np.abs(r) ** 2))
    if rms == 0:
        return 0.0 if np.all(g == 0) else np.inf
    return float(np.max(np.abs(g - r) - U_IO[io] * np.abs(r)) / (U_IO[io] * rms))


def assert_gate(got, ref, io, extra=""):
    """Every part: L2 error <= GATE_DB[io] and per-sample residual <= PEAK_K[io]."""
    from oracle import metrics
    for k, (g, r) in enumerate(zip(got, ref)):
        assert len(g) == len(r)
        e = metrics.err_db(g, r)
        pk = peak_residual(g, r, io)
        print("part %d: %s err %.1f dB (gate %.0f), peak %.2f u (bound %.0f) %s"
              % (k, io, e, GATE_DB[io], pk, PEAK_K[io], extra), flush=True)
        assert e <= GATE_DB[io], "part %d: %.1f dB" % (k, e)
        assert pk <= PEAK_K[io], "part %d: per-sample residual %.2f u" % (k, pk)
