"""Throughput of the batched mixed-precision FC filter banks on one MI355X.

One step = one pass of the hot path over one batch of synthetic input:
  TX: symbol-synchronised FC synthesis of 256 independent carriers of uneven
      width (1-106 PRB), numerology (15/30/60 kHz) and long transform
      (1024-4096), one slot each, FP16 I/Q storage, repeated over
      --tx-batches slot-batches (one call: one launch per kernel class, the
      classes running concurrently);
  RX: symbol-synchronised FC analysis of a 100 MHz / 30 kHz carrier (N = 4096)
      into 8 subbands, one 10 ms frame each, BF16 I/Q storage, --rx-frames
      frames (one kernel launch).
Both calls are autotuned by the library, captured as HIP graphs and timed as
graph replays with HIP events on the stream they run on.
value = (high-rate samples produced by TX + consumed by RX) / step time.
The plain form (FP32, one plan and launch per carrier / per subband, no
batching) is timed on the same work and reported beside it.

Prints ONE JSON line. --gpus above 1 is refused (single-GPU build).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# published FP32 vector peak: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x
# 2 (packed FP32) x 2.4 GHz; the kernels do not use packed FP32, whose rate
# without packing is half of it
ALU_PEAK_TFLOPS = 157.3
ALU_PEAK_NONPACKED_TFLOPS = 78.6
EVM_GATE_DB = -50.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tx-batches", type=int, default=32)
    ap.add_argument("--rx-frames", type=int, default=100)
    ap.add_argument("--burst-slots", type=int, default=4096, help="slots of the plain FP32 continuous burst")
    ap.add_argument("--subframes", type=int, default=4000, help="mixed-numerology subframes (TX + RX)")
    ap.add_argument("--opt-slots", type=int, default=64, help="slots per carrier of the weight optimisation")
    ap.add_argument("--cf-slots", type=int, default=4096, help="slots of the 52-PRB channel-filter comparison")
    ap.add_argument("--opt-steps", type=int, default=10, help="Adam steps of the weight optimisation")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tuning", default=None,
                    help="tx_run_len,tx_conc,rx_run_len,rx_conc: apply instead of autotuning (profiling runs)")
    ap.add_argument("--no-latency", action="store_true", help="skip the single-unit latency graphs")
    ap.add_argument("--quick", action="store_true",
                    help="profiling runs: only the step, the demodulating RX and the grid-input TX")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------ workloads ---
def tx_workload(n_batches):
    from fcsynth import workloads as W
    sbs, meta = W.batched_carriers()
    out = []
    for b in range(n_batches):
        for k, s in enumerate(sbs):
            out.append(dict(s, stream=b * len(sbs) + k))
    return sbs, out, meta


def rx_workload(n_frames):
    from fcsynth import workloads as W
    sbs, meta = W.rx_filterbank()
    out = []
    for f in range(n_frames):
        for s in sbs:
            out.append(dict(s, stream=f))
    return sbs, out, meta


def tx_input(plan, sbs, meta):
    """CP-OFDM input of one batch (complex128) from the plan's CP schedule."""
    import fcsynth
    rng = np.random.default_rng(meta["seed"])
    xs = []
    for i, s in enumerate(sbs):
        _, lcp, _ = plan.symbols(i)
        g = fcsynth.qam_grid(rng, meta["qam"], s["n_symbols"], s["n_active"])
        xs.append(fcsynth.cp_ofdm(g, s["n_short"], lcp))
    return xs


def tx_input_grids(plan, sbs, meta):
    """CP-OFDM input (complex128) and the QAM grids behind it, from the plan's
    CP schedule."""
    import fcsynth
    rng = np.random.default_rng(meta["seed"])
    xs, gs = [], []
    for i, s in enumerate(sbs):
        _, lcp, _ = plan.symbols(i)
        g = fcsynth.qam_grid(rng, meta["qam"], s["n_symbols"], s["n_active"])
        gs.append(g)
        xs.append(fcsynth.cp_ofdm(g, s["n_short"], lcp))
    return xs, gs


def tx_grids(sbs, meta):
    """The QAM grids behind tx_input (same seed, same draw order)."""
    import fcsynth
    rng = np.random.default_rng(meta["seed"])
    return [fcsynth.qam_grid(rng, meta["qam"], s["n_symbols"], s["n_active"]) for s in sbs]


def rx_input(plan, sbs, meta):
    """One frame: the 8 subbands' 256-QAM CP-OFDM from one 4096-point IDFT per
    symbol, placed where the plan expects the first useful sample, plus AWGN."""
    import fcsynth
    rng = np.random.default_rng(meta["seed"])
    ncp, _, _ = plan.symbols(0)
    grids = [fcsynth.qam_grid(rng, meta["qam"], s["n_symbols"], s["n_active"]) for s in sbs]
    sig = fcsynth.cp_ofdm_highrate(grids, [s["center_bin"] for s in sbs], sbs[0]["n_long"], ncp)
    lo, hi = plan.layout(1)
    Q = int(hi[1] - hi[0])
    N = sbs[0]["n_long"]
    lead = N // 4 - ncp[0]
    y = np.zeros(Q, dtype=complex)
    y[lead:lead + len(sig)] = sig
    p = np.mean(np.abs(sig) ** 2)
    y += fcsynth.awgn(rng, Q, p * 10 ** (-meta["snr_db"] / 10))
    return y


def burst_workload(n_slots):
    """The plain FP32 single-subband form as a continuous burst: the plain
    slot's subband (24 PRB, L = 512, N = 2048, continuous OLS) carrying
    n_slots x 14 symbols (the CP schedule repeats every 7 symbols at 15 kHz,
    so the input is the one-slot signal repeated)."""
    from fcsynth import workloads as W
    sbs, meta = W.plain_tx_slot()
    return sbs[0], dict(sbs[0], n_symbols=14 * n_slots), meta


def subframes_workload(n_sub):
    """Mixed numerology, one 1 ms subframe per stream, n_sub streams: subband
    A (15 kHz, 48 PRB, L 1024, N 2048) and B (30 kHz, 24 PRB, L 512, N 1024)
    on each stream, synchronised OLA TX and CP-removing RX, FP32."""
    from fcsynth import workloads as W
    sbs, meta = W.mixed_numerology("sync_ola")
    return sbs, [dict(s, stream=k) for k in range(n_sub) for s in sbs], meta


def to_dev(a, io, reps=1):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if io == "c64":
        d = t.to(torch.complex64)
    else:
        dt = torch.float16 if io == "f16" else torch.bfloat16
        d = torch.view_as_real(t).to(torch.float32).to(dt).contiguous()
    d = d.cuda()
    if reps > 1:
        d = d.repeat((reps,) + (1,) * (d.dim() - 1)).contiguous()
    return d


# ----------------------------------------------------- algorithmic cost ---
def tx_cost(sbs, bytes_per_sample):
    """Algorithmic bytes (input read once + output written once) and flops of
    synchronised TX (two blocks per symbol): nominal per block
    5 L log2 L + 2 L + 5 N log2 N (the paper's chain with a full long IFFT),
    and executed per block 5 L log2 L + 2 L + 5 N log2 L + 6 N (the long IFFT
    pruned to the band's L bins)."""
    from paper_2008_00672_amd import Plan, OP_TX
    p = Plan(sbs, io="c64", device=-1)
    lo, hi = p.layout(OP_TX)
    nominal = executed = 0.0
    for s in sbs:
        L, N = s["n_short"], s["n_long"]
        short = 5 * L * math.log2(L) + 2 * L
        nominal += 2 * s["n_symbols"] * (short + 5 * N * math.log2(N))
        executed += 2 * s["n_symbols"] * (short + 5 * N * math.log2(L) + 6 * N)
    return (lo[-1] + hi[-1]) * bytes_per_sample, nominal, executed, int(hi[-1])


def rx_cost(sbs, bytes_per_sample):
    """Algorithmic bytes and flops of synchronised RX: per block one long FFT
    per stream (5 N log2 N) and per subband 5 L log2 L + 2 L."""
    from paper_2008_00672_amd import Plan, OP_RX
    p = Plan(sbs, io="c64", device=-1)
    lo, hi = p.layout(OP_RX)
    flops = 0.0
    for st in sorted(set(s["stream"] for s in sbs)):
        s0 = next(s for s in sbs if s["stream"] == st)
        N = s0["n_long"]
        flops += 2 * s0["n_symbols"] * 5 * N * math.log2(N)
    for s in sbs:
        L = s["n_short"]
        flops += 2 * s["n_symbols"] * (5 * L * math.log2(L) + 2 * L)
    return (lo[-1] + hi[-1]) * bytes_per_sample, flops, int(hi[-1])


def block_flops(L, N, pruned=True):
    """Flops of one TX block: short FFT + weights, then the long IFFT, pruned
    to the band (5 N log2 L + 6 N, executed) or full (5 N log2 N)."""
    long = 5 * N * math.log2(L) + 6 * N if pruned else 5 * N * math.log2(N)
    return 5 * L * math.log2(L) + 2 * L + long


def rx_block_flops(L, N):
    """Flops of one RX block of a one-subband group: long FFT + short IFFT."""
    return 5 * N * math.log2(N) + 5 * L * math.log2(L) + 2 * L


def rxd_cost(sbs):
    """Flops of the demodulating RX per call: per symbol two long FFTs per
    stream and per subband one short IFFT and one FFT (5 L log2 L each) plus
    the bin-wise products of the joint form (A, V, x: 18 L)."""
    flops = 0.0
    for st in sorted(set(s["stream"] for s in sbs)):
        s0 = next(s for s in sbs if s["stream"] == st)
        flops += 2 * s0["n_symbols"] * 5 * s0["n_long"] * math.log2(s0["n_long"])
    for s in sbs:
        L = s["n_short"]
        flops += s["n_symbols"] * (2 * 5 * L * math.log2(L) + 18 * L)
    return flops


def wgrad_cost(sbs):
    """Flops of the weight gradient per call: per TX block the long FFT of the
    output cotangent (5 N log2 N), the forward short FFT of the input block
    (5 L log2 L) and the bin-wise products with the phase (4 L + 6 L)."""
    flops = 0.0
    for s in sbs:
        L, N = s["n_short"], s["n_long"]
        flops += 2 * s["n_symbols"] * (5 * N * math.log2(N) + 5 * L * math.log2(L) + 10 * L)
    return flops


def plan_of(tune):
    """1 when a tuning runs transform plan 1 anywhere (the op's plan or a
    kernel class chosen by the autotuner), else 0."""
    return 1 if tune.get("plan", 0) or tune.get("classes_plan1", 0) else 0


def traffic(op, run_len, plan=0):
    """HBM bytes per call of op at run_len blocks per task from the committed
    rocprofv3 counter summary (profiles/traffic_<op>.json), or None when the
    kernel sources changed since the counters were taken, no counters were
    taken at that run length, or the op runs transform plan 1 (the counters
    are taken with plan 0)."""
    if plan:
        return None
    from paper_2008_00672_amd.profsum import kernel_hash
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % op)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    rec = d.get("by_run_len", {}).get(str(int(run_len)))
    if d.get("kernel_hash") != kernel_hash() or rec is None:
        return None
    return round(rec["bytes_per_launch"])


# ------------------------------------------------------------ CPU leg ---
def _time_tx_carriers(budget_s, tx_sbs, xs, order, reference="fc"):
    """Oracle TX of carriers in `order` until budget_s has passed: (samples,
    seconds, carriers done, outputs)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from fc_cases import oracle_tx
    from oracle.weights import rc_weights
    t0 = time.time()
    samples, outs = 0, {}
    for k in order:
        s = dict(tx_sbs[k], stream=0)
        ref = oracle_tx([s], [xs[k]], [rc_weights(s["n_short"], s["n_active"], s["n_tb"])], reference=reference)[0]
        outs[int(k)] = ref
        samples += len(ref)
        if time.time() - t0 > budget_s:
            break
    return samples, time.time() - t0, len(outs), outs


def paper_complexity():
    """The paper's complexity per QAM symbol (Sec. V formula, real
    multiplications, split-radix transforms) for the benchmark's configs:
    context, not a target."""
    from oracle import metrics
    rxw = [4, 12, 24, 33, 51, 66, 11, 72]
    rxl = [64, 256, 512, 512, 1024, 1024, 256, 1024]
    bank = [(l, l, 8, 12 * w) for w, l in zip(rxw, rxl)]
    r1 = lambda v: round(float(v), 1)
    return {"unit": "real multiplications per QAM symbol (Sec. V)",
            "plain_slot_cont_ols": r1(metrics.complexity_per_symbol(2048, [(512, 512, 8, 288)], alpha=31 / 14)),
            "mixed_numerology_A": r1(metrics.complexity_per_symbol(2048, [(1024, 1024, 8, 576)])),
            "mixed_numerology_B": r1(metrics.complexity_per_symbol(1024, [(512, 512, 8, 288)])),
            "rx_filterbank_beta_1": r1(metrics.complexity_per_symbol(4096, bank)),
            "rx_filterbank_beta_half": r1(metrics.complexity_per_symbol(4096, bank, beta=0.5)),
            "direct_fir_per_output_sample_N2048": 4 * 2048}


def cpu_baseline(budget_s, tx_sbs, tx_meta, gpu_tx_out, tx_plan_one, rx_sbs, rx_meta, gpu_rx_out, rx_plan_one,
                 rx_in, burst, subframes):
    """The FP64 oracle on the host: timed on a bounded sample of the same work
    at all host threads and at one thread, the plain linear-convolution
    reference (O-LIN) timed beside it; and the GPU outputs checked against the
    oracle on unquantised input (EVM): the headline TX carriers and RX
    symbols, the FP32 burst and the mixed-numerology subframe."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from fc_cases import make_inputs, oracle_rx, oracle_tx, quantize, rx_frame_input, stream_offsets
    from oracle import metrics
    from oracle.weights import rc_weights
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    # the oracle's inputs come from the same seeded generators, with the CP
    # schedule from the oracle's own numerology; they must equal what the GPU
    # was given (built from the library's schedule)
    xs = make_inputs(tx_sbs, tx_meta["qam"], tx_meta["seed"], "rc")[0]
    xs_gpu = tx_input(tx_plan_one, tx_sbs, tx_meta)
    if not all(np.array_equal(a, b) for a, b in zip(xs, xs_gpu)):
        raise RuntimeError("TX inputs differ between the oracle's and the library's CP schedule")
    rx_ref_in = rx_frame_input(rx_sbs, rx_meta["qam"], rx_meta["seed"], rx_meta["snr_db"])
    if not np.array_equal(rx_ref_in, rx_in):
        raise RuntimeError("RX input differs between the oracle's and the library's CP schedule")
    lo, hi = tx_plan_one.layout(0)
    order = np.argsort([s["n_long"] for s in tx_sbs])      # cheap carriers first
    # all host threads: TX carriers, then the RX frame's first 14 symbols
    smp, t_tx, n_done, outs = _time_tx_carriers(budget_s * 0.4, tx_sbs, xs, order)
    evm_tx = [metrics.err_db(gpu_tx_out[hi[k]:hi[k + 1]], ref) for k, ref in outs.items()]
    t1 = time.time()
    B = 14
    sub = [dict(s, n_symbols=B) for s in rx_sbs]
    _, lens_sub, _ = stream_offsets(sub)
    seg = rx_ref_in[:lens_sub[0]]
    refs = oracle_rx(sub, [seg], [rc_weights(s["n_short"], s["n_active"], s["n_tb"]) for s in rx_sbs])
    t_rx = time.time() - t1
    lo_rx, _ = rx_plan_one.layout(1)
    evm_rx = [metrics.err_db(gpu_rx_out[lo_rx[i]:lo_rx[i] + len(r)], r) for i, r in enumerate(refs)]
    rate = (smp + len(seg)) / (t_tx + t_rx) / 1e6
    # one thread (BLAS limited to one), the same carriers from the start
    with threadpool_limits(limits=1):
        smp1, t1s, n1, _ = _time_tx_carriers(budget_s * 0.25, tx_sbs, xs, order)
    # the plain definition: direct linear convolution (np.convolve, one thread)
    with threadpool_limits(limits=1):
        smpl, tl, nl, _ = _time_tx_carriers(budget_s * 0.15, tx_sbs, xs, order, reference="lin")
    # first few carriers: out-of-band power ratio of GPU and FP64 outputs, and
    # the error split: storage (oracle on the FP16-rounded input against the
    # unquantised one), compute and output rounding (GPU against the oracle on
    # the rounded input), and the distance to plain linear convolution
    split = []
    for k in order[:4]:
        s = dict(tx_sbs[k], stream=0)
        D = [rc_weights(s["n_short"], s["n_active"], s["n_tb"])]
        ref = outs[int(k)]
        ref_q = oracle_tx([s], [quantize(xs[k], tx_meta["io"])], D)[0]
        ref_lin = oracle_tx([s], [xs[k]], D, reference="lin")[0]
        got = gpu_tx_out[hi[k]:hi[k + 1]]
        band = [(s["center_bin"], s["n_active"], s["n_tb"])]
        split.append(dict(carrier=int(k), L=s["n_short"], N=s["n_long"],
                          oob_gpu=round(float(metrics.oob_ratio_db(got, s["n_long"], band)), 2),
                          oob_fp64=round(float(metrics.oob_ratio_db(ref, s["n_long"], band)), 2),
                          storage=round(float(metrics.err_db(ref_q, ref)), 2),
                          compute_and_output=round(float(metrics.err_db(got, ref_q)), 2),
                          total=round(float(metrics.err_db(got, ref)), 2),
                          fc_vs_linear=round(float(metrics.err_db(ref, ref_lin)), 2)))
    # the FP32 burst: a three-slot burst of the oracle has the burst's start
    # (first two slots) and end (last slot and tail); the slots in between
    # were checked bitwise on the GPU to repeat the second slot
    b1, b_meta, head, tail = burst["slot"], burst["meta"], burst["head"], burst["tail"]
    xb = make_inputs([b1], b_meta["qam"], b_meta["seed"], "rc")[0][0]
    if not np.array_equal(xb, burst["x_slot"]):
        raise RuntimeError("burst input differs between the oracle's and the library's CP schedule")
    D1 = [rc_weights(b1["n_short"], b1["n_active"], b1["n_tb"])]
    y3 = oracle_tx([dict(b1, n_symbols=42)], [np.tile(xb, 3)], D1)[0]
    evm_burst = [metrics.err_db(head, y3[:len(head)]), metrics.err_db(tail, y3[-len(tail):])]
    # the mixed-numerology subframe: TX of stream 0 against the oracle, and the
    # RX of the GPU's TX output against the oracle's RX of the oracle's TX
    m_sbs, m_meta = subframes["subbands"], subframes["meta"]
    xm, Dm, _ = make_inputs(m_sbs, m_meta["qam"], m_meta["seed"], "rc")
    ym_ref = oracle_tx(m_sbs, xm, Dm)[0]
    zm_ref = np.concatenate(oracle_rx(m_sbs, [ym_ref], Dm))
    evm_sub = [metrics.err_db(subframes["tx"], ym_ref), metrics.err_db(subframes["rx"], zm_ref)]
    cpu = dict(value=rate, unit="Msamples/s", cores=threads, kind="oracle",
               sample="FP64 dense-DFT oracle: TX of %d of the 256 carriers (one slot each, cheapest first) + RX "
                      "of the first 14 symbols of one 8-subband frame; %.1f s" % (n_done, t_tx + t_rx),
               os_cpu_count=os.cpu_count(), blas_threads=threads,
               one_thread={"value": round(smp1 / t1s / 1e6, 4), "unit": "Msamples/s", "threads": 1,
                           "sample": "TX of the first %d carriers, %.1f s" % (n1, t1s)},
               olin={"value": round(smpl / tl / 1e6, 4), "unit": "Msamples/s", "threads": 1,
                     "sample": "plain reference: direct linear convolution with one period of the FC kernel "
                               "(np.convolve) + the same inputs, first %d carriers, %.1f s" % (nl, tl)},
               paper_complexity=paper_complexity())
    evm = dict(tx_max=float(np.max(evm_tx)), tx_mean=float(np.mean(evm_tx)), rx_max=float(np.max(evm_rx)),
               tx_carriers=n_done, rx_per_subband=[round(float(e), 2) for e in evm_rx], tx_split=split,
               burst_fp32=[round(float(e), 1) for e in evm_burst],
               subframe_fp32_tx_rx=[round(float(e), 1) for e in evm_sub])
    return cpu, evm


def method_check():
    """Part of the oracle leg: the wide-band comparison of continuous and
    symbol-synchronised processing (52 PRB at N = 1024, 15 kHz, 64-QAM, one
    slot, no noise), four TX/RX chains through the library and through the
    FP64 oracle: EVM of the active subcarriers and out-of-band power ratio."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from wideband import OOB_GUARD, Setup, gpu_chains, oracle_chains
    S = Setup()
    _, ref = oracle_chains(S)
    _, got = gpu_chains(S)
    r3 = lambda d: {k: round(float(v), 3) for k, v in d.items()}
    return {"workload": "one 52-PRB subband (624 active subcarriers, 8-bin raised-cosine transition bands), "
                        "N = L = 1024, 15 kHz, 14 symbols of 64-QAM, FP32 I/O",
            "evm_db_gpu": r3(got["evm_db"]), "evm_db_fp64": r3(ref["evm_db"]),
            "oob_db_gpu": r3(got["oob_db"]), "oob_db_fp64": r3(ref["oob_db"]),
            "oob": "Welch PSD (Blackman-Harris, N bins, hop N/2): power outside the active and transition "
                   "bins +- %d bins, over the total" % OOB_GUARD,
            "paper": "continuous out-of-band PSD about 5 dB below synchronised; passband EVM 63.8 dB "
                     "(continuous) and 63.4 dB (synchronised) with its own optimised weights"}


def time_graph(fn, gs, warmup, steps):
    """Capture fn(stream) as a HIP graph on gs, replay it warmup times, then
    time `steps` replays with HIP events on gs: ms per replay."""
    import torch
    from paper_2008_00672_amd import Graph
    with Graph(gs) as g:
        fn(gs)
    for _ in range(warmup):
        g.launch(gs)
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a0.record(gs)
    for _ in range(steps):
        g.launch(gs)
    a1.record(gs)
    torch.cuda.synchronize()
    ms = a0.elapsed_time(a1) / steps
    g.close()
    return ms


def repeats_bitwise(t, n_rep, n_each, start=0):
    """True if the n_rep consecutive pieces of n_each samples of t from
    `start` are bitwise equal to the first."""
    import torch
    v = t[start:start + n_rep * n_each]
    v = torch.view_as_real(v) if v.is_complex() else v
    v = v.contiguous().view(torch.int32 if v.dtype == torch.float32 else torch.int16).reshape(n_rep, -1)
    return bool(torch.equal(v, v[:1].expand_as(v)))


def frac(tf):
    return {"frac": round(tf / ALU_PEAK_TFLOPS, 4), "frac_non_packed": round(tf / ALU_PEAK_NONPACKED_TFLOPS, 4)}


def single_unit_latency(ptx1, prx1, x_dev, r_dev, gs):
    """One slot of the 256 carriers (TX) and one frame (RX): graph replays,
    median of 20 after two warm-ups."""
    import torch
    from paper_2008_00672_amd import Graph, OP_RX, OP_TX
    x1 = x_dev[:int(ptx1.layout(OP_TX)[0][-1])]
    y1 = ptx1.empty(int(ptx1.layout(OP_TX)[1][-1]))
    r1 = r_dev[:int(prx1.layout(OP_RX)[1][-1])]
    z1 = prx1.empty(int(prx1.layout(OP_RX)[0][-1]))
    with Graph(gs) as g1_tx:
        ptx1.tx(x1, y1, gs)
    with Graph(gs) as g1_rx:
        prx1.rx(r1, z1, gs)

    def median_ms(g):
        ts = []
        for _ in range(22):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(gs)
            g.launch(gs)
            b.record(gs)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts[2:]))
    return {"tx_one_slot_256_carriers_ms": round(median_ms(g1_tx), 4), "rx_one_frame_ms": round(median_ms(g1_rx), 4)}


def extra_sections(args, torch, dev, gs, ptx, x_dev, hi, tx_all, tx_samples, tune, repeat_ok):
    """Timed beside the step: the weight gradient on the batched TX workload,
    the plain FP32 single-subband form as a continuous burst, and the
    mixed-numerology TX + RX. Returns their result records and what the
    oracle leg needs to check them."""
    from paper_2008_00672_amd import OP_ADJ, OP_RX, OP_TX, Plan
    # the weight gradient through the adjoint (Sec. III: the output is linear
    # in D) on the batched TX workload: a seeded random cotangent of the
    # output. Its blocks per task are fixed (a fixed summation tree); its
    # launches run on the side streams like the other operations.
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    g_dev = torch.randn((int(hi[-1]), 2), generator=gen, device=dev).to(torch.float16)
    gw = torch.empty(sum(s["n_short"] for s in tx_all), dtype=torch.float32, device=dev)
    ptx.set_tuning(OP_ADJ, 0, 4)
    tune["weight_grad"] = {"run_len": 4, "conc": 4}
    for _ in range(args.warmup):
        ptx.weight_grad(x_dev, g_dev, gw, gs)
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a0.record(gs)
    for _ in range(args.steps):
        ptx.weight_grad(x_dev, g_dev, gw, gs)
    a1.record(gs)
    torch.cuda.synchronize()
    wg_ms = a0.elapsed_time(a1) / args.steps
    wg_flops = wgrad_cost(tx_all)
    weight_grad = dict({"ms": round(wg_ms, 4), "value": round(tx_samples / (wg_ms * 1e-3) / 1e6, 1),
                        "unit": "Msamples/s (high-rate cotangent samples)",
                        "achieved_tflops": round(wg_flops / wg_ms / 1e9, 2), "algorithmic_flops": int(wg_flops),
                        "form": "dJ/dD of all 8192 carrier-slots' weights from the input and a cotangent of the "
                                "output (FP16), adjoint kernels + per-bin products, partial sums reduced in "
                                "block order"},
                       **frac(wg_flops / wg_ms / 1e9))
    del g_dev, gw
    log("weight grad: %.3f ms (%.1f TFLOP/s)" % (wg_ms, weight_grad["achieved_tflops"]))

    # ---------------- the plain FP32 single-subband form ----------------
    # one continuous OLS subband (24 PRB, L 512, N 2048) carrying a burst of
    # --burst-slots slots, FP32 I/O, one call (graph replay)
    b1, bN, b_meta = burst_workload(args.burst_slots)
    pb1 = Plan([b1], io="c64", device=0)
    pb = Plan([bN], io="c64", device=0)
    xb_slot = tx_input(pb1, [b1], b_meta)[0]
    xb = to_dev(xb_slot, "c64", reps=args.burst_slots)
    lo_b, hi_b = pb.layout(OP_TX)
    assert xb.shape[0] == lo_b[-1]
    yb = pb.empty(int(hi_b[-1]))
    tune["burst"] = pb.get_tuning(OP_TX) if args.tuning else pb.autotune(OP_TX, xb, yb, stream=gs)
    b_ms = time_graph(lambda st: pb.tx(xb, yb, st), gs, args.warmup, args.steps)
    I_b = b1["n_long"] // b1["n_short"]
    period = len(xb_slot) * I_b                              # high-rate samples per slot
    n0 = I_b * b1["n_short"] * b1["overlap"][0] // b1["overlap"][1]   # first sample of x: I L_O
    repeat_ok["burst_slots"] = repeats_bitwise(yb, args.burst_slots - 2, period, start=n0 + period)
    b_samples = args.burst_slots * period
    b_bytes = 8 * (int(lo_b[-1]) + int(hi_b[-1]))
    b_flops = pb.stats(OP_TX)["blocks"] * block_flops(b1["n_short"], b1["n_long"])
    burst_tail = int(hi_b[-1]) - (n0 + args.burst_slots * period)
    b_head = yb[:n0 + 2 * period].cpu().numpy().astype(np.complex128)
    b_tail = yb[-(period + burst_tail):].cpu().numpy().astype(np.complex128)
    del xb, yb
    burst = dict({"ms": round(b_ms, 4), "value": round(b_samples / (b_ms * 1e-3) / 1e6, 1), "unit": "Msamples/s",
                  "hbm_gbs": round(b_bytes / b_ms / 1e6, 1), "hbm_frac": round(b_bytes / b_ms / 1e6 / HBM_PEAK_GBS, 4),
                  "achieved_tflops": round(b_flops / b_ms / 1e9, 2), "algorithmic_bytes": b_bytes,
                  "algorithmic_flops": int(b_flops), "samples": b_samples,
                  "form": "plain FP32 single-subband form: one continuous overlap-save subband (24 PRB, L 512, "
                          "N 2048, 50 %% overlap, QPSK) carrying %d slots, FP32 I/O, one call" % args.burst_slots},
                 **frac(b_flops / b_ms / 1e9))
    log("plain FP32 burst: %.3f ms, %.0f Msamples/s, %.0f GB/s" % (b_ms, burst["value"], burst["hbm_gbs"]))

    # ---------------- mixed numerology: TX + RX of --subframes subframes ----
    m_one, m_all, m_meta = subframes_workload(args.subframes)
    pm1 = Plan(m_one, io="c64", device=0)
    pm = Plan(m_all, io="c64", device=0)
    xm = to_dev(np.concatenate(tx_input(pm1, m_one, m_meta)), "c64", reps=args.subframes)
    lo_m, hi_m = pm.layout(OP_TX)
    assert xm.shape[0] == lo_m[-1]
    ym = pm.empty(int(hi_m[-1]))
    lo_mr, _ = pm.layout(OP_RX)
    zm = pm.empty(int(lo_mr[-1]))
    if args.tuning:
        tune["subframes"] = {"tx": pm.get_tuning(OP_TX), "rx": pm.get_tuning(OP_RX)}
    else:
        tune["subframes"] = {"tx": pm.autotune(OP_TX, xm, ym, stream=gs)}
        pm.tx(xm, ym, gs)
        tune["subframes"]["rx"] = pm.autotune(OP_RX, ym, zm, stream=gs)
    pm.tx(xm, ym, gs)
    pm.rx(ym, zm, gs)
    torch.cuda.synchronize()
    m_tx_ms = time_graph(lambda st: pm.tx(xm, ym, st), gs, args.warmup, args.steps)
    m_rx_ms = time_graph(lambda st: pm.rx(ym, zm, st), gs, args.warmup, args.steps)
    len_st = int(hi_m[1] - hi_m[0])
    n_rx1 = int(lo_mr[len(m_one)])
    repeat_ok["subframes_tx"] = repeats_bitwise(ym, args.subframes, len_st)
    repeat_ok["subframes_rx"] = repeats_bitwise(zm, args.subframes, n_rx1)
    m_samples = args.subframes * 30720                      # 1 ms at 30.72 MS/s per subframe
    m_tx_bytes = 8 * (int(lo_m[-1]) + int(hi_m[-1]))
    m_rx_bytes = 8 * (int(hi_m[-1]) + int(lo_mr[-1]))
    m_tx_flops = sum(2 * s["n_symbols"] * block_flops(s["n_short"], s["n_long"]) for s in m_all)
    m_rx_flops = sum(2 * s["n_symbols"] * rx_block_flops(s["n_short"], s["n_long"]) for s in m_all)
    m_tx0 = ym[:len_st].cpu().numpy().astype(np.complex128)
    m_rx0 = zm[:n_rx1].cpu().numpy().astype(np.complex128)
    del xm, ym, zm
    subframes = {"tx_ms": round(m_tx_ms, 4), "rx_ms": round(m_rx_ms, 4),
                 "value": round(2 * m_samples / ((m_tx_ms + m_rx_ms) * 1e-3) / 1e6, 1), "unit": "Msamples/s",
                 "tx": dict({"value": round(m_samples / (m_tx_ms * 1e-3) / 1e6, 1),
                             "hbm_gbs": round(m_tx_bytes / m_tx_ms / 1e6, 1),
                             "achieved_tflops": round(m_tx_flops / m_tx_ms / 1e9, 2)}, **frac(m_tx_flops / m_tx_ms / 1e9)),
                 "rx": dict({"value": round(m_samples / (m_rx_ms * 1e-3) / 1e6, 1),
                             "hbm_gbs": round(m_rx_bytes / m_rx_ms / 1e6, 1),
                             "achieved_tflops": round(m_rx_flops / m_rx_ms / 1e9, 2)}, **frac(m_rx_flops / m_rx_ms / 1e9)),
                 "form": "mixed numerology (15 kHz 48 PRB + 30 kHz 24 PRB on one 30.72 MS/s stream), synchronised "
                         "OLA TX then CP-removing RX of its output, %d subframes, FP32 I/O" % args.subframes}
    log("mixed numerology: TX %.3f ms, RX %.3f ms" % (m_tx_ms, m_rx_ms))

    weight_opt = weight_opt_section(args, torch, gs)
    channel_filter = channel_filter_section(args, torch, gs, repeat_ok)
    checks = dict(burst=dict(slot=b1, meta=b_meta, x_slot=xb_slot, head=b_head, tail=b_tail),
                  subframes=dict(subbands=m_one, meta=m_meta, tx=m_tx0, rx=m_rx0))
    return weight_grad, burst, subframes, weight_opt, channel_filter, checks


def channel_filter_section(args, torch, gs, repeat_ok):
    """The full-band channel filter with a 768 = 3 x 256 point transform
    against 1024 points (Sec. VI-C): one 52-PRB subband (624 active
    subcarriers, 8-bin transition bands) at 15 kHz, L = N (I = 1), --cf-slots
    slots as independent streams, FP32 I/O; synchronised OLA TX, then the
    demodulating RX of its output."""
    from fcsynth import workloads as W
    from paper_2008_00672_amd import OP_RXD, OP_TX, Plan
    out = {}
    for n in (768, 1024):
        sb1, meta = W.wideband_slot("sync_ola", n)
        sbs = [dict(sb1[0], stream=k) for k in range(args.cf_slots)]
        p1 = Plan(sb1, io="c64", device=0)
        p = Plan(sbs, io="c64", device=0)
        x = to_dev(tx_input(p1, sb1, meta)[0], "c64", reps=args.cf_slots)
        lo, hi = p.layout(OP_TX)
        assert x.shape[0] == lo[-1]
        y = p.empty(int(hi[-1]))
        z = p.empty(int(p.layout(OP_RXD)[0][-1]))
        tx_ms = time_graph(lambda st: p.tx(x, y, st), gs, args.warmup, args.steps)
        rx_ms = time_graph(lambda st: p.rx_demod(y, z, st), gs, args.warmup, args.steps)
        repeat_ok["channel_filter_%d" % n] = (repeats_bitwise(y, args.cf_slots, int(hi[1] - hi[0]))
                                              and repeats_bitwise(z, args.cf_slots, 14 * n))
        out["L%d" % n] = {"tx_ms": round(tx_ms, 4), "rx_demod_ms": round(rx_ms, 4),
                          "us_per_slot": round(1e3 * (tx_ms + rx_ms) / args.cf_slots, 4),
                          "high_rate_samples_per_slot": int(hi[1] - hi[0])}
        del x, y, z
    out["time_768_over_1024"] = round((out["L768"]["tx_ms"] + out["L768"]["rx_demod_ms"])
                                      / (out["L1024"]["tx_ms"] + out["L1024"]["rx_demod_ms"]), 3)
    out["form"] = ("52-PRB full-band channel filter, L = N (I = 1), %d slots of 64-QAM as streams, FP32 I/O: "
                   "synchronised OLA TX + demodulating RX" % args.cf_slots)
    log("channel filter 768 vs 1024: %s" % out)
    return out


def weight_opt_section(args, torch, gs):
    """Transition-weight optimisation of the 256 batched carriers (N_tb ~
    U{4..16}, FP32, 16-QAM, --opt-slots slots each): Adam on J = mean EVM +
    mean OOB through the library's backward kernels; time per optimisation
    step (forward, objective, backward, update) and the objective's values."""
    from fcsynth import workloads as W
    from paper_2008_00672_amd import Plan, fc_tx
    from paper_2008_00672_amd.weight_opt import TransitionWeights, TxObjective
    sbs, meta = W.weight_opt_carriers(n_slots=args.opt_slots)
    t = time.time()
    pw = Plan(sbs, io="c64", device=0)
    xs, grids = tx_input_grids(pw, sbs, meta)
    xw = to_dev(np.concatenate(xs), "c64")
    del xs
    tw = TransitionWeights(pw)
    obj = TxObjective(pw, grids, mu_oob=meta["mu_oob"])
    log("weight optimisation set-up: %.1f s" % (time.time() - t))
    theta = tw.theta0.clone().requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=0.02)
    st = torch.cuda.current_stream()
    js, evm_db, oob_db, ts = [], [], [], []
    for it in range(args.opt_steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        opt.zero_grad()
        J, evm, oob = obj(fc_tx(pw, xw, tw.full(theta)))
        J.backward()
        opt.step()
        b.record(st)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
        js.append(float(J))
        evm_db.append(round(10 * math.log10(float(evm.mean())), 3))
        oob_db.append(round(10 * math.log10(float(oob.mean())), 3))
    # the library's share of a step: one forward and one weight gradient
    y = pw.tx(xw)
    gy = torch.randn_like(y)
    gw = torch.empty(sum(s["n_short"] for s in sbs), dtype=torch.float32, device=xw.device)
    f_ms = time_graph(lambda s_: pw.tx(xw, y, s_), gs, 2, 5)
    pw.weight_grad(xw, gy, gw)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(st)
    for _ in range(5):
        pw.weight_grad(xw, gy, gw)
    b.record(st)
    torch.cuda.synchronize()
    g_ms = a.elapsed_time(b) / 5
    out = {"ms_per_step": round(float(np.median(ts[1:] if len(ts) > 1 else ts)), 3), "steps": args.opt_steps,
           "J": [float("%.6e" % v) for v in js], "evm_db_mean": evm_db, "oob_db_mean": oob_db,
           "carriers": len(sbs), "slots": args.opt_slots, "parameters": int(tw.idx.numel()),
           "tx_forward_ms": round(f_ms, 3), "weight_grad_ms": round(g_ms, 3),
           "form": "256 batched carriers, N_tb ~ U{4..16}, %d slots of 16-QAM each, FP32 I/O: Adam (lr 0.02) on "
                   "J = mean EVM + mean OOB (linear; EVM at a mid-CP window after a least-squares gain, OOB from a "
                   "Welch PSD) over the 2 N_tb transition weights per carrier; forward, adjoint and weight gradient "
                   "in the library's kernels, the objective in PyTorch" % args.opt_slots}
    log("weight optimisation: %.1f ms per step, J %s" % (out["ms_per_step"], out["J"]))
    del xw, y, gy, gw, obj
    return out


# ------------------------------------------------------------------ main ---
def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        return 2
    import torch
    from paper_2008_00672_amd import Graph, Plan, OP_ADJ, OP_RX, OP_RXD, OP_TX, OP_TXG

    if args.copy_calib:
        n = 256 << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}))
        return 0

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # ---------------- batched TX ----------------
    tx_one, tx_all, tx_meta = tx_workload(args.tx_batches)
    t = time.time()
    ptx = Plan(tx_all, io="f16", device=0)
    plan_s = {"tx": round(time.time() - t, 3)}
    ptx1 = Plan(tx_one, io="f16", device=0)
    xs = tx_input(ptx1, tx_one, tx_meta)
    x_dev = to_dev(np.concatenate(xs), "f16", reps=args.tx_batches)
    lo, hi = ptx.layout(OP_TX)
    assert x_dev.shape[0] == lo[-1]
    y_dev = ptx.empty(int(hi[-1]))
    log("TX plan: %d carriers, %s, %.1f s" % (len(tx_all), ptx.stats(OP_TX), time.time() - t))

    # ---------------- batched RX ----------------
    rx_one, rx_all, rx_meta = rx_workload(args.rx_frames)
    t = time.time()
    prx = Plan(rx_all, io="bf16", device=0)
    plan_s["rx"] = round(time.time() - t, 3)
    prx1 = Plan(rx_one, io="bf16", device=0)
    rx_in = rx_input(prx1, rx_one, rx_meta)
    r_dev = to_dev(rx_in, "bf16", reps=args.rx_frames)
    lo_r, hi_r = prx.layout(OP_RX)
    assert r_dev.shape[0] == hi_r[-1]
    z_dev = prx.empty(int(lo_r[-1]))
    log("RX plan: %d frames, %s, %.1f s" % (args.rx_frames, prx.stats(OP_RX), time.time() - t))

    # work split chosen by the library's autotuner on these buffers, then one
    # TX call and one RX call captured as HIP graphs on a side stream
    gs = torch.cuda.Stream()
    torch.cuda.synchronize()
    tl = tc = rl = rc = 0
    if args.tuning:
        tl, tc, rl, rc = [int(v) for v in args.tuning.split(",")]
        ptx.set_tuning(OP_TX, tl, tc)
        prx.set_tuning(OP_RX, rl, rc)
        tune = {"tx": ptx.get_tuning(OP_TX), "rx": prx.get_tuning(OP_RX), "source": "--tuning"}
    else:
        tune = {"tx": ptx.autotune(OP_TX, x_dev, y_dev, stream=gs), "rx": prx.autotune(OP_RX, r_dev, z_dev, stream=gs),
                "source": "autotune"}
    log("tuning: %s" % tune)
    with Graph(gs) as g_tx:
        ptx.tx(x_dev, y_dev, gs)
    with Graph(gs) as g_rx:
        prx.rx(r_dev, z_dev, gs)

    for _ in range(args.warmup):
        g_tx.launch(gs)
        g_rx.launch(gs)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(gs)
    for k in range(args.steps):
        ev[k][0].record(gs)
        g_tx.launch(gs)
        ev[k][1].record(gs)
        g_rx.launch(gs)
        ev[k][2].record(gs)
    e1.record(gs)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    tx_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    rx_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    tx_bytes, tx_flops_nominal, tx_flops, tx_samples = tx_cost(tx_all, 4)
    rx_bytes, rx_flops, rx_samples = rx_cost(rx_all, 4)
    value = (tx_samples + rx_samples) / (ms * 1e-3) / 1e6
    log("step %.3f ms: TX %.3f ms (%.0f GB/s, %.1f TFLOP/s), RX %.3f ms (%.0f GB/s, %.1f TFLOP/s)" % (
        ms, tx_ms, tx_bytes / tx_ms / 1e6, tx_flops / tx_ms / 1e9, rx_ms, rx_bytes / rx_ms / 1e6,
        rx_flops / rx_ms / 1e9))

    # every slot-batch / frame repeats one input: its output must repeat bit
    # for bit (this extends the oracle's sampled EVM check to the whole output)
    n1_tx, n1_rx = int(ptx1.layout(OP_TX)[1][-1]), int(prx1.layout(OP_RX)[0][-1])
    repeat_ok = {"tx_batches": repeats_bitwise(y_dev, args.tx_batches, n1_tx),
                 "rx_frames": repeats_bitwise(z_dev, args.rx_frames, n1_rx)}

    # the demodulating receiver (Sec. V-A simplified form) on the same RX
    # workload, outside the step: subcarriers instead of time-domain symbols
    zd_dev = prx.empty(int(prx.layout(OP_RXD)[0][-1]))
    if args.tuning:
        prx.set_tuning(OP_RXD, rl, rc)
        tune["rx_demod"] = prx.get_tuning(OP_RXD)
    else:
        tune["rx_demod"] = prx.autotune(OP_RXD, r_dev, zd_dev, stream=gs)
    rxd_ms = time_graph(lambda st: prx.rx_demod(r_dev, zd_dev, st), gs, args.warmup, args.steps)
    rxd_flops = rxd_cost(rx_all)
    rx_demod = dict({"ms": round(rxd_ms, 4), "value": round(rx_samples / (rxd_ms * 1e-3) / 1e6, 1),
                     "unit": "Msamples/s", "achieved_tflops": round(rxd_flops / rxd_ms / 1e9, 2),
                     "algorithmic_flops": int(rxd_flops), "kernel": "fc_rxd_kernel<bf16, N=4096>",
                     "algorithmic_bytes": int(rx_bytes),
                     "traffic": traffic("fc_rxd", tune["rx_demod"]["run_len"], plan_of(tune["rx_demod"])),
                     "form": "synchronised RX + OFDM demodulation, one short IFFT + one FFT per symbol (Sec. V-A)"},
                    **frac(rxd_flops / rxd_ms / 1e9))
    log("rx demod: %.3f ms (%.1f TFLOP/s)" % (rxd_ms, rx_demod["achieved_tflops"]))

    # the grid-input TX (QAM grid -> OFDM IFFT + truncated CP -> FC in the
    # kernels) on the same TX workload, outside the step
    g_in = to_dev(np.concatenate([g.ravel() for g in tx_grids(tx_one, tx_meta)]), "f16", reps=args.tx_batches)
    y_g = ptx.empty(int(hi[-1]))
    if args.tuning:
        ptx.set_tuning(OP_TXG, tl, tc)
        tune["tx_grid"] = ptx.get_tuning(OP_TXG)
    else:
        tune["tx_grid"] = ptx.autotune(OP_TXG, g_in, y_g, stream=gs)
    txg_ms = time_graph(lambda st: ptx.tx_grid(g_in, y_g, st), gs, args.warmup, args.steps)
    del y_g, g_in
    txg_flops = tx_flops + sum(2 * s["n_symbols"] * 5 * s["n_short"] * math.log2(s["n_short"]) for s in tx_all)
    tx_grid = dict({"ms": round(txg_ms, 4), "value": round(tx_samples / (txg_ms * 1e-3) / 1e6, 1),
                    "unit": "Msamples/s", "achieved_tflops": round(txg_flops / txg_ms / 1e9, 2),
                    "algorithmic_flops": int(txg_flops),
                    "traffic": traffic("fc_tx_grid", tune["tx_grid"]["run_len"], plan_of(tune["tx_grid"])),
                    "form": "QAM grid in (FP16): OFDM IFFT + truncated CP + synchronised FC TX in the kernels "
                            "(the OFDM IFFT is run for each of a symbol's two blocks)"},
                   **frac(txg_flops / txg_ms / 1e9))
    log("tx grid: %.3f ms (%.1f TFLOP/s)" % (txg_ms, tx_grid["achieved_tflops"]))

    # beside the step: the weight gradient, the plain FP32 burst and the
    # mixed-numerology TX + RX
    weight_grad, burst, subframes, weight_opt, channel_filter, checks, latency = (None,) * 7
    if args.quick:
        args.no_plain = args.no_cpu = args.no_latency = True
    else:
        weight_grad, burst, subframes, weight_opt, channel_filter, checks = extra_sections(
            args, torch, dev, gs, ptx, x_dev, hi, tx_all, tx_samples, tune, repeat_ok)

    # single-unit latency: one slot of the 256 carriers, one RX frame (graph
    # replays, median of 20)
    if not args.no_latency:
        latency = single_unit_latency(ptx1, prx1, x_dev, r_dev, gs)
        log("latency: %s" % latency)

    # dominant kernel: the RX analysis is one kernel launch per call and the
    # longest single dispatch of the step; the TX call is a set of concurrent
    # per-class launches, reported beside it
    dk, d_ms, d_bytes, d_flops = "fc_rx", rx_ms, rx_bytes, rx_flops
    ai = d_flops / d_bytes
    ridge = ALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    hbm_gbs = d_bytes / d_ms / 1e6
    alu_tf = d_flops / d_ms / 1e9
    if ai > ridge:
        roof = {"bound": "alu", "achieved": round(alu_tf, 2), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(alu_tf / ALU_PEAK_TFLOPS, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    roof["traffic"] = traffic(dk, tune["rx"]["run_len"], plan_of(tune["rx"]))
    roof["kernel"] = "fc_rx_kernel<bf16, N=4096> (one launch per RX call)"
    roof["algorithmic_bytes"] = int(d_bytes)
    roof["algorithmic_flops"] = int(d_flops)
    roof["hbm_gbs"] = round(hbm_gbs, 1)
    roof["hbm_frac"] = round(hbm_gbs / HBM_PEAK_GBS, 4)
    roof["peak_non_packed"] = ALU_PEAK_NONPACKED_TFLOPS
    roof["frac_non_packed"] = round(alu_tf / ALU_PEAK_NONPACKED_TFLOPS, 4)
    roof["flop_per_byte"] = round(ai, 2)
    tx_tf = tx_flops / tx_ms / 1e9
    roof["tx_call"] = dict({"ms": round(tx_ms, 4), "launches": ptx.stats(OP_TX)["launches"],
                            "achieved_tflops": round(tx_tf, 2), "flops": "executed (long IFFT pruned to the band)",
                            "achieved_tflops_nominal": round(tx_flops_nominal / tx_ms / 1e9, 2),
                            "hbm_gbs": round(tx_bytes / tx_ms / 1e6, 1), "algorithmic_bytes": int(tx_bytes),
                            "algorithmic_flops": int(tx_flops),
                            "traffic": traffic("fc_tx", tune["tx"]["run_len"], plan_of(tune["tx"]))},
                           **frac(tx_tf))

    # ---------------- launch overhead of unbatched calls ----------------
    # one FP32 plan and one eager launch per carrier (TX) / per subband (RX):
    # mostly host launch cost, reported as such
    overhead = None
    if not args.no_plain:
        plans = [Plan([dict(s, stream=0)], io="c64", device=0) for s in tx_one]
        xin = [to_dev(x, "c64") for x in xs]
        outs = [p.empty(int(p.layout(OP_TX)[1][-1])) for p in plans]
        rplans = [Plan([dict(s, stream=0)], io="c64", device=0) for s in rx_one]
        rin = to_dev(rx_in, "c64")
        routs = [p.empty(int(p.layout(OP_RX)[0][-1])) for p in rplans]

        def plain_step():
            for p, xi, o in zip(plans, xin, outs):
                p.tx(xi, o, stream)
            for p, o in zip(rplans, routs):
                p.rx(rin, o, stream)
        for _ in range(2):
            plain_step()
        torch.cuda.synchronize()
        n_plain = max(2, args.steps // 4)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(n_plain):
            plain_step()
        b.record(stream)
        torch.cuda.synchronize()
        pms = a.elapsed_time(b) / n_plain
        p_samples = tx_samples / args.tx_batches + rx_samples / args.rx_frames
        overhead = {"value": round(p_samples / (pms * 1e-3) / 1e6, 1), "unit": "Msamples/s",
                    "ms_per_batch": round(pms, 3), "launches": len(plans) + len(rplans),
                    "form": "FP32 I/O, one plan and one eager launch per carrier (TX) / per subband (RX), one "
                            "slot-batch + one frame: mostly host launch cost"}
        log("unbatched eager calls: %.3f ms per (1 TX batch + 1 RX frame) -> %.0f Msamples/s" % (pms, overhead["value"]))

    # ---------------- CPU oracle + EVM on a sample ----------------
    cpu, evm, method = None, None, None
    if not args.no_cpu:
        import torch as _t
        yh = y_dev[:n1_tx].to(_t.float32).cpu().numpy()
        zh = z_dev[:n1_rx].to(_t.float32).cpu().numpy()
        cpu, evm = cpu_baseline(args.cpu_seconds, tx_one, tx_meta, yh[:, 0] + 1j * yh[:, 1], ptx1,
                                rx_one, rx_meta, zh[:, 0] + 1j * zh[:, 1], prx1, rx_in, checks["burst"],
                                checks["subframes"])
        cpu["value"] = round(cpu["value"], 3)
        log("cpu oracle %.3f Msamples/s on %d threads; EVM vs FP64: %s" % (cpu["value"], cpu["cores"], evm))
        method = method_check()
        log("method check (wide-band, 52 PRB): %s" % method)

    # the metric's condition: EVM <= -50 dB against the FP64 oracle on the
    # sampled outputs, and every repeated batch / frame / slot / subframe
    # bitwise equal to the checked one; otherwise no value is reported
    gate = {"evm_gate_db": EVM_GATE_DB, "repeats_bitwise": repeat_ok}
    failed = [k for k, ok in repeat_ok.items() if not ok]
    if evm is None:
        gate["status"] = "unchecked (--no-cpu): value withheld"
    else:
        worst = max([evm["tx_max"], evm["rx_max"]] + evm["burst_fp32"] + evm["subframe_fp32_tx_rx"])
        gate["worst_evm_db"] = round(worst, 2)
        if worst > EVM_GATE_DB:
            failed.append("evm")
        gate["status"] = "pass" if not failed else "FAIL: " + ", ".join(failed)
    if failed and "status" in gate and not gate["status"].startswith("FAIL"):
        gate["status"] = "FAIL: " + ", ".join(failed)
    ok = evm is not None and not failed
    if burst is not None:
        burst["batched_vs_plain_fp32"] = round(value / burst["value"], 2)

    out = {
        "metric": "FC-OFDM Msamples/s on 1 GPU, batched vs plain, at EVM <= -50 dB vs FP64",
        "value": round(value, 1) if ok else None, "unit": "Msamples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched FC TX (256 uneven carriers x %d slot-batches, FP16 I/Q) + batched FC RX "
                               "(8 subbands of a 100 MHz 30 kHz carrier x %d frames, BF16 I/Q)"
                               % (args.tx_batches, args.rx_frames),
                   "storage": "f16 (TX) / bf16 (RX) interleaved I/Q", "timing": "HIP graph replays, HIP events",
                   "tx_samples": tx_samples, "rx_samples": rx_samples, "tx_ms": round(tx_ms, 4),
                   "plan_create_s": plan_s,
                   "rx_ms": round(rx_ms, 4), "tuning": tune, "latency": latency},
        "gate": gate, "value_measured": round(value, 1),
        "roofline": roof, "plain_fp32": burst, "mixed_numerology": subframes, "rx_demod": rx_demod,
        "tx_grid": tx_grid, "weight_grad": weight_grad, "weight_opt": weight_opt, "channel_filter": channel_filter,
        "launch_overhead": overhead,
        "evm_db": evm,
        "method_check": method, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if evm is not None and failed:
        log("bench.py: gate failed: %s" % gate["status"])
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())
