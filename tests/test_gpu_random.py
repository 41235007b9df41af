"""Seeded random plans against the FP64 oracle: modes, sizes (powers of two,
and mixed radix), centres, overlaps, smooth edges, CP schedules, and
subbands sharing a stream.

Each configuration is drawn from a fixed seed and kept only if a host-only
plan accepts it (so every drawn case is one the library declares valid); the
TX, the RX, and where the mode has them the adjoint, the weight gradient and
the demodulating RX are compared with the oracle under the FP32 gate."""
import numpy as np
import pytest

from fcsynth import workloads as W
from fc_cases import assert_gate
from test_gpu_parity import run_rx, run_tx

pytestmark = pytest.mark.gpu

MODES = ["cont_ola", "cont_ols", "sync_ola", "sync_ols"]


def draw(seed, mixed_radix=False):
    """One valid plan (list of subbands) from the seed: power-of-two sizes, or
    (mixed_radix) N in {768, 1536, 3072} with L in {768, 1536}."""
    from paper_2008_00672_amd import FcError, Plan
    rng = np.random.default_rng(seed)
    while True:
        mode = MODES[int(rng.integers(0, 4))]
        sync = mode.startswith("sync")
        n_sb = int(rng.integers(1, 4))
        N = int(768 << rng.integers(0, 3)) if mixed_radix else int(2 ** rng.integers(6, 11))   # 64 .. 1024
        n_sym = int(rng.integers(1, 5))
        lam = (1, 2) if sync or rng.random() < 0.6 else (1, 4)
        # one CP schedule per plan (subbands sharing a stream share it)
        if sync:
            ncp = [int(v) for v in rng.integers(1, N // 4, n_sym)]
        else:
            step = N // 16
            ncp = [int(step * v) for v in rng.integers(1, 4, n_sym)]
        taper = 0
        if mode == "sync_ols" and rng.random() < 0.5:
            taper = 2 * int(rng.integers(1, max(2, (N // 4 - max(ncp)) // 2 + 1)))
        sbs = []
        for m in range(n_sb):
            if mixed_radix:
                L = int(min(N, 768 << rng.integers(0, 2)))  # 768, 1536
            else:
                L = int(min(N, 2 ** rng.integers(4, 9)))   # 16 .. 256
            n_tb = int(rng.integers(0, 5))
            K = 2 * int(rng.integers(0, (L - 2 * n_tb) // 2 + 1))
            cmax = N // 2 - L // 2
            c = int(rng.integers(-cmax, cmax + 1))
            s = W.subband(15, n_sym, K, n_tb, L, N, c, mode, stream=0 if rng.random() < 0.7 else m,
                          overlap=lam, taper=taper)
            s["ncp_high"] = ncp
            sbs.append(s)
        # streams numbered densely
        ids = sorted({s["stream"] for s in sbs})
        for s in sbs:
            s["stream"] = ids.index(s["stream"])
        try:
            Plan(sbs, device=-1)
        except FcError:
            continue
        return sbs


SEEDS = list(range(100, 124))
MIXED_SEEDS = list(range(200, 208))


def _check_wgrad(sbs, seed):
    """Weight gradient on six random bins per subband against the oracle.
    The bins are drawn from the input's active band and transition bins
    (outside it the input has almost no energy and the gradient almost
    vanishes, so its relative error measures FP32 noise on near-zero values);
    subbands without active subcarriers are skipped."""
    import torch
    from fc_cases import make_inputs, oracle_wgrad, stream_offsets, to_device
    from oracle import metrics
    from test_gpu_parity import _cat, _plan, _split
    xs, Ds, _ = make_inputs(sbs, 16, seed, "random")
    p = _plan(sbs, "c64", Ds)
    _, lens, _ = stream_offsets(sbs)
    rng = np.random.default_rng(seed + 1)
    gs = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in lens]
    gw = p.weight_grad(to_device(_cat(xs), "c64"), to_device(_cat(gs), "c64"))
    torch.cuda.synchronize()
    offs = np.concatenate([[0], np.cumsum([s["n_short"] for s in sbs])])
    got = _split(gw.cpu().numpy().astype(np.float64), offs)
    bins = []
    for s in sbs:
        L, K, ntb = s["n_short"], s["n_active"], s["n_tb"]
        band = np.arange(L // 2 - K // 2 - ntb, L // 2 + K // 2 + ntb)
        bins.append(sorted(rng.choice(band, size=min(6, len(band)), replace=False).tolist()) if K else [])
    for k, (g, r, b) in enumerate(zip(got, oracle_wgrad(sbs, xs, gs, bins), bins)):
        if not b:
            continue
        e = metrics.err_db(g[b], r[b])
        print("random weight gradient %d, subband %d: err %.1f dB" % (seed, k, e), flush=True)
        assert e <= -90.0


@pytest.mark.parametrize("seed", SEEDS + MIXED_SEEDS)
def test_random_plan(seed):
    sbs = draw(seed, mixed_radix=seed in MIXED_SEEDS)
    desc = ", ".join("%s L%d N%d c%d K%d tb%d B%d%s" % (s["mode"], s["n_short"], s["n_long"], s["center_bin"],
                                                        s["n_active"], s["n_tb"], s["n_symbols"],
                                                        " taper%d" % s["taper"] if s["taper"] else "")
                     for s in sbs)
    print("seed %d: %s" % (seed, desc), flush=True)
    got, ref = run_tx(sbs, "c64", seed=seed, weights="random")
    assert_gate(got, ref, "c64", "random TX %d" % seed)
    got, ref = run_rx(sbs, "c64", seed=seed, weights="random")
    assert_gate(got, ref, "c64", "random RX %d" % seed)
    if all(s["mode"] != "sync_ols" for s in sbs):
        got, ref = run_rx(sbs, "c64", seed=seed, weights="random", adjoint=True)
        assert_gate(got, ref, "c64", "random adjoint %d" % seed)
        _check_wgrad(sbs, seed)
    if all(s["mode"].startswith("sync") for s in sbs):
        got, ref = run_rx(sbs, "c64", seed=seed, weights="random", demod=True)
        assert_gate(got, ref, "c64", "random demod RX %d" % seed)


def draw_wide(seed):
    """One valid synchronised plan with wide groups (three to six subbands
    of 256 to 2048 points sharing one 2048- or 4096-point transform): the
    demodulating RX's subband regions then take 20 to 64 KB, so in FP16 /
    BF16 storage its second-block terms go to device scratch (and groups
    beyond 8192 region entries are split)."""
    from paper_2008_00672_amd import FcError, Plan
    rng = np.random.default_rng(seed)
    while True:
        mode = ("sync_ola", "sync_ols")[int(rng.integers(0, 2))]
        N = int(2048 << rng.integers(0, 2))
        n_sym = int(rng.integers(1, 4))
        ncp = [int(v) for v in rng.integers(1, N // 8, n_sym)]
        sbs = []
        for m in range(int(rng.integers(3, 7))):
            L = int(min(N // 2, 256 << rng.integers(0, 4)))       # 256 .. 2048
            n_tb = int(rng.integers(0, 9))
            K = 2 * int(rng.integers(0, (L - 2 * n_tb) // 2 + 1))
            cmax = N // 2 - L // 2
            s = W.subband(30, n_sym, K, n_tb, L, N, int(rng.integers(-cmax, cmax + 1)), mode)
            s["ncp_high"] = ncp
            sbs.append(s)
        try:
            Plan(sbs, device=-1)
        except FcError:
            continue
        return sbs


@pytest.mark.parametrize("io", ["f16", "bf16"])
@pytest.mark.parametrize("seed", list(range(300, 306)))
def test_random_demod_half_storage(seed, io):
    sbs = draw_wide(seed)
    print("seed %d %s: %s" % (seed, io, ", ".join("%s L%d N%d c%d K%d tb%d B%d" % (
        s["mode"], s["n_short"], s["n_long"], s["center_bin"], s["n_active"], s["n_tb"], s["n_symbols"])
        for s in sbs)), flush=True)
    got, ref = run_rx(sbs, io, seed=seed, weights="random", demod=True)
    assert_gate(got, ref, io, "random demod RX %d" % seed)
