"""GPU weight gradient and autograd through the C ABI against the oracle.

The weight gradient dJ/dD_p = Re <g, b_p> (oracle: the definition, bin by
bin, see oracle/grad.py) is compared as a vector: 10 log10 of the squared
error norm over the squared reference norm. Gate -90 dB: every term is a
product of two FP32 transforms (each about -125 dB, see the parity gate)
summed over blocks; the 35 dB margin covers cancellation in those sums.
"""
import numpy as np
import pytest

from fc_cases import make_inputs, oracle_adj, oracle_wgrad, stream_offsets, to_device
from fcsynth import workloads as W
from oracle import metrics
from test_gpu_parity import TINY_TX, _cat, _plan, _split

pytestmark = pytest.mark.gpu

GRAD_GATE_DB = -90.0


def _g_streams(subbands, seed):
    rng = np.random.default_rng(seed)
    _, lens, _ = stream_offsets(subbands)
    return [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in lens]


def gpu_wgrad(subbands, xs, Ds, gs):
    import torch
    p = _plan(subbands, "c64", Ds)
    gw = p.weight_grad(to_device(_cat(xs), "c64"), to_device(_cat(gs), "c64"))
    torch.cuda.synchronize()
    offs = np.cumsum([0] + [s["n_short"] for s in subbands])
    return _split(gw.cpu().numpy().astype(np.float64), offs)


def assert_grad(got, ref, what, bins=None):
    for k, (g, r) in enumerate(zip(got, ref)):
        if bins is not None:
            g, r = g[bins[k]], r[bins[k]]
        e = metrics.err_db(g, r)
        print("%s subband %d: weight-gradient err %.1f dB (gate %.0f)" % (what, k, e, GRAD_GATE_DB), flush=True)
        assert e <= GRAD_GATE_DB, "%s subband %d: %.1f dB" % (what, k, e)


# (synchronised OLS has no adjoint operator, hence no gradient entry points)
GRAD_CASES = sorted(k for k, v in TINY_TX.items() if all(s["mode"] != "sync_ols" for s in v))


@pytest.mark.parametrize("name", GRAD_CASES)
def test_weight_grad_tiny(name):
    sbs = TINY_TX[name]
    xs, Ds, _ = make_inputs(sbs, 16, 21, "random")
    gs = _g_streams(sbs, 22)
    assert_grad(gpu_wgrad(sbs, xs, Ds, gs), oracle_wgrad(sbs, xs, gs), name)


# single-subband groups at larger interpolation factors: continuous OLS / OLA
# (accumulating adjoint), a quarter overlap, I = 64, and L = 1024
SINGLE = {
    "cont_ols_64_256": W.subband(15, 3, 40, 8, 64, 256, -40, "cont_ols"),
    "cont_ola_quarter_64_512": W.subband(15, 3, 40, 8, 64, 512, 50, "cont_ola", overlap=(1, 4)),
    "sync_ola_16_1024": W.subband(15, 5, 8, 2, 16, 1024, -300, "sync_ola"),
    "sync_ola_1024_2048": W.subband(15, 3, 600, 8, 1024, 2048, 200, "sync_ola"),
}
SINGLE_CP = {"cont_ols_64_256": [20, 16, 16], "cont_ola_quarter_64_512": [24, 16, 16]}


@pytest.mark.parametrize("name", sorted(SINGLE))
def test_weight_grad_single_subband(name):
    s = dict(SINGLE[name])
    if name in SINGLE_CP:
        s["ncp_high"] = SINGLE_CP[name]
    sbs = [s]
    xs, Ds, _ = make_inputs(sbs, 16, 25, "random")
    gs = _g_streams(sbs, 26)
    L = s["n_short"]
    bins = None
    if L > 64:
        rng = np.random.default_rng(27)
        bins = [sorted(rng.choice(L, 12, replace=False).tolist())]
    assert_grad(gpu_wgrad(sbs, xs, Ds, gs), oracle_wgrad(sbs, xs, gs, bins), name, bins)


def test_weight_grad_mixed_numerology_sampled():
    """Both subbands of the 20 MHz mixed-numerology subframe; the oracle
    evaluates the transition bins and a seeded sample of the others."""
    sbs, meta = W.mixed_numerology("sync_ola")
    xs, Ds, _ = make_inputs(sbs, meta["qam"], meta["seed"], "rc")
    gs = _g_streams(sbs, 23)
    rng = np.random.default_rng(24)
    bins = []
    for s in sbs:
        L, K, ntb = s["n_short"], s["n_active"], s["n_tb"]
        tb = [(K // 2 - 1 + i + L // 2) % L for i in range(1, ntb + 1)] + \
             [(-K // 2 - i + L // 2) % L for i in range(1, ntb + 1)]
        bins.append(sorted(set(tb) | set(rng.choice(L, 8, replace=False).tolist())))
    ref = oracle_wgrad(sbs, xs, gs, bins)
    assert_grad(gpu_wgrad(sbs, xs, Ds, gs), ref, "mixed numerology", bins)


def test_weight_grad_largest_carrier_sampled():
    """The largest carrier shape of the batched TX (L = 2048 in N = 4096, one
    slot, FP16 storage of input and cotangent), sampled bins."""
    import torch
    from fc_cases import quantize
    s = W.subband(30, 14, 1272, 8, 2048, 4096, -700, "sync_ola")
    xs, Ds, _ = make_inputs([s], 64, 31, "rc")
    xq = [quantize(xs[0], "f16")]
    gq = [quantize(_g_streams([s], 32)[0], "f16")]
    L, K = 2048, 1272
    bins = [sorted({(K // 2 - 1 + i + L // 2) % L for i in range(1, 9)} | {L // 2, L // 2 + 7})]
    ref = oracle_wgrad([s], xq, gq, bins)
    p = _plan([s], "f16", Ds)
    gw = p.weight_grad(to_device(xq[0], "f16"), to_device(gq[0], "f16"))
    torch.cuda.synchronize()
    got = [gw.cpu().numpy().astype(np.float64)]
    assert_grad(got, ref, "L 2048 N 4096 f16", bins)


@pytest.mark.parametrize("name", ["cont_ols_16_64", "sync_ola_64_256", "two_sb_one_group"])
def test_autograd_matches_oracle(name):
    """J = sum |y - t|^2 through fc_tx: grad_x against the oracle adjoint of
    g = 2 (y - t), grad_w against the oracle weight gradient of the same g."""
    import torch
    from paper_2008_00672_amd import Plan, fc_tx
    sbs = TINY_TX[name]
    xs, Ds, _ = make_inputs(sbs, 16, 31, "random")
    plan = Plan(sbs, io="c64", device=0)
    x = to_device(_cat(xs), "c64").requires_grad_(True)
    w = torch.tensor(np.concatenate(Ds), dtype=torch.float32, device="cuda:0", requires_grad=True)
    y = fc_tx(plan, x, w)
    t = torch.randn(y.shape, dtype=torch.complex64, device="cuda:0", generator=torch.Generator("cuda:0").manual_seed(5))
    J = (y - t).abs().pow(2).sum()
    J.backward()
    torch.cuda.synchronize()
    g = [(2.0 * (y - t)).detach().cpu().numpy().astype(np.complex128)]
    _, lens, _ = stream_offsets(sbs)
    g = _split(g[0], np.cumsum([0] + lens))
    lo, _ = plan.layout(0)
    gx_ref = oracle_adj(sbs, g, [D.astype(np.float32).astype(np.float64) for D in Ds])
    gx = _split(x.grad.cpu().numpy().astype(np.complex128), lo)
    for k, (a, b) in enumerate(zip(gx, gx_ref)):
        e = metrics.err_db(a, b)
        print("%s grad_x part %d: err %.1f dB" % (name, k, e), flush=True)
        assert e <= -100.0
    x64 = [xx for xx in xs]
    gw_ref = oracle_wgrad(sbs, x64, g)
    offs = np.cumsum([0] + [s["n_short"] for s in sbs])
    assert_grad(_split(w.grad.cpu().numpy().astype(np.float64), offs), gw_ref, name + " autograd")


def test_weight_grad_finite_difference_fp32():
    """Central differences of J through the GPU forward in FP32 (h = 1e-3)
    against the GPU weight gradient, relative error <= 1e-3 on the bins with
    the largest gradients."""
    import torch
    from paper_2008_00672_amd import Plan, fc_tx
    sbs = TINY_TX["sync_ola_64_256"]
    xs, Ds, _ = make_inputs(sbs, 16, 41, "random")
    plan = Plan(sbs, io="c64", device=0)
    x = to_device(_cat(xs), "c64")
    w0 = torch.tensor(np.concatenate(Ds), dtype=torch.float32, device="cuda:0")
    t = torch.randn(plan.layout(0)[1][-1], dtype=torch.complex64, device="cuda:0",
                    generator=torch.Generator("cuda:0").manual_seed(6))

    def loss(w):
        y = fc_tx(plan, x, w)
        return float((y.to(torch.complex128) - t.to(torch.complex128)).abs().pow(2).sum())

    w = w0.clone().requires_grad_(True)
    J = (fc_tx(plan, x, w) - t).abs().pow(2).sum()
    J.backward()
    gw = w.grad.cpu().numpy().astype(np.float64)
    h = 1e-3
    for p in np.argsort(-np.abs(gw))[:6]:
        e = torch.zeros_like(w0)
        e[p] = h
        fd = (loss(w0 + e) - loss(w0 - e)) / (2 * h)
        print("bin %d: analytic %.6g fd %.6g" % (p, gw[p], fd), flush=True)
        assert abs(fd - gw[p]) <= 1e-3 * abs(gw[p])


def test_weight_optimisation_reduces_objective():
    """Transition-weight optimisation through the adjoint on four carriers
    (one slot of 16-QAM each): J = mean in-band EVM + mean out-of-band power
    ratio (both linear) of the synchronised TX output, the passband weights
    fixed at one and the 2 N_tb transition weights per carrier learned from
    the raised-cosine start with Adam; gradients come from the library's
    backward kernels, the objective is evaluated in float64 on the CPU."""
    import torch
    from paper_2008_00672_amd import OP_TX, Plan, fc_tx
    from oracle import numerology as nu
    from oracle import weights as ow
    sbs = [W.subband(15, 14, 12 * Wp, ntb, L, N, c, "sync_ola", stream=k)
           for k, (Wp, ntb, L, N, c) in enumerate([(4, 8, 64, 1024, -200), (10, 4, 128, 1024, 150),
                                                   (20, 8, 256, 2048, -300), (40, 8, 512, 2048, 400)])]
    xs, _, grids = make_inputs(sbs, 16, 41, "rc")
    plan = Plan(sbs, io="c64", device=0)
    _, hi = plan.layout(OP_TX)
    x = to_device(_cat(xs), "c64")
    # passband (fixed) and transition bins (learned), fftshifted order
    fixed, tb_idx, theta0 = [], [], []
    off = 0
    for s in sbs:
        L, K, ntb = s["n_short"], s["n_active"], s["n_tb"]
        D = ow.rc_weights(L, K, ntb)
        idx = [L // 2 + K // 2 - 1 + i for i in range(1, ntb + 1)] + [L // 2 - K // 2 - i for i in range(1, ntb + 1)]
        Dp = D.copy()
        Dp[idx] = 0.0
        fixed.append(Dp)
        tb_idx += [off + i for i in idx]
        theta0 += list(D[idx])
        off += L
    fixed = torch.tensor(np.concatenate(fixed), dtype=torch.float32, device="cuda:0")
    tb_idx = torch.tensor(tb_idx, device="cuda:0")
    theta = torch.tensor(theta0, dtype=torch.float32, device="cuda:0", requires_grad=True)

    def objective(y):
        evm, oob = [], []
        for k, s in enumerate(sbs):
            N, L, K, c, ntb = s["n_long"], s["n_short"], s["n_active"], s["center_bin"], s["n_tb"]
            yk = y[int(hi[k]):int(hi[k + 1])].cpu().to(torch.complex128)
            ncp = nu.nr_cp_list(N, 0, 0, 14)
            sig = nu.sync_sigma(ncp, N)
            kap = torch.tensor(np.arange(-K // 2, K // 2) % N)
            # symbol m's useful part starts at sigma_m + N/4; undo the carrier
            # phase at the window start
            sc = torch.stack([torch.fft.fft(yk[sig[m] + N // 4:sig[m] + N // 4 + N])[(kap + c) % N]
                              * np.exp(-2j * np.pi * c * (sig[m] + N // 4) / N) for m in range(14)])
            q = torch.tensor(grids[k], dtype=torch.complex128)
            a = torch.sum(q.conj() * sc) / torch.sum(q.conj() * q)
            evm.append(torch.sum(torch.abs(sc - a * q) ** 2) / torch.sum(torch.abs(a * q) ** 2))
            # Welch periodogram over N bins (hop N/2), Blackman window
            win = torch.tensor(np.blackman(N), dtype=torch.float64)
            segs = torch.stack([yk[t:t + N] * win for t in range(0, len(yk) - N + 1, N // 2)])
            psd = torch.sum(torch.abs(torch.fft.fft(segs, dim=1)) ** 2, dim=0)
            inb = torch.zeros(N, dtype=torch.bool)
            inb[torch.arange(c - K // 2 - ntb - 8, c + K // 2 + ntb + 8) % N] = True
            oob.append(torch.sum(psd[~inb]) / torch.sum(psd))
        return torch.stack(evm).mean() + torch.stack(oob).mean()

    opt = torch.optim.Adam([theta], lr=0.02)
    js = []
    for it in range(12):
        opt.zero_grad()
        w = fixed.index_put((tb_idx,), theta)
        J = objective(fc_tx(plan, x, w))
        J.backward()
        assert torch.isfinite(theta.grad).all()
        js.append(float(J.detach()))
        opt.step()
    print("objective:", ["%.4e" % v for v in js], flush=True)
    assert js[-1] < js[0]
