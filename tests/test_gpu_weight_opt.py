"""Transition-weight optimisation at the shape of the weight-optimisation
workload: all 256 batched carriers, N_tb ~ U{4..16}, FP32 I/O, 16-QAM, the
objective J = mean EVM + mean OOB of paper_2008_00672_amd.weight_opt (two
slots per carrier here; the bench runs 64).

* The gradient from the library's backward kernels matches the oracle's
  weight gradient (Re <g, b_p>, with g the objective's cotangent of the
  output) on sampled carriers and transition bins, <= -90 dB.
* It matches central finite differences of the objective through the GPU
  forward in FP32 (h = 1e-3), relative error <= 1e-3, on the bins with the
  largest gradients.
* A few Adam steps lower J.
"""
import numpy as np
import pytest

from fc_cases import make_inputs, oracle_wgrad, to_device
from fcsynth import workloads as W
from oracle import metrics

pytestmark = pytest.mark.gpu

SLOTS = 2


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2008_00672_amd import Plan
    sbs, meta = W.weight_opt_carriers(n_slots=SLOTS)
    print("case: weight optimisation, %d carriers x %d slots, FP32" % (len(sbs), SLOTS), flush=True)
    xs, Ds, grids = make_inputs(sbs, meta["qam"], meta["seed"], "rc")
    plan = Plan(sbs, io="c64", device=0)
    x = to_device(np.concatenate(xs), "c64")
    torch.cuda.synchronize()
    return dict(sbs=sbs, xs=xs, grids=grids, plan=plan, x=x)


def _grad(setup, dtype):
    import torch
    from paper_2008_00672_amd import fc_tx
    from paper_2008_00672_amd.weight_opt import TransitionWeights, TxObjective
    plan = setup["plan"]
    tw = TransitionWeights(plan)
    obj = TxObjective(plan, setup["grids"], dtype=dtype)
    w = tw.full(tw.theta0).requires_grad_(True)
    y = fc_tx(plan, setup["x"], w)
    y.retain_grad()
    J, evm, oob = obj(y)
    J.backward()
    torch.cuda.synchronize()
    return tw, obj, w, y, J, evm, oob


def test_gradient_matches_oracle(setup):
    """J is a sum of per-carrier terms, so carrier k's cotangent depends on
    its own output only. For sampled carriers the cotangent is taken on the
    oracle side (the objective on the CPU in FP64, applied to the oracle's
    output); the same cotangent, placed on those carriers of the full
    256-carrier plan, goes through the library's weight gradient and the
    oracle's, on sampled transition bins."""
    import torch
    from fc_cases import oracle_tx
    from paper_2008_00672_amd import Plan
    from paper_2008_00672_amd.weight_opt import TxObjective, transition_bins
    from oracle import weights as ow
    plan, sbs, xs = setup["plan"], setup["sbs"], setup["xs"]
    _, hi = plan.layout(0)
    w_off = np.concatenate([[0], np.cumsum([s["n_short"] for s in sbs])])
    g_full = np.zeros(int(hi[-1]), dtype=np.complex128)
    rng = np.random.default_rng(12)
    checks = []
    for k in (0, 77, 128, 255):
        s = dict(sbs[k], stream=0)
        D = ow.rc_weights(s["n_short"], s["n_active"], s["n_tb"])
        y_ref = oracle_tx([s], [xs[k]], [D])[0]
        obj = TxObjective(Plan([s], io="c64", device=-1), [setup["grids"][k]], dtype=torch.complex128, device="cpu")
        y = torch.tensor(y_ref, dtype=torch.complex128, requires_grad=True)
        J, _, _ = obj(y)
        J.backward()
        g = y.grad.numpy()
        assert len(g) == int(hi[k + 1] - hi[k])
        g_full[int(hi[k]):int(hi[k + 1])] = g
        tb = transition_bins(s["n_short"], s["n_active"], s["n_tb"])
        bins = sorted(rng.choice(tb, size=4, replace=False).tolist())
        checks.append((k, s, g, bins, float(J)))
    gw = plan.weight_grad(setup["x"], to_device(g_full, "c64"))
    torch.cuda.synchronize()
    gw = gw.cpu().numpy().astype(np.float64)
    for k, s, g, bins, J in checks:
        ref = oracle_wgrad([s], [xs[k]], [g], [bins])[0]
        got = gw[w_off[k] + np.array(bins)]
        e = metrics.err_db(got, ref[bins])
        print("carrier %d (L %d N %d N_tb %d, J_k %.3e) bins %s: err %.1f dB" % (
            k, s["n_short"], s["n_long"], s["n_tb"], J, bins, e), flush=True)
        assert e <= -90.0


def test_gradient_matches_finite_differences(setup):
    import torch
    from paper_2008_00672_amd import fc_tx
    tw, obj, w, y, J, evm, oob = _grad(setup, torch.complex128)
    plan, sbs = setup["plan"], setup["sbs"]
    gw = w.grad.cpu().numpy().astype(np.float64)
    n = len(sbs)
    owner = np.concatenate([[k] * s["n_short"] for k, s in enumerate(sbs)])
    tb_idx = tw.idx.cpu().numpy()
    w0 = tw.full(tw.theta0)
    h = 1e-3
    # J = mean EVM + mean OOB, and a weight of subband k moves only its own
    # terms: dJ/dw_p = (EVM_k + OOB_k)' / n, differenced per subband
    for p in tb_idx[np.argsort(-np.abs(gw[tb_idx]))[:6]]:
        k = int(owner[p])

        def jk(delta):
            e = torch.zeros_like(w0)
            e[p] = delta
            with torch.no_grad():
                _, ev, oo = obj(fc_tx(plan, setup["x"], w0 + e))
            return float(ev[k] + oo[k])
        fd = (jk(h) - jk(-h)) / (2 * h) / n
        print("weight %d (carrier %d): analytic %.6g fd %.6g" % (p, k, gw[p], fd), flush=True)
        assert abs(fd - gw[p]) <= 1e-3 * abs(gw[p])


def test_adam_lowers_objective(setup):
    from paper_2008_00672_amd.weight_opt import optimise
    theta, js = optimise(setup["plan"], setup["x"], setup["grids"], steps=5, lr=0.02)
    print("J per step:", ["%.5e" % v for v in js], flush=True)
    assert np.all(np.isfinite(js)) and js[-1] < js[0]
