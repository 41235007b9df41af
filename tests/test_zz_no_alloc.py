"""fc_tx_weight_grad_noalloc through the C ABI: the weight gradient with the
library's fixed device scratch instead of plan-owned scratch.

Two calls in a row, the second on a smaller plan, each bitwise equal to
fc_tx_weight_grad on the same inputs (same kernels, same fixed summation
tree); a plan whose partial sums exceed the fixed scratch is rejected with
FC_E_LIMIT before any work is queued.
"""
import numpy as np
import pytest

from fc_cases import make_inputs, stream_offsets, to_device
from fcsynth import workloads as W

pytestmark = pytest.mark.gpu

FC_E_LIMIT = -7                      # fc_status value of include/fc.h


def _case(n_carriers, batches=1, seed=21):
    from paper_2008_00672_amd import Plan
    sbs, meta = W.batched_carriers(n_carriers=n_carriers)
    allsb = [dict(s, stream=b * len(sbs) + k) for b in range(batches) for k, s in enumerate(sbs)]
    p = Plan(allsb, io="f16", device=0)
    xs, _, _ = make_inputs(sbs, meta["qam"], meta["seed"], "rc")
    _, lens, _ = stream_offsets(allsb)
    rng = np.random.default_rng(seed)
    x = to_device(np.concatenate(xs * batches), "f16")
    g = to_device(rng.standard_normal(sum(lens)) + 1j * rng.standard_normal(sum(lens)), "f16")
    return p, x, g


def test_noalloc_matches_weight_grad():
    import torch
    cases = [("48 carriers", _case(48)), ("12 carriers", _case(12, seed=22))]   # second call: smaller
    for name, (p, x, g) in cases:
        print("case: weight gradient without allocation, %s" % name, flush=True)
        ref = p.weight_grad(x, g)
        out = torch.full_like(ref, float("nan"))
        torch.cuda.synchronize()
        p.weight_grad_noalloc(x, g, out)
        torch.cuda.synchronize()
        same = torch.equal(out.view(torch.int32), ref.view(torch.int32))
        print("%s: %d weights, bitwise equal to fc_tx_weight_grad: %s" % (name, out.numel(), same), flush=True)
        assert torch.isfinite(ref).all() and ref.abs().max() > 0
        assert same


def test_noalloc_rejects_plans_beyond_the_limit():
    import torch
    from paper_2008_00672_amd import FcError
    # 12 batches of the 256 carriers: about 1.73 M partial-sum floats per
    # batch, 83 MB in all, beyond the 64 MiB scratch
    p, x, g = _case(256, batches=12)
    out = torch.zeros(sum(s["n_short"] for s in p.subbands), dtype=torch.float32, device=x.device)
    print("case: weight gradient without allocation beyond the limit", flush=True)
    with pytest.raises(FcError) as ei:
        p.weight_grad_noalloc(x, g, out)
    assert ei.value.status == FC_E_LIMIT
    torch.cuda.synchronize()
    assert torch.count_nonzero(out) == 0          # nothing was queued
