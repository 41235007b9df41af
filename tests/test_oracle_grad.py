"""Pins of the weight-gradient oracle (no GPU).

The oracle's gradient is the definition Re <g, b_p> (output linear in D);
it is pinned to central finite differences of a nonlinear loss and to the
linearity identity J(D) = sum_p D_p dJ/dD_p of the loss J = Re <g, y(D)>.
"""
import os

import numpy as np
import pytest

from fc_cases import make_inputs, oracle_wgrad, sub_params, subband_forward
from fcsynth import workloads as W
from oracle import grad as ogr


def _tiny(mode, L=16, N=64, c=5, ncp=None, n_sym=3):
    s = W.subband(15, n_sym, 8, 2, L, N, c, mode)
    s["ncp_high"] = ncp
    return s


CASES = {
    "cont_ols": _tiny("cont_ols", ncp=[8, 4, 4]),
    "cont_ola": _tiny("cont_ola", ncp=[8, 4, 4]),
    "sync_ola": _tiny("sync_ola", ncp=[9, 5, 6]),
    "sync_ola_c_neg": _tiny("sync_ola", L=32, N=128, c=-21, ncp=[20, 18, 18]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_grad_matches_central_difference(name):
    """J = ||y(D) - t||^2, g = 2 (y - t): the definition against FD (FP64, h = 1e-6)."""
    s = CASES[name]
    xs, Ds, _ = make_inputs([s], 16, 7, "random")
    fwd = subband_forward(s, xs[0])
    rng = np.random.default_rng(8)
    y0 = fwd(Ds[0])
    t = rng.standard_normal(len(y0)) + 1j * rng.standard_normal(len(y0))
    loss = lambda D: float(np.sum(np.abs(fwd(D) - t) ** 2))
    L = sub_params(s)["L"]
    g = 2.0 * (y0 - t)
    an = ogr.weight_grad(fwd, g, L)
    fd = ogr.central_difference(loss, Ds[0], 1e-6, range(L))
    assert np.max(np.abs(an - fd)) <= 1e-6 * np.max(np.abs(fd))


@pytest.mark.parametrize("name", sorted(CASES))
def test_linear_loss_identity(name):
    """J(D) = Re <g, y(D)> is linear in D, so J(D) = sum_p D_p dJ/dD_p."""
    s = CASES[name]
    xs, Ds, _ = make_inputs([s], 16, 9, "random")
    fwd = subband_forward(s, xs[0])
    rng = np.random.default_rng(10)
    n = len(fwd(Ds[0]))
    g = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    grad = ogr.weight_grad(fwd, g, sub_params(s)["L"])
    J = np.real(np.vdot(g, fwd(Ds[0])))
    assert abs(J - grad @ Ds[0]) <= 1e-10 * np.sum(np.abs(grad * Ds[0]))


def test_stream_gradient_splits_by_subband():
    """Two subbands summed into one stream: each subband's gradient only sees
    its own output (the stream is linear in every subband's weights)."""
    sbs = [W.subband(15, 3, 8, 2, 16, 128, -20, "sync_ola"), W.subband(15, 3, 16, 4, 32, 128, 25, "sync_ola")]
    for s in sbs:
        s["ncp_high"] = [9, 9, 9]
    xs, Ds, _ = make_inputs(sbs, 16, 12, "random")
    rng = np.random.default_rng(13)
    from fc_cases import oracle_tx, stream_offsets
    _, lens, _ = stream_offsets(sbs)
    g = [rng.standard_normal(lens[0]) + 1j * rng.standard_normal(lens[0])]
    grads = oracle_wgrad(sbs, xs, g)
    J = np.real(np.vdot(g[0], oracle_tx(sbs, xs, Ds)[0]))
    assert abs(J - sum(gr @ D for gr, D in zip(grads, Ds))) <= 1e-10 * abs(J) + 1e-12


def test_zero_input_zero_gradient():
    s = CASES["sync_ola"]
    L = sub_params(s)["L"]
    xs, _, _ = make_inputs([s], 16, 1, "random")
    fwd = subband_forward(s, np.zeros_like(xs[0]))
    n = len(fwd(np.ones(L)))
    assert np.all(ogr.weight_grad(fwd, np.ones(n), L) == 0.0)


GRAD_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "grad.py")
GRAD_MUTATIONS = {
    "imag_part": ("out[p] = np.real(np.vdot(g, basis_response(forward, L, p)))",
                  "out[p] = np.imag(np.vdot(g, basis_response(forward, L, p)))"),
    "no_conjugate": ("out[p] = np.real(np.vdot(g, basis_response(forward, L, p)))",
                     "out[p] = np.real(np.sum(g * basis_response(forward, L, p)))"),
    "basis_off_by_one": ("e[p] = 1.0", "e[(p + 1) % L] = 1.0"),
    "half_gradient": ("out[p] = np.real(np.vdot(g, basis_response(forward, L, p)))",
                      "out[p] = 0.5 * np.real(np.vdot(g, basis_response(forward, L, p)))"),
}


@pytest.mark.parametrize("name", sorted(GRAD_MUTATIONS))
def test_grad_mutation_is_caught(name, monkeypatch):
    """A planted mistake in the gradient oracle fails the finite-difference pin."""
    import types
    old, new = GRAD_MUTATIONS[name]
    src = open(GRAD_SRC).read()
    assert src.count(old) == 1
    mod = types.ModuleType("oracle.grad_mutant")
    exec(compile(src.replace(old, new), GRAD_SRC + ":" + name, "exec"), mod.__dict__)
    monkeypatch.setattr(ogr, "weight_grad", mod.weight_grad)
    with pytest.raises(AssertionError):
        test_grad_matches_central_difference("sync_ola")
