"""Gradient of a real loss with respect to the real subband weights D (oracle).

Test infrastructure only (see ``oracle/__init__``).

Sec. III: every FC block applies the diagonal weight matrix D between the short
transform and the bin mapping, and the transmitter sums the blocks, so the
output is linear in D: y(D) = sum_p D_p b_p with b_p the output for the unit
weight vector e_p. For a real loss J and the complex gradient g that PyTorch
propagates for y (g = 2 dJ/d conj(y), the conjugate Wirtinger convention),

    dJ/dD_p = Re <g, b_p> = Re sum_t conj(g_t) b_p[t].

``weight_grad`` evaluates that definition bin by bin with any forward function
D -> y (for example ``oracle.fc.tx_sync`` with the input fixed).
``central_difference`` is the independent numerical check.
"""
import numpy as np


def basis_response(forward, L, p):
    """Output of the forward map for the unit weight vector e_p."""
    e = np.zeros(L)
    e[p] = 1.0
    return forward(e)


def weight_grad(forward, g, L, bins=None):
    """dJ/dD_p = Re <g, b_p> for p in ``bins`` (default all L); other entries 0."""
    g = np.asarray(g, dtype=complex)
    out = np.zeros(L)
    for p in (range(L) if bins is None else bins):
        out[p] = np.real(np.vdot(g, basis_response(forward, L, p)))
    return out


def central_difference(loss, D, h, bins):
    """(J(D + h e_p) - J(D - h e_p)) / 2h for p in ``bins``."""
    D = np.asarray(D, dtype=float)
    out = np.zeros(len(D))
    for p in bins:
        e = np.zeros(len(D))
        e[p] = h
        out[p] = (loss(D + e) - loss(D - e)) / (2.0 * h)
    return out
