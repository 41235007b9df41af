"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign or index, a wrong
operand) into a copy of the oracle's FC source, loads the copy as a module and
runs every pin on it; at least one pin must fail. Runs on the CPU only.
"""
import importlib.util
import os
import types

import numpy as np
import pytest

from oracle_pins import ALL_PINS, TOL

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "fc.py")

MUTATIONS = {
    "dft_index": ("e = np.outer(k, k) % n", "e = np.outer(k, (k + 1) % n) % n"),
    "tx_drop_sqrtI": ("yb = np.sqrt(ov.I) * phi * blocks[:, r]", "yb = phi * blocks[:, r]"),
    "phi_sign": ("phi = unit_phase(r * c * ov.L_S, L)\n        yb", "phi = unit_phase(-r * c * ov.L_S, L)\n        yb"),
    "xi_off_by_one": ("return (c - (-(-L // 2)) + np.arange(L)) % N", "return (c - (-(-L // 2)) + np.arange(L) + 1) % N"),
    "tx_wrong_direction": ("return idft_matrix(N)[:, xi(L, N, c)] @ inner", "return dft_matrix(N)[:, xi(L, N, c)] @ inner / N"),
    "drop_shift": ("inner = D[:, None] * (shift_matrix(L) @ dft_matrix(L))", "inner = D[:, None] * dft_matrix(L)"),
    "weights_reversed": ("inner = D[:, None] * (shift_matrix(L) @ dft_matrix(L))", "inner = D[::-1, None] * (shift_matrix(L) @ dft_matrix(L))"),
    "theta_dropped": ("theta = unit_phase(c * sigma[n], N)\n        wn", "theta = 1.0\n        wn"),
    "theta_sign": ("theta = unit_phase(c * sigma[n], N)\n        wn", "theta = unit_phase(-c * sigma[n], N)\n        wn"),
    "first_window_no_cp": ("a = [np.r_[np.zeros(S_L), np.ones(ov.L_S + lcp[n]), np.zeros(ov.L_T)],",
                           "a = [np.r_[np.zeros(ov.L_L), np.ones(ov.L_S), np.zeros(ov.L_T)],"),
    "windows_swapped": ("seg = z[r * L // 2:r * L // 2 + L] * a[r]", "seg = z[r * L // 2:r * L // 2 + L] * a[1 - r]"),
    "sync_second_block_offset": ("wn[r * N // 2:r * N // 2 + N] += np.sqrt(ov.I)", "wn[r * N // 4:r * N // 4 + N] += np.sqrt(ov.I)"),
    "sync_padding_wrong": ("S_L = ov.L_L - lcp[n]\n        z = np.r_", "S_L = ov.L_L - lcp[n] - 1\n        z = np.r_"),
    "ola_window_dropped": ("    if ola:\n        segs = segs * a[:, None]", "    if False:\n        segs = segs * a[:, None]"),
    "ols_keep_shifted": ("        if not ola:\n            yb = s * yb", "        if not ola:\n            yb = np.roll(s, 1) * yb"),
    "rx_phase_not_conj": ("phi = np.conj(unit_phase(r * c * ov.L_S, L))\n        zr", "phi = unit_phase(r * c * ov.L_S, L)\n        zr"),
    "rx_scale": ("zr = phi * z[:, r] / np.sqrt(ov.I)", "zr = phi * z[:, r] * np.sqrt(ov.I)"),
    "rx_no_unshift": ("Pinv = shift_matrix(L).T", "Pinv = np.eye(L)"),
    "rx_wrong_gather": ("return left @ dft_matrix(N)[xi(L, N, c), :]", "return left @ dft_matrix(N)[xi(L, N, -c), :]"),
    "rx_sync_theta_missing": ("theta = np.conj(unit_phase(c * sigma[n], N))", "theta = 1.0"),
    "concat_wrong_half": ("P[rows, L // 4 + np.arange(L // 2)] = 1.0", "P[rows, np.arange(L // 2)] = 1.0"),
    "keep_cp_off_by_one": ("out.append(np.r_[z[0][S_L:3 * L // 4], z[1][L // 4:3 * L // 4]])",
                           "out.append(np.r_[z[0][S_L + 1:3 * L // 4 + 1], z[1][L // 4:3 * L // 4]])"),
    "demod_no_scale": ("return rx_sync(yh, L, N, c, D, ncp) @ dft_matrix(L) / np.sqrt(L)",
                       "return rx_sync(yh, L, N, c, D, ncp) @ dft_matrix(L)"),
    "demod_inverse": ("return rx_sync(yh, L, N, c, D, ncp) @ dft_matrix(L) / np.sqrt(L)",
                      "return rx_sync(yh, L, N, c, D, ncp) @ idft_matrix(L) * np.sqrt(L)"),
    "reduced_window_second_half": ("S_hat = np.diag(np.r_[np.ones(L // 2), np.zeros(L // 2)])",
                                   "S_hat = np.diag(np.r_[np.zeros(L // 2), np.ones(L // 2)])"),
    "reduced_omega_sign": ("return np.exp(-2j * np.pi * ((phi * np.arange(L)) % L) / L)",
                           "return np.exp(2j * np.pi * ((phi * np.arange(L)) % L) / L)"),
    "reduced_block_swap": ("for g0, g1 in g:", "for g1, g0 in g:"),
    "blocks_freq_no_phase": ("g.append(phi_r * th_n * (Gf @ wn[r * N // 2:r * N // 2 + N]) / np.sqrt(ov.I))",
                             "g.append(th_n * (Gf @ wn[r * N // 2:r * N // 2 + N]) / np.sqrt(ov.I))"),
    "ols_first_window_no_cp": ("np.r_[np.zeros(ov.N_L - ncp[n]), np.ones(ov.N_S + ncp[n]), np.zeros(ov.N_T)]",
                               "np.r_[np.zeros(ov.N_L), np.ones(ov.N_S), np.zeros(ov.N_T)]"),
    "ols_block_offset": ("blk = T @ zpad[r * L // 2:r * L // 2 + L]", "blk = T @ zpad[r * L // 4:r * L // 4 + L]"),
    "ols_phase_dropped": ("ph_r = unit_phase(r * c * ov.L_S, L)", "ph_r = 1.0"),
    "ofdm_no_scale": ("x = np.sqrt(L) * (Winv @ X)", "x = Winv @ X"),
    "ofdm_forward": ("x = np.sqrt(L) * (Winv @ X)", "x = (dft_matrix(L) @ X) / np.sqrt(L)"),
    "ofdm_cp_from_start": ("out.append(np.r_[x[L - lcp[n]:], x])\n    return np.concatenate(out)\n\n\ndef tx_sync_grid",
                           "out.append(np.r_[x[:lcp[n]], x])\n    return np.concatenate(out)\n\n\ndef tx_sync_grid"),
    "ofdm_subcarrier_shift": ("X[np.arange(-K // 2, K // 2) % L] = grid[n]\n        x = np.sqrt(L)",
                              "X[np.arange(-K // 2 + 1, K // 2 + 1) % L] = grid[n]\n        x = np.sqrt(L)"),
    "blocks_freq_theta_sign": ("th_n = np.conj(unit_phase(c * sigma[n], N))", "th_n = unit_phase(c * sigma[n], N)"),
    "taper_falling_not_mirrored": ("s_win[1][e1 - h:e1 + h] = ramp[::-1]", "s_win[1][e1 - h:e1 + h] = ramp"),
    "taper_edge_off_by_one": ("s_win[0][e0 - h:e0 + h] = ramp", "s_win[0][e0 - h + 1:e0 + h + 1] = ramp"),
    "taper_shape_offset": ("return np.sin(np.pi * (i + 0.5) / (2 * T)) ** 2", "return np.sin(np.pi * (i + 1) / (2 * T)) ** 2"),
}


def load_mutant(name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor for %s must match exactly once" % name
    mod = types.ModuleType("oracle.fc_mutant_" + name)
    mod.__package__ = "oracle"
    mod.__file__ = SRC
    exec(compile(src.replace(old, new), SRC + ":" + name, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    mod = load_mutant(name, *MUTATIONS[name])
    failed = []
    for pin, fn in ALL_PINS.items():
        try:
            err = fn(mod)
            if not np.isfinite(err) or err > TOL:
                failed.append(pin)
        except Exception:
            failed.append(pin)
    assert failed, "no pin caught mutation %s" % name
