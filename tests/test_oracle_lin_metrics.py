"""The linear-convolution reference and the metrics of the oracle against
their pins (``lin_metric_pins``), and planted mistakes that the pins must
catch. CPU only.
"""
import importlib
import os
import types

import numpy as np
import pytest

from lin_metric_pins import LIN_PINS, METRIC_PINS, TOL
from oracle import lin, metrics

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


@pytest.mark.parametrize("name", sorted(LIN_PINS))
def test_lin_pin(name):
    err = LIN_PINS[name](lin)
    print("%s: %.2e" % (name, err))
    assert err < TOL


@pytest.mark.parametrize("name", sorted(METRIC_PINS))
def test_metric_pin(name):
    err = METRIC_PINS[name](metrics)
    print("%s: %.2e" % (name, err))
    assert err < TOL


LIN_MUTATIONS = {
    "proto_sign": ("return (np.exp(2j * np.pi * np.outer(d, kappa) / N) @ D) / N",
                   "return (np.exp(-2j * np.pi * np.outer(d, kappa) / N) @ D) / N"),
    "proto_kappa_off": ("kappa = np.arange(L) - (-(-L // 2))", "kappa = np.arange(L) - (-(-L // 2)) + 1"),
    "proto_scale": ("return (np.exp(2j * np.pi * np.outer(d, kappa) / N) @ D) / N",
                    "return (np.exp(2j * np.pi * np.outer(d, kappa) / N) @ D) / L"),
    "carrier_sign": ("return np.exp(2j * np.pi * ((c * t) % N) / N)", "return np.exp(-2j * np.pi * ((c * t) % N) / N)"),
    "filter_not_centred": ("seg = full[N // 2:N // 2 + length]", "seg = full[N // 2 + 1:N // 2 + 1 + length]"),
    "tx_cont_place": ("v[ov.I * (ov.L_O + np.arange(len(x)))] = x", "v[ov.I * (ov.L_L + np.arange(len(x)))] = x"),
    "tx_cont_no_sqrtI": ("    return np.sqrt(ov.I) * _carrier(c, N, t) * _filter_stuffed(v, prototype(L, N, D), N, Q)\n\n\ndef _sync",
                         "    return _carrier(c, N, t) * _filter_stuffed(v, prototype(L, N, D), N, Q)\n\n\ndef _sync"),
    "sync_pad_wrong": ("        S_L = ov.L_L - lc\n", "        S_L = ov.L_L - lc + 1\n"),
    "sync_stride": ("pos.append(sigma[n] + ov.I * (S_L + np.arange(L + lc)))",
                    "pos.append(sigma[n] + ov.I * S_L + np.arange(L + lc))"),
    "sync_no_sqrtI": ("    return np.sqrt(ov.I) * _carrier(c, N, t) * _filter_stuffed(v, prototype(L, N, D), N, Q)\n\n\ndef rx_cont",
                      "    return _carrier(c, N, t) * _filter_stuffed(v, prototype(L, N, D), N, Q)\n\n\ndef rx_cont"),
    "rx_cont_no_conj": ("f = _filter_stuffed(np.conj(_carrier(c, N, t)) * yh, prototype(L, N, D), N, len(yh))\n    return np.sqrt(ov.I) * f[ov.I",
                        "f = _filter_stuffed(_carrier(c, N, t) * yh, prototype(L, N, D), N, len(yh))\n    return np.sqrt(ov.I) * f[ov.I"),
    "rx_cont_sample_off": ("return np.sqrt(ov.I) * f[ov.I * (ov.L_O + np.arange(n_x))]",
                           "return np.sqrt(ov.I) * f[ov.I * (ov.L_O + np.arange(n_x)) + 1]"),
    "rx_cont_scale": ("return np.sqrt(ov.I) * f[ov.I * (ov.L_O + np.arange(n_x))]",
                      "return f[ov.I * (ov.L_O + np.arange(n_x))] / np.sqrt(ov.I)"),
    "rx_sync_grid_from_cp": ("f[s + ov.N_L + ov.I * np.arange(L)]", "f[s + ov.N_L - ov.I + ov.I * np.arange(L)]"),
    "rx_sync_no_conj": ("f = _filter_stuffed(np.conj(_carrier(c, N, t)) * yh, prototype(L, N, D), N, len(yh))\n    sigma",
                        "f = _filter_stuffed(_carrier(c, N, t) * yh, prototype(L, N, D), N, len(yh))\n    sigma"),
    "rx_sync_no_sqrtI": ("np.stack([np.sqrt(ov.I) * f[s + ov.N_L", "np.stack([f[s + ov.N_L"),
}

METRIC_MUTATIONS = {
    "bh_a2_sign": ("+ a[2] * np.cos(4 * np.pi * k / n)", "- a[2] * np.cos(4 * np.pi * k / n)"),
    "bh_symmetric": ("k = np.arange(n)\n    a = (", "k = np.arange(n) * n / (n - 1)\n    a = ("),
    "bh_coefficient": ("a = (0.35875, 0.48829, 0.14128, 0.01168)", "a = (0.35875, 0.48829, 0.14128, 0.0168)"),
    "welch_no_window": ("frames = [y[s:s + N] * w for s", "frames = [y[s:s + N] for s"),
    "welch_hop_n": ("for s in range(0, len(y) - N + 1, N // 2)]", "for s in range(0, len(y) - N + 1, N)]"),
    "welch_power_not_squared": ("return np.sum(np.abs(dft_matrix(N) @ F) ** 2, axis=1)",
                                "return np.sum(np.abs(dft_matrix(N) @ F), axis=1)"),
    "oob_guard_high": ("inband[np.arange(lo, c + K // 2 + n_tb + guard) % N] = True",
                       "inband[np.arange(lo, c + K // 2 + n_tb + guard + 1) % N] = True"),
    "oob_guard_low": ("lo = c - K // 2 - n_tb - guard\n", "lo = c - K // 2 - n_tb - guard + 1\n"),
    "oob_no_tb": ("lo = c - K // 2 - n_tb - guard\n", "lo = c - K // 2 - guard\n"),
    "oob_inband_over_total": ("return 10.0 * np.log10(np.sum(psd[~inband]) / tot)",
                              "return 10.0 * np.log10(np.sum(psd[inband]) / tot)"),
    "complexity_no_tb": ("+ 6 * alpha * ntb +", "+ 6 * ntb +"),
    "complexity_beta_on_ofdm": ("+ split_radix_mults(Lo)\n", "+ beta * split_radix_mults(Lo)\n"),
    "complexity_alpha_high_dropped": ("hi = alpha * split_radix_mults(n_long)", "hi = split_radix_mults(n_long)"),
    "complexity_wrong_denominator": ("return (hi + lo) / sum(k for *_, k in subbands)",
                                     "return (hi + lo) / sum(lm for lm, *_ in subbands)"),
}


def load_mutant(modname, name, old, new):
    path = os.path.join(ORACLE, modname + ".py")
    src = open(path).read()
    assert src.count(old) == 1, "mutation anchor for %s must match exactly once" % name
    mod = types.ModuleType("oracle.%s_mutant_%s" % (modname, name))
    mod.__package__ = "oracle"
    mod.__file__ = path
    exec(compile(src.replace(old, new), path + ":" + name, "exec"), mod.__dict__)
    return mod


def _caught(mod, pins):
    failed = []
    for pin, fn in pins.items():
        try:
            with np.errstate(all="ignore"):
                err = fn(mod)
            if not np.isfinite(err) or err > TOL:
                failed.append(pin)
        except Exception:
            failed.append(pin)
    return failed


@pytest.mark.parametrize("name", sorted(LIN_MUTATIONS))
def test_lin_mutation_is_caught(name):
    mod = load_mutant("lin", name, *LIN_MUTATIONS[name])
    assert _caught(mod, LIN_PINS), "no pin caught mutation %s" % name


@pytest.mark.parametrize("name", sorted(METRIC_MUTATIONS))
def test_metric_mutation_is_caught(name):
    mod = load_mutant("metrics", name, *METRIC_MUTATIONS[name])
    assert _caught(mod, METRIC_PINS), "no pin caught mutation %s" % name


def test_unmutated_modules_load_clean():
    # the loader itself does not perturb the modules: an identity replacement
    # passes every pin
    for modname, pins in (("lin", LIN_PINS), ("metrics", METRIC_PINS)):
        mod = load_mutant(modname, "identity", "import numpy as np", "import numpy as np")
        assert not _caught(mod, pins)
