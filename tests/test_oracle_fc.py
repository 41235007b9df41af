"""Oracle pins (CPU only): the FP64 FC oracle against the paper's invariants,
closed forms, textbook special cases and brute force."""
import numpy as np
import pytest

from oracle import fc, lin, metrics, numerology as nu, weights
import fcsynth
from oracle_pins import ALL_PINS, TOL, rel


@pytest.mark.parametrize("name", sorted(ALL_PINS))
def test_pin(name):
    assert ALL_PINS[name](fc) < TOL


def test_dft_matrix_closed_forms():
    for n in (8, 12, 64):
        W = fc.dft_matrix(n)
        assert rel(W @ np.conj(W).T, n * np.eye(n)) < 1e-12            # W W^H = n I
        k0 = 3
        tone = np.exp(-2j * np.pi * k0 * np.arange(n) / n)
        e = np.zeros(n)
        e[(-k0) % n] = n
        assert rel(W @ tone, e) < 1e-12
        assert rel(fc.idft_matrix(n) @ W, np.eye(n)) < 1e-12
        # library special case: numpy's FFT computes the same matrix product
        v = np.random.default_rng(n).standard_normal(n) + 0j
        assert rel(W @ v, np.fft.fft(v)) < 1e-12


def test_shift_and_mapping_matrices():
    for L in (8, 16):
        P = fc.shift_matrix(L)
        v = np.arange(L) + 0j
        assert np.array_equal(P @ v, np.fft.fftshift(v))      # DC moves to L/2
    L, N, c = 8, 32, -5
    M = fc.mapping_matrix(L, N, c, phi=1.0)
    assert np.all(M.sum(axis=0) == 1) and M.sum() == L
    # Xi is 1-based in the paper: Xi(p) = (c - ceil(L/2) + p - 1 mod N) + 1
    for p1 in range(1, L + 1):
        q1 = ((c - L // 2 + p1 - 1) % N) + 1
        assert M[q1 - 1, p1 - 1] == 1
    # the column-selection form equals the dense M product
    D = np.random.default_rng(0).uniform(size=L)
    dense = fc.idft_matrix(N) @ M @ np.diag(D) @ fc.shift_matrix(L) @ fc.dft_matrix(L)
    assert rel(fc.block_core(L, N, c, D), dense) < 1e-12
    dense_rx = (fc.idft_matrix(L) @ fc.shift_matrix(L).T @ np.diag(D) @ M.T @ fc.dft_matrix(N))
    assert rel(fc.block_core_rx(L, N, c, D), dense_rx) < 1e-12


def test_rc_weights():
    D = weights.rc_weights(64, 40, 8)
    assert D.shape == (64,)
    assert np.all(D[32 - 20:32 + 20] == 1.0)
    assert np.all((D >= 0) & (D <= 1))
    assert D[32 + 20 + 8:].sum() == 0 and D[:32 - 20 - 8].sum() == 0
    # symmetric transition: kappa = K/2-1+i and -K/2-i carry the same weight
    for i in range(1, 9):
        assert D[32 + 19 + i] == D[32 - 20 - i]
        assert 0 < D[32 + 19 + i] < 1
    with pytest.raises(ValueError):
        weights.rc_weights(64, 50, 8)


def test_lin_i1_is_np_convolve():
    """The plain reference itself reduces to np.convolve at I = 1, c = 0."""
    from oracle_pins import short_fir
    rng = np.random.default_rng(3)
    h, D = short_fir(rng, 32, 3)
    x = rng.standard_normal(90) + 1j * rng.standard_normal(90)
    y = lin.tx_cont_lin(x, 32, 32, 0, D)
    ov = nu.Overlap(32, 32)
    conv = np.convolve(x, h)
    assert rel(y[ov.L_O - 3:ov.L_O - 3 + len(conv)], conv) < 1e-12


def _plain_slot_signal():
    sbs, meta = fcsynth.workloads.plain_tx_slot()
    s = sbs[0]
    L, N, K = s["n_short"], s["n_long"], s["n_active"]
    ncp = nu.nr_cp_list(N, 0, 0, 14)
    lcp = nu.lowrate_cp(ncp, N // L, exact=True)
    g = fcsynth.qam_grid(np.random.default_rng(meta["seed"]), meta["qam"], 14, K)
    return s, fcsynth.cp_ofdm(g, L, lcp), weights.rc_weights(L, K, s["n_tb"])


def test_fc_approximates_linear_convolution():
    """O-FC against O-LIN: FC is an approximation of linear convolution; with
    50 % overlap and an 8-bin RC transition it is close (bounded, not exact)."""
    s, x, D = _plain_slot_signal()
    L, N = s["n_short"], s["n_long"]
    e_ols = metrics.err_db(fc.tx_cont(x, L, N, 0, D, ola=False), lin.tx_cont_lin(x, L, N, 0, D))
    e_ola = metrics.err_db(fc.tx_cont(x, L, N, 0, D, ola=True), lin.tx_cont_lin(x, L, N, 0, D))
    assert -90 < e_ols < -70 and -90 < e_ola < -60
    # a brick-wall D (no transition band) is much further from linear convolution
    Dbw = weights.rc_weights(L, 288, 0)
    e_bw = metrics.err_db(fc.tx_cont(x, L, N, 0, Dbw), lin.tx_cont_lin(x, L, N, 0, Dbw))
    assert e_bw > e_ols + 20


def test_sync_fc_vs_linear_and_inband_evm():
    """Synchronised TX of a CP-OFDM burst: close to per-symbol linear
    convolution, and the FFT of each received symbol (window at mid-CP) returns
    the QAM grid to within the filter's in-band distortion."""
    L, N, K, c = 512, 2048, 288, 100
    ncp = nu.nr_cp_list(N, 0, 0, 4)
    lcp = nu.lowrate_cp(ncp, N // L, exact=True)
    rng = np.random.default_rng(7)
    g = fcsynth.qam_grid(rng, 16, 4, K)
    x = fcsynth.cp_ofdm(g, L, lcp)
    D = weights.rc_weights(L, K, 16)
    y = fc.tx_sync(x, L, N, c, D, ncp)
    assert metrics.err_db(y, lin.tx_sync_lin(x, L, N, c, D, ncp)) < -60
    ov = nu.Overlap(L, N)
    sig = nu.sync_sigma(ncp, N)
    kap = np.arange(-K // 2, K // 2)
    evm = []
    for n in range(4):
        h = ncp[n] // 2
        t = sig[n] + ov.N_L - h + np.arange(N)          # FFT window at mid-CP
        seg = y[t] * np.exp(-2j * np.pi * c * t / N)
        X = (fc.dft_matrix(N) @ seg) / np.sqrt(N)
        got = X[kap % N] * np.exp(2j * np.pi * kap * h / N)
        evm.append(metrics.err_db(got, g[n]))
    assert max(evm) < -45


def test_rx_loopback_sync():
    """RX(TX(x)) with the same RC window returns the CP-free symbols. The RX
    takes the useful part that starts at the end of the CP, where the zero-phase
    filter's pre-ringing limits the in-band error to about -35 dB."""
    L, N, K, c = 256, 1024, 144, -60
    ncp = nu.nr_cp_list(N, 1, 0, 6)
    lcp = nu.lowrate_cp(ncp, N // L, exact=False)
    g = fcsynth.qam_grid(np.random.default_rng(8), 16, 6, K)
    x = fcsynth.cp_ofdm(g, L, lcp)
    D = weights.rc_weights(L, K, 8)
    y = fc.tx_sync(x, L, N, c, D, ncp)
    z = fc.rx_sync(y, L, N, c, D, ncp)
    got = metrics.ofdm_demod(z)[:, np.arange(-K // 2, K // 2) % L]
    assert metrics.err_db(got, g) < -30


def test_superposition_over_subbands():
    """Two subbands on one stream: the stream is the sum of the single-subband
    outputs (Sec. III-B, x = sum_m w_m); RX of each subband rejects the other."""
    L, N = 64, 256
    rng = np.random.default_rng(9)
    ncp = [18, 18, 18]
    lcp = nu.lowrate_cp(ncp, 4, exact=False)
    K = 24
    D = weights.rc_weights(L, K, 8)
    gA = fcsynth.qam_grid(rng, 4, 3, K)
    gB = fcsynth.qam_grid(rng, 4, 3, K)
    xA, xB = fcsynth.cp_ofdm(gA, L, lcp), fcsynth.cp_ofdm(gB, L, lcp)
    yA = fc.tx_sync(xA, L, N, -60, D, ncp)
    y = fc.place([(0, yA), (0, fc.tx_sync(xB, L, N, 60, D, ncp))])
    zA = fc.rx_sync(y, L, N, -60, D, ncp)
    zA_alone = fc.rx_sync(yA, L, N, -60, D, ncp)
    assert metrics.err_db(zA, zA_alone) < -80           # B is rejected by A's RX
    got = metrics.ofdm_demod(zA)[:, np.arange(-K // 2, K // 2) % L]
    assert metrics.err_db(got, gA) < -30


def test_metrics():
    y = np.ones(10) + 0j
    assert metrics.err_db(y, y) == -np.inf
    assert abs(metrics.err_db(1.1 * y, y) - 10 * np.log10(0.01)) < 1e-12
    N = 64
    t = np.arange(4 * N)
    psd = metrics.welch_psd(np.exp(2j * np.pi * 5 * t / N), N)
    assert np.argmax(psd) == 5
    assert metrics.oob_ratio_db(np.exp(2j * np.pi * 5 * t / N), N, [(5, 2, 1)], guard=4) < -60
    # complexity formula reproduces mu-based counts
    c = metrics.complexity_per_symbol(128, [(16, 16, 0, 12)], alpha=2, beta=1)
    assert c == (2 * 516 + 2 * 20 + 20) / 12
