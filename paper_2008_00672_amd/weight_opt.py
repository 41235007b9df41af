"""Transition-weight optimisation through the library's adjoint.

The FC synthesis is linear in the real weights D of every subband (Sec. III
block operator W_N^{-1} M(phi) D P W_L A), so the 2 N_tb transition weights
of each subband can be learned by gradient descent on any differentiable
objective of the output. Here the objective is the synchronised transmitter's
quality:

    J = mean_k EVM_k + mu_oob * mean_k OOB_k        (both linear, per subband k)

EVM_k: the subband's active subcarriers, demodulated from its own high-rate
output (an N-point DFT per symbol, window starting half-way into the CP with
the linear phase of that shift removed, the carrier phase at the window start
removed), against the transmitted QAM symbols after a least-squares complex
gain. OOB_k: Welch PSD of the subband's output (4-term Blackman-Harris window
of N samples, hop N/2), power outside [c - K/2 - N_tb - guard,
c + K/2 + N_tb + guard) over the total.

The FC forward, its adjoint and the weight gradient run in libfc.so
(``autograd.fc_tx``); the objective itself is an ordinary PyTorch loss on the
GPU (batched over subbands of the same N and CP schedule), as a user of the
library would write it.
"""
import numpy as np
import torch

from .autograd import fc_tx
from .fc import OP_TX

# 4-term Blackman-Harris window coefficients (Harris, Proc. IEEE 1978)
_BH = (0.35875, 0.48829, 0.14128, 0.01168)


def transition_bins(L, K, ntb):
    """Indices (fftshifted order, p = kappa + L/2) of the 2 N_tb transition
    bins: kappa = K/2 - 1 + i above the band and -K/2 - i below it, i = 1..N_tb."""
    return [L // 2 + K // 2 - 1 + i for i in range(1, ntb + 1)] + [L // 2 - K // 2 - i for i in range(1, ntb + 1)]


class TransitionWeights:
    """The learnable part of a plan's weights: theta holds the 2 N_tb
    transition weights of every subband (plan order); full(theta) is the whole
    weight vector (passband and stopband fixed at the plan's current values)."""

    def __init__(self, plan):
        dev = torch.device("cuda", plan.device)
        fixed, idx, theta0, off = [], [], [], 0
        for k, s in enumerate(plan.subbands):
            L = s["n_short"]
            D = plan.get_weights(k).astype(np.float32)
            tb = transition_bins(L, s["n_active"], s["n_tb"])
            theta0.append(D[tb].copy())
            D[tb] = 0.0
            fixed.append(D)
            idx += [off + i for i in tb]
            off += L
        self.fixed = torch.tensor(np.concatenate(fixed), device=dev)
        self.idx = torch.tensor(idx, dtype=torch.int64, device=dev)
        self.theta0 = torch.tensor(np.concatenate(theta0), device=dev)

    def full(self, theta):
        return self.fixed.index_put((self.idx,), theta)


def _bh_window(N, device, dtype):
    k = torch.arange(N, dtype=torch.float64, device=device)
    w = (_BH[0] - _BH[1] * torch.cos(2 * np.pi * k / N) + _BH[2] * torch.cos(4 * np.pi * k / N)
         - _BH[3] * torch.cos(6 * np.pi * k / N))
    return w.to(dtype)


def _sigma(ncp, N):
    """High-rate start of each synchronised symbol: sigma_n = n N + sum_{q=1..n} N_CP,q."""
    return np.arange(len(ncp)) * N + np.concatenate([[0], np.cumsum(ncp[1:])])


class TxObjective:
    """J of a plan whose subbands are synchronised, one per stream, with the
    transmitted QAM grids ``grids`` ((n_symbols, K) per subband). ``dtype``
    (complex64 or complex128) is the precision of the objective; ``device``
    where it is evaluated (default: the plan's GPU; the plan's layout and CP
    schedule are all it reads, so a host-only plan serves a CPU objective)."""

    def __init__(self, plan, grids, mu_oob=1.0, guard=8, dtype=torch.complex64, device=None):
        sbs = plan.subbands
        if any(s["mode"] not in ("sync_ola", "sync_ols") for s in sbs):
            raise ValueError("the objective takes synchronised subbands")
        if sorted(s["stream"] for s in sbs) != list(range(len(sbs))):
            raise ValueError("the objective takes one subband per stream")
        self.mu_oob, self.dtype = mu_oob, dtype
        rdt = torch.float64 if dtype == torch.complex128 else torch.float32
        dev = torch.device(device) if device is not None else torch.device("cuda", plan.device)
        _, hi = plan.layout(OP_TX)
        groups = {}
        for k, s in enumerate(sbs):
            ncp, _, off = plan.symbols(k)
            if off != 0:
                raise ValueError("one subband per stream expected")
            groups.setdefault((s["n_long"], tuple(int(v) for v in ncp)), []).append(k)
        self.n = len(sbs)
        # streams in order (one subband each): y splits into them in one view
        self.stream_lens = [int(v) for v in np.diff(hi)]
        self.stream_of = [s["stream"] for s in sbs]
        self.groups = []
        for (N, ncp), ks in groups.items():
            ncp = np.array(ncp)
            B = len(ncp)
            Q = int(hi[sbs[ks[0]]["stream"] + 1] - hi[sbs[ks[0]]["stream"]])
            t0 = _sigma(ncp, N) + N // 4                      # start of each symbol's useful part
            d = ncp // 2                                      # window start: half-way into the CP
            win_start = t0 - d
            Kmax = max(sbs[k]["n_active"] for k in ks)
            bins = np.zeros((len(ks), Kmax), dtype=np.int64)
            mask = np.zeros((len(ks), Kmax), dtype=bool)
            qam = np.zeros((len(ks), B, Kmax), dtype=np.complex128)
            inband = np.zeros((len(ks), N), dtype=bool)
            ph = np.zeros((len(ks), B, Kmax))
            for g, k in enumerate(ks):
                s = sbs[k]
                K, c, ntb = s["n_active"], s["center_bin"], s["n_tb"]
                kb = np.arange(-K // 2, K // 2) + c           # bin of subcarrier kappa
                bins[g, :K] = kb % N
                mask[g, :K] = True
                qam[g, :, :K] = grids[k]
                inband[g, np.arange(c - K // 2 - ntb - guard, c + K // 2 + ntb + guard) % N] = True
                # + 2 pi kb d_m / N (the window's cyclic shift) - 2 pi c t0_m / N
                # (carrier phase at the useful part's start), integer-reduced
                ph[g, :, :K] = 2 * np.pi * ((np.outer(d, kb) - c * t0[:, None]) % N) / N
            # the symbols' windows do not overlap (each starts at most half a
            # CP before its useful part): the output splits into windows and
            # the gaps between them
            cuts = np.ravel(np.column_stack([win_start, win_start + N]))
            pieces = np.diff(np.concatenate([[0], cuts, [Q]])).tolist()
            if min(pieces) < 0:
                raise ValueError("symbol windows overlap")
            self.groups.append(dict(
                N=N, ks=torch.tensor(ks, device=dev), ks_list=list(ks), Q=Q, pieces=pieces,
                bins=torch.tensor(bins, device=dev)[:, None, :].expand(len(ks), B, Kmax),
                mask=torch.tensor(mask, device=dev)[:, None, :],
                qam=torch.tensor(qam, dtype=dtype, device=dev),
                phase=torch.polar(torch.ones(ph.shape, dtype=rdt), torch.tensor(ph, dtype=rdt)).to(dev),
                inband=torch.tensor(inband, device=dev),
                window=_bh_window(N, dev, rdt)))

    def __call__(self, y):
        """(J, EVM per subband, OOB per subband) of the TX output y."""
        y = y.to(self.dtype)
        evm = y.new_zeros(self.n, dtype=y.real.dtype)
        oob = y.new_zeros(self.n, dtype=y.real.dtype)
        # one split of the output into its streams (its backward is a single
        # concatenation, where slicing per subband would build a full-size
        # gradient per slice)
        streams = torch.split(y, self.stream_lens)
        for G in self.groups:
            N = G["N"]
            Y = torch.stack([streams[self.stream_of[k]] for k in G["ks_list"]])   # (n_g, Q)
            W = torch.stack(torch.split(Y, G["pieces"], dim=1)[1::2], dim=1)   # (n_g, B, N) symbol windows
            Z = torch.fft.fft(W, dim=-1)
            Z = torch.gather(Z, 2, G["bins"]) * G["phase"]              # active subcarriers
            q = G["qam"]
            m = G["mask"]
            a = (torch.sum(q.conj() * Z * m, dim=(1, 2)) / torch.sum((q.abs() ** 2) * m, dim=(1, 2)))
            e = torch.sum(torch.abs(Z - a[:, None, None] * q) ** 2 * m, dim=(1, 2))
            evm = evm.index_put((G["ks"],), e / (torch.abs(a) ** 2 * torch.sum(q.abs() ** 2 * m, dim=(1, 2))))
            F = torch.fft.fft(Y.unfold(1, N, N // 2) * G["window"], dim=-1)   # (n_g, frames, N), hop N/2
            psd = torch.sum(torch.abs(F) ** 2, dim=1)
            oob = oob.index_put((G["ks"],), torch.sum(psd * ~G["inband"], dim=1) / torch.sum(psd, dim=1))
        return evm.mean() + self.mu_oob * oob.mean(), evm, oob


def optimise(plan, x, grids, steps=10, lr=0.02, mu_oob=1.0, dtype=torch.complex64, stream_sync=True):
    """Adam over the transition weights from the plan's current weights.
    Returns (theta, J per step)."""
    tw = TransitionWeights(plan)
    obj = TxObjective(plan, grids, mu_oob=mu_oob, dtype=dtype)
    theta = tw.theta0.clone().requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=lr)
    js = []
    for _ in range(steps):
        opt.zero_grad()
        J, _, _ = obj(fc_tx(plan, x, tw.full(theta)))
        J.backward()
        opt.step()
        js.append(J.detach())
    if stream_sync:
        torch.cuda.synchronize()
    return theta.detach(), [float(j) for j in js]
