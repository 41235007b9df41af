"""Wide-band method check on the GPU: the four TX/RX chains of the 52-PRB
case (continuous and symbol-synchronised processing, Sec. VI) through the
library, against the FP64 oracle on the same input.

The TX waveforms meet the FP32 gate; the out-of-band power ratio of each TX
scheme and the EVM of each chain agree with the oracle's to well within the
FP32 rounding (GPU noise sits ~80 dB below the filter distortion measured
here, so the tolerances are loose bounds, not fitted values)."""
import pytest

from fc_cases import assert_gate
from wideband import Setup, gpu_chains, oracle_chains

pytestmark = pytest.mark.gpu


def test_wideband_chains():
    S = Setup()
    print("case: wide-band 52 PRB, L = N = 1024, four chains", flush=True)
    y_ref, ref = oracle_chains(S)
    y_gpu, got = gpu_chains(S)
    for k in ("cont", "sync"):
        print("%s TX: OOB %.2f dB (oracle %.2f)" % (k, got["oob_db"][k], ref["oob_db"][k]), flush=True)
        assert_gate([y_gpu[k]], [y_ref[k]], "c64", "%s TX" % k)
        assert abs(got["oob_db"][k] - ref["oob_db"][k]) < 0.1
    for k, v in ref["evm_db"].items():
        print("%s: EVM %.3f dB (oracle %.3f)" % (k, got["evm_db"][k], v), flush=True)
        assert abs(got["evm_db"][k] - v) < 0.05
    assert got["oob_db"]["cont"] < got["oob_db"]["sync"]
