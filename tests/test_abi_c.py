"""The C ABI used from C: a C99 program compiled against include/fc.h and
linked with libfc.so builds a host-only plan (no GPU), reads its layout and
CP schedule, and reports the status strings of invalid calls; the results
must equal what the Python binding reports for the same subband."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2008_00672_amd")

PROG = r"""
#include "fc.h"
#include <stdio.h>
int main(void) {
  fc_subband sb = {0};
  sb.scs_khz = 15; sb.n_symbols = 14; sb.n_active = 288; sb.n_tb = 8;
  sb.n_short = 512; sb.n_long = 2048; sb.center_bin = 0;
  sb.overlap_num = 1; sb.overlap_den = 2; sb.mode = FC_SYNC_OLA;
  fc_plan* plan = 0;
  fc_status st = fc_plan_create(&sb, 1, FC_IO_F16, -1, &plan);
  if (st != FC_OK) { printf("create %d\n", st); return 1; }
  int64_t lo[2], hi[2];
  if (fc_plan_layout(plan, FC_OP_TX, lo, hi) != FC_OK) return 2;
  printf("tx %lld %lld\n", (long long)lo[1], (long long)hi[1]);
  if (fc_plan_layout(plan, FC_OP_RX, lo, hi) != FC_OK) return 3;
  printf("rx %lld %lld\n", (long long)lo[1], (long long)hi[1]);
  int32_t ncp[14], lcp[14];
  int64_t off;
  if (fc_plan_symbols(plan, 0, ncp, lcp, &off) != FC_OK) return 4;
  printf("cp %d %d %d %d\n", ncp[0], ncp[1], lcp[0], lcp[1]);
  /* a compute call on a host-only plan is a state error, not a crash */
  printf("state %d\n", fc_tx_synthesize(plan, (const void*)1, (void*)1, 0));
  fc_plan_destroy(plan);
  sb.n_short = 96;                                   /* not a power of two */
  printf("bad %d %s\n", fc_plan_create(&sb, 1, FC_IO_F16, -1, &plan), fc_status_str(FC_E_UNSUPPORTED));
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_program(tmp_path):
    from fcsynth import workloads as W
    from paper_2008_00672_amd import OP_RX, OP_TX, Plan
    from paper_2008_00672_amd import fc as fcmod
    fcmod.lib()            # the library is built
    src = tmp_path / "t.c"
    src.write_text(PROG)
    exe = tmp_path / "t"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-L", LIBDIR, "-lfc", "-Wl,-rpath," + LIBDIR, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    s = dict(W.plain_tx_slot()[0][0], mode="sync_ola")
    p = Plan([s], io="f16", device=-1)
    lo, hi = p.layout(OP_TX)
    assert out[0] == "tx %d %d" % (lo[-1], hi[-1])
    lo, hi = p.layout(OP_RX)
    assert out[1] == "rx %d %d" % (lo[-1], hi[-1])
    ncp, lcp, _ = p.symbols(0)
    assert out[2] == "cp %d %d %d %d" % (ncp[0], ncp[1], lcp[0], lcp[1])
    assert out[3] == "state -6"
    assert out[4].startswith("bad -3 ")
