"""Host checks of the transform plans and LDS budgets that the kernels take
from csrc/fc_internal.h (compile-time functions shared by the planner and the
device code): a C++ program built with g++ evaluates them for every size and
reports what it finds.

* every radix plan factors its size into powers of two, within its cap;
* the per-pass twiddle-base table regions are disjoint and inside the table;
* the plans the kernels use keep every thread within 16 values and keep
  every lane busy where the size allows it (one wave from 256 points up,
  the workgroup's 256 threads from 1024 points up);
* the LDS of every TX pruned class and weight-gradient group fits its budget.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_00672_amd", "csrc")

PROG = r"""
#include "fc_internal.h"
#include <cstdio>
#include <vector>
using namespace fcx;
static int bad = 0;
#define CHECK(c, ...) do { if (!(c)) { ++bad; std::printf(__VA_ARGS__); std::printf("\n"); } } while (0)

// values per thread and busy threads of each pass of a P-point plan on NT threads
static void check_layout(int NT, int P, int RM, bool all_busy, const char* what) {
  for (int s = 0; s < npass(P, RM); ++s) {
    const int R = radix_of(P, s, RM), total = P / R;
    const int maxit = (total + NT - 1) / NT;
    CHECK(maxit * R <= 16, "%s P=%d RM=%d pass %d: %d values per thread", what, P, RM, s, maxit * R);
    if (all_busy) CHECK(total >= NT, "%s P=%d RM=%d pass %d: %d of %d threads busy", what, P, RM, s, total, NT);
  }
}

int main() {
  std::vector<int> used(twb_total(), 0);
  for (int RM : {16, 8, 4}) {
    for (int P = 2; P <= kMaxPoints; P <<= 1) {
      long prod = 1;
      for (int s = 0; s < npass(P, RM); ++s) {
        const int R = radix_of(P, s, RM);
        CHECK(R >= 2 && (R & (R - 1)) == 0 && R <= 16, "RM=%d P=%d pass %d radix %d", RM, P, s, R);
        if (RM < 16) CHECK(R <= RM, "RM=%d P=%d pass %d radix %d above the cap", RM, P, s, R);
        CHECK(ns_of(P, s, RM) == prod, "RM=%d P=%d pass %d ns", RM, P, s);
        prod *= R;
        if (s >= 1) {
          const int off = twb_off(P, s, RM), n = twb_size(P, s, RM);
          CHECK(n == 4 * ns_of(P, s, RM), "RM=%d P=%d pass %d base count", RM, P, s);
          CHECK(off >= 0 && off + n <= twb_total(), "RM=%d P=%d pass %d bases outside the table", RM, P, s);
          for (int i = 0; i < n && off + i < twb_total(); ++i) used[off + i]++;
        }
      }
      CHECK(prod == P, "RM=%d P=%d: radices multiply to %ld", RM, P, prod);
    }
  }
  for (int i = 0; i < twb_total(); ++i) CHECK(used[i] == 1, "twiddle base slot %d used %d times", i, used[i]);
  for (int P = 16; P <= 1024; P <<= 1) check_layout(64, P, wave_radix_cap(P), P >= 256, "wave");
  for (int P = 16; P <= kMaxPoints; P <<= 1) check_layout(kThreads, P, radix_cap(P), P >= 1024, "workgroup");
  // pruned TX long IFFT: 2^LOGI interleaved L-point transforms on the workgroup
  for (int N = 64; N <= kMaxPoints; N <<= 1)
    for (int L = 16; L <= N / 2; L <<= 1) {
      const int RM = radix_cap(N);
      for (int s = 0; s < npass(L, RM); ++s) {
        const int R = radix_of(L, s, RM), total = (L / R) * (N / L);
        CHECK(((total + kThreads - 1) / kThreads) * R <= 16, "pruned N=%d L=%d pass %d", N, L, s);
      }
      const int lds = pruned_lds_bytes(L, N);
      CHECK(lds <= 163840 / 2 || !pruned_wave_short(L, N), "pruned N=%d L=%d: %d B for grouped blocks", N, L, lds);
      CHECK(lds <= 163840, "pruned N=%d L=%d: %d B LDS", N, L, lds);
      CHECK(pruned_waves_per_simd(L, N) >= 1 && pruned_waves_per_simd(L, N) <= 3, "pruned N=%d L=%d waves", N, L);
      if (L <= 1024) {
        const int nb = wgg_group_blocks(L, N);
        CHECK(nb == 1 || wgg_lds_entries(L, N, nb) * 8 <= 80 * 1024, "wgrad N=%d L=%d nb=%d over 80 KiB", N, L, nb);
      }
    }
  std::printf(bad ? "FAILED %d\n" : "ok\n", bad);
  return bad ? 1 : 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no C++ compiler")
def test_radix_plans_and_lds_budgets(tmp_path):
    src = tmp_path / "plans.cpp"
    src.write_text(PROG)
    exe = tmp_path / "plans"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    print(res.stdout)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stdout[-2000:]
