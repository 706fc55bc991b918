"""The FP64 flight-time logarithm of the HIP path (paper_1901_08140_amd/csrc/unit_log.hpp), built
for the host with the library's own compiler and flags: it uses only IEEE-exact operations, so
the host build computes the bits the kernels compute.  Its error is measured against the
x87 extended-precision logarithm on the inputs the kernels see, x = 1 - u with u a 53-bit
uniform (eq. random_time), and on edge values (1, 1 - 2^-53, 2^-53, the near-1 switch, table
cell edges, powers of two)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1901_08140_amd", "csrc")

HOST_PROGRAM = r"""
#include <cstdio>
#include <cstdint>
#include <cmath>
#include <random>
#include "unit_log.hpp"
using namespace swarm_impl;

static double ulp_err(double x, const double* tab) {
  const long double ref = logl(static_cast<long double>(x));
  const double got = unit_log(x, tab);
  if (ref == 0.0L) return got == 0.0 ? 0.0 : 1e9;
  int e;
  frexpl(ref, &e);
  const long double ulp = ldexpl(1.0L, e - 53);          // ulp of a double near ref
  return static_cast<double>(fabsl(static_cast<long double>(got) - ref) / ulp);
}

int main() {
  double tab[kUnitLogStride * kUnitLogEntries];
  unit_log_table(tab);
  printf("entry0 %.17g %.17g\n", tab[0], tab[1]);
  std::mt19937_64 g(12345);
  double worst = 0.0, worst_x = 1.0;
  const int n = 2000000;
  for (int k = 0; k < n; ++k) {
    const uint64_t v = g() >> 11;                          // 53-bit integer
    double u = ldexp(static_cast<double>(v), -53);
    if (k % 4 == 1) u = ldexp(u, -(int)(g() % 60));        // also short flights
    const double x = 1.0 - u;                              // exact
    if (!(x > 0.0)) continue;
    const double err = ulp_err(x, tab);
    if (err > worst) { worst = err; worst_x = x; }
  }
  printf("random %.4f %a\n", worst, worst_x);
  double ew = 0.0;
  const double edges[] = {1.0, 1.0 - 0x1p-53, 0x1p-53, 0.5, 0.5 + 0x1p-54, 0x1.fcp-1, 0x1.fcp-1 + 0x1p-53,
                          0x1.fcp-1 - 0x1p-53, 0.75, 0.25, 0x1p-20, 0.999, 0.001};
  for (double x : edges) ew = fmax(ew, ulp_err(x, tab));
  for (int i = 0; i < kUnitLogEntries; ++i)
    for (int ex = -53; ex <= -1; ++ex) {
      const double c = ldexp(1.0 + i / 64.0, ex);
      for (double x : {c, nextafter(c, 0.0), nextafter(c, 2.0)})
        if (x > 0.0 && x <= 1.0) ew = fmax(ew, ulp_err(x, tab));
    }
  printf("edges %.4f\n", ew);
  printf("zero %a\n", unit_log(1.0, tab));
  return 0;
}
"""


@pytest.fixture(scope="module")
def host_output(tmp_path_factory):
    d = tmp_path_factory.mktemp("unit_log")
    src = d / "drv.cpp"
    src.write_text(HOST_PROGRAM)
    exe = d / "drv"
    cmd = ["hipcc", "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", CSRC, str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    return {ln.split()[0]: ln.split()[1:] for ln in out.stdout.splitlines()}


def test_error_on_kernel_inputs_is_within_two_ulp(host_output):
    assert float(host_output["random"][0]) <= 2.0, host_output["random"]


def test_error_on_edge_values_is_within_two_ulp(host_output):
    assert float(host_output["edges"][0]) <= 2.0, host_output["edges"]


def test_table_and_exact_zero(host_output):
    assert [float(v) for v in host_output["entry0"]] == [1.0, 0.0]     # c_0 = 1: no table term
    assert float.fromhex(host_output["zero"][0]) == 0.0                 # ln 1 = 0 exactly
