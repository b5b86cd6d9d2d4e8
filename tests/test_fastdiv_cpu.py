"""The kernels' division by run-time sizes (csrc/fastdiv.hpp: multiply-high and
shifts) against the hardware division, on the host: every divisor up to 4096
with the dividends 0..69,999 and the 5,000 largest 32-bit values, and the
network's sizes (channels, image sides, 3x3 taps times channels) plus large
divisors with 2 million pseudo-random dividends each."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SRC = r"""
#include "fastdiv.hpp"
#include <cstdio>
int main() {
  long bad = 0, n_checked = 0;
  const uint32_t ds[] = {1, 2, 3, 5, 7, 8, 9, 24, 32, 48, 64, 96, 128, 192, 256, 288, 384, 512, 1000, 1152,
                         2304, 4095, 65535, 65536, 1u << 20, (1u << 31) - 1, 12345679};
  for (uint32_t d = 1; d <= 4096; ++d) {
    const pat::FastDiv f = pat::make_fastdiv(d);
    for (uint32_t n = 0; n < 70000; ++n, ++n_checked) bad += pat::fast_div(n, f) != n / d;
    for (uint64_t n = 0xFFFFFFFFull; n > 0xFFFFFFFFull - 5000; --n, ++n_checked)
      bad += pat::fast_div((uint32_t)n, f) != (uint32_t)n / d;
  }
  uint32_t x = 12345;
  for (uint32_t d : ds) {
    const pat::FastDiv f = pat::make_fastdiv(d);
    for (int i = 0; i < 2000000; ++i, ++n_checked) {
      x = x * 1664525u + 1013904223u;
      uint32_t q, r;
      pat::fast_divmod(x, f, q, r);
      bad += q != x / d || r != x % d;
    }
  }
  const pat::FastDiv z = pat::make_fastdiv(0);  // an unused size: taken as 1
  bad += pat::fast_div(77, z) != 77;
  printf("%ld of %ld wrong\n", bad, n_checked);
  return bad != 0;
}
"""


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not found")
def test_fast_division_is_exact(tmp_path):
    src = tmp_path / "fastdiv_check.cpp"
    src.write_text(SRC)
    exe = tmp_path / "fastdiv_check"
    r = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2",
                        f"-I{os.path.join(ROOT, 'paper_1707_02245_amd', 'csrc')}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("0 of ")
