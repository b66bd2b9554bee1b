"""The host-side launch check (csrc/fstat_launch.hpp) on the CPU: a launch the queue
would reject (a zero or oversize grid or workgroup dimension, a workgroup above the
kernel's compiled maximum, more LDS than a workgroup may hold, a grid dimension over
2^32 - 1 work-items) is named, a valid one passes.  The header is plain C++, compiled
here with g++ into a small driver that reads one case per line."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1410_3677_amd", "csrc")

DRIVER = r"""
#include <iostream>
#include "fstat_launch.hpp"
int main() {
  fstat::DeviceLaunchLimits d;           // the limits a gfx950 reports
  d.max_threads_per_block = 1024;
  d.max_block[0] = d.max_block[1] = d.max_block[2] = 1024;
  d.max_grid[0] = 2147483647; d.max_grid[1] = 65536; d.max_grid[2] = 65536;
  d.max_lds_per_block = 163840;
  long long kmax, klds, g0, g1, g2, b0, b1, b2, dyn;
  while (std::cin >> kmax >> klds >> g0 >> g1 >> g2 >> b0 >> b1 >> b2 >> dyn) {
    fstat::KernelLaunchLimits k;
    k.max_threads_per_block = kmax;
    k.static_lds = klds;
    const int64_t g[3] = {g0, g1, g2}, b[3] = {b0, b1, b2};
    const std::string why = fstat::launch_problem(d, k, g, b, dyn);
    std::cout << (why.empty() ? "OK" : why) << "\n";
  }
}
"""

CASES = [
    # kernel max, static LDS, grid, block, dynamic LDS -> expected substring ("OK" = allowed)
    ((256, 0, 4096, 1, 1, 256, 1, 1, 0), "OK"),
    ((512, 39824, 4096, 1, 1, 512, 1, 1, 0), "OK"),                     # the scoring kernel today
    ((256, 77552, 4096, 1, 1, 256, 1, 1, 0), "OK"),                     # 75.7 KiB of LDS is allowed
    ((1024, 0, 1, 1, 1, 1024, 1, 1, 0), "OK"),
    ((256, 0, 0, 1, 1, 256, 1, 1, 0), "grid x dimension 0"),            # an empty grid
    ((256, 0, 16, 0, 1, 256, 1, 1, 0), "grid y dimension 0"),
    ((256, 0, 16, 1, 1, 0, 1, 1, 0), "workgroup x dimension 0"),
    ((256, 0, 16, 1, 1, 512, 1, 1, 0), "kernel's compiled maximum 256"),  # 512 threads on a 256 kernel
    ((1024, 0, 16, 1, 1, 2048, 1, 1, 0), "above the device's 1024"),
    ((1024, 0, 16, 1, 1, 64, 32, 1, 0), "2048 work-items per workgroup above the device's 1024"),
    ((256, 0, 16, 70000, 1, 256, 1, 1, 0), "grid y dimension 70000 above the device's 65536"),
    ((256, 0, 1 << 24, 1, 1, 256, 1, 1, 0), "exceeds 2^32 - 1"),          # 2^32 work-items along x
    ((256, 0, (1 << 24) - 1, 1, 1, 256, 1, 1, 0), "OK"),
    ((256, 100000, 16, 1, 1, 256, 1, 1, 65536), "bytes of LDS (100000 static + 65536 dynamic)"),
    ((256, 163840, 16, 1, 1, 256, 1, 1, 0), "OK"),
    ((256, 163840, 16, 1, 1, 256, 1, 1, 1), "above the 163840"),
]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("launch")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def test_launch_problems_are_named_and_valid_launches_pass(driver):
    inp = "\n".join(" ".join(str(v) for v in c) for c, _ in CASES) + "\n"
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout.splitlines()
    assert len(out) == len(CASES)
    for (case, want), got in zip(CASES, out):
        if want == "OK":
            assert got == "OK", (case, got)
        else:
            assert want in got, (case, got)
