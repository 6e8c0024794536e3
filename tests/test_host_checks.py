"""Host-side argument checks (csrc/host_checks.h), compiled with g++ and compared with
brute force: a batched view {base + i*stride + [0, n)} overlaps another exactly when
some byte belongs to both."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2402_16683_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "host_checks.h"
int main(int argc, char** argv) {
  // each input line: sa na sb nb batch d -> prints 0/1
  long long sa, na, sb, nb, batch, d;
  static char buf[1 << 16];
  while (std::scanf("%lld %lld %lld %lld %lld %lld", &sa, &na, &sb, &nb, &batch, &d) == 6) {
    const char* a = buf + 20000;
    const char* b = a + d;
    std::printf("%d\n", icr::overlaps_batched(a, sa, na, b, sb, nb, batch) ? 1 : 0);
  }
  return 0;
}
"""


def brute(sa, na, sb, nb, batch, d):
    A = {i * sa + k for i in range(batch) for k in range(na)}
    return any((d + j * sb + k) in A for j in range(batch) for k in range(nb))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("hc")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", f"-I{HDR}", str(src), "-o", str(exe)], check=True)
    return str(exe)


def _run(exe, cases):
    inp = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split()
    return [o == "1" for o in out]


def test_equal_strides_are_exact(driver):
    rng = np.random.default_rng(0)
    cases = []
    for _ in range(3000):
        s = int(rng.integers(1, 40))
        na, nb = int(rng.integers(0, s + 1)), int(rng.integers(0, s + 1))
        batch = int(rng.integers(0, 7))
        d = int(rng.integers(-6 * s, 6 * s))
        cases.append((s, na, s, nb, batch, d))
    got = _run(driver, cases)
    for c, g in zip(cases, got):
        assert g == brute(*c), c


def test_other_layouts_never_miss_an_overlap(driver):
    # unequal strides or rows longer than the stride: conservative, never a false "disjoint"
    rng = np.random.default_rng(1)
    cases = []
    for _ in range(3000):
        sa, sb = int(rng.integers(1, 30)), int(rng.integers(1, 30))
        na, nb = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        batch = int(rng.integers(0, 6))
        d = int(rng.integers(-150, 150))
        cases.append((sa, na, sb, nb, batch, d))
    got = _run(driver, cases)
    for c, g in zip(cases, got):
        if brute(*c):
            assert g, c


def test_interleaved_level_slices_are_accepted(driver):
    # two consecutive per-level slices of one [batch][W] workspace (element size 4)
    W, lo, mid, hi = 1000, 100, 400, 900
    c = (4 * W, 4 * (mid - lo), 4 * W, 4 * (hi - mid), 16, 4 * (mid - lo))
    assert _run(driver, [c]) == [False]
    c2 = (4 * W, 4 * (mid - lo) + 4, 4 * W, 4 * (hi - mid), 16, 4 * (mid - lo))  # one element shared
    assert _run(driver, [c2]) == [True]
