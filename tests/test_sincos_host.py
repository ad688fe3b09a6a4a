"""The double pendulum kernels' sin/cos (sincos_cw in systems_dp.h, a
Cody-Waite reduction and Taylor polynomials written for the stage loop's
register budget), compiled for the host from the same header and checked
against 50-digit values: within 1 ulp for ordinary arguments up to 1e9,
an absolute error below 1e-30 next to multiples of pi/2, NaN from 2^32 on
and for non-finite arguments."""
import math
import os
import shutil
import subprocess

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = r'''
#include <hip/hip_runtime.h>
#include "systems_dp.h"
#include <cstdio>
int main() {
  int n;
  if (scanf("%d", &n) != 1) return 1;
  for (int i = 0; i < n; ++i) {
    double x, s, c;
    if (scanf("%la", &x) != 1) return 1;
    chx::sincos_cw(x, s, c);
    printf("%a %a\n", s, c);
  }
  return 0;
}
'''


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("sincos")
    src = d / "t.hip"
    src.write_text(SRC)
    out = d / "t"
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950",
                    "-I", os.path.join(ROOT, "paper_2507_00622_amd", "csrc"),
                    str(src), "-o", str(out)], check=True, capture_output=True)
    return str(out)


def run(exe, xs):
    inp = "%d\n" % len(xs) + "\n".join(float(x).hex() for x in xs)
    lines = subprocess.run([exe], input=inp, capture_output=True, text=True,
                           check=True).stdout.split("\n")
    return [tuple(float.fromhex(t) for t in l.split()) for l in lines[:len(xs)]]


def ulp(v):
    return mp.mpf(2) ** (mp.floor(mp.log(abs(v), 2)) - 52)


def test_ordinary_arguments_within_one_ulp(exe):
    mp.mp.dps = 50
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(-10, 10, 1500), rng.uniform(-1e4, 1e4, 800),
                         rng.uniform(-1e9, 1e9, 500), [0.25, -math.pi / 4, math.pi / 4, 1e-8]])
    worst = 0.0
    for x, (s, c) in zip(xs, run(exe, xs)):
        S, C = mp.sin(x), mp.cos(x)
        worst = max(worst, float(abs(mp.mpf(s) - S) / ulp(S)), float(abs(mp.mpf(c) - C) / ulp(C)))
    assert worst < 1.0


def test_near_multiples_of_half_pi(exe):
    mp.mp.dps = 60
    ks = list(range(-64, 65)) + [10 ** 5 + 1, 3 * 10 ** 6 + 7, 123456789]
    xs = [float(mp.mpf(k) * mp.pi / 2) for k in ks]
    for x, (s, c) in zip(xs, run(exe, xs)):
        assert abs(mp.mpf(s) - mp.sin(x)) < 1e-30 or abs(mp.mpf(s) - mp.sin(x)) <= ulp(mp.sin(x))
        assert abs(mp.mpf(c) - mp.cos(x)) < 1e-30 or abs(mp.mpf(c) - mp.cos(x)) <= ulp(mp.cos(x))


def test_signed_zero_tiny_and_out_of_range(exe):
    res = run(exe, [0.0, -0.0, 5e-324, 2.0 ** 32, -2.0 ** 40, float("inf"), float("nan")])
    assert res[0] == (0.0, 1.0) and math.copysign(1, res[0][0]) == 1
    assert res[1][1] == 1.0 and res[1][0] == 0.0
    assert res[2] == (5e-324, 1.0)
    for s, c in res[3:]:
        assert math.isnan(s) and math.isnan(c)
