"""The kernels' sine/cosine routines (csrc/ile_sincos.h), compiled for the
host and checked against long-double libm over 3M angles, including floats
up to 1e6 rad: the full FP64 series to a few ulp, the sky-direction series
to 1e-11 (delays of <= 90 window samples then move by < 1e-9 of a sample),
the FP32 series to about one FP32 ulp."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SRC = r'''
#include "ile_sincos.h"
#include <cstdio>
#include <cmath>
#include <random>
int main() {
  std::mt19937_64 g(2);
  double ws = 0, wsky = 0, wf = 0;
  std::uniform_real_distribution<double> u(-7, 7), v(-1e6, 1e6);
  for (int i = 0; i < 3000000; i++) {
    const double x = (i % 3 == 2) ? v(g) : u(g);
    const float xf = (float)x;
    const double xd = xf;
    const long double ls = sinl((long double)xd), lc = cosl((long double)xd);
    double s, c;
    ile::sincos_rad(xd, &s, &c);
    ws = fmax(ws, fmax(fabs((double)(s - ls)), fabs((double)(c - lc))));
    ile::sincos_rad_sky(xd, &s, &c);
    wsky = fmax(wsky, fmax(fabs((double)(s - ls)), fabs((double)(c - lc))));
    float sf, cf;
    ile::sincos_rad(xf, &sf, &cf);
    wf = fmax(wf, fmax(fabs((double)(sf - ls)), fabs((double)(cf - lc))));
  }
  double s, c;
  ile::sincos_rad(0.0, &s, &c);
  printf("%.6g %.6g %.6g %.17g %.17g\n", ws, wsky, wf, s, c);
  return 0;
}
'''


def test_sincos_accuracy(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "t.cpp"
    src.write_text(SRC)
    exe = tmp_path / "t"
    subprocess.check_call([hipcc, "-O2", "-I", os.path.join(ROOT, "paper_2505_11655_amd", "csrc"), str(src),
                           "-o", str(exe)], stderr=subprocess.DEVNULL)
    full, sky, f32, s0, c0 = (float(v) for v in subprocess.check_output([str(exe)]).split())
    assert full <= 3e-16, full
    assert sky <= 1e-11, sky
    assert f32 <= 1.5e-7, f32
    assert s0 == 0.0 and c0 == 1.0
