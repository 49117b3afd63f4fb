"""The register DFTs of the HIP passes (csrc/dft_regs.hpp), compiled for the host with g++ and
checked against the DFT's definition summed in long double (the transforms of the split-step
method, Sec. II.C Eq. (evoloperat) and Appendix A, are built from these blocks).  The header is
included as it is; a small stand-in for <hip/hip_runtime.h> supplies double2, make_double2 and
the host-side qualifiers.  CPU only: this runs no GPU code."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1903_02581_amd", "csrc", "dft_regs.hpp")

SHIM = r"""
#pragma once
#include <cmath>
#define __device__
#define __host__
#define __forceinline__ inline
struct double2 { double x, y; };
inline double2 make_double2(double a, double b) { return {a, b}; }
using std::fma;
"""

DRIVER = r"""
#include "HEADER"
#include <complex>
#include <cstdio>
#include <random>
using namespace hom4d_dev;
typedef std::complex<long double> cl;
static const long double kPi = 3.14159265358979323846264338327950288L;
// largest |dft<R, DIR>(v) - sum_n v[n] exp(DIR 2 pi i n k / R)| over 200 random vectors, and
// largest |dft<R, +1>(dft<R, -1>(v)) - R v|
template <int R, int DIR> void check(std::mt19937_64& g) {
    std::normal_distribution<double> nd;
    double err = 0.0, inv = 0.0;
    for (int rep = 0; rep < 200; ++rep) {
        double2 v[R], w[R];
        for (int i = 0; i < R; ++i) v[i] = w[i] = make_double2(nd(g), nd(g));
        dft<R, DIR>(v);
        for (int k = 0; k < R; ++k) {
            cl acc = 0;
            for (int n = 0; n < R; ++n)
                acc += cl(w[n].x, w[n].y) * std::polar<long double>(1.0L, DIR * 2.0L * kPi * ((n * k) % R) / R);
            err = std::max(err, (double)std::abs(cl(v[k].x, v[k].y) - acc));
        }
        dft<R, -DIR>(v);
        for (int k = 0; k < R; ++k)
            inv = std::max(inv, std::hypot(v[k].x - R * w[k].x, v[k].y - R * w[k].y));
    }
    std::printf("%d %d %.3e %.3e\n", R, DIR, err, inv);
}
int main() {
    std::mt19937_64 g(20260501);
#define BOTH(R) check<R, -1>(g); check<R, 1>(g);
    BOTH(1) BOTH(2) BOTH(3) BOTH(4) BOTH(6) BOTH(8) BOTH(12) BOTH(16) BOTH(24)
    return 0;
}
"""


@pytest.fixture(scope="module")
def dft_errors(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    d = tmp_path_factory.mktemp("dftcpu")
    os.makedirs(d / "hip")
    (d / "hip" / "hip_runtime.h").write_text(SHIM)
    (d / "t.cpp").write_text(DRIVER.replace("HEADER", HEADER))
    exe = d / "t"
    res = subprocess.run([gxx, "-O2", "-std=c++17", "-I", str(d), str(d / "t.cpp"), "-o", str(exe)],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    rows = {}
    for line in out.split("\n"):
        if line.strip():
            r, sign, err, inv = line.split()
            rows[(int(r), int(sign))] = (float(err), float(inv))
    return rows


@pytest.mark.parametrize("r", [1, 2, 3, 4, 6, 8, 12, 16, 24])
@pytest.mark.parametrize("sign", [-1, 1])
def test_register_dft_matches_definition(dft_errors, r, sign):
    err, inv = dft_errors[(r, sign)]
    # unit-variance complex inputs: entries of size ~sqrt(R); rounding of a few ulps per stage
    assert err <= 2e-15 * r, (r, sign, err)
    # the two directions are inverse up to the factor R
    assert inv <= 4e-15 * r * r, (r, sign, inv)
