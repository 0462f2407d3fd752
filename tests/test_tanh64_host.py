"""The FP64 tanh of the network activations (csrc/tanh64.h), built for the host.

The device code calls the same inline function; here hipcc compiles it into
a host program (no GPU needed) that is checked against numpy's tanh: at most
4 ulp on a dense grid over [-25, 25], on random points of every magnitude
down to 1e-300, and exact special values (signed zeros, saturation, NaN).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HARNESS = r"""
#include "tanh64.h"
#include <cstdio>
#include <vector>
int main(int argc, char **argv)
{
    FILE *f = std::fopen(argv[1], "rb");
    std::vector<double> x;
    double v;
    while (std::fread(&v, 8, 1, f) == 1) x.push_back(v);
    std::fclose(f);
    FILE *g = std::fopen(argv[2], "wb");
    for (double a : x) {
        double t = dp::tanh_f64(a);
        std::fwrite(&t, 8, 1, g);
    }
    std::fclose(g);
    return 0;
}
"""


@pytest.fixture(scope="module")
def tanh_host(tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("tanh64")
    src = d / "h.hip"
    src.write_text(HARNESS)
    exe = d / "h"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O2", "-I",
                           os.path.join(ROOT, "paper_2201_01446_amd", "csrc"), str(src), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)

    def run(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        xi, yo = d / "x.bin", d / "y.bin"
        x.tofile(xi)
        subprocess.check_call([str(exe), str(xi), str(yo)])
        return np.fromfile(yo)
    return run


def _ulp(y, ref):
    return np.abs(y - ref) / np.spacing(np.abs(ref))


def test_grid_and_random_within_4_ulp(tanh_host):
    rng = np.random.default_rng(7)
    x = np.concatenate([np.linspace(-25, 25, 200001),
                        rng.normal(size=100000) * 3,
                        np.exp(rng.uniform(-690, 3.5, 100000)) * rng.choice([-1, 1], 100000)])
    y = tanh_host(x)
    assert _ulp(y, np.tanh(x)).max() <= 4


def test_special_values(tanh_host):
    x = np.array([0.0, -0.0, 5e-324, -5e-324, 19.5, 20.0, -20.0, 1e300, np.inf, -np.inf, np.nan])
    y = tanh_host(x)
    assert y[0] == 0 and not np.signbit(y[0])
    assert y[1] == 0 and np.signbit(y[1])
    assert y[2] == 5e-324 and y[3] == -5e-324
    assert list(y[4:10]) == [1.0, 1.0, -1.0, 1.0, 1.0, -1.0]
    assert np.isnan(y[10])


def test_odd_symmetry(tanh_host):
    x = np.linspace(1e-6, 22, 50001)
    assert np.array_equal(tanh_host(-x), -tanh_host(x))
