"""The library's construction of the physics-based interface functions
(`csrc/physics_space.h`, plain C++ run at set-up) against the oracle's
(section 3.1, eqs. (new_basis1)-(new_basis6)), on the CPU: the header is
compiled with g++ into a small driver that reads face conductances and
prints the functions of the slots.

Both sides classify the faces against the same median and evaluate the
same closed forms; the values agree to rounding (the ramps are formed with
the same operations in the same order) and the slot counts exactly.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.discretization import physics_space

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2104_04653_amd", "csrc")

DRIVER = r'''
#include <cstdio>
#include <vector>
#include "physics_space.h"
int main() {
  int n_case, M;
  if (std::scanf("%d", &n_case) != 1) return 1;
  for (int c = 0; c < n_case; ++c) {
    if (std::scanf("%d", &M) != 1) return 1;
    std::vector<double> t(M);
    for (int j = 0; j < M; ++j) if (std::scanf("%lf", &t[j]) != 1) return 1;
    std::vector<double> out((mrcm::phys::PHYS_P + mrcm::phys::PHYS_U) * M, 0.0);
    int np_ = 0, nu = 0;
    mrcm::phys::physics_space(t, out.data(), M, np_, nu);
    std::printf("%d %d\n", np_, nu);
    for (double v : out) std::printf("%.17g\n", v);
  }
  return 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("phys")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", HDR, str(src), "-o", str(exe)], check=True)
    return exe


def run_driver(exe, cases):
    text = "%d\n" % len(cases) + "".join(
        "%d %s\n" % (t.size, " ".join(repr(float(v)) for v in t)) for t in cases)
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout.split()
    res, q = [], 0
    for t in cases:
        m = t.size
        n_p, n_u = int(out[q]), int(out[q + 1])
        q += 2
        vals = np.array([float(v) for v in out[q:q + 8 * m]]).reshape(8, m)
        q += 8 * m
        res.append((n_p, n_u, vals))
    return res


def random_conductances(rng, m):
    """Background of one scale with channels and barriers of random widths."""
    t = np.exp(rng.uniform(-0.5, 0.5, m))
    for _ in range(rng.integers(0, 4)):
        j0 = int(rng.integers(0, m))
        w = int(rng.integers(1, 6))
        t[j0:j0 + w] *= 10.0 ** rng.choice([-3, -2, 2, 4])
    return t


def test_library_functions_match_the_oracle(driver):
    rng = np.random.default_rng(7)
    cases = [random_conductances(rng, int(rng.choice([8, 16, 32]))) for _ in range(300)]
    # cases with a structure touching an end, and none at all
    t = np.ones(16)
    t[:4] = 1e4
    cases.append(t)
    t = np.ones(16)
    t[12:] = 1e-3
    cases.append(t)
    cases.append(np.full(32, 3.0))
    n_struct = 0
    for t, (n_p, n_u, vals) in zip(cases, run_driver(driver, cases)):
        ps, us = physics_space(t)
        assert (n_p, n_u) == (ps.shape[0], us.shape[0])
        assert np.allclose(vals[:n_p], ps, rtol=0, atol=1e-15)
        assert np.allclose(vals[4:4 + n_u], us, rtol=0, atol=1e-15)
        assert not vals[n_p:4].any() and not vals[4 + n_u:].any()
        n_struct += (n_p > 2) or (n_u > 2)
    assert n_struct > 100          # the random cases exercise the structures
