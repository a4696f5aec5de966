"""CPU checks of the library's own random-number and elementary-function code (the same
source as the GPU kernels, compiled for the host): Philox against its published
known-answer vectors, sin/cos(2 pi u) and log(u) against the host libm within a few ulp."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "mathcheck.cpp")
OUT = os.path.join(ROOT, "tests", "_build", "libmathcheck.so")
GOLD = os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")


@pytest.fixture(scope="module")
def mc():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    r = subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_1006_0532_amd", "csrc"), SRC, "-o", OUT],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("hipcc host build unavailable: " + r.stderr[-300:])
    return C.CDLL(OUT)


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def test_library_philox_known_answers(mc):
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        ctr = np.array(v[0:4], np.uint32)
        key = np.array(v[4:6], np.uint32)
        out = np.zeros(4, np.uint32)
        mc.mc_philox(_p(ctr, C.c_uint32), _p(key, C.c_uint32), _p(out, C.c_uint32))
        assert out.tolist() == v[6:10]


def _uniform_words(n, seed=3):
    rng = np.random.default_rng(seed)
    w = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    edge = np.array([0, 1, 2, 0x3FFFFFFF, 0x40000000, 0x7FFFFFFF, 0x80000000, 0xBFFFFFFF, 0xC0000000,
                     0xFFFFFFFE, 0xFFFFFFFF], np.uint32)
    return np.concatenate([edge, w])


def _ulp_err(got, ref):
    return np.abs(got - ref) / np.spacing(np.maximum(np.abs(ref), 1e-300))


def test_sincos_2pi_accuracy(mc):
    w = _uniform_words(400000)
    u = (w.astype(np.float64) + 0.5) * 2.0 ** -32
    s, c = np.empty_like(u), np.empty_like(u)
    mc.mc_sincos_2pi(_p(u, C.c_double), len(u), _p(s, C.c_double), _p(c, C.c_double))
    # reference in x87 extended precision with a 36-digit pi (the angle 2 pi u is exact there
    # to about 1e-19, unlike in double)
    pi_ld = np.longdouble("3.14159265358979323846264338327950288")
    ang = 2 * pi_ld * u.astype(np.longdouble)
    rs, rc = np.sin(ang).astype(np.float64), np.cos(ang).astype(np.float64)
    assert np.abs(s - rs).max() < 3e-16 and np.abs(c - rc).max() < 3e-16
    assert np.abs(s * s + c * c - 1).max() < 4e-16
    # quarter angles are exact
    for uu, es, ec in [(0.25, 1.0, 0.0), (0.5, 0.0, -1.0), (0.75, -1.0, 0.0), (0.0, 0.0, 1.0)]:
        a = np.array([uu]); s1 = np.empty(1); c1 = np.empty(1)
        mc.mc_sincos_2pi(_p(a, C.c_double), 1, _p(s1, C.c_double), _p(c1, C.c_double))
        assert abs(s1[0] - es) < 1e-16 and abs(c1[0] - ec) < 1e-16


def test_log_unit_accuracy(mc):
    w = _uniform_words(400000)
    u = (w.astype(np.float64) + 0.5) * 2.0 ** -32
    u = np.concatenate([u, [1.0, 0.5, 0.25, 2.0 ** -33, np.sqrt(0.5), np.nextafter(np.sqrt(0.5), 1)]])
    o = np.empty_like(u)
    mc.mc_log_unit(_p(u, C.c_double), len(u), _p(o, C.c_double))
    ref = np.log(u)
    err = _ulp_err(o, ref)
    assert err.max() <= 4, err.max()
    assert o[len(u) - 6] == 0.0


def test_box_muller_matches_textbook_form(mc):
    a = _uniform_words(100000, 5)
    b = _uniform_words(100000, 6)
    z = np.empty(2 * len(a))
    mc.mc_box_muller(_p(a, C.c_uint32), _p(b, C.c_uint32), len(a), _p(z, C.c_double))
    u1 = (a.astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (b.astype(np.float64) + 0.5) * 2.0 ** -32
    r = np.sqrt(-2 * np.log(u1))
    ref = np.stack([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)], 1).ravel()
    assert np.abs(z - ref).max() < 1e-14 * max(1.0, np.abs(ref).max())
