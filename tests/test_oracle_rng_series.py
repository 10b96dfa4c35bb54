"""Pins of the oracle's random numbers and screening series against sources
other than the oracle itself: rocRAND's independent Philox4x32-10 engine,
scipy's special functions, closed forms, and distribution tests."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import special, stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _build_rocrand_ref(tmp_path_factory):
    src = os.path.join(HERE, "pins", "philox_rocrand.cpp")
    out = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    inc = "/opt/rocm/include"
    if shutil.which("g++") and os.path.isdir(os.path.join(inc, "rocrand")):
        r = subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + inc, src, "-o", out],
                           capture_output=True, text=True)
        if r.returncode == 0:
            return out
    if shutil.which("hipcc"):
        subprocess.run(["hipcc", "-x", "hip", "--cuda-host-only", "-O1", src, "-o", out],
                       check=True, capture_output=True)
        return out
    pytest.skip("no compiler for the rocRAND reference engine")


def test_philox_matches_rocrand_engine(oracle, tmp_path_factory):
    """Philox4x32-10 of the oracle equals rocRAND's header-only engine on
    random counters and keys (the two are written independently)."""
    exe = _build_rocrand_ref(tmp_path_factory)
    rng = np.random.default_rng(123)
    cases = []
    for _ in range(300):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] = c[1] % (1 << 30)  # keep the engine's 64-bit offset in range
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        cases.append([int(v) for v in c] + [int(v) for v in k])
    cases += [[0, 0, 0, 0, 0, 0], [5, 7, 11, 0, 0xDEADBEEF, 0xCAFEF00D], [0, 0, 0, 0, 0xFFFFFFFF, 0xFFFFFFFF]]
    inp = "\n".join(" ".join(f"{v:x}" for v in c) for c in cases) + "\n"
    r = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
    ref = [[int(t, 16) for t in line.split()] for line in r.stdout.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, want in zip(cases, ref):
        assert oracle.philox(c[:4], c[4:]) == want, c


def test_uniform_is_exact_open_interval(oracle):
    """Uniforms are odd multiples of 2^-24 strictly inside (0, 1), so they are
    exact in FP32 and FP64 alike."""
    for x in [0, 1, 511, 512, 2**31, 2**32 - 1, 0x12345678]:
        u = oracle.uniform(x)
        assert 0.0 < u < 1.0
        assert u == float(np.float32(u))
        m = u * 2**24
        assert m == int(m) and int(m) % 2 == 1
    assert oracle.uniform(0) == 2.0**-24
    assert oracle.uniform(2**32 - 1) == 1.0 - 2.0**-24


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7, 8])
def test_direction_is_uniform_on_sphere(oracle, d):
    """Unit norm, E[v] = 0, E[v v^T] = I/d, and the first coordinate follows
    the marginal of a uniform direction: (v_1 + 1)/2 ~ Beta((d-1)/2, (d-1)/2)."""
    n = 6000
    V = np.array([oracle.direction(d, 77, k % 5, k // 5, 3, 1) for k in range(n)])
    assert np.allclose((V ** 2).sum(1), 1.0, atol=1e-14)
    assert np.all(np.abs(V.mean(0)) < 5.0 / math.sqrt(n * d))
    M = V.T @ V / n
    assert np.allclose(M, np.eye(d) / d, atol=6.0 / math.sqrt(n) / d + 2e-3)
    a = (d - 1) / 2.0
    for i in range(d):
        p = stats.kstest((V[:, i] + 1) / 2, stats.beta(a, a).cdf).pvalue
        assert p > 1e-4, (d, i, p)


def test_direction_depends_on_every_counter_word(oracle):
    base = oracle.direction(5, 9, 3, 4, 5, 6)
    for args in [(5, 10, 3, 4, 5, 6), (5, 9, 4, 4, 5, 6), (5, 9, 3, 5, 5, 6), (5, 9, 3, 4, 6, 6),
                 (5, 9, 3, 4, 5, 7)]:
        assert not np.allclose(base, oracle.direction(*args))


@pytest.mark.parametrize("b", [1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0, 4.5, 5.0])
def test_hyp0f1_matches_scipy(oracle, b):
    for y in [0.0, 1e-8, 0.01, 0.3, 1.0, 4.9, 19.7, 60.0, 250.0]:
        want = special.hyp0f1(b, y)
        assert oracle.hyp0f1(b, y) == pytest.approx(want, rel=1e-13)


def _C_bessel(d, sigma, R):
    """Value at the centre of a ball of radius R of the solution of
    Laplacian(u) = sigma u with u = 1 on the sphere:
    (z/2)^nu / (Gamma(nu+1) I_nu(z)), z = sqrt(sigma) R, nu = d/2 - 1."""
    nu = d / 2.0 - 1.0
    z = math.sqrt(sigma) * R
    if z == 0:
        return 1.0
    return (z / 2.0) ** nu / (special.gamma(nu + 1.0) * special.iv(nu, z))


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7, 8])
def test_screening_weight_is_ball_centre_value(oracle, d):
    for sigma in [0.0, 0.5, 2.0, 8.0]:
        for R in [1e-3, 0.1, 0.5, 1.0, 2.0, math.pi]:
            assert oracle.screening_C(d, sigma, R) == pytest.approx(_C_bessel(d, sigma, R), rel=1e-12)


def test_screening_weight_closed_forms(oracle):
    for z in [1e-3, 0.3, 1.0, 2.5, 7.0]:
        # d = 3: z / sinh z; d = 5: z^3 / (3 (z cosh z - sinh z)); d = 2: 1 / I0(z)
        assert oracle.screening_C(3, 1.0, z) == pytest.approx(z / math.sinh(z), rel=1e-12)
        if z > 0.05:
            assert oracle.screening_C(5, 1.0, z) == pytest.approx(
                z ** 3 / (3 * (z * math.cosh(z) - math.sinh(z))), rel=1e-10)
        assert oracle.screening_C(2, 1.0, z) == pytest.approx(1.0 / special.i0(z), rel=1e-12)
        # first-sphere gradient factor: d = 3 uses I_{3/2}; C1(d) = C(d + 2)
        assert oracle.screening_C1(3, 1.0, z) == pytest.approx(oracle.screening_C(5, 1.0, z), rel=1e-14)
        assert oracle.screening_C1(2, 1.0, z) == pytest.approx(z / 2 / special.i1(z), rel=1e-12)
    assert oracle.screening_C(7, 0.0, 2.0) == 1.0 and oracle.screening_C1(7, 0.0, 2.0) == 1.0


@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_dlnC_dsigma_matches_derivative_of_bessel_form(oracle, d):
    for sigma in [0.0, 0.7, 2.0, 8.0]:
        for R in [0.05, 0.6, 1.7]:
            if sigma == 0.0:
                h = 1e-6  # one-sided difference of the Bessel form, O(h) accurate
                fd = math.log(_C_bessel(d, h, R)) / h
                want = -R * R / (2 * d)
                assert fd == pytest.approx(want, rel=1e-4)
                assert oracle.dlnC_dsigma(d, sigma, R) == pytest.approx(want, rel=1e-14)
            else:
                h = 1e-5
                fd = (math.log(_C_bessel(d, sigma + h, R)) - math.log(_C_bessel(d, sigma - h, R))) / (2 * h)
                assert oracle.dlnC_dsigma(d, sigma, R) == pytest.approx(fd, rel=1e-6, abs=1e-10)
