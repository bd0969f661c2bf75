"""Pins of the oracle's counter-based sampler (Philox4x32-10 + Box-Muller).

The raw words are checked bit for bit against rocRAND's header-only Philox4x32-10
engine (an independent implementation of the same published generator, compiled
here for the host); the round function is checked to be a bijection; the
uniform and normal transforms are checked against their definitions' moments.
"""
import os
import subprocess

import numpy as np
import pytest

from oracle import rng

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = [(0, 0), (0, 1), (1, 0), (123456789, 42), (2**32 + 7, 2**32 + 3), (2**64 - 1, 2**40),
         (99, 2 * (17 * 40 + 5) + 1), (4, 2**33 - 1)]


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    header = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include", "rocrand",
                          "rocrand_philox4x32_10.h")
    if not (os.path.exists(hipcc) and os.path.exists(header)):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = tmp_path_factory.mktemp("probe") / "philox_probe"
    # Host-only build of a host-only program (no device code).
    inc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")
    subprocess.run([hipcc, "-O1", "-x", "c++", "-D__HIP_PLATFORM_AMD__", f"-I{inc}",
                    os.path.join(HERE, "rocrand_philox_probe.cpp"), "-o", str(exe)], check=True,
                   capture_output=True)
    return str(exe)


def test_philox_words_match_rocrand(rocrand_probe):
    inp = "".join(f"{s} {n}\n" for s, n in CASES)
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True)
    got = [tuple(int(x) for x in line.split()) for line in out.stdout.strip().splitlines()]
    for (s, n), words in zip(CASES, got):
        assert rng.philox_words(s, n) == words, (s, n)


def test_vectorised_rounds_equal_scalar_rounds():
    n = np.array([0, 1, 2**32 - 1, 2**32, 12345678901], dtype=np.uint64)
    seed = 2**40 + 17
    w = rng.philox4x32_10_np(n & np.uint64(0xFFFFFFFF), n >> np.uint64(32), 0 * n, 0 * n,
                             seed & 0xFFFFFFFF, seed >> 32)
    for i, ni in enumerate(n.tolist()):
        assert tuple(int(x[i]) for x in w) == rng.philox_words(seed, ni)


def test_philox_round_is_a_bijection_on_small_counters():
    """Distinct counters give distinct outputs (the rounds are invertible)."""
    outs = {rng.philox_words(7, n) for n in range(4096)}
    assert len(outs) == 4096


def test_uniforms_are_exact_float32_in_open_interval():
    u = rng.uniform23([0, 511, 512, 0xFFFFFFFF])
    assert u[0] == 2.0 ** -24 and u[1] == u[0]
    assert u[2] == 3 * 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24
    np.testing.assert_array_equal(u.astype(np.float32).astype(np.float64), u)


def test_box_muller_on_hand_values():
    za, zb = rng.box_muller(np.exp(-0.5), 0.25)      # r = 1, angle pi/2
    assert za == pytest.approx(0.0, abs=1e-15) and zb == pytest.approx(1.0, rel=1e-15)
    za, zb = rng.box_muller(np.exp(-2.0), 0.0)        # r = 2, angle 0
    assert za == pytest.approx(2.0, rel=1e-15) and zb == 0.0


def test_noise_moments_and_layout():
    K, H = 512, 16
    sigma = np.array([0.5, 0.5, 0.5, 0.25, 0.5, 1.0, 0.5])
    eps = rng.sample_noise(11, K, H, sigma)
    assert eps.shape == (K, H, 7)
    z = eps / sigma
    n = K * H
    assert abs(z.mean()) < 5 / np.sqrt(7 * n)
    np.testing.assert_allclose(z.reshape(-1, 7).var(axis=0), 1.0, atol=6 * np.sqrt(2 / n))
    # Joints are uncorrelated.
    c = np.corrcoef(z.reshape(-1, 7).T)
    assert np.max(np.abs(c - np.eye(7))) < 6 / np.sqrt(n)
    # Element (m, k) comes from counters 2(mH + k) and 2(mH + k) + 1.
    for m, k in ((0, 0), (3, 7), (K - 1, H - 1)):
        np.testing.assert_allclose(eps[m, k], sigma * rng.step_normals(11, m, k, H), rtol=1e-15)
    # Different seeds give different streams.
    assert not np.allclose(rng.sample_noise(12, 4, 4, 0.5), rng.sample_noise(11, 4, 4, 0.5))
