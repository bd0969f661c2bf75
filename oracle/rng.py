"""Counter-based disturbance sampling for the SMPC plan step (oracle, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Algorithm 1's sampling step draws eps_k^(m) ~ D; the paper only asks for a
zero-mean distribution.  When the plan step samples on the device, both sides
implement this one generator from its published definitions:

* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): 128-bit counter (c0..c3), 64-bit key (k0, k1), ten rounds
  of two 32x32->64-bit multiplications (constants 0xD2511F53, 0xCD9E8D57) with
  xor-mixing, the key bumped by the Weyl constants 0x9E3779B9, 0xBB67AE85
  between rounds;
* key = (seed mod 2^32, seed >> 32); the draw for rollout m, step k uses the
  counters n = 2 (m H + k) + b, b in {0, 1}, as (n mod 2^32, n >> 32, 0, 0);
* uniforms u = ((w >> 9) + 1/2) 2^-23 in (0, 1) from each 32-bit word w (every
  value, 2^-24 .. 1 - 2^-24, is exact in float32);
* Box-Muller: (u_a, u_b) -> sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b); the
  words of counter b = 0 give normals for joints 0..3, those of b = 1 joints 4..6
  (the last normal is unused);
* eps_j = sigma_j z_j.

Integer work is exact (Python ints); the transform is float64.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """Ten Philox rounds on one 4-word counter with a 2-word key; returns 4 words."""
    c0, c1, c2, c3 = (int(x) & MASK for x in counter)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox4x32_10_np(c0, c1, c2, c3, k0, k1):
    """The same rounds on arrays of counters (uint64 arrays holding 32-bit words)."""
    m32 = np.uint64(MASK)
    c0, c1, c2, c3 = (np.asarray(x, np.uint64) & m32 for x in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & MASK)
    k1 = np.uint64(int(k1) & MASK)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & m32
            k1 = (k1 + np.uint64(W1)) & m32
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m32
        hi1, lo1 = p1 >> np.uint64(32), p1 & m32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def philox_words(seed: int, n: int):
    """The 4 words of counter index n under the key taken from `seed`."""
    return philox4x32_10((n & MASK, (n >> 32) & MASK, 0, 0), (seed & MASK, (seed >> 32) & MASK))


def uniform23(words) -> np.ndarray:
    """u = ((w >> 9) + 1/2) * 2^-23 for each 32-bit word (exactly representable in float32)."""
    w = np.asarray(words, dtype=np.uint64)
    return ((w >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(ua, ub):
    r = np.sqrt(-2.0 * np.log(ua))
    t = 2.0 * np.pi * ub
    return r * np.cos(t), r * np.sin(t)


def step_normals(seed: int, m: int, k: int, H: int) -> np.ndarray:
    """Seven standard normals of rollout m, step k (float64)."""
    z = []
    for b in (0, 1):
        u = uniform23(philox_words(seed, 2 * (m * H + k) + b))
        za, zb = box_muller(u[0], u[1])
        zc, zd = box_muller(u[2], u[3])
        z.extend([za, zb, zc, zd])
    return np.array(z[:7])


def sample_noise(seed: int, K: int, H: int, sigma) -> np.ndarray:
    """eps [K][H][7] = sigma * z for the plan step's on-device sampling (float64)."""
    sigma = np.broadcast_to(np.asarray(sigma, np.float64), (7,))
    item = np.arange(K * H, dtype=np.uint64)
    z = []
    for b in (0, 1):
        n = np.uint64(2) * item + np.uint64(b)
        w = philox4x32_10_np(n & np.uint64(MASK), n >> np.uint64(32), 0 * n, 0 * n,
                             seed & MASK, (seed >> 32) & MASK)
        u = [uniform23(x) for x in w]
        za, zb = box_muller(u[0], u[1])
        zc, zd = box_muller(u[2], u[3])
        z.extend([za, zb, zc, zd])
    return (np.stack(z[:7], axis=-1) * sigma).reshape(K, H, 7)
