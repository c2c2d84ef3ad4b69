"""Random objects of the estimator, defined once for the oracle side.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes only the distributions:

* CountSketch (Section 3.4, "CountSketch" paragraph, and the OSE theorem cited
  there): S in R^{r x n} has exactly one nonzero per column, at row h(i), with
  value s_i = +-1; h must be 2-wise independent and the signs 4-wise
  independent.
* Gaussian embeddings (Section 3.4, "Gaussian embeddings"): S = G / sqrt(r)
  with G i.i.d. N(0,1).  Algorithm 3 applies G (m x r) to SA; Algorithm 8
  applies a JL Gaussian Pi_2 to R^{-1}.

Which concrete generators realise those distributions is left open, so this
module fixes one reading (each written from its published definition, no
code shared with the GPU library, which implements the same definitions on
its own):

* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) expands the user seed into
  the words w0, w1, ... that parameterise everything below.
* Bucket hash: the Carter-Wegman family h(i) = ((a*i + c) mod P) mod r with
  P the smallest prime >= max(n, 2), a in [1, P-1], c in [0, P-1].  For
  i != j in [0, n) the pair ((a*i+c) mod P, (a*j+c) mod P) is uniform over
  distinct pairs, so h is pairwise independent up to the rounding of
  "mod r" (relative error O(r/P)).
* Sign: s(i) = +1 if g(i) is even else -1, with g a uniformly random cubic
  polynomial over GF(p61), p61 = 2^61 - 1 (4-wise independent values).
* Gaussians: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011), counter =
  floor(e / 2) for the row-major element index e, key = a SplitMix64 word;
  two 53-bit uniforms per counter; Box-Muller in FP64, cosine branch for
  even e and sine branch for odd e.
* SRHT (Section 3.4, "SRHT"): F = sqrt(r / t) P H D with D = diag(+-1),
  H the r x r Walsh-Hadamard matrix scaled by 1 / sqrt(r) and P a uniform
  sample of t of the r coordinates.  The sign of coordinate j is the top
  bit of the SplitMix64 finaliser of key_d + j * gamma; the sample takes
  coordinates pi(0), ..., pi(t - 1) of a keyed permutation pi of [0, r): a
  four-round Feistel network (Luby-Rackoff) on 2h-bit words, h = max(1,
  ceil(log2(r) / 2)), round functions from the finaliser of key_p + (round
  * 2^32 + half) * gamma, walked along its cycle until the value is < r
  (Black-Rogaway cycle walking), so pi is a bijection of [0, r).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

MASK64 = (1 << 64) - 1
MASK32 = (1 << 32) - 1
P61 = (1 << 61) - 1


# --------------------------------------------------------------------------
# SplitMix64 (Steele, Lea, Flood 2014): state += golden gamma, then a
# variant-13 finaliser of the new state.
# --------------------------------------------------------------------------
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    """The SplitMix64 output finaliser (variant 13) of a 64-bit word."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_words(seed: int, count: int) -> list[int]:
    """The first ``count`` outputs of SplitMix64 started from ``seed``."""
    state = seed & MASK64
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        z = z ^ (z >> 31)
        out.append(z)
    return out


def is_prime(x: int) -> bool:
    """Trial division; fine for x < 2^32."""
    if x < 2:
        return False
    if x % 2 == 0:
        return x == 2
    f = 3
    while f * f <= x:
        if x % f == 0:
            return False
        f += 2
    return True


def next_prime(x: int) -> int:
    """Smallest prime >= x."""
    p = max(2, x)
    while not is_prime(p):
        p += 1
    return p


@dataclass(frozen=True)
class SketchRandomness:
    """Everything the estimator draws, derived from one 64-bit seed."""

    seed: int
    n: int
    r_cs: int
    P: int          # prime modulus of the bucket hash, P >= n
    a: int          # bucket hash multiplier, 1 <= a <= P-1
    c: int          # bucket hash offset, 0 <= c <= P-1
    sign_coef: tuple  # (c0, c1, c2, c3) in GF(p61)
    key_m: tuple    # Philox key (k0, k1) of the Gaussian transform G_m
    key_k: tuple    # Philox key (k0, k1) of the JL Gaussian G_k
    key_d: int      # SRHT signs D
    key_p: int      # SRHT coordinate sample P


def derive(seed: int, n: int, r_cs: int) -> SketchRandomness:
    w = splitmix64_words(seed, 10)
    P = next_prime(max(n, 2))
    a = 1 + (w[0] % (P - 1))
    c = w[1] % P
    coef = tuple(w[2 + t] % P61 for t in range(4))
    key_m = (w[6] & MASK32, w[6] >> 32)
    key_k = (w[7] & MASK32, w[7] >> 32)
    return SketchRandomness(seed, n, r_cs, P, a, c, coef, key_m, key_k, w[8], w[9])


# --------------------------------------------------------------------------
# SRHT signs and coordinate sample
# --------------------------------------------------------------------------
def srht_sign(rnd: SketchRandomness, j: int) -> int:
    """D_jj = +1 when the top bit of mix64(key_d + j * gamma) is clear."""
    return -1 if mix64(rnd.key_d + j * GOLDEN_GAMMA) >> 63 else 1


def _feistel_half_bits(r: int) -> int:
    k = max(0, (r - 1).bit_length())  # r = 2^k
    return max(1, (k + 1) // 2)


def _feistel(rnd: SketchRandomness, x: int, h: int) -> int:
    mask = (1 << h) - 1
    left, right = x >> h, x & mask
    for t in range(4):
        f = mix64(rnd.key_p + ((t << 32) + right) * GOLDEN_GAMMA) & mask
        left, right = right, left ^ f
    return (left << h) | right


def srht_coordinate(rnd: SketchRandomness, r: int, j: int) -> int:
    """pi(j) for 0 <= j < r: the Feistel permutation of [0, 2^{2h}) walked
    along its cycle until it lands in [0, r)."""
    h = _feistel_half_bits(r)
    y = _feistel(rnd, j, h)
    while y >= r:
        y = _feistel(rnd, y, h)
    return y


# --------------------------------------------------------------------------
# CountSketch hash and signs
# --------------------------------------------------------------------------
def bucket_of(rnd: SketchRandomness, i: int) -> int:
    """h(i) = ((a*i + c) mod P) mod r_cs, by definition (Python ints)."""
    return ((rnd.a * i + rnd.c) % rnd.P) % rnd.r_cs


def sign_of(rnd: SketchRandomness, i: int) -> int:
    """s(i) = +1 if g(i) = c3 i^3 + c2 i^2 + c1 i + c0 (mod p61) is even."""
    c0, c1, c2, c3 = rnd.sign_coef
    g = (c3 * i ** 3 + c2 * i ** 2 + c1 * i + c0) % P61
    return 1 if g % 2 == 0 else -1


def buckets(rnd: SketchRandomness) -> np.ndarray:
    """h(i) for every row, vectorised.  a*i + c < 2^32 * 2^31 + 2^32 < 2^64."""
    i = np.arange(rnd.n, dtype=np.uint64)
    x = (np.uint64(rnd.a) * i + np.uint64(rnd.c)) % np.uint64(rnd.P)
    return (x % np.uint64(rnd.r_cs)).astype(np.int64)


def signs(rnd: SketchRandomness) -> np.ndarray:
    """s(i) for every row as float64 +-1 (vectorised Horner over GF(p61))."""
    c0, c1, c2, c3 = rnd.sign_coef
    i = np.arange(rnd.n, dtype=np.uint64)  # i < 2^31 < p61
    g = np.full(rnd.n, c3, dtype=np.uint64)
    for coef in (c2, c1, c0):
        g = (_mulmod_p61_vec(g, i) + np.uint64(coef)) % np.uint64(P61)
    return np.where(g % np.uint64(2) == 0, 1.0, -1.0)


def _mulmod_p61_vec(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Elementwise (x * y) mod p61 for uint64 arrays, y < 2^32."""
    x = x.astype(np.uint64)
    y = y.astype(np.uint64)
    x0, x1 = x & np.uint64(MASK32), x >> np.uint64(32)   # x1 < 2^29
    p = np.uint64(P61)
    hi = x1 * y                                          # < 2^61; weight 2^32
    lo = x0 * y                                          # < 2^64; weight 1
    hi_part = (hi >> np.uint64(29)) + ((hi & np.uint64((1 << 29) - 1)) << np.uint64(32))
    lo_part = (lo & p) + (lo >> np.uint64(61))
    return ((hi_part % p) + (lo_part % p)) % p


def countsketch_matrix_entries(rnd: SketchRandomness):
    """(rows, cols, vals) of S: S[h(i), i] = s(i) (Section 3.4)."""
    return buckets(rnd), np.arange(rnd.n, dtype=np.int64), signs(rnd)


# --------------------------------------------------------------------------
# Philox4x32-10 and Box-Muller
# --------------------------------------------------------------------------
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on uint32 numpy arrays.

    ``ctr`` is a tuple of four uint32 arrays, ``key`` a pair of ints.  One
    round multiplies words 0 and 2 by the two Philox constants (full 64-bit
    products), and outputs (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^
    k1, lo(M0*x0)); the key is advanced by the Weyl constants between rounds.
    """
    x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) & np.uint64(MASK32) for v in ctr)
    k0, k1 = key[0] & MASK32, key[1] & MASK32
    m32 = np.uint64(MASK32)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = np.uint64(PHILOX_M0) * x0
        p1 = np.uint64(PHILOX_M1) * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m32
        hi1, lo1 = p1 >> np.uint64(32), p1 & m32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0)
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def gaussian_matrix(key, rows: int, cols: int, scale: float = 1.0) -> np.ndarray:
    """rows x cols matrix of N(0,1) * scale in FP64, row-major index e."""
    total = rows * cols
    e = np.arange(total, dtype=np.uint64)
    q = e >> np.uint64(1)
    zero = np.zeros_like(q)
    x0, x1, x2, x3 = philox4x32_10((q & np.uint64(MASK32), q >> np.uint64(32), zero, zero), key)
    u53a = (x0.astype(np.uint64) << np.uint64(21)) | (x1.astype(np.uint64) >> np.uint64(11))
    u53b = (x2.astype(np.uint64) << np.uint64(21)) | (x3.astype(np.uint64) >> np.uint64(11))
    u1 = (u53a.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = (u53b.astype(np.float64) + 0.5) * 2.0 ** -53
    radius = np.sqrt(-2.0 * np.log(u1))
    angle = 2.0 * math.pi * u2
    even = (e & np.uint64(1)) == 0
    z = np.where(even, radius * np.cos(angle), radius * np.sin(angle))
    return (z * scale).reshape(rows, cols)


def gaussian_transform(rnd: SketchRandomness, m: int) -> np.ndarray:
    """G_m / sqrt(m), m x r_cs (the Gaussian of Algorithm 3, scaled as a
    Gaussian embedding of Section 3.4)."""
    return gaussian_matrix(rnd.key_m, m, rnd.r_cs, 1.0 / math.sqrt(m))


def jl_gaussian(rnd: SketchRandomness, d: int, k: int) -> np.ndarray:
    """G_k / sqrt(k), d x k; row j multiplies pivot position j (Algorithm 8,
    Pi_2, applied in the k-dimensional space of the selected columns)."""
    return gaussian_matrix(rnd.key_k, d, k, 1.0 / math.sqrt(k))
