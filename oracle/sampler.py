"""Seeded sampling of the scheme's random inputs (oracle side).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.

The paper draws the secret key, the uniform polynomials a and the errors e of
encryption and key generation (Sec. 2.3, Sec. 2.4.1) but fixes no generator,
and gives no error distribution's width.  Reading (shared with the library,
which implements it independently in C++): every draw comes from a SHAKE-256
stream (FIPS 202; here Python's ``hashlib.shake_256``) keyed by

    seed (32 bytes) || tag || index || limb     (each a little-endian uint32),

read front to back, with

* uniform below m (m >= 2): an 8-byte little-endian word masked to
  bitlen(m - 1) bits, rejected while >= m;
* uniform ternary: a byte b, v = b & 3, rejected while v = 3; 0, 1, 2 map to
  0, +1, -1;
* h-sparse ternary over N positions: positions 0..N-1 in a list; for
  i = 0..h-1 swap entry i with entry i + u, u uniform below N - i; then per
  chosen position (in that order) one byte whose bit 0 gives the sign
  (0: +1, 1: -1);
* discrete Gaussian of sigma = 3.2 cut at |e| <= 19: the cumulative table
  T[k] = floor(2^63 * P(|X| <= k)), k = 0..18, with P(|X| = k) proportional
  to exp(-k^2 / 2 sigma^2) (twice for k > 0) summed in order in FP64, and
  T[19] = 2^63; u = (8-byte word) >> 1, |e| = the least k with u < T[k];
  a non-zero |e| takes its sign from bit 0 of one more byte.

Tags and indices: 1 the secret (index 0), 2 a switching key's a (index
256 g + j for Galois element g, 0 for relinearisation, digit j; limb = prime
index over Q then P), 3 its error (index as a, limb 0), 4 the a of an
encryption (index 0, limb = prime index), 5 its error (index 0, limb 0).
"""
from __future__ import annotations

import hashlib
import math
import struct

import numpy as np

TAG_SECRET, TAG_KEY_A, TAG_KEY_E, TAG_ENC_A, TAG_ENC_E = 1, 2, 3, 4, 5
SIGMA, BOUND = 3.2, 19


class Stream:
    """The bytes of SHAKE-256(seed || tag || index || limb), read in order."""

    def __init__(self, seed: bytes, tag: int, index: int, limb: int):
        assert len(seed) == 32
        self.msg = bytes(seed) + struct.pack("<III", tag, index, limb)
        self.buf = b""
        self.pos = 0

    def read(self, n: int) -> bytes:
        while self.pos + n > len(self.buf):           # re-squeeze a longer prefix
            self.buf = hashlib.shake_256(self.msg).digest(max(4096, 2 * len(self.buf)))
        out = self.buf[self.pos:self.pos + n]
        self.pos += n
        return out

    def word(self) -> int:
        return struct.unpack("<Q", self.read(8))[0]


def uniform_below(st: Stream, m: int) -> int:
    mask = (1 << (m - 1).bit_length()) - 1
    while True:
        v = st.word() & mask
        if v < m:
            return v


def uniform_poly(seed: bytes, tag: int, index: int, limb: int, q: int, n: int) -> np.ndarray:
    """n draws uniform below q from one stream: the words of uniform_below in
    stream order, taken `need` words at a time (every word read is one draw's
    candidate, so this is the same sequence)."""
    st = Stream(seed, tag, index, limb)
    mask = np.uint64((1 << (q - 1).bit_length()) - 1)
    parts, need = [], n
    while need:
        cand = np.frombuffer(st.read(8 * need), dtype="<u8") & mask
        ok = cand[cand < np.uint64(q)]
        parts.append(ok)
        need -= ok.size
    return np.concatenate(parts).astype(np.uint64) if parts else np.zeros(0, np.uint64)


def ternary_uniform(seed: bytes, tag: int, index: int, n: int) -> np.ndarray:
    st = Stream(seed, tag, index, 0)
    out = np.zeros(n, dtype=np.int8)
    for i in range(n):
        while True:
            v = st.read(1)[0] & 3
            if v != 3:
                break
        out[i] = (0, 1, -1)[v]
    return out


def ternary_sparse(seed: bytes, tag: int, index: int, n: int, h: int) -> np.ndarray:
    assert 0 <= h <= n
    st = Stream(seed, tag, index, 0)
    pos = list(range(n))
    for i in range(h):
        if n - i > 1:
            u = uniform_below(st, n - i)
            pos[i], pos[i + u] = pos[i + u], pos[i]
    out = np.zeros(n, dtype=np.int8)
    for i in range(h):
        out[pos[i]] = -1 if st.read(1)[0] & 1 else 1
    return out


def gaussian_table(sigma: float = SIGMA, bound: int = BOUND) -> list:
    rho = [math.exp(-(k * k) / (2.0 * sigma * sigma)) for k in range(bound + 1)]
    total = rho[0]
    for k in range(1, bound + 1):
        total += 2.0 * rho[k]
    t, acc = [], 0.0
    for k in range(bound):
        acc += (rho[k] if k == 0 else 2.0 * rho[k]) / total
        t.append(int(math.floor(acc * 2.0 ** 63)))
    t.append(1 << 63)
    return t


def gaussian_poly(seed: bytes, tag: int, index: int, n: int) -> np.ndarray:
    st = Stream(seed, tag, index, 0)
    table = gaussian_table()
    out = np.zeros(n, dtype=np.int64)
    for i in range(n):
        u = st.word() >> 1
        k = next(j for j, t in enumerate(table) if u < t)
        if k and st.read(1)[0] & 1:
            k = -k
        out[i] = k
    return out


def secret(seed: bytes, n: int, h: int) -> np.ndarray:
    """The secret key: h-sparse ternary, or uniform ternary for h < 0."""
    return ternary_uniform(seed, TAG_SECRET, 0, n) if h < 0 else ternary_sparse(seed, TAG_SECRET, 0, n, h)


def key_inputs(seed: bytes, ext_mods, n: int, beta: int, galois: int):
    """(a, e) of a switching key: a[j][m] uniform below ext_mods[m], e[j]
    Gaussian, as the switching-key generation of the oracle takes them."""
    a = np.stack([np.stack([uniform_poly(seed, TAG_KEY_A, 256 * galois + j, m, int(q), n)
                            for m, q in enumerate(ext_mods)]) for j in range(beta)])
    e = np.stack([gaussian_poly(seed, TAG_KEY_E, 256 * galois + j, n) for j in range(beta)])
    return a, e


def encryption_inputs(seed: bytes, mods, n: int):
    """(a, e) of a secret-key encryption at the level of `mods`."""
    a = np.stack([uniform_poly(seed, TAG_ENC_A, 0, i, int(q), n) for i, q in enumerate(mods)])
    return a, gaussian_poly(seed, TAG_ENC_E, 0, n)
