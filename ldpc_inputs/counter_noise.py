"""Counter-based channel noise for Monte-Carlo error-rate runs (host side).

The device library draws its own channel noise (ldpc_simulate); this module
draws the same noise on the host from the same published definitions, so that
tests can check the device's channel against it.  It holds none of the
decoder's arithmetic.

* Philox4x32-10 (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
  "Parallel random numbers: as easy as 1, 2, 3", SC 2011): a counter of four
  32-bit words and a key of two go through ten rounds; each round multiplies
  counter words 0 and 2 by fixed 32-bit multipliers into 64-bit products,
  swaps and mixes the halves with words 1 and 3 and the round key, and the
  key advances by two Weyl constants between rounds.
* Uniforms u = ((x >> 9) + 0.5) 2^-23 in (0, 1), then the Box-Muller
  transform: z0 = r cos(2 pi u1), z1 = r sin(2 pi u1), r = sqrt(-2 ln u0).
* Frame f (global index), bits 4q..4q+3: counter (q, f mod 2^32, f >> 32, 0),
  key (seed mod 2^32, seed >> 32); outputs (x0, x1) give bits 4q, 4q+1 and
  (x2, x3) bits 4q+2, 4q+3.
* All-zero codeword over BPSK/AWGN: y = 1 + sigma z and L = 2y/sigma^2, with
  sigma^2 from Eb/N0 and the nominal rate (n - m)/n (Eqs. (3)-(4)).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32 with 10 rounds.  counter: [..., 4] integers < 2^32; key: [..., 2].

    Returns [..., 4] uint32.
    """
    ctr = np.asarray(counter, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i] for i in range(4))
    k0, k1 = k[..., 0], k[..., 1]
    for _ in range(10):
        p0 = c0 * _M0          # < 2^64: exact in uint64
        p1 = c2 * _M1
        c0, c1, c2, c3 = ((p1 >> _S32) ^ c1 ^ k0) & _MASK, p1 & _MASK, ((p0 >> _S32) ^ c3 ^ k1) & _MASK, p0 & _MASK
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def unit_open(x: np.ndarray) -> np.ndarray:
    """Uniforms in (0, 1) from the top 23 bits of 32-bit words (exact in float32)."""
    return ((np.asarray(x, dtype=np.uint32) >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def frame_normals(n: int, frames: int, seed: int, first_frame: int = 0) -> np.ndarray:
    """Standard normals [frames][n] (float64) of global frames first_frame .. + frames - 1."""
    quads = (n + 3) // 4
    f = np.uint64(first_frame) + np.arange(frames, dtype=np.uint64)
    ctr = np.empty((frames, quads, 4), dtype=np.uint64)
    ctr[..., 0] = np.arange(quads, dtype=np.uint64)[None, :]
    ctr[..., 1] = (f & _MASK)[:, None]
    ctr[..., 2] = (f >> _S32)[:, None]
    ctr[..., 3] = 0
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    x = philox4x32_10(ctr, key)
    u = unit_open(x)
    z = np.empty((frames, quads, 4))
    for a, b in ((0, 1), (2, 3)):
        r = np.sqrt(-2.0 * np.log(u[..., a]))
        z[..., a] = r * np.cos(2.0 * np.pi * u[..., b])
        z[..., b] = r * np.sin(2.0 * np.pi * u[..., b])
    return z.reshape(frames, quads * 4)[:, :n]


def sim_channel_llr(n: int, m: int, frames: int, ebn0_db: float, seed: int, first_frame: int = 0) -> np.ndarray:
    """Channel LLRs [frames][n] float32 of the all-zero codeword, as drawn by ldpc_simulate.

    L = k0 + k1 z with k0 = 2/sigma^2 and k1 = 2/sigma rounded to float32 (the
    device evaluates the same expression in float32 with its own transcendentals,
    so the two agree to a few units in the last place).
    """
    rate = (n - m) / n
    sigma2 = 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))
    k0 = float(np.float32(2.0 / sigma2))
    k1 = float(np.float32(2.0 / np.sqrt(sigma2)))
    z = frame_normals(n, frames, seed, first_frame)
    return (k1 * z + k0).astype(np.float32)
