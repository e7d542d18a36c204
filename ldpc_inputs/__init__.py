"""Seeded synthetic inputs for the irregular-LDPC decoder: codes, codewords, channel.

This module is shared by the tests, the benchmark and the FP64 oracle's checks.
It holds none of the decoder's arithmetic: it builds parity-check matrices H
(as COO row/column lists), draws codewords and passes them through a BPSK/AWGN
channel to produce channel LLRs.  Everything is driven by explicit seeds
(NumPy PCG64 generators), so every caller sees the same inputs.

Conventions (Broulim et al., "OpenCL/CUDA algorithms for parallel decoding of
any irregular LDPC code using GPU", Sec. II-A and Sec. IV):

* H is m x n, H[i, j] = 1 joins check i to bit j (Eqs. (1)-(2)).
* BPSK maps bit c to x = 1 - 2c; the channel adds N(0, sigma^2) noise.
* sigma^2 = (1/R) * N0/2 with R = k/n (Eqs. (3)-(4)); with unit-energy
  symbols this is sigma^2 = 1 / (2 R 10^(EbN0/10)).
* The LLR handed to the decoder is L = 2y/sigma^2 = ln P(c=0|y)/P(c=1|y),
  the log-ratio form of the AWGN probabilities of Algorithm 3.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from .counter_noise import sim_channel_llr  # noqa: E402  (counter-based noise of Monte-Carlo runs)

__all__ = [
    "Code", "socket_code", "ebn0_to_sigma2", "awgn_llr", "code_14_7",
    "tiny_code", "large_code", "extreme_code", "batch_codes", "BATCH_SPECS",
    "tree_code", "spc_code", "path_code", "random_small_code", "sim_channel_llr",
    "lifted_code", "large_qc_code", "headline_workload", "HEADLINE_POINTS_DB",
]


@dataclasses.dataclass
class Code:
    """A binary parity-check matrix in COO form (one entry per Tanner-graph edge)."""
    m: int
    n: int
    rows: np.ndarray   # int32 [E], check index of each edge
    cols: np.ndarray   # int32 [E], bit index of each edge
    name: str = ""
    # quasi-cyclic codes: (Z, shifts) with shifts int32 [m/Z][n/Z], -1 for a zero block
    qc: tuple | None = None

    @property
    def nnz(self) -> int:
        return int(self.rows.shape[0])

    @property
    def rate(self) -> float:
        """Nominal rate (n - m) / n."""
        return (self.n - self.m) / self.n

    def dense(self) -> np.ndarray:
        H = np.zeros((self.m, self.n), dtype=np.uint8)
        H[self.rows, self.cols] = 1
        return H

    def check_degrees(self) -> np.ndarray:
        return np.bincount(self.rows, minlength=self.m)

    def bit_degrees(self) -> np.ndarray:
        return np.bincount(self.cols, minlength=self.n)

    def syndrome(self, words: np.ndarray) -> np.ndarray:
        """H c^T over GF(2) for each row of `words` ([F][n] of 0/1)."""
        words = np.atleast_2d(np.asarray(words, dtype=np.uint8))
        out = np.zeros((words.shape[0], self.m), dtype=np.uint8)
        np.bitwise_xor.at(out.T, self.rows, words[:, self.cols].T)
        return out


# ---------------------------------------------------------------------------
# channel
# ---------------------------------------------------------------------------

def ebn0_to_sigma2(ebn0_db: float, rate: float) -> float:
    """Noise variance for unit-energy BPSK at the given Eb/N0 (Eqs. (3)-(4))."""
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def awgn_llr(n: int, frames: int, sigma2: float, seed: int,
             codewords: np.ndarray | None = None) -> np.ndarray:
    """Channel LLRs [frames][n] float32 for BPSK over AWGN.

    `codewords` ([frames][n] of 0/1) defaults to the all-zero word.  The
    noise is drawn from PCG64(seed) as one [frames][n] block in float64,
    so a given seed gives the same noise whatever codeword is sent.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((frames, n))
    x = np.ones((frames, n)) if codewords is None else 1.0 - 2.0 * np.asarray(codewords, dtype=np.float64)
    y = x + np.sqrt(sigma2) * noise
    return (2.0 * y / sigma2).astype(np.float32)


# ---------------------------------------------------------------------------
# code construction
# ---------------------------------------------------------------------------

def even_check_degrees(E: int, m: int) -> np.ndarray:
    """Check degrees 'as even as possible': ceil(E/m) for the first E mod m checks."""
    d = np.full(m, E // m, dtype=np.int64)
    d[: E % m] += 1
    return d


def socket_code(bit_deg, check_deg, seed: int, name: str = "") -> Code:
    """Random Tanner graph with the given node degrees (socket matching).

    Bit sockets are listed bit by bit; a seeded permutation assigns them to
    check sockets.  Repeated (check, bit) pairs are removed by swapping the
    check end of a repeated edge with that of a random edge whenever the swap
    makes no new repeat, until none remain.  Short cycles are allowed.
    """
    bit_deg = np.asarray(bit_deg, dtype=np.int64)
    check_deg = np.asarray(check_deg, dtype=np.int64)
    n, m = bit_deg.size, check_deg.size
    E = int(bit_deg.sum())
    if E != int(check_deg.sum()):
        raise ValueError("bit and check socket counts differ")
    if check_deg.size and check_deg.max() > n:
        raise ValueError("a check degree exceeds n")
    rng = np.random.Generator(np.random.PCG64(seed))
    cols = np.repeat(np.arange(n, dtype=np.int64), bit_deg)
    rows = np.repeat(np.arange(m, dtype=np.int64), check_deg)[rng.permutation(E)]

    for _sweep in range(10000):
        key = rows * n + cols
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = order[1:][ks[1:] == ks[:-1]]
        if dup.size == 0:
            break
        uniq, counts = np.unique(key, return_counts=True)
        count = dict(zip(uniq.tolist(), counts.tolist()))
        for k in dup.tolist():
            r1, c1 = int(rows[k]), int(cols[k])
            if count.get(r1 * n + c1, 0) < 2:
                continue        # already repaired by an earlier swap
            for _try in range(100000):
                k2 = int(rng.integers(E))
                r2, c2 = int(rows[k2]), int(cols[k2])
                if r1 == r2 or c1 == c2:
                    continue
                if count.get(r2 * n + c1, 0) or count.get(r1 * n + c2, 0):
                    continue
                count[r1 * n + c1] -= 1
                count[r2 * n + c2] -= 1
                count[r2 * n + c1] = 1
                count[r1 * n + c2] = 1
                rows[k], rows[k2] = r2, r1
                break
            else:
                raise RuntimeError("could not repair a repeated edge")
    else:
        raise RuntimeError("repeated-edge repair did not converge")
    return Code(m=m, n=n, rows=rows.astype(np.int32), cols=cols.astype(np.int32), name=name)


def _block_profile(n: int, counts_by_degree):
    """Bit degrees in blocks, highest degree first (information-first order)."""
    degs = []
    for d, c in sorted(counts_by_degree.items(), key=lambda kv: -kv[0]):
        degs.extend([d] * c)
    if len(degs) != n:
        raise ValueError("profile does not cover n bits")
    return np.array(degs, dtype=np.int64)


def tiny_code(seed: int = 1001) -> Code:
    """n=1024, m=512; 50% degree-2, 30% degree-3, 20% degree-8 bits; even checks."""
    n, m = 1024, 512
    n2, n3 = round(0.5 * n), round(0.3 * n)
    bd = _block_profile(n, {8: n - n2 - n3, 3: n3, 2: n2})
    return socket_code(bd, even_check_degrees(int(bd.sum()), m), seed, "tiny-1024")


def large_code(seed: int = 1002) -> Code:
    """n=64800, m=32400 rate 1/2: 12960 degree-8, 19440 degree-3, 32400 degree-2 bits."""
    n, m = 64800, 32400
    bd = _block_profile(n, {8: 12960, 3: 19440, 2: 32400})
    return socket_code(bd, even_check_degrees(int(bd.sum()), m), seed, "large-64800")


def lifted_code(base: Code, Z: int, seed: int, name: str = "") -> Code:
    """Quasi-cyclic lifting of a base graph (a protograph without parallel edges).

    Every base edge (i, j) becomes a Z x Z circulant with a seeded shift
    s_ij in [0, Z): check i*Z + r joins bit j*Z + ((r + s_ij) mod Z).  Rows and
    bits keep the base order block by block, so a block of Z consecutive checks
    touches Z consecutive (rotated) bits of each of its column blocks.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    shifts = rng.integers(0, Z, size=base.nnz)
    r = np.arange(Z, dtype=np.int64)
    rows = (base.rows.astype(np.int64)[:, None] * Z + r[None, :]).ravel()
    cols = (base.cols.astype(np.int64)[:, None] * Z + (r[None, :] + shifts[:, None]) % Z).ravel()
    order = np.lexsort((cols, rows))
    table = np.full((base.m, base.n), -1, np.int32)
    table[base.rows, base.cols] = shifts
    return Code(m=base.m * Z, n=base.n * Z, rows=rows[order].astype(np.int32),
                cols=cols[order].astype(np.int32), name=name, qc=(int(Z), table))


def large_qc_code(seed: int = 1012) -> Code:
    """n=64800, m=32400 rate 1/2 with the large code's degree profile, lifted by Z=360
    from a 90 x 180 base graph (36 degree-8, 54 degree-3, 90 degree-2 columns;
    every base row of degree 7)."""
    bd = _block_profile(180, {8: 36, 3: 54, 2: 90})
    base = socket_code(bd, even_check_degrees(int(bd.sum()), 90), seed, "base-90-180")
    return lifted_code(base, 360, seed + 1, "qc-64800")


def _power_law(rng, lo, hi, alpha, size):
    d = np.arange(lo, hi + 1)
    p = d.astype(np.float64) ** (-alpha)
    return rng.choice(d, size=size, p=p / p.sum())


def extreme_code(seed: int = 1003, n: int = 16200, m: int = 8100, hubs: int = 8) -> Code:
    """Extreme irregularity: power-law bit degrees on [2,64], check degrees 4..512.

    Bit degrees are i.i.d. with P(d) ~ d^-2.0 on [2, 64].  `hubs` checks get
    degrees uniform in [257, 512]; the others are drawn with P(d) ~ d^-2.26 on
    [4, 256] and then moved by +-1 on random non-hub checks (staying inside
    [4, 256]) until the check sockets match the bit sockets.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    bd = np.sort(_power_law(rng, 2, 64, 2.0, n))[::-1].astype(np.int64)
    E = int(bd.sum())
    cd = np.empty(m, dtype=np.int64)
    cd[:hubs] = rng.integers(257, 513, size=hubs)
    cd[hubs:] = _power_law(rng, 4, 256, 2.26, m - hubs)
    diff = E - int(cd.sum())
    while diff != 0:
        step = 1 if diff > 0 else -1
        idx = rng.integers(hubs, m, size=abs(diff))
        for i in idx.tolist():
            if 4 <= cd[i] + step <= 256:
                cd[i] += step
                diff -= step
                if diff == 0:
                    break
    rng.shuffle(cd)
    return socket_code(bd, cd, seed + 7, "extreme-16200")


# (n, m) of the eight codes of the batched / served workloads; rates 1/3 .. 9/10
BATCH_SPECS = [(576, 384), (1152, 576), (2304, 768), (4608, 768),
               (8192, 2048), (16200, 1620), (32400, 10800), (64800, 32400)]


def batch_code(n: int, m: int, seed: int) -> Code:
    """m degree-2 bits; the other n-m bits split 0.6 / 0.4 into degree 3 / 8."""
    rest = n - m
    n3 = round(0.6 * rest)
    bd = _block_profile(n, {8: rest - n3, 3: n3, 2: m})
    return socket_code(bd, even_check_degrees(int(bd.sum()), m), seed, f"batch-{n}-{m}")


def batch_codes():
    return [batch_code(n, m, 1101 + i) for i, (n, m) in enumerate(BATCH_SPECS)]


def batch_frame_split(total: int = 4096, k: int = 8):
    """Zipf(s=1) split of `total` frames over k codes ranked by ascending n.

    Largest-remainder rounding, so the counts sum to `total`.
    """
    w = 1.0 / np.arange(1, k + 1)
    exact = total * w / w.sum()
    f = np.floor(exact).astype(np.int64)
    short = total - int(f.sum())
    f[np.argsort(-(exact - f), kind="stable")[:short]] += 1
    return f


# ---------------------------------------------------------------------------
# small structured codes used to pin the oracle
# ---------------------------------------------------------------------------

def code_14_7() -> Code:
    """The (14,7) example code, edges in the paper's Table I order (bit-sorted)."""
    pairs = [(0, 5), (0, 3), (0, 2), (0, 0), (1, 4), (1, 0), (2, 5), (2, 1), (3, 6), (3, 4),
             (3, 1), (4, 4), (4, 3), (5, 1), (5, 0), (6, 4), (6, 2), (7, 6), (7, 5), (8, 5),
             (8, 4), (9, 2), (9, 1), (10, 6), (10, 0), (11, 3), (11, 1), (12, 6), (12, 3),
             (13, 5), (13, 0)]
    cols = np.array([p[0] for p in pairs], dtype=np.int32)
    rows = np.array([p[1] for p in pairs], dtype=np.int32)
    return Code(m=7, n=14, rows=rows, cols=cols, name="paper-14-7")


def tree_code(n_checks: int, seed: int, max_check_deg: int = 4) -> Code:
    """A random cycle-free Tanner graph; every check has degree >= 2.

    Grown from one bit: each new check hangs off a random existing bit and
    brings 1..max_check_deg-1 new bits, so the graph stays a tree.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    rows, cols = [], []
    n = 1
    for c in range(n_checks):
        parent = int(rng.integers(n))
        k = int(rng.integers(1, max_check_deg))
        rows.append(c)
        cols.append(parent)
        for _ in range(k):
            rows.append(c)
            cols.append(n)
            n += 1
    perm = rng.permutation(len(rows))
    return Code(m=n_checks, n=n, rows=np.array(rows, np.int32)[perm],
                cols=np.array(cols, np.int32)[perm], name=f"tree-{seed}")


def spc_code(d: int) -> Code:
    """Single parity check on d bits."""
    return Code(m=1, n=d, rows=np.zeros(d, np.int32), cols=np.arange(d, dtype=np.int32), name=f"spc-{d}")


def path_code(n: int) -> Code:
    """Repetition code as a path: check i ties bits i and i+1."""
    rows = np.repeat(np.arange(n - 1, dtype=np.int32), 2)
    cols = np.stack([np.arange(n - 1), np.arange(1, n)], axis=1).reshape(-1).astype(np.int32)
    return Code(m=n - 1, n=n, rows=rows, cols=cols, name=f"path-{n}")


def random_small_code(n: int, m: int, bit_deg: int, seed: int) -> Code:
    """Regular-bit-degree random code with even checks (small test cases)."""
    bd = np.full(n, bit_deg, dtype=np.int64)
    return socket_code(bd, even_check_degrees(int(bd.sum()), m), seed, f"rand-{n}-{m}")


# ---------------------------------------------------------------------------
# systematic GF(2) encoder (C, gf2enc.c)
# ---------------------------------------------------------------------------

import ctypes as _ct
import os as _os
import subprocess as _sp

_ENC_SRC = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "gf2enc.c")
_ENC_SO = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "libgf2enc.so")
_enc_lib = None


def build_encoder() -> str:
    tmp = _ENC_SO + ".tmp"
    _sp.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _ENC_SRC])
    _os.replace(tmp, _ENC_SO)
    return _ENC_SO


def _enc():
    global _enc_lib
    if _enc_lib is None:
        if not _os.path.exists(_ENC_SO):
            build_encoder()
        lib = _ct.CDLL(_ENC_SO)
        P = _ct.c_void_p
        lib.gf2enc_create.argtypes = [_ct.c_int, _ct.c_int, _ct.c_long, P, P, _ct.POINTER(P), _ct.POINTER(_ct.c_int)]
        lib.gf2enc_create.restype = _ct.c_int
        lib.gf2enc_encode.argtypes = [P, _ct.c_int, P, P]
        lib.gf2enc_encode.restype = _ct.c_int
        lib.gf2enc_info_columns.argtypes = [P, P]
        lib.gf2enc_info_columns.restype = _ct.c_int
        lib.gf2enc_free.argtypes = [P]
        _enc_lib = lib
    return _enc_lib


class Encoder:
    """Systematic encoder of a Code: k = n - rank(H) information columns."""

    def __init__(self, code: Code):
        lib = _enc()
        self._lib = lib
        rows = np.ascontiguousarray(code.rows, np.int32)
        cols = np.ascontiguousarray(code.cols, np.int32)
        self._h = _ct.c_void_p()
        k = _ct.c_int()
        st = lib.gf2enc_create(code.m, code.n, rows.size, rows.ctypes.data_as(_ct.c_void_p),
                               cols.ctypes.data_as(_ct.c_void_p), _ct.byref(self._h), _ct.byref(k))
        if st != 0:
            raise ValueError(f"encoder construction failed (status {st})")
        self.k, self.n = int(k.value), code.n
        self.info_cols = np.zeros(self.k, np.int32)
        lib.gf2enc_info_columns(self._h, self.info_cols.ctypes.data_as(_ct.c_void_p))

    def encode(self, info: np.ndarray) -> np.ndarray:
        info = np.ascontiguousarray(np.atleast_2d(info), np.uint8)
        if info.shape[1] != self.k:
            raise ValueError("info width must be k")
        cw = np.zeros((info.shape[0], self.n), np.uint8)
        st = self._lib.gf2enc_encode(self._h, info.shape[0], info.ctypes.data_as(_ct.c_void_p),
                                     cw.ctypes.data_as(_ct.c_void_p))
        if st != 0:
            raise RuntimeError(f"encoding failed (status {st})")
        return cw

    def random_codewords(self, frames: int, seed: int) -> np.ndarray:
        rng = np.random.Generator(np.random.PCG64(seed))
        return self.encode(rng.integers(0, 2, size=(frames, self.k), dtype=np.uint8))

    def __del__(self):
        try:
            if self._h:
                self._lib.gf2enc_free(self._h)
                self._h = _ct.c_void_p()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# the rate-1/2 n = 64800 workload (random codewords at four Eb/N0 points)
# ---------------------------------------------------------------------------

HEADLINE_POINTS_DB = (0.8, 1.0, 1.2, 1.4)


def headline_workload(frames: int = 256, points=HEADLINE_POINTS_DB):
    """(code, codewords, llrs): the large rate-1/2 code, `frames` random
    codewords per Eb/N0 point (information seed 3002 + i through the systematic
    GF(2) encoder) and their channel LLRs (noise seed 2002 + 10 i), one
    [frames][n] float32 array per point."""
    code = large_code()
    enc = Encoder(code)
    cws = [enc.random_codewords(frames, seed=3002 + i) for i in range(len(points))]
    llrs = [awgn_llr(code.n, frames, ebn0_to_sigma2(eb, code.rate), seed=2002 + 10 * i, codewords=cws[i])
            for i, eb in enumerate(points)]
    return code, cws, llrs
