"""Philox4x32-10 and the sparse-sign index stream -- oracle side (test infrastructure only).

Philox4x32-10 is written from its published definition (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key; each of
the ten rounds multiplies counter words 0 and 2 by 0xD2511F53 and 0xCD9E8D57, splits each 64-bit
product into hi/lo halves and permutes
    (c0, c1, c2, c3) -> (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)),
and the key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds.
Pinned by the published known-answer vectors (tests/golden/philox4x32_10_kat.txt).

Sparse sign embedding (paper, Section 4.2, "Choice of embedding"): every column s_j of
S = zeta^{-1/2} [s_1 ... s_m] has zeta nonzeros +-1 in uniformly random positions of [0, d).  The
paper fixes no generator; this project's stream (identical on the HIP side, implemented there
independently) is:
  * key = (seed mod 2^32, seed >> 32);
  * row positions of column j: words of Philox(counter=(j mod 2^32, j >> 32, t, 0)), t = 0, 1, ...,
    taken in order w0..w3; a word w maps to floor(w * d / 2^32) and is rejected when
    (w * d) mod 2^32 < 2^32 mod d (Lemire's unbiased multiply-shift) or when the value equals a
    position already accepted for this column; accept until zeta positions;
  * if T_MAX blocks (4 * T_MAX words) do not yield zeta positions, the remaining ones are the
    smallest unused positions in increasing order (unreachable for zeta << d in practice);
  * signs: bit k of the 128-bit block Philox(counter=(j mod 2^32, j >> 32, k // 128, 1)), bit
    (k mod 32) of word (k mod 128) // 32; bit 1 means -1.  Sign k belongs to the k-th accepted
    position.
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
SH32 = np.uint64(32)
T_MAX = 64


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10; arguments are uint64 arrays/scalars holding 32-bit values."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for rnd in range(10):
        p0 = M0 * c0                   # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> SH32, p0 & MASK32
        hi1, lo1 = p1 >> SH32, p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        if rnd < 9:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
    return c0, c1, c2, c3


def _key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.uint64(seed & 0xFFFFFFFF), np.uint64(seed >> 32)


def sparse_sign_indices(m: int, d: int, zeta: int, seed: int, col0: int = 0, ncols=None):
    """Row positions (int32, shape (ncols, zeta)) and signs (+1/-1 int8) of columns col0.. of S."""
    if not (1 <= zeta <= d):
        raise ValueError("need 1 <= zeta <= d")
    if ncols is None:
        ncols = m - col0
    k0, k1 = _key(seed)
    j = np.arange(col0, col0 + ncols, dtype=np.uint64)
    jlo, jhi = j & MASK32, j >> SH32
    d64 = np.uint64(d)
    thresh = np.uint64((1 << 32) % d)
    rows = np.full((ncols, zeta), -1, dtype=np.int64)
    cnt = np.zeros(ncols, dtype=np.int64)
    active = np.arange(ncols)
    for t in range(T_MAX):
        if active.size == 0:
            break
        words = philox4x32_10(jlo[active], jhi[active], np.uint64(t), np.uint64(0), k0, k1)
        for w in words:
            prod = w * d64
            cand = (prod >> SH32).astype(np.int64)
            ok = (prod & MASK32) >= thresh
            # distinctness against positions accepted so far in this column
            ra = rows[active]
            dup = (ra == cand[:, None]).any(axis=1)
            ok &= ~dup
            ok &= cnt[active] < zeta
            acc = active[ok]
            rows[acc, cnt[acc]] = cand[ok]
            cnt[acc] += 1
        active = active[cnt[active] < zeta]
    for c in active:  # deterministic completion (practically unreachable)
        used = set(int(v) for v in rows[c, : cnt[c]])
        nxt = 0
        while cnt[c] < zeta:
            if nxt not in used:
                rows[c, cnt[c]] = nxt
                cnt[c] += 1
            nxt += 1
    signs = np.empty((ncols, zeta), dtype=np.int8)
    for blk in range((zeta + 127) // 128):
        words = philox4x32_10(jlo, jhi, np.uint64(blk), np.uint64(1), k0, k1)
        for k in range(blk * 128, min(zeta, blk * 128 + 128)):
            kk = k - blk * 128
            bit = (words[kk // 32] >> np.uint64(kk % 32)) & np.uint64(1)
            signs[:, k] = np.where(bit == 1, -1, 1).astype(np.int8)
    return rows.astype(np.int32), signs
