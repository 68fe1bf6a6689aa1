"""Pins for the oracle's Philox4x32-10 and sparse-sign index stream (CPU only)."""

import os

import numpy as np
import pytest

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            vals = [int(t, 16) for t in line.split()]
            rows.append((vals[:6], vals[6:]))
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_philox_known_answers(row):
    (c0, c1, c2, c3, k0, k1), expect = row
    out = philox.philox4x32_10(c0, c1, c2, c3, k0, k1)
    assert [int(o) for o in out] == expect


def test_philox_vectorised_matches_scalar():
    c = np.arange(1000, dtype=np.uint64) * np.uint64(2654435761) & np.uint64(0xFFFFFFFF)
    out = philox.philox4x32_10(c, c ^ np.uint64(7), np.uint64(3), np.uint64(9), np.uint64(11), np.uint64(13))
    for i in (0, 17, 999):
        s = philox.philox4x32_10(int(c[i]), int(c[i]) ^ 7, 3, 9, 11, 13)
        assert [int(o[i]) for o in out] == [int(v) for v in s]


def test_lemire_map_reference_scalar():
    """Row positions follow the documented word -> position rule, recomputed with Python ints."""
    m, d, zeta, seed = 300, 37, 5, 0xDEADBEEF12345
    rows, signs = philox.sparse_sign_indices(m, d, zeta, seed)
    k0, k1 = seed & 0xFFFFFFFF, seed >> 32
    thresh = (1 << 32) % d
    for j in (0, 1, 150, 299):
        acc = []
        t = 0
        while len(acc) < zeta:
            words = philox.philox4x32_10(j & 0xFFFFFFFF, j >> 32, t, 0, k0, k1)
            for w in words:
                w = int(w)
                prod = w * d
                if len(acc) < zeta and (prod & 0xFFFFFFFF) >= thresh and (prod >> 32) not in acc:
                    acc.append(prod >> 32)
            t += 1
        assert list(rows[j]) == acc
        sw = [int(w) for w in philox.philox4x32_10(j & 0xFFFFFFFF, j >> 32, 0, 1, k0, k1)]
        exp = [(-1 if (sw[k // 32] >> (k % 32)) & 1 else 1) for k in range(zeta)]
        assert list(signs[j]) == exp


def test_indices_distinct_in_range_and_seeded():
    m, d, zeta = 20000, 600, 8
    r1, s1 = philox.sparse_sign_indices(m, d, zeta, 12345)
    r2, s2 = philox.sparse_sign_indices(m, d, zeta, 12345)
    r3, _ = philox.sparse_sign_indices(m, d, zeta, 12346)
    assert np.array_equal(r1, r2) and np.array_equal(s1, s2)
    assert not np.array_equal(r1, r3)
    assert r1.min() >= 0 and r1.max() < d
    srt = np.sort(r1, axis=1)
    assert np.all(np.diff(srt, axis=1) > 0), "positions within a column must be distinct"
    assert set(np.unique(s1)) == {-1, 1}


def test_index_statistics():
    """Row hits ~ Binomial(m zeta, 1/d) and fair signs (uniform positions, Section 4.2)."""
    m, d, zeta = 60000, 600, 8
    rows, signs = philox.sparse_sign_indices(m, d, zeta, 7)
    hits = np.bincount(rows.reshape(-1), minlength=d)
    mean = m * zeta / d
    assert abs(hits.mean() - mean) < 1e-9
    # chi-square against uniform; 599 dof -> mean 599, sd ~34.6
    chi2 = np.sum((hits - mean) ** 2 / mean)
    assert 450 < chi2 < 760
    frac_neg = np.mean(signs == -1)
    assert abs(frac_neg - 0.5) < 0.01
    # sign independent of slot
    assert np.all(np.abs((signs == -1).mean(axis=0) - 0.5) < 0.03)


def test_dense_zeta_equals_d_completes():
    """zeta = d forces the deterministic completion path: each column is a permutation of [0, d)."""
    rows, _ = philox.sparse_sign_indices(5, 6, 6, 3)
    for r in rows:
        assert sorted(r.tolist()) == list(range(6))
