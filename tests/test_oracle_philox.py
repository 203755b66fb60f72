"""Pin of the oracle's counter-based generator against published known-answer vectors."""

import os

import numpy as np
import pytest

from oracle import philox

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_known_answers(ctr, key, out):
    got = philox.philox4x32_10(np.array(ctr, dtype=np.uint32), np.array(key, dtype=np.uint32))
    assert [int(x) for x in got] == out


def test_gaussian_moments_and_independence():
    z = philox.gaussian_block(20000, 8, 1.0, seed=5, stream=17)
    assert abs(z.mean()) < 0.01
    assert abs(z.std() - 1.0) < 0.01
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(8))) < 0.03
    # row offsets address the same block
    part = philox.gaussian_block(100, 8, 1.0, seed=5, stream=17, row0=500)
    assert np.array_equal(part, z[500:600])
    # different streams differ
    assert not np.allclose(philox.gaussian_block(10, 8, 1.0, 5, 18), z[:10])


def test_uniforms_in_open_interval():
    u = philox.uniforms(100000, seed=3, stream=2)
    assert u.min() > 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 0.005


def test_round_bf16():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.14159265], dtype=np.float64)
    r = philox.round_bf16(x)
    # bfloat16 keeps 8 significant bits: ties go to the even neighbour
    assert list(r[:4]) == [1.0, 1.0, 1.0 + 4 * 2 ** -8, -2.5]
    assert r[4] == np.float32(3.140625)
