"""Pins of the oracle's encoder: the brute-force Kronecker product and the
involution F^{(x)m} F^{(x)m} = I over GF(2) (Section III, eq. (3))."""

import numpy as np
import pytest

import oracle

F = np.array([[1, 0], [1, 1]], dtype=np.int64)


def kron_power(m):
    G = np.ones((1, 1), dtype=np.int64)
    for _ in range(m):
        G = np.kron(G, F)
    return G


@pytest.mark.parametrize("m", [1, 2, 3, 4, 6])
def test_encode_equals_kronecker_product(m):
    n = 1 << m
    rng = np.random.default_rng(m)
    u = rng.integers(0, 2, size=(50, n)).astype(np.uint8)
    want = (u.astype(np.int64) @ kron_power(m)) % 2
    assert np.array_equal(oracle.encode(u), want.astype(np.uint8))


def test_unit_vectors_give_rows_of_G():
    m = 5
    G = kron_power(m)
    assert np.array_equal(oracle.encode(np.eye(32, dtype=np.uint8)), G)


@pytest.mark.parametrize("m", [1, 5, 10, 14])
def test_involution(m):
    rng = np.random.default_rng(100 + m)
    u = rng.integers(0, 2, size=(4, 1 << m)).astype(np.uint8)
    assert np.array_equal(oracle.encode(oracle.encode(u)), u)
