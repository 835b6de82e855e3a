"""Pins of the oracle's algebra (Appendix) against facts outside its own code.

* Hamilton's basis table (i^2 = j^2 = k^2 = ijk = -1) -- textbook identity.
* Quaternions as 2x2 complex matrices, dual quaternions as 4x4 block upper
  triangular complex matrices [[A, B], [0, A]] (e^2 = 0 is the nilpotent block):
  products by numpy's matmul, which knows nothing of the oracle.
* Eq. quatsq against the Hamilton product q q.
* Associativity, identity and e^2 = 0 of the dual-quaternion product.
* a b + b a = 2 (a0 b0 - a.b, a0 b + b0 a): the cross-product-free square used by
  the GPU kernels, checked against the oracle's two literal Hamilton products.
"""
import numpy as np
import pytest

ONE = np.array([1.0, 0, 0, 0])
I = np.array([0, 1.0, 0, 0])
J = np.array([0, 0, 1.0, 0])
K = np.array([0, 0, 0, 1.0])


def test_hamilton_basis_table(oracle_mod):
    q = oracle_mod.quat_mul
    for u in (I, J, K):
        np.testing.assert_array_equal(q(u, u), -ONE)
    np.testing.assert_array_equal(q(q(I, J), K), -ONE)
    # ij = k, jk = i, ki = j and the anti-commuted products
    np.testing.assert_array_equal(q(I, J), K)
    np.testing.assert_array_equal(q(J, K), I)
    np.testing.assert_array_equal(q(K, I), J)
    np.testing.assert_array_equal(q(J, I), -K)
    np.testing.assert_array_equal(q(K, J), -I)
    np.testing.assert_array_equal(q(I, K), -J)
    for u in (ONE, I, J, K):
        np.testing.assert_array_equal(q(ONE, u), u)
        np.testing.assert_array_equal(q(u, ONE), u)


def quat_matrix(q):
    """Textbook 2x2 complex representation of q = s + x i + y j + z k."""
    s, x, y, z = q
    return np.array([[s + 1j * x, y + 1j * z], [-y + 1j * z, s - 1j * x]])


def dq_matrix(zeta):
    A = quat_matrix(zeta[:4])
    B = quat_matrix(zeta[4:])
    Z = np.zeros((2, 2), complex)
    return np.block([[A, B], [Z, A]])


def matrix_to_quat(M):
    return np.array([M[0, 0].real, M[0, 0].imag, M[0, 1].real, M[0, 1].imag])


def matrix_to_dq(M):
    return np.concatenate([matrix_to_quat(M[:2, :2]), matrix_to_quat(M[:2, 2:])])


def test_matrix_representation_is_faithful():
    # i^2 = j^2 = k^2 = ijk = -1 in the representation itself (so it pins the table,
    # not the other way round)
    Mi, Mj, Mk = quat_matrix(I), quat_matrix(J), quat_matrix(K)
    E = np.eye(2)
    for M in (Mi, Mj, Mk):
        np.testing.assert_allclose(M @ M, -E)
    np.testing.assert_allclose(Mi @ Mj @ Mk, -E)


def test_quat_mul_matches_matrix_product(oracle_mod):
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b = rng.normal(size=4), rng.normal(size=4)
        ref = matrix_to_quat(quat_matrix(a) @ quat_matrix(b))
        np.testing.assert_allclose(oracle_mod.quat_mul(a, b), ref, rtol=0, atol=1e-14)


def test_dq_mul_matches_block_matrix_product(oracle_mod):
    rng = np.random.default_rng(2)
    for _ in range(200):
        x, y = rng.normal(size=8), rng.normal(size=8)
        ref = matrix_to_dq(dq_matrix(x) @ dq_matrix(y))
        np.testing.assert_allclose(oracle_mod.dq_mul(x, y), ref, rtol=0, atol=1e-13)


def test_eq_quatsq_equals_hamilton_square(oracle_mod):
    rng = np.random.default_rng(3)
    for _ in range(200):
        q = rng.normal(size=4)
        np.testing.assert_allclose(oracle_mod.quat_square_eq(q), oracle_mod.quat_mul(q, q),
                                   rtol=0, atol=4e-15 * max(1.0, np.dot(q, q)))


def test_dq_product_associative_identity_nilpotent(oracle_mod):
    rng = np.random.default_rng(4)
    m = oracle_mod.dq_mul
    one = np.array([1.0, 0, 0, 0, 0, 0, 0, 0])
    eps = np.array([0, 0, 0, 0, 1.0, 0, 0, 0])
    np.testing.assert_array_equal(m(eps, eps), np.zeros(8))
    for _ in range(200):
        x, y, z = rng.normal(size=8), rng.normal(size=8), rng.normal(size=8)
        lhs, rhs = m(m(x, y), z), m(x, m(y, z))
        assert np.max(np.abs(lhs - rhs)) <= 1e-13 * max(1.0, np.max(np.abs(lhs)))
        np.testing.assert_array_equal(m(one, x), x)
        np.testing.assert_array_equal(m(x, one), x)
        # dual unit times anything keeps only the real part, moved to the dual slots
        ex = m(eps, x)
        np.testing.assert_array_equal(ex[:4], np.zeros(4))
        np.testing.assert_array_equal(ex[4:], x[:4])


def test_zero_dual_part_reduces_to_hamilton(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(100):
        a, b = rng.normal(size=4), rng.normal(size=4)
        x = np.concatenate([a, np.zeros(4)])
        y = np.concatenate([b, np.zeros(4)])
        r = oracle_mod.dq_mul(x, y)
        np.testing.assert_array_equal(r[:4], oracle_mod.quat_mul(a, b))
        np.testing.assert_array_equal(r[4:], np.zeros(4))


def test_square_dual_part_is_cross_free(oracle_mod):
    """a b + b a = 2 (a0 b0 - a.b, a0 b + b0 a) -- the form the GPU kernels use."""
    rng = np.random.default_rng(6)
    for _ in range(200):
        z = rng.normal(size=8)
        a, b = z[:4], z[4:]
        expect = 2.0 * np.concatenate([[a[0] * b[0] - np.dot(a[1:], b[1:])],
                                       a[0] * b[1:] + b[0] * a[1:]])
        sq = oracle_mod.dq_square(z)
        np.testing.assert_allclose(sq[4:], expect, rtol=0, atol=1e-14)
        np.testing.assert_allclose(sq[:4], oracle_mod.quat_square_eq(a), rtol=0, atol=1e-14)


def test_square_is_not_componentwise(oracle_mod):
    """The product-rule square differs from the printed component-wise q_a^2 + q_b^2 e."""
    z = np.array([0.5, 0.1, 0.2, 0.3, 0.7, -0.2, 0.4, 0.1])
    sq = oracle_mod.dq_square(z)
    assert not np.allclose(sq[4:], oracle_mod.quat_square_eq(z[4:]))
