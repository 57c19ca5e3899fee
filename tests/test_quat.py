"""Pin of the oracle's quaternion algebra against 2x2 complex matrices
(paper Sec. 2: U = a0 1 + i a.sigma, Tr U = 2 a0, det U = a^2)."""
import numpy as np

SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]], complex),
       np.array([[1, 0], [0, -1]], complex)]


def mat(a):
    return a[0] * np.eye(2) + 1j * (a[1] * SIG[0] + a[2] * SIG[1] + a[3] * SIG[2])


def test_product_matches_matrices(orc):
    rng = np.random.default_rng(3)
    for _ in range(500):
        a, b = rng.standard_normal(4), rng.standard_normal(4)
        c = orc.qmul(a, b)
        assert np.allclose(mat(c), mat(a) @ mat(b), atol=1e-13)


def test_su2_properties(orc):
    rng = np.random.default_rng(4)
    for _ in range(100):
        a = rng.standard_normal(4)
        a /= np.linalg.norm(a)
        M = mat(a)
        assert np.allclose(M @ M.conj().T, np.eye(2), atol=1e-14)
        assert abs(np.linalg.det(M) - 1) < 1e-14
        assert abs(np.trace(M).real / 2 - a[0]) < 1e-15
        ad = np.array([a[0], -a[1], -a[2], -a[3]])
        assert np.allclose(mat(ad), M.conj().T)
        assert np.allclose(orc.qmul(a, ad), [1, 0, 0, 0], atol=1e-15)
