"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds no arithmetic of the method: it only draws random unit 4-vectors
(configurations to upload) and permutations with numpy's PCG64 generator.
"""
import numpy as np


def random_config(dims, seed):
    """[V, 4, 4] float64 links, each an independent uniformly random unit
    4-vector (normalised Gaussian 4-vector)."""
    V = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((V, 4, 4))
    return z / np.linalg.norm(z, axis=2, keepdims=True)


def near_identity_config(dims, seed, eps):
    """Links (1, eps*g)/norm with g Gaussian: an ordered, weak-coupling-like
    configuration."""
    V = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    z = np.zeros((V, 4, 4))
    z[..., 0] = 1.0
    z[..., 1:] = eps * rng.standard_normal((V, 4, 3))
    return z / np.linalg.norm(z, axis=2, keepdims=True)


def permutation(n, seed):
    return np.random.default_rng(seed).permutation(n).astype(np.int64)


# workload shapes named by the benchmark configurations
C1 = dict(dims=(8, 8, 8, 8), beta=2.3, start="cold", sweeps=20, seed=1)
C2 = dict(dims=(32, 32, 32, 32), beta=2.6, start="hot", sweeps=200, seed=2)
C4 = dict(dims=(24, 24, 24, 48), beta=2.5, start="hot", seed=4, ape_alpha=0.7,
          ape_steps=25, Rmax=12, Tmax=16)


def c3_betas():
    return [2.1 + 0.4 * i / 15 for i in range(16)]


def c5_shapes():
    combos = []
    for L in (8, 12, 16, 24):
        for Nt in (4, 6, 8, L):
            combos.append((L, L, L, Nt))
    dims = [combos[i % 16] for i in range(64)]
    betas = [2.2 + 0.6 * i / 63 for i in range(64)]
    return dims, betas
