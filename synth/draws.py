"""Seeded random draws.  Every random number the method consumes comes from here.

* start vectors: the random initial Lanczos vector f_1 (Alg. 1 requires a random
  vector of norm 1; the normalisation is the method's job, not this module's);
* batch draws: U/t and filling of each instance of the batched workload;
* network initialisation and minibatch draws for the learned start vector.
"""

import numpy as np

# 32 occupation bits (16 up, 16 down) -> 3 hidden layers of 128 -> 1 amplitude
MLP_SIZES = (32, 128, 128, 128, 1)


def start_vector(seed: int, dim: int) -> np.ndarray:
    """Uniform(-1, 1) entries in float64, ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, int(dim))


def batch_instances(n: int = 64, seed: int = 1000, u_max: float = 8.0, fillings=(3, 4, 5, 6)):
    """(U, N) pairs of the batched workload: all U drawn first, then all fillings.

    The start-vector seed of instance i is ``seed + i``.
    """
    rng = np.random.default_rng(seed)
    us = rng.uniform(0.0, u_max, n)
    ns = rng.choice(np.asarray(fillings, dtype=np.int64), n)
    return [(float(u), int(k), seed + i) for i, (u, k) in enumerate(zip(us, ns))]


def mlp_init(seed: int, sizes=MLP_SIZES):
    """He-uniform weights W_l (fan_out x fan_in) and zero biases, float64."""
    rng = np.random.default_rng(seed)
    ws, bs = [], []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / fan_in)
        ws.append(rng.uniform(-lim, lim, (fan_out, fan_in)))
        bs.append(np.zeros(fan_out))
    return ws, bs


def minibatch_uniforms(seed: int, n_iters: int, batch: int) -> np.ndarray:
    """Uniform [0,1) numbers, two per sample: (selector, position).

    The selector chooses between the |psi|^2-weighted and the uniform proposal;
    the position is inverted through the chosen cumulative distribution.
    Shape (n_iters, batch, 2), float64.
    """
    rng = np.random.default_rng(seed)
    return rng.random((n_iters, batch, 2))


def start_vector_complex(seed: int, dim: int) -> np.ndarray:
    """Complex start vector: ``start_vector(seed, 2 * dim)`` read as interleaved (re, im) pairs,
    the memory layout of a complex128 array."""
    return start_vector(seed, 2 * int(dim)).view(np.complex128)
