"""Seeded synthetic workloads shaped like the paper's test matrices.

This module holds no arithmetic of the method (no polynomial, coefficient,
power, norm-based plan or error measure).  It only draws matrices; the same
arrays are handed to the GPU library and to the CPU oracle by the tests and
the benchmark.  Generator: numpy PCG64 seeded with 17396 + 100*case + k.

Workloads (synthetic stand-ins; the paper's own collections -- Anymatrix, the
matrices-expm group, MATLAB gallery matrices, the cosine test set -- are not
available, see the paper's sections 3.3 and 4):
  single_64        one 64x64 N(0,1) matrix rescaled to ||A||_1 = 1
  dense_1024(t)    one 1024x1024 N(0,1) matrix rescaled to ||A||_1 = t,
                   t in {0.1, 1, 8, 64}; squarings sigma = max(0, ceil(log2 t))
                   so that ||A / 2^sigma||_1 <= 1
  batch_uneven     4096 matrices, n drawn uniformly from {8, 16, ..., 256},
                   N(0,1) entries rescaled to ||A||_1 ~ U[0.05, 4]
  orthosim_2048    A = Q diag(lambda) Q^T, Q Haar orthogonal (QR of N(0,1) with
                   the signs of diag(R) folded in), lambda ~ U[-2, 2]; and the
                   nonnormal variant diag(lambda) + triu(N(0,1), 1)/sqrt(n)
  grad_batch_512   64 matrices 512x512 with N(0,1)/sqrt(n) entries (float32)
                   and upstream gradients G with N(0,1) entries
  class_b(n)       the paper's class B generator 100*triu(N(0,1), 1)
  shifted_1024     -t I + E, E a 1024x1024 N(0,1) matrix rescaled to
                   ||E||_1 = eps (t = 0.5, eps = 0.05): a matrix near a
                   negative scalar, the kind for which Algorithm 2's
                   variable-s branch raises s above ceil(sqrt(m))
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 17396


def rng(case: int, k: int = 0) -> np.random.Generator:
    return np.random.default_rng(BASE_SEED + 100 * case + k)


def _colsum_max(G: np.ndarray) -> float:
    return float(np.max(np.sum(np.abs(G), axis=0)))


def rescaled_normal(n: int, target: float, g: np.random.Generator) -> np.ndarray:
    G = g.standard_normal((n, n))
    return G * (target / _colsum_max(G))


def squarings_for(target: float) -> int:
    """sigma with ||A||_1 / 2^sigma <= 1 for ||A||_1 = target."""
    return max(0, int(math.ceil(math.log2(target)))) if target > 0 else 0


def single_64() -> np.ndarray:
    return rescaled_normal(64, 1.0, rng(0))


DENSE_NORMS = (0.1, 1.0, 8.0, 64.0)


def dense_1024(t: float, n: int = 1024) -> np.ndarray:
    k = DENSE_NORMS.index(t) if t in DENSE_NORMS else int(round(1000 * t))
    return rescaled_normal(n, t, rng(1, k))


def batch_uneven(count: int = 4096, nmin: int = 8, nmax: int = 256, step: int = 8):
    """Returns (list of float64 arrays, list of target norms)."""
    g = rng(2)
    sizes = g.integers(nmin // step, nmax // step + 1, count) * step
    norms = g.uniform(0.05, 4.0, count)
    mats = [rescaled_normal(int(n), float(t), g) for n, t in zip(sizes, norms)]
    return mats, [float(t) for t in norms]


def haar_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    Q, R = np.linalg.qr(g.standard_normal((n, n)))
    return Q * np.sign(np.diag(R))[None, :]


def orthosim_2048(n: int = 2048, nonnormal: bool = False) -> np.ndarray:
    g = rng(3, 1 if nonnormal else 0)
    lam = g.uniform(-2.0, 2.0, n)
    if nonnormal:
        return np.diag(lam) + np.triu(g.standard_normal((n, n)), 1) / math.sqrt(n)
    Q = haar_orthogonal(n, g)
    return (Q * lam[None, :]) @ Q.T


def grad_batch_512(batch: int = 64, n: int = 512):
    """Returns (A, G) as float32 arrays of shape (batch, n, n)."""
    g = rng(4)
    A = (g.standard_normal((batch, n, n)) / math.sqrt(n)).astype(np.float32)
    G = g.standard_normal((batch, n, n)).astype(np.float32)
    return A, G


def class_b(n: int, k: int = 0) -> np.ndarray:
    return 100.0 * np.triu(rng(5, k).standard_normal((n, n)), 1)


def shifted_1024(t: float = 0.5, eps: float = 0.05, n: int = 1024) -> np.ndarray:
    return -t * np.eye(n) + rescaled_normal(n, eps, rng(8))


def gaussian(rows: int, cols: int, k: int = 0) -> np.ndarray:
    """N(0,1) entries: the matrices and right-hand sides of the linear solve."""
    return rng(6, k).standard_normal((rows, cols))
