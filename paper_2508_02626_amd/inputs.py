"""Seeded synthetic workloads (host FP64 arrays) shared by the GPU path and the
checks.  This module holds no arithmetic of the method: it only draws points
and charges.

Distributions (the paper uses only synthetic particles, Sec. 3.5):
  uniform   x ~ U[0,1)^3
  gaussian  x ~ N(0, I_3) (the paper's Sec. 3.5 workload, unit deviation)
  plummer   radius a / sqrt(u^(-2/3) - 1), u ~ U(0,1), redrawn while > rmax,
            isotropic direction from a normalised N(0, I_3); centred at 0
  clusters  mixture of k Gaussian clusters (sigma each), centres ~ U[0.1,0.9]^3,
            equal weights
Charges are q ~ U(-1, 1), drawn after the positions from the same generator.
"""
import numpy as np


def uniform(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3))
    q = rng.uniform(-1.0, 1.0, n)
    return x, q


def gaussian(n, seed, sigma=1.0):
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, sigma, (n, 3))
    q = rng.uniform(-1.0, 1.0, n)
    return x, q


def _plummer_radii(rng, n, a, rmax):
    r = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        u = rng.random(todo.size)
        u = np.where(u == 0.0, 0.5, u)
        rr = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        ok = rr <= rmax
        r[todo[ok]] = rr[ok]
        todo = todo[~ok]
    return r


def plummer(n, seed, a=0.05, rmax=1.0):
    rng = np.random.default_rng(seed)
    r = _plummer_radii(rng, n, a, rmax)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    x = v * r[:, None]
    q = rng.uniform(-1.0, 1.0, n)
    return x, q


def clusters(n, seed, k=8, sigma=0.02):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.1, 0.9, (k, 3))
    lab = rng.integers(0, k, n)
    x = c[lab] + rng.normal(0.0, sigma, (n, 3))
    q = rng.uniform(-1.0, 1.0, n)
    return x, q


def batch_problem(i):
    """Problem i of the 256-problem batch: N log-uniform in [1e3, 2e5], half
    uniform cube and half 8-cluster mixtures, p from {4, 6, 8}; seed 1000+i."""
    rng = np.random.default_rng(1000 + i)
    n = int(np.floor(np.exp(rng.uniform(np.log(1e3), np.log(2e5)))))
    p = int(rng.choice([4, 6, 8]))
    if i % 2 == 0:
        x, q = uniform(n, 1000 + i)
    else:
        x, q = clusters(n, 1000 + i)
    return x, q, p


def served_request(i):
    """Request i of the served stream: N log-uniform in [1e3, 1e6], uniform or
    Plummer, requested relative error from {1e-4, 1e-7, 1e-9}; seed 10000+i."""
    rng = np.random.default_rng(10000 + i)
    n = int(np.floor(np.exp(rng.uniform(np.log(1e3), np.log(1e6)))))
    err = float(rng.choice([1e-4, 1e-7, 1e-9]))
    if rng.random() < 0.5:
        x, q = uniform(n, 10000 + i)
    else:
        x, q = plummer(n, 10000 + i)
    return x, q, err


def poisson_arrivals(count, rate, seed=5):
    """Arrival times (s) of a Poisson stream of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))
