"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws data: it holds none of the solver's arithmetic and is
shared by the oracle tests, the GPU tests and the benchmark.  The recipe
follows the synthetic set-up of the experiments section (Sec. 4, "Long
convolutional sparse coding signals"): Gaussian atoms normalised to unit
norm, Bernoulli-Gaussian activations, additive white Gaussian noise, with the
sizes of each workload below.

Draw order for ``generate`` with ``numpy.random.Generator(PCG64(seed))``:
  1. D ~ N(0, 1)^{K x P x W}, each atom scaled to unit Frobenius norm;
  2. Z_true = Bernoulli(rho) * N(0, sigma_z^2), shape K x L, L = T - W + 1;
  3. X = sum_k Z_true_k * D_k (full convolution, length T) + N(0, sigma_noise^2).
The solvers consume the float32 casts of X and D.
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    P: int
    K: int
    W: int
    T: int
    rho: float
    sigma_noise: float
    sigma_z: float = 10.0
    lam_rel: float = 0.1
    eps: float = 1e-6
    n_seg: int = 0


# Workload sizes (the paper's default shape is W=200, K=25, P=7).
SMALL = Workload("small: P=1 K=5 W=32 T=4096, 4 segments", 1, 5, 32, 4096,
                 0.01, 0.1, n_seg=4)
PAPER = Workload("paper-shaped: P=7 K=25 W=200 T=150000", 7, 25, 200, 150_000,
                 0.007, 0.1)
LONG = Workload("long: P=7 K=25 W=200 T=5000000", 7, 25, 200, 5_000_000,
                0.007, 0.1)
BATCH_ATOM = dict(P=7, K=25, W=64, rho=0.005, sigma_noise=0.1)


def dictionary(rng, K, P, W):
    D = rng.standard_normal((K, P, W))
    D /= np.sqrt(np.sum(D * D, axis=(1, 2), keepdims=True))
    return D


def activations(rng, K, L, rho, sigma_z):
    mask = rng.random((K, L)) < rho
    vals = rng.standard_normal((K, L)) * sigma_z
    return np.where(mask, vals, 0.0)


def synthesize(D, Z, T):
    """sum_k Z_k * D_k, shape (P, T); scatters each non-zero activation."""
    K, P, W = D.shape
    X = np.zeros((P, T))
    for k in range(K):
        idx = np.flatnonzero(Z[k])
        if idx.size == 0:
            continue
        z = Z[k, idx]
        for tau in range(W):
            X[:, idx + tau] += np.outer(D[k, :, tau], z)
    return X


def generate(P, K, W, T, rho, sigma_noise, seed, sigma_z=10.0, D=None):
    """Returns (X float32 [P,T], D float32 [K,P,W], Z_true float64 [K,L]).

    If ``D`` is given it is used as the dictionary (shared-dictionary batches)
    and step 1 is skipped.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if D is None:
        D = dictionary(rng, K, P, W)
    else:
        D = np.asarray(D, dtype=np.float64)
    L = T - W + 1
    Z = activations(rng, K, L, rho, sigma_z)
    X = synthesize(D, Z, T) + sigma_noise * rng.standard_normal((P, T))
    return X.astype(np.float32), D.astype(np.float32), Z


def synthesize_fast(D, Z, T):
    """sum_k Z_k * D_k like ``synthesize``, summed per channel with one
    bincount over all non-zero activations (other summation order)."""
    K, P, W = D.shape
    ks, ts = np.nonzero(Z)
    order = np.argsort(ts, kind="stable")
    ks, ts = ks[order], ts[order]
    z = Z[ks, ts]
    X = np.zeros((P, T))
    step = max(1, (1 << 22) // W)  # bounded temporaries
    for a in range(0, z.size, step):
        k, t, v = ks[a:a + step], ts[a:a + step], z[a:a + step]
        lo = int(t[0])
        idx = (t[:, None] - lo + np.arange(W)[None, :]).ravel()
        n = int(t[-1]) - lo + W
        for p in range(P):
            X[p, lo:lo + n] += np.bincount(idx, weights=(v[:, None] * D[k, p, :]).ravel(),
                                           minlength=n)
    return X


def generate_fast(P, K, W, T, rho, sigma_noise, seed, D, sigma_z=10.0):
    """The same distributions as ``generate`` with a shared dictionary, drawn in
    float32 and with Gaussian values only for the non-zero activations (a
    different random stream from ``generate``): for the large batched and
    served workloads.  Returns X float32 [P, T]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = np.asarray(D, dtype=np.float64)
    L = T - W + 1
    mask = rng.random((K, L), dtype=np.float32) < rho
    Z = np.zeros((K, L))
    Z[mask] = rng.standard_normal(int(mask.sum())) * sigma_z
    X = synthesize_fast(D, Z, T)
    X += sigma_noise * rng.standard_normal((P, T), dtype=np.float32)
    return X.astype(np.float32)


def generate_conv(P, K, W, T, rho, sigma_noise, seed, D, sigma_z=10.0):
    """The draws of ``generate_fast`` (same seed, same Z and noise) with the
    sum of convolutions formed by one transposed convolution in float32 on the
    CPU (torch): seconds for millions of samples, for the largest benchmark
    workloads.  Differs from ``generate_fast`` by float32 rounding only.
    Returns X float32 [P, T]."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    L = T - W + 1
    mask = rng.random((K, L), dtype=np.float32) < rho
    ks, ts = np.nonzero(mask)
    vals = rng.standard_normal(ks.size) * sigma_z
    Z = torch.zeros(1, K, L, dtype=torch.float32)
    Z[0, torch.from_numpy(ks), torch.from_numpy(ts)] = torch.from_numpy(vals.astype(np.float32))
    X = torch.nn.functional.conv_transpose1d(
        Z, torch.from_numpy(np.ascontiguousarray(D, dtype=np.float32)))[0].numpy()
    X += sigma_noise * rng.standard_normal((P, T), dtype=np.float32)
    return np.ascontiguousarray(X, dtype=np.float32)


def workload(w: Workload, seed: int):
    return generate(w.P, w.K, w.W, w.T, w.rho, w.sigma_noise, seed, w.sigma_z)


def batch_lengths(n, lo, hi, seed):
    """Signal lengths for the uneven batch: uniform integers in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=n)


def served_lengths(n, lo, hi, seed):
    """Request lengths log-uniform in [lo, hi] (served encode stream)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))).astype(np.int64)


def poisson_arrivals(n, rate, seed):
    """Arrival times (s) of a Poisson stream with the given rate (1/s)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def segment_sequence(M, n, seed):
    """Uniform random segment choices for the SeqDICOD schedule (Algorithm 3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, M, size=n).astype(np.int32)
