"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws data: Gaussian-mixture point sets shaped like the
workloads the method is evaluated on (low-dimensional clustered data and
higher-dimensional mixtures), subsample index lists, and the workload
descriptions (n, d, sigma, L, seeds).  It holds none of the method's
arithmetic and imports neither the GPU library nor the oracle.

Recipe (numpy PCG64, FP64 draws cast to FP32 at the end):
  1. component means ~ U[mean_lo, mean_hi]^d, per-component isotropic std
     ~ U[std_lo, std_hi] (or explicit means/stds);
  2. exact per-component counts (n // C each, the remainder to the first
     components);
  3. points = mean + std * N(0, I_d), concatenated by component;
  4. a seeded permutation of the rows, so that index order carries no
     cluster information (the partition tree is built over index order).
The kernel scale of each workload is gamma = 1 / (2 sigma^2).
"""
import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np


def mixture(n: int, d: int, n_comp: int, seed: int, mean_range=(-5.0, 5.0), std_range=(1.0, 1.0),
            means: Optional[np.ndarray] = None, stds: Optional[Sequence[float]] = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if means is None:
        means = rng.uniform(mean_range[0], mean_range[1], size=(n_comp, d))
    else:
        means = np.asarray(means, dtype=np.float64).reshape(n_comp, d)
    if stds is None:
        stds = rng.uniform(std_range[0], std_range[1], size=n_comp)
    else:
        stds = np.asarray(stds, dtype=np.float64).reshape(n_comp)
    counts = np.full(n_comp, n // n_comp, dtype=np.int64)
    counts[: n % n_comp] += 1
    parts = []
    for c in range(n_comp):
        if counts[c] == 0:
            continue
        parts.append(means[c] + stds[c] * rng.standard_normal(size=(int(counts[c]), d)))
    X = np.concatenate(parts, axis=0)
    X = X[rng.permutation(n)]
    return np.ascontiguousarray(X, dtype=np.float32)


def subsample(n: int, m: int, seed: int) -> np.ndarray:
    """m distinct row indices of [0, n), sorted, seeded."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(m, n), replace=False)).astype(np.int32)


def two_moons(n: int, noise: float, seed: int):
    """Two interleaved half circles in R^2 (the synthetic shape of the
    paper's experiments): n // 2 points at angle t ~ U[0, pi] on the outer
    moon (cos t, sin t), the rest on the inner moon (1 - cos t, 1/2 - sin t),
    plus isotropic Gaussian noise of std `noise`, rows in seeded random order.
    Returns (X float32 [n, 2], moon label [n])."""
    rng = np.random.default_rng(seed)
    n_out = n // 2
    t = rng.uniform(0.0, math.pi, size=n)
    X = np.empty((n, 2), dtype=np.float64)
    X[:n_out, 0] = np.cos(t[:n_out])
    X[:n_out, 1] = np.sin(t[:n_out])
    X[n_out:, 0] = 1.0 - np.cos(t[n_out:])
    X[n_out:, 1] = 0.5 - np.sin(t[n_out:])
    X += noise * rng.standard_normal(size=(n, 2))
    lab = np.concatenate([np.zeros(n_out, dtype=np.int64), np.ones(n - n_out, dtype=np.int64)])
    perm = rng.permutation(n)
    return np.ascontiguousarray(X[perm], dtype=np.float32), lab[perm]


def depth_of(n: int) -> int:
    """ceil(log2 n): the number of halvings from n points to one."""
    return 0 if n <= 1 else int(math.ceil(math.log2(n)))


@dataclass
class Workload:
    name: str
    n: int
    d: int
    sigma: float
    L: int
    data_seed: int
    philox_seed: int
    n_comp: int
    mean_range: tuple = (-5.0, 5.0)
    std_range: tuple = (1.0, 1.0)
    means: Optional[list] = None
    stds: Optional[list] = None
    extra: dict = field(default_factory=dict)

    @property
    def gamma(self) -> float:
        return 1.0 / (2.0 * self.sigma * self.sigma)

    def points(self) -> np.ndarray:
        return mixture(self.n, self.d, self.n_comp, self.data_seed, self.mean_range, self.std_range,
                       self.means, self.stds)

    def describe(self) -> dict:
        return {"workload": self.name, "n": self.n, "d": self.d, "sigma": self.sigma, "gamma": self.gamma,
                "L": self.L, "components": self.n_comp, "data_seed": self.data_seed,
                "philox_seed": self.philox_seed}


def tiny_blobs() -> Workload:
    """n=1000 in R^2: two isotropic blobs at (0,0) and (4,0), std 1, sigma 1, L 10."""
    return Workload("blobs2d-n1000", 1000, 2, 1.0, 10, 1000, 2000, 2,
                    means=[[0.0, 0.0], [4.0, 0.0]], stds=[1.0, 1.0])


def mixture32() -> Workload:
    """n=100,000 in R^32: 10 components, means U[-5,5], std U[0.5,1.5], sigma 2, L 17."""
    return Workload("mix32-n100k", 100_000, 32, 2.0, 17, 1001, 2001, 10, (-5.0, 5.0), (0.5, 1.5))


def mixture64() -> Workload:
    """n=1,000,000 in R^64: 50 components, means U[-10,10], std U[0.5,2.0], sigma 3, L 20."""
    w = Workload("mix64-n1m", 1_000_000, 64, 3.0, 20, 1002, 2002, 50, (-10.0, 10.0), (0.5, 2.0))
    w.extra["subsample"] = 20_000
    w.extra["subsample_seed"] = 1003
    return w


def batched_sets(count: int = 256, seed: int = 1003):
    """Independent sets: n log-uniform in [1e3, 6.4e4], d in {8,32,128}, 5 components,
    means U[-5,5], std 1, sigma = sqrt(d)/2, L = ceil(log2 n)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(6.4e4)))))
        d = int(rng.choice([8, 32, 128]))
        out.append(Workload(f"set{s}-n{n}-d{d}", n, d, math.sqrt(d) / 2.0, depth_of(n), seed * 1000 + s,
                            2003 * 1000 + s, 5, (-5.0, 5.0), (1.0, 1.0)))
    return out


def serving_trace(seconds: float = 60.0, rate: float = 50.0, seed: int = 1004):
    """Seeded open-loop request trace: Poisson arrivals at `rate` per second
    for `seconds`; 80% builds of a point set from a pool of 64 (n log-uniform
    in [2e3, 2e5], d 64, 20 components, means U[-10,10], std U[0.5,2], sigma
    3, L ceil(log2 n)), 20% KDE queries of 10,000 points of the same mixture
    family against a finished set; precision 50/50 per request.  Returns
    (pool of Workloads, requests as dicts with arrival time t, kind, pool
    index, precision, Philox seed and a uniform `pick` for the KDE target)."""
    rng = np.random.default_rng(seed)
    pool = []
    for k in range(64):
        n = int(round(math.exp(rng.uniform(math.log(2e3), math.log(2e5)))))
        pool.append(Workload(f"pool{k}-n{n}", n, 64, 3.0, depth_of(n), seed * 1000 + k, seed * 1000 + 500 + k,
                             20, (-10.0, 10.0), (0.5, 2.0)))
    t, reqs = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= seconds:
            break
        kind = "build" if rng.random() < 0.8 else "kde"
        prec = "bf16_split" if rng.random() < 0.5 else "plain_fp64"
        reqs.append({"t": t, "kind": kind, "pool": int(rng.integers(len(pool))), "prec": prec,
                     "seed": int(rng.integers(1 << 62)), "pick": float(rng.random())})
    return pool, reqs


def serving_queries(w: Workload, m: int = 10_000) -> np.ndarray:
    """The KDE query points of a serving request against pool set w: m fresh
    points of the set's mixture family (its own seed + 7)."""
    return mixture(m, w.d, w.n_comp, w.data_seed + 7, w.mean_range, w.std_range)


WORKLOADS = {"blobs2d-n1000": tiny_blobs, "mix32-n100k": mixture32, "mix64-n1m": mixture64}
