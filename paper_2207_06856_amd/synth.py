"""Seeded synthetic workloads shaped like the paper's GP regression problems.

This module only draws random inputs; it holds none of the method's
arithmetic, and both the oracle-based tests and the device path take their
inputs from it.  The paper trains on standardised UCI regression sets with
RBF-ARD kernels (Sec. 6, Table 1; App. C); those sets are not available, so
each workload below is a synthetic stand-in with the same kind of shape.

Random generator: numpy ``Generator(PCG64(seed))`` with
seed = 20220 + 100 * workload + replicate unless a seed is passed.
Probe vectors are Rademacher (+-1), as used for Hutchinson estimates (Sec. 2.2).
"""

from dataclasses import dataclass, field

import numpy as np

RBF = 0
MATERN52 = 1


def rng_for(workload, replicate=0, seed=None):
    s = 20220 + 100 * workload + replicate if seed is None else seed
    return np.random.Generator(np.random.PCG64(s))


@dataclass
class Problem:
    """One GP solve: points X (n x d), right-hand sides B (n x R), hyperparameters."""
    X: np.ndarray
    B: np.ndarray
    kind: int
    lengthscale: np.ndarray
    outputscale: float
    noise: float
    name: str = ""
    extra: dict = field(default_factory=dict)

    def __post_init__(self):
        # hyperparameters are float32 values, exactly as the library receives them
        self.lengthscale = np.asarray(self.lengthscale, dtype=np.float32)
        self.outputscale = float(np.float32(self.outputscale))
        self.noise = float(np.float32(self.noise))

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]

    @property
    def r(self):
        return self.B.shape[1]


def rademacher(rng, n, m):
    return (rng.integers(0, 2, size=(n, m)) * 2 - 1).astype(np.float32)


def plain_solve(n=2000, replicate=0, seed=None):
    """Small plain solve: X ~ U[-1,1]^3, y = sin(3 x1) + cos(2 x2) + 0.1 eps,
    RBF l=0.5, a^2=1, s^2=0.01, one right-hand side."""
    g = rng_for(1, replicate, seed)
    X = g.uniform(-1.0, 1.0, size=(n, 3)).astype(np.float32)
    y = np.sin(3 * X[:, 0]) + np.cos(2 * X[:, 1]) + 0.1 * g.standard_normal(n)
    return Problem(X, y.astype(np.float32)[:, None], RBF, np.array([0.5], np.float32),
                   1.0, 0.01, name=f"plain_n{n}_d3_r1")


def mixed_precision(n=100_000, kind=MATERN52, replicate=0, seed=None, probes=15):
    """Mixed-precision solve: X ~ N(0, I)^8 column-standardised,
    y = sum_j sin(x_j)/sqrt(8) + 0.05 eps, RHS = [y, 15 Rademacher probes];
    l = 1, a^2 = 1, s^2 = 0.05 (Matern-5/2 or RBF)."""
    g = rng_for(2, replicate, seed)
    d = 8
    X = g.standard_normal((n, d))
    X = (X - X.mean(0)) / X.std(0)
    y = np.sin(X).sum(1) / np.sqrt(d) + 0.05 * g.standard_normal(n)
    B = np.concatenate([y[:, None], rademacher(g, n, probes)], axis=1).astype(np.float32)
    return Problem(X.astype(np.float32), B, kind, np.array([1.0], np.float32), 1.0, 0.05,
                   name=f"mixed_n{n}_d{d}_r{probes + 1}_{'matern52' if kind == MATERN52 else 'rbf'}")


def large_single(n=1_800_000, replicate=0, seed=None, probes=15, features=512):
    """Large problem: X ~ N(0, I)^11 with pairs (1,2), (3,4), (5,6) correlated at
    rho = 0.8; y = random-Fourier-feature function (512 features, lengthscale
    1.5) + 0.1 eps; RHS = [y, 15 probes]; RBF l=1.5, a^2=1, s^2=0.01."""
    g = rng_for(3, replicate, seed)
    d = 11
    X = g.standard_normal((n, d)).astype(np.float32)
    rho = np.float32(0.8)
    for i in (0, 2, 4):
        X[:, i + 1] = rho * X[:, i] + np.sqrt(np.float32(1) - rho * rho) * X[:, i + 1]
    W = g.standard_normal((features, d)).astype(np.float32)
    b = g.uniform(0, 2 * np.pi, features).astype(np.float32)
    a = g.standard_normal(features).astype(np.float32)
    y = np.empty(n, dtype=np.float32)
    step = 65536
    for s in range(0, n, step):
        ph = X[s:s + step] @ (W.T / np.float32(1.5)) + b
        y[s:s + step] = np.sqrt(2.0 / features) * (np.cos(ph) @ a)
    y += (0.1 * g.standard_normal(n)).astype(np.float32)
    B = np.concatenate([y[:, None], rademacher(g, n, probes)], axis=1).astype(np.float32)
    return Problem(X, B, RBF, np.array([1.5], np.float32), 1.0, 0.01,
                   name=f"large_n{n}_d{d}_r{probes + 1}_rbf")


def batched(nprob=256, replicate=0, seed=None, probes=7, kind=RBF, n_lo=500, n_hi=20_000):
    """Many independent problems: N log-uniform in [500, 20000], d uniform in
    {2..16}, X ~ N(0, I), y as in the mixed-precision workload with its own d,
    l log-uniform in [0.3, 3], s^2 uniform in [0.01, 0.1], a^2 = 1, RHS = [y, 7 probes]."""
    g = rng_for(4, replicate, seed)
    out = []
    for p in range(nprob):
        n = int(round(np.exp(g.uniform(np.log(n_lo), np.log(n_hi)))))
        d = int(g.integers(2, 17))
        X = g.standard_normal((n, d))
        y = np.sin(X).sum(1) / np.sqrt(d) + 0.05 * g.standard_normal(n)
        B = np.concatenate([y[:, None], rademacher(g, n, probes)], axis=1).astype(np.float32)
        ls = float(np.exp(g.uniform(np.log(0.3), np.log(3.0))))
        s2 = float(g.uniform(0.01, 0.1))
        out.append(Problem(X.astype(np.float32), B, kind, np.array([ls], np.float32), 1.0, s2,
                           name=f"batch{p}_n{n}_d{d}"))
    return out


def served_requests(count=10_000, replicate=0, seed=None, rate_hz=200.0,
                    n_lo=1_000, n_hi=200_000):
    """Request stream: Poisson arrivals at ``rate_hz``; N log-uniform in
    [1000, 200000], d uniform in {4..12}, R uniform in {1..32} (y plus R-1
    probes), RBF or Matern-5/2 and tolerance 1.0 or 0.1 with equal odds;
    l = 1, a^2 = 1, s^2 = 0.05.  Returns descriptors; ``materialise`` draws the
    arrays of one request from its own seed."""
    g = rng_for(5, replicate, seed)
    t = np.cumsum(g.exponential(1.0 / rate_hz, size=count))
    reqs = []
    for i in range(count):
        reqs.append(dict(
            arrival_s=float(t[i]),
            n=int(round(np.exp(g.uniform(np.log(n_lo), np.log(n_hi))))),
            d=int(g.integers(4, 13)),
            r=int(g.integers(1, 33)),
            kind=int(g.integers(0, 2)),
            tol=float([1.0, 0.1][int(g.integers(0, 2))]),
            seed=int(g.integers(0, 2 ** 31 - 1)),
        ))
    return reqs


def materialise(req):
    """Draw X, B of one served request (y as in the mixed-precision workload)."""
    g = np.random.Generator(np.random.PCG64(req["seed"]))
    n, d, r = req["n"], req["d"], req["r"]
    X = g.standard_normal((n, d))
    y = np.sin(X).sum(1) / np.sqrt(d) + 0.05 * g.standard_normal(n)
    B = np.concatenate([y[:, None], rademacher(g, n, r - 1)], axis=1).astype(np.float32)
    return Problem(X.astype(np.float32), B, req["kind"], np.array([1.0], np.float32), 1.0, 0.05,
                   name=f"req_n{n}_d{d}_r{r}")


def training(n=100_000, d=8, replicate=0, seed=None):
    """Hyperparameter-training data shaped like the paper's standardised UCI
    regressions (Sec. 6, Table 1): X ~ N(0, I)^d column-standardised,
    y = sum_j c_j sin(2 x_j) + 0.1 eps with relevance c_j = 1 / (1 + j)
    (later inputs matter less, so ARD lengthscales separate), then y
    standardised to mean 0 and variance 1.  Returns (X float32 n x d, y float32 n)."""
    g = rng_for(6, replicate, seed)
    X = g.standard_normal((n, d))
    X = (X - X.mean(0)) / X.std(0)
    c = 1.0 / (1.0 + np.arange(d))
    y = np.sin(2.0 * X) @ c + 0.1 * g.standard_normal(n)
    y = (y - y.mean()) / y.std()
    return X.astype(np.float32), y.astype(np.float32)


def compact_support(n=1_000_000, d=2, half_width=10.0, probes=15, replicate=0, seed=None):
    """Support-truncation workload (Sec. 4.1, Fig. 1 and Fig. 2c): points
    uniform in [-w, w]^d (w = 10, the Fig. 1 range, in d = 2), y = sin(x_1) +
    cos(x_2) + 0.1 eps, RHS = [y, 15 probes]; RBF l = 1, a^2 = 1, s^2 = 0.05.
    At l = 1 the binary16 support radius (6.0) covers about a fifth of the
    pairs, so about three quarters of the product is exact zeros."""
    g = rng_for(7, replicate, seed)
    X = g.uniform(-half_width, half_width, size=(n, d))
    y = np.sin(X[:, 0]) + (np.cos(X[:, 1]) if d > 1 else 0.0) + 0.1 * g.standard_normal(n)
    B = np.concatenate([y[:, None], rademacher(g, n, probes)], axis=1).astype(np.float32)
    return Problem(X.astype(np.float32), B, RBF, np.array([1.0], np.float32), 1.0, 0.05,
                   name=f"support_n{n}_d{d}_r{probes + 1}_rbf")


def random_points(n, d, seed, scale=1.0, dist="normal"):
    """Generic seeded inputs for parity tests."""
    g = np.random.Generator(np.random.PCG64(seed))
    if dist == "normal":
        return (scale * g.standard_normal((n, d))).astype(np.float32)
    return g.uniform(-scale, scale, size=(n, d)).astype(np.float32)


def random_rhs(n, r, seed, dist="normal"):
    g = np.random.Generator(np.random.PCG64(seed + 7919))
    if dist == "rademacher":
        return rademacher(g, n, r)
    return g.standard_normal((n, r)).astype(np.float32)
