"""Seeded synthetic inputs shared by the tests and the benchmark.

This module holds workload shapes and numpy random generators only; it
contains none of the method's arithmetic, so the HIP path and the CPU oracle
can both be fed from it without sharing any code with each other.

The paper measures on the DTLZ suite, whose definitions it does not give.
The problems used here (ids 1..3) are this repository's own stand-ins of the
same shape (m objectives, d variables in [0,1], m-1 position variables and
d-m+1 distance variables); the problem id plays the role of the DTLZ
instance each workload names:
    1  linear front, multimodal distance term   (in place of DTLZ1)
    2  sphere front, unimodal distance term     (in place of DTLZ2)
    3  sphere front, multimodal distance term   (in place of DTLZ3)
"""
import numpy as np

LINEAR_MULTIMODAL = 1
SPHERE_UNIMODAL = 2
SPHERE_MULTIMODAL = 3

# Workloads of the paper's scale: name -> shape.  K = N = Das-Dennis count.
CONFIGS = {
    # 105 reference vectors (H=13, m=3), d=12, 100 generations
    "small_m3_d12_n105": dict(problem=SPHERE_UNIMODAL, m=3, d=12, H=13, N=105, K=105,
                              gens=100, seed=0),
    # headline: H=140 -> K=N=10,011, d=500, 100 generations
    "large_m3_d500_n10011": dict(problem=LINEAR_MULTIMODAL, m=3, d=500, H=140, N=10011,
                                 K=10011, gens=100, seed=0),
    # big population: H=446 -> K=N=100,128, d=5,000, 50 generations
    "big_m3_d5000_n100128": dict(problem=SPHERE_MULTIMODAL, m=3, d=5000, H=446, N=100128,
                                 K=100128, gens=50, seed=0),
}

# The paper's two scaling sweeps (its Tables 3 and 4, DTLZ1, m = 3, 100
# generations), each point a population size n and a dimension d.  Reading:
# the population is N = n individuals and the reference vectors are the
# smallest Das-Dennis lattice with at least n of them (K >= N, so every
# initial individual has a slot; empty slots take no part).
#   Series 1: d = 100, n = 2^5 .. 2^14;  Series 2: n = 100, d = 2^9 .. 2^18.
def lattice_count(H, m):
    from math import comb

    return comb(H + m - 1, m - 1)


def smallest_lattice_at_least(n, m):
    """(H, K): the fewest divisions H whose lattice count K = C(H+m-1, m-1) >= n."""
    H = 1
    while lattice_count(H, m) < n:
        H += 1
    return H, lattice_count(H, m)


def sweep_point(series, n, d, m=3, gens=100, seed=0):
    H, K = smallest_lattice_at_least(n, m)
    return dict(name=f"series{series}_m{m}_d{d}_n{n}", series=series, problem=LINEAR_MULTIMODAL,
                m=m, d=d, n=n, N=n, K=K, H=H, gens=gens, seed=seed)


SERIES1 = [sweep_point(1, 2 ** e, 100) for e in range(5, 15)]
SERIES2 = [sweep_point(2, 100, 2 ** e) for e in range(9, 19)]

# Neuroevolution-shaped workload: N = 4,096 policies (32 -> 64 -> 64 -> 8 tanh,
# d = 6,728 weights, second hidden layer without bias), m = 2, K = N (H = 4,095),
# E = 16 rollouts of T = 200 steps on the linear system of ``lq_system``.
POLICY_LQ = 100
POLICY_D = 6728
POLICY_CONFIG = dict(problem=POLICY_LQ, m=2, d=POLICY_D, H=4095, N=4096, K=4096, gens=50,
                     seed=0, E=16, T=200, sigma=0.1, lb=-1.0, ub=1.0)

DEFAULT_PARAMS = dict(alpha=2.0, fr=0.1, t_max=100, eta_c=20.0, eta_m=20.0, p_c=1.0,
                      p_m=1.0, lb=0.0, ub=1.0)


def rng(seed):
    return np.random.default_rng(np.uint64(seed))


def population(seed, K, d, lb=0.0, ub=1.0):
    """K x d float32 genes uniform in [lb, ub]."""
    r = rng(seed)
    return r.uniform(lb, ub, size=(K, d)).astype(np.float32)


def valid_mask(seed, K, frac_valid=1.0):
    """uint8 mask with about frac_valid of the K slots set (at least one)."""
    r = rng(seed)
    v = (r.random(K) < frac_valid).astype(np.uint8)
    if v.sum() == 0:
        v[r.integers(0, K)] = 1
    return v


def objectives(seed, M, m, radius=(0.5, 2.0), offset=0.0):
    """M x m float32 objective vectors: positive-orthant directions (|normal|)
    with radii uniform in ``radius``, shifted by ``offset``."""
    r = rng(seed)
    g = np.abs(r.standard_normal((M, m)))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    rad = r.uniform(radius[0], radius[1], size=(M, 1))
    return (g * rad + offset).astype(np.float32)


def gamma_like(seed, K, lo=0.02, hi=0.2):
    """Positive per-vector angles, for feeding selection in isolation."""
    return rng(seed).uniform(lo, hi, size=K)


def lq_system(seed, E=16, n=32, q=8, rho=0.95):
    """Stable linear system x' = A x + B u: A = rho G / spectral_radius(G) with
    G ~ N(0,1)^{n x n} (eigenvalues in binary64), B ~ N(0, 0.1^2)^{n x q},
    E start states x0 ~ N(0, I).  float32 arrays A (n x n), B (n x q), x0 (E x n)."""
    r = rng(seed)
    G = r.standard_normal((n, n))
    A = rho * G / np.max(np.abs(np.linalg.eigvals(G)))
    B = 0.1 * r.standard_normal((n, q))
    x0 = r.standard_normal((E, n))
    return dict(A=A.astype(np.float32), B=B.astype(np.float32), x0=x0.astype(np.float32))


def policy_population(seed, n, sigma=0.1, lb=-1.0, ub=1.0):
    """n x 6728 float32 policy weights N(0, sigma^2) clipped to [lb, ub]."""
    r = rng(seed)
    return np.clip(sigma * r.standard_normal((n, POLICY_D)), lb, ub).astype(np.float32)


def seeds(n, base=0):
    return [base + i for i in range(n)]


# Served workload: independent runs arriving as a Poisson stream.  Each draws
# its problem (the three stand-ins above, in place of DTLZ1-7), m from
# {2,3,5,8}, d uniform in [30, 2000] and the lattice divisions H uniformly
# over the values whose count C(H+m-1, m-1) lies in [100, 10011]; N = K.
SERVE_H_RANGE = {2: (99, 10010), 3: (13, 140), 5: (5, 19), 8: (3, 8)}


def serving_specs(n=256, rate=20.0, seed=0, gens=100):
    """List of dicts: rid, arrival (s), problem, m, d, N, K, seed, gens."""
    r = rng(seed)
    arrivals = np.cumsum(r.exponential(1.0 / rate, size=n)) if rate > 0 else np.zeros(n)
    out = []
    for i in range(n):
        m = int(r.choice([2, 3, 5, 8]))
        lo, hi = SERVE_H_RANGE[m]
        H = int(r.integers(lo, hi + 1))
        K = lattice_count(H, m)
        out.append(dict(rid=i, arrival=float(arrivals[i]), problem=int(r.integers(1, 4)), m=m,
                        d=int(r.integers(30, 2001)), N=K, K=K, seed=1000 + i, gens=gens))
    return out
