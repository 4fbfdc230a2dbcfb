"""Quality indicators on the device against the oracle: the hypervolume of
App. C.2 (reference point ones on normalised objectives, m = 2 and 3) and
the expected utility over a weight set.

Both sides read the same binary32 objective rows and normalise them in
binary64 with the same operations.  The hypervolume is a sum of
non-negative binary64 terms on both sides, taken in different orders, so
they agree to a relative 8 n 2^-53 (n rows); the expected utility's best
utility per weight is the same fma chain on both sides, and only the mean's
summation order differs (relative 1e-13)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2404_01159_amd as P

    return P


@pytest.fixture(scope="module")
def O():
    import oracle as O

    O.lib()
    return O


def hv_tol(n):
    return max(1e-13, 8 * max(n, 1) * 2.0 ** -53)


def random_rows(rng, n, m, kind):
    F = rng.random((n, m)).astype(np.float32)
    valid = (rng.random(n) < 0.9).astype(np.uint8)
    if kind == "ties":  # coordinates on a coarse grid: equal x, y and z values
        F = (np.round(F * 8) / 8).astype(np.float32)
    elif kind == "dups":  # whole rows repeated
        F[n // 2:2 * (n // 2)] = F[:n // 2]
    elif kind == "outside":  # rows at or beyond the reference point, non-finite rows
        F[rng.random(n) < 0.15] *= 1.6
        F[rng.random(n) < 0.05, 0] = 1.0
        F[rng.random(n) < 0.05, m - 1] = np.nan
        F[rng.random(n) < 0.03, 0] = np.inf
    elif kind == "shifted":  # objectives outside [0, 1], normalised by lo / hi
        F = (F * 7.0 - 2.0).astype(np.float32)
    return F, valid


@pytest.mark.parametrize("m", [2, 3])
@pytest.mark.parametrize("n", [1, 7, 64, 65, 1000, 4097])
@pytest.mark.parametrize("kind", ["plain", "ties", "dups", "outside", "shifted"])
def test_hypervolume_matches_oracle(P, O, m, n, kind):
    rng = np.random.default_rng(1000 * m + n + len(kind))
    F, valid = random_rows(rng, n, m, kind)
    lo = hi = None
    if kind == "shifted":
        lo, hi = np.full(m, -2.5), np.linspace(4.0, 5.5, m)
    got = P.hypervolume(F, valid, lo, hi)
    want = O.hypervolume(F.astype(np.float64), valid, lo, hi)
    assert abs(got - want) <= hv_tol(n) * abs(want) + 1e-300, (got, want)
    got_all = P.hypervolume(F, None, lo, hi)
    want_all = O.hypervolume(F.astype(np.float64), None, lo, hi)
    assert abs(got_all - want_all) <= hv_tol(n) * abs(want_all) + 1e-300


def test_hypervolume_edge_cases(P, O):
    # nothing counts: no rows, no valid rows, every row outside the box
    assert P.hypervolume(np.zeros((0, 3), np.float32)) == 0.0
    F = np.random.default_rng(0).random((50, 2)).astype(np.float32)
    assert P.hypervolume(F, np.zeros(50, np.uint8)) == 0.0
    assert P.hypervolume(F + 1.0) == 0.0
    # one box and the front sample of the sphere problems' front
    assert P.hypervolume(np.array([[0.25, 0.5, 0.75]], np.float32)) == 0.75 * 0.5 * 0.25
    Fs = O.front(2, 3, 30).astype(np.float32)
    want = O.hypervolume(Fs.astype(np.float64))
    assert abs(P.hypervolume(Fs) - want) <= hv_tol(len(Fs)) * want
    from paper_2404_01159_amd.rvea import RveaError

    with pytest.raises(RveaError):
        P.hypervolume(np.zeros((4, 4), np.float32))  # m = 4
    with pytest.raises(RveaError):
        P.hypervolume(F, lo=np.ones(2), hi=np.ones(2))  # empty range


def test_hypervolume_of_final_populations(P, O):
    """The 105-vector workload after 100 generations (m = 3, objectives taken
    as they are) and a 4,096-vector m = 2 run after 30 generations (still far
    from its front: normalised by lo = 0 and hi = 1.1 times the survivors'
    largest values): the device's value of the run's final survivors equals
    the oracle's."""
    for (problem, m, d, N, K, gens) in [(2, 3, 12, 105, 105, 100), (3, 2, 30, 4096, 4096, 30)]:
        run = P.Run(problem, m, d, N, K, seed=5, params=P.default_params(t_max=gens))
        run.run(gens)
        st = run.get_state(genes=False)
        run.close()
        lo = hi = None
        if problem == 3:
            lo = np.zeros(m)
            hi = 1.1 * st["F"][st["valid"] == 1].astype(np.float64).max(axis=0)
        got = P.hypervolume(st["F"], st["valid"], lo, hi)
        want = O.hypervolume(st["F"].astype(np.float64), st["valid"], lo, hi)
        assert want > 0 and abs(got - want) <= hv_tol(K) * want, (problem, got, want)
        print(f"problem {problem}, K={K}: HV {got:.10f} (oracle {want:.10f})")


def simplex_weights(O, H, m):
    V = O.unit_vectors(H, m)
    return V / V.sum(axis=1, keepdims=True)


@pytest.mark.parametrize("m,n,H", [(2, 1, 9), (2, 300, 99), (3, 1000, 13), (5, 257, 4),
                                   (8, 64, 2)])
def test_expected_utility_matches_oracle(P, O, m, n, H):
    rng = np.random.default_rng(n + m)
    F, valid = random_rows(rng, n, m, "shifted" if m == 3 else "outside")
    lo, hi = np.full(m, -2.5), np.full(m, 5.0)
    W = simplex_weights(O, H, m)
    got = P.expected_utility(F, W, valid, lo, hi)
    want = O.expected_utility(F.astype(np.float64), W, valid, lo, hi)
    assert abs(got - want) <= 1e-13 * abs(want), (got, want)


def test_expected_utility_closed_forms(P, O):
    rng = np.random.default_rng(3)
    F = rng.random((500, 3)).astype(np.float32)
    # one-hot weights: the mean over objectives of the negated smallest value
    got = P.expected_utility(F, np.eye(3))
    want = -np.mean(F.astype(np.float64).min(axis=0))
    assert abs(got - want) <= 1e-15 * abs(want)
    # no row counts: -inf
    assert P.expected_utility(F, np.eye(3), np.zeros(500, np.uint8)) == -np.inf
    assert P.expected_utility(np.zeros((0, 3), np.float32), np.eye(3)) == -np.inf
