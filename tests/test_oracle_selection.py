"""Pins of the oracle's selection (Alg. 1, Eqs. 2-5) and adaptation.

Selection is pinned against a brute force written from the definitions by a
different route (angles from 2*atan2(|a^-b^|, |a^+b^|), survivors by
sorting members on (APD, index)), against a hand-worked example, and by
invariances (translation, power-of-two scaling, permutation, masking).
"""
import math

import numpy as np
import pytest


def brute_select(m, K, N, t, t_max, alpha, Fm, mvalid, V, gam):
    M = K + N
    take = [bool(mvalid[i]) and bool(np.all(np.isfinite(Fm[i]))) for i in range(M)]
    z = np.min(Fm[np.array(take)], axis=0)
    assoc = [-1] * M
    apd = [math.inf] * M
    for i in range(M):
        if not take[i]:
            continue
        f = Fm[i] - z
        nf = math.sqrt(sum(x * x for x in f))
        if nf == 0.0:
            assoc[i], apd[i] = 0, 0.0
            continue
        best, bj = math.inf, -1
        for j in range(K):
            a = f / nf
            b = V[j] / math.sqrt(sum(x * x for x in V[j]))
            ang = 2.0 * math.atan2(np.linalg.norm(a - b), np.linalg.norm(a + b))
            if ang < best:
                best, bj = ang, j
        assoc[i] = bj
        apd[i] = (1.0 + m * (t / t_max) ** alpha * best / gam[bj]) * nf
    surv = [-1] * K
    for j in range(K):
        members = sorted((apd[i], i) for i in range(M) if assoc[i] == j)
        if members:
            surv[j] = members[0][1]
    return z, np.array(assoc), np.array(apd), np.array(surv)


def _random_case(seed, K_H=(4, 3), N=None, frac_valid=0.8):
    import oracle as O
    from workloads import objectives, valid_mask

    H, m = K_H
    V = O.unit_vectors(H, m)
    K = V.shape[0]
    N = K if N is None else N
    Fm = objectives(seed, K + N, m).astype(np.float64)
    mv = np.ones(K + N, np.uint8)
    mv[:K] = valid_mask(seed + 1, K, frac_valid)
    return m, K, N, Fm, mv, V, O.gamma(V)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shape", [(4, 3), (5, 2), (2, 4)])
def test_selection_matches_bruteforce(ora, seed, shape):
    m, K, N, Fm, mv, V, gam = _random_case(seed, shape)
    t, t_max = 1 + seed * 7, 50
    r = ora.select(m, K, N, t, t_max, 2.0, Fm, mv, V, gam)
    z, assoc, apd, surv = brute_select(m, K, N, t, t_max, 2.0, Fm, mv, V, gam)
    assert np.array_equal(r["zstar"], z)
    assert np.array_equal(r["assoc"], assoc)
    fin = np.isfinite(apd)
    assert np.allclose(r["apd"][fin], apd[fin], rtol=1e-12)
    assert np.array_equal(r["surv"], surv)


def test_hand_worked_example(ora):
    # V = {(1,0), (1,1)/sqrt2, (0,1)}: gamma = pi/4 for each
    s = 1 / math.sqrt(2)
    V = np.array([[1.0, 0.0], [s, s], [0.0, 1.0]])
    gam = ora.gamma(V)
    assert np.allclose(gam, math.pi / 4)
    # merged rows: three parents and one offspring
    Fm = np.array([[1.0, 1.0], [3.0, 1.0], [1.0, 4.0], [2.0, 1.5]])
    r = ora.select(2, 3, 1, 10, 10, 2.0, Fm, np.ones(4, np.uint8), V, gam)
    assert list(r["zstar"]) == [1.0, 1.0]
    # f' = (0,0) -> A=0, APD 0; (2,0) -> A=0, theta 0, APD 2; (0,3) -> A=2, APD 3
    # (1, 0.5): angle atan(1/2) to axis 0, pi/4 - atan(1/2) to the diagonal -> A=1
    th = math.pi / 4 - math.atan(0.5)
    want = [0.0, 2.0, 3.0, (1 + 2 * 1.0 * th / (math.pi / 4)) * math.hypot(1.0, 0.5)]
    assert list(r["assoc"]) == [0, 0, 2, 1]
    assert r["apd"] == pytest.approx(want, rel=1e-14)
    assert list(r["surv"]) == [0, 3, 2]
    # without penalty (t -> 0) APD is the norm of f'
    r0 = ora.select(2, 3, 1, 0, 10, 2.0, Fm, np.ones(4, np.uint8), V, gam)
    assert r0["apd"] == pytest.approx([0.0, 2.0, 3.0, math.hypot(1.0, 0.5)], rel=1e-15)


def test_selection_invariants_random(ora):
    for seed in range(4):
        m, K, N, Fm, mv, V, gam = _random_case(100 + seed, (13, 3), frac_valid=0.6)
        r = ora.select(m, K, N, 7, 100, 2.0, Fm, mv, V, gam)
        surv, assoc, apd = r["surv"], r["assoc"], r["apd"]
        took = set(np.nonzero(mv)[0].tolist())
        assert all(assoc[i] == -1 for i in range(K + N) if i not in took)
        for j in range(K):
            members = np.nonzero(assoc == j)[0]
            if len(members) == 0:
                assert surv[j] == -1
                continue
            s = surv[j]
            assert assoc[s] == j and apd[s] == apd[members].min()
            assert s == members[apd[members] == apd[s]].min()
        used = surv[surv >= 0]
        assert len(np.unique(used)) == len(used)


def test_translation_scaling_permutation(ora):
    m, K, N, Fm, mv, V, gam = _random_case(7, (13, 3))
    base = ora.select(m, K, N, 30, 100, 2.0, Fm, mv, V, gam)
    # power-of-two scaling is exact: APD scales, choices do not change
    sc = ora.select(m, K, N, 30, 100, 2.0, Fm * 4.0, mv, V, gam)
    assert np.array_equal(sc["assoc"], base["assoc"]) and np.array_equal(sc["surv"], base["surv"])
    fin = np.isfinite(base["apd"])
    assert np.array_equal(sc["apd"][fin], base["apd"][fin] * 4.0)
    # translation: z* absorbs it
    tr = ora.select(m, K, N, 30, 100, 2.0, Fm + 3.0, mv, V, gam)
    assert np.array_equal(tr["assoc"], base["assoc"]) and np.array_equal(tr["surv"], base["surv"])
    assert np.allclose(tr["apd"][fin], base["apd"][fin], rtol=1e-13)
    # permuting the offspring rows permutes the outputs
    perm = np.random.default_rng(0).permutation(N)
    Fp = Fm.copy()
    Fp[K:] = Fm[K:][perm]
    pr = ora.select(m, K, N, 30, 100, 2.0, Fp, mv, V, gam)
    assert np.array_equal(pr["assoc"][K:], base["assoc"][K:][perm])
    inv = np.empty(N, np.int64)
    inv[perm] = np.arange(N)
    mapped = np.array([s if s < K or s < 0 else K + inv[s - K] for s in base["surv"]])
    assert np.array_equal(pr["surv"], mapped)


def test_duplicates_nonfinite_and_masked_rows(ora):
    s = 1 / math.sqrt(2)
    V = np.array([[1.0, 0.0], [s, s], [0.0, 1.0]])
    gam = ora.gamma(V)
    Fm = np.array([[2.0, 1.0], [0.0, 5.0], [np.nan, 1.0], [2.0, 1.0], [5.0, 0.0], [-9, -9]])
    mv = np.array([1, 1, 1, 1, 1, 0], np.uint8)
    r = ora.select(2, 3, 3, 5, 10, 2.0, Fm, mv, V, gam)
    assert r["assoc"][2] == -1 and r["assoc"][5] == -1  # NaN row and masked row
    assert list(r["zstar"]) == [0.0, 0.0]  # masked row does not enter z*
    assert r["assoc"][0] == r["assoc"][3]
    assert r["surv"][r["assoc"][0]] == 0  # identical rows: the lower index wins


def test_zero_norm_row(ora):
    s = 1 / math.sqrt(2)
    V = np.array([[0.0, 1.0], [s, s], [1.0, 0.0]])
    Fm = np.array([[1.0, 1.0], [2.0, 3.0], [4.0, 1.0], [1.5, 1.5]])
    r = ora.select(2, 3, 1, 5, 10, 2.0, Fm, np.ones(4, np.uint8), V, ora.gamma(V))
    assert r["assoc"][0] == 0 and r["apd"][0] == 0.0 and r["theta"][0] == pytest.approx(math.pi / 2)


def test_adaptation(ora):
    V0 = ora.unit_vectors(13, 3)
    K = V0.shape[0]
    rng = np.random.default_rng(2)
    valid = np.ones(K, np.uint8)
    F = rng.uniform(0, 1, size=(K, 3))
    F[0], F[1] = [0, 0, 0], [1, 1, 1]  # ranges exactly 1 -> V = V0
    V, ch = ora.adapt(V0, F, valid, V0 * 0.0)
    assert ch and np.allclose(V, V0, atol=2e-16)
    # scaling objective 0 by 3: V_j ~ (3 v0_j0, v0_j1, v0_j2)
    F2 = F.copy()
    F2[:, 0] *= 3.0
    V, ch = ora.adapt(V0, F2, valid, V0)
    want = V0 * np.array([3.0, 1.0, 1.0])
    want /= np.linalg.norm(want, axis=1, keepdims=True)
    assert ch and np.allclose(V, want, atol=1e-15)
    assert np.allclose(np.linalg.norm(V, axis=1), 1.0, atol=4e-16)
    # an invalid slot does not enter the ranges
    F3 = F.copy()
    F3[5] = [50, 50, 50]
    v3 = valid.copy()
    v3[5] = 0
    V, _ = ora.adapt(V0, F3, v3, V0)
    assert np.allclose(V, V0, atol=2e-16)
    # a zero range leaves V unchanged
    F4 = F.copy()
    F4[:, 2] = 0.25
    Vin = V0 * 1.0
    V, ch = ora.adapt(V0, F4, valid, Vin)
    assert not ch and np.array_equal(V, Vin)


def test_adaptation_period(ora):
    assert ora.adapt_period(0.1, 100) == 10
    assert ora.adapt_period(0.1, 50) == 5
    assert ora.adapt_period(0.3, 10) == 3
    assert ora.adapt_period(1.0, 7) == 7
    assert ora.adapt_period(0.01, 10) == 1
    assert ora.adapt_period(0.25, 10) == 3
