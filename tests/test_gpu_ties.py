"""Ties and degenerate rows of the selection (Alg. 1) against the oracle.

Forced through rvea_set_state, each case is one generation compared with the
oracle stage by stage, plus explicit checks of the rule it exercises:
  - objective rows duplicated between parents and offspring: equal APDs go to
    the lower merged index, so no offspring survives (the device compares a
    packed (APD, row) word whose lowest bits hold the row);
  - rows equal to the ideal point: association to vector 0, APD 0, the lowest
    such row survives;
  - rows whose two best vectors are mirror images across a 32-vector tile or
    chunk boundary, or inside one tile: identical association to the oracle's
    (lowest vector index on exact cosine ties).
"""
import numpy as np
import pytest

from parity import lockstep, new_stats

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


@pytest.mark.parametrize("case", [(2, 3, 12, 105, 105, 31), (1, 2, 20, 64, 64, 32),
                                  (3, 5, 40, 126, 126, 33)])
def test_duplicates_across_parents_and_offspring(P, O, case):
    """With p_c = 0 and p_m = 0 every child copies a parent's genes.  Each
    parent slot is given the objectives its copies get from the offspring
    evaluation, and the generation is replayed from that state: every child
    then duplicates a parent's objective row bit for bit, and every survivor
    must be a parent (the lower merged index)."""
    problem, m, d, N, K, seed = case
    prm = P.default_params(t_max=20, p_c=0.0, p_m=0.0)
    run = P.Run(problem, m, d, N, K, seed=seed, params=prm)
    st = run.get_state()
    run.step()
    off = run.get_offspring()
    half = (N + 1) // 2
    src = np.array([off["parents"][o, 0] if o < half else off["parents"][o - half, 1]
                    for o in range(N)])
    assert np.array_equal(off["X"], st["X"][src]), "children are not copies"
    run.select()
    run.adapt()
    F = st["F"].copy()
    F[src] = off["F"]
    run.set_state(st["X"], F, st["valid"], V=st["V"], gamma=st["gamma"], t=0)
    stats = lockstep(O, run, prm, 1, new_stats(), exact_survivors=True)
    off2 = run.get_offspring()
    assert np.array_equal(off2["parents"], off["parents"])
    assert np.array_equal(off2["F"].view(np.uint32), F[src].view(np.uint32)), \
        "replayed children do not duplicate their parents' objectives"
    sel = run.get_selection()
    s = sel["surv"]
    assert np.all(s < K), f"offspring survived a tie with its parent: {s[s >= K][:8]}"
    assert np.all(sel["apd"][K:] == sel["apd"][src])
    assert stats["near_ties"] == 0
    run.close()


def test_rows_at_the_ideal_point(P, O):
    """Two parent rows equal to each other and below every other row in all
    objectives are the ideal point: translated they are zero, go to vector 0
    with APD 0, and the lower of the two survives there."""
    problem, m, d, N, K = 2, 3, 12, 105, 105
    prm = P.default_params()
    run = P.Run(problem, m, d, N, K, seed=41, params=prm)
    st = run.get_state()
    F = st["F"].copy()
    F[[40, 7]] = -1.0
    run.set_state(st["X"], F, st["valid"], t=0)
    lockstep(O, run, prm, 1, new_stats(), exact_survivors=True)
    sel = run.get_selection()
    assert np.array_equal(sel["zstar"], np.full(m, -1.0, np.float32))
    assert sel["assoc"][7] == 0 and sel["assoc"][40] == 0
    assert sel["apd"][7] == 0.0 and sel["apd"][40] == 0.0
    assert sel["surv"][0] == 7
    assert np.all(sel["apd"][np.isfinite(sel["apd"])] >= 0.0)
    run.close()


@pytest.mark.parametrize("K,tune", [(64, False), (80, False), (4096, False), (4096, True),
                                    (1026, True)])
def test_mirror_ties_across_tiles(P, O, K, tune):
    """m = 2: vectors j and K-1-j are mirror images, so the middle pair
    (K/2-1, K/2) straddles a 32-vector tile boundary for K = 64 and 4096
    (and a chunk boundary for the shorter chunks) and sits inside one tile
    for K = 80.  Rows along (1, 1) scaled by powers of two have bitwise equal
    dot products with the two; with the ideal point pinned at 0 each must get
    the oracle's association, one of the middle pair, and the oracle's
    survivors."""
    problem, m, d, N = 2, 2, 12, K
    prm = P.default_params(t_max=40)
    run = P.Run(problem, m, d, N, K, seed=43, params=prm)
    st = run.get_state()
    F = st["F"].copy()
    assert np.all(F[st["valid"] == 1] >= 0)
    F[0] = (0.0, 3.0)
    F[1] = (3.0, 0.0)
    rows = np.arange(2, 12)
    F[rows] = np.ldexp(1.0, (rows % 5) - 2)[:, None]
    F[12] = F[13] = (0.5, 0.5)
    run.set_state(st["X"], F, st["valid"], t=5)
    if tune:
        t = run.autotune()
        print(f"K={K}: chunk {t['chunk_vectors']}, rows per lane {t['rows_per_lane']}")
    stats = lockstep(O, run, prm, 1, new_stats())
    sel = run.get_selection()
    assert np.array_equal(sel["zstar"], np.zeros(m, np.float32))
    a = sel["assoc"][2:14]
    assert np.all(a == a[0]) and a[0] in (K // 2 - 1, K // 2), a
    assert stats["near_ties"] <= 1, stats
    run.close()
