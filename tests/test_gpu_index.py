"""The indexed association (the grid for three objectives, the line for
two) against the full scan through the C ABI: the same association, APD (bit for bit) and survivors every
generation, adaptations included, at small shapes, at the 10,011-vector
shape, after a host-set V whose index is unscaled, inside a batch (whose
phases keep the index rebuilt as each run adapts) and after a run leaves the
batch.  Both paths are
also checked against the oracle by the other GPU tests (the index is the
default for m = 3)."""
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


def same_selection(a, b, t):
    sa, sb = a.get_selection(), b.get_selection()
    for k in ("zstar", "assoc", "surv"):
        assert np.array_equal(sa[k], sb[k]), f"{k} differs at t={t}"
    assert np.array_equal(sa["apd"].view(np.uint64), sb["apd"].view(np.uint64)), \
        f"apd differs at t={t}"


def twin(P, problem, m, d, N, K, seed, t_max):
    prm = P.default_params(t_max=t_max)
    a = P.Run(problem, m, d, N, K, seed=seed, params=prm)
    b = P.Run(problem, m, d, N, K, seed=seed, params=prm)
    b.set_index(False)
    return a, b


def lock(a, b, gens):
    for _ in range(gens):
        a.step()
        b.step()
        a.select()
        b.select()
        same_selection(a, b, a.counters()["generations"])
        a.adapt()
        b.adapt()
    sa, sb = a.get_state(), b.get_state()
    for k in ("X", "F", "valid", "V", "gamma"):
        assert np.array_equal(sa[k], sb[k], equal_nan=True), k


@pytest.mark.parametrize("case", [(1, 3, 30, 105, 105, 25, 30), (2, 3, 12, 40, 55, 25, 20),
                                  (3, 3, 64, 300, 351, 21, 20), (1, 3, 10, 3, 3, 12, 10),
                                  (1, 2, 30, 100, 100, 25, 30), (2, 2, 31, 60, 64, 25, 20),
                                  (3, 2, 64, 300, 301, 21, 20), (1, 2, 10, 3, 3, 12, 10),
                                  (2, 2, 20, 2, 2, 8, 10)],
                         ids=lambda c: "p%d_m%d_d%d_N%d_K%d" % (c[0], c[1], c[2], c[3], c[4]))
def test_index_matches_full_scan(P, case):
    problem, m, d, N, K, gens, t_max = case
    print(f"index vs scan {case}", flush=True)
    a, b = twin(P, problem, m, d, N, K, 7, t_max)
    lock(a, b, gens)
    assert a.counters()["full_rescans"] == 0
    a.close()
    b.close()


def test_index_matches_full_scan_headline(P):
    print("index vs scan at 10,011 vectors", flush=True)
    a, b = twin(P, 1, 3, 500, 10011, 10011, 3, 100)
    lock(a, b, 12)  # one adaptation (generation 10)
    assert a.counters()["full_rescans"] == 0
    a.close()
    b.close()


def test_line_index_matches_full_scan_10000_vectors(P):
    print("line index vs scan at 10,000 vectors", flush=True)
    a, b = twin(P, 1, 2, 100, 10000, 10000, 3, 100)
    lock(a, b, 12)  # one adaptation (generation 10)
    assert a.counters()["full_rescans"] == 0
    a.close()
    b.close()


def test_line_index_after_host_set_vectors(P):
    # an adapted-looking V set from the host: the line is rebuilt unscaled
    import oracle as O

    a, b = twin(P, 2, 2, 20, 200, 200, 11, 40)
    st = a.get_state()
    V = O.unit_vectors(O.lattice_H(200, 2), 2) * np.array([30.0, 0.2])
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = st["F"] * np.array([30.0, 0.2], np.float32)
    for r in (a, b):
        r.set_state(st["X"], F, st["valid"], V=V, t=0)
    lock(a, b, 9)
    a.close()
    b.close()


def test_line_walk_limit_and_outside_vectors_fall_back(P):
    """Two objectives: vectors crowded near one axis (1 : 1e-3, set from the
    host, so the line is unscaled) while the rows spread over the quadrant,
    so most rows step past the walk limit and scan all vectors; then a V with
    one vector outside the quadrant, which the line leaves out, so every row
    scans.  The selection equals the full-scan run's throughout (counted
    rescans)."""
    import oracle as O

    a, b = twin(P, 1, 2, 16, 300, 301, 9, 50)
    st = a.get_state()
    V = O.unit_vectors(O.lattice_H(301, 2), 2) * np.array([1.0, 1e-3])
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    for r in (a, b):
        r.set_state(st["X"], st["F"], st["valid"], V=V, t=1)
    lock(a, b, 2)
    n1 = a.counters()["full_rescans"]
    assert n1 > 0
    V2 = O.unit_vectors(O.lattice_H(301, 2), 2)
    V2[7] = np.array([-0.6, 0.8])
    st = a.get_state()
    for r in (a, b):
        r.set_state(st["X"], st["F"], st["valid"], V=V2, t=1)
    a.step()
    b.step()
    a.select()
    b.select()
    same_selection(a, b, 2)
    assert a.counters()["full_rescans"] - n1 >= 300
    a.close()
    b.close()


def test_index_after_host_set_vectors(P):
    # an adapted-looking V set from the host: the index is rebuilt unscaled
    import oracle as O

    a, b = twin(P, 2, 3, 20, 200, 231, 11, 40)
    st = a.get_state()
    V = O.unit_vectors(O.lattice_H(231, 3), 3) * np.array([30.0, 1.0, 0.2])
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = st["F"] * np.array([30.0, 1.0, 0.2], np.float32)
    for r in (a, b):
        r.set_state(st["X"], F, st["valid"], V=V, t=0)
    lock(a, b, 9)
    a.close()
    b.close()


def test_index_rebuilt_after_a_batch(P):
    prm = P.default_params(t_max=20)
    a = P.Run(1, 3, 40, 105, 105, seed=5, params=prm)
    b = P.Run(1, 3, 40, 105, 105, seed=5, params=prm)
    for _ in range(3):
        a.generation()
        b.generation()
    bt = P.Batch(2)
    bt.admit(a)
    bt.step(8)  # adaptations at 4 and 8 in the batch
    bt.retire(a)
    bt.close()
    for _ in range(8):
        b.generation()
    lock(a, b, 6)
    a.close()
    b.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_index_in_a_batch_matches_full_scan(P, graphs):
    """Indexed and full-scan twins advanced in one batch (with other runs of
    other objective counts): the same selection every tick, adaptations
    included, and the same state at the end."""
    specs = [(1, 3, 40, 105, 105, 3, 20), (3, 3, 64, 300, 351, 4, 20),
             (1, 3, 500, 10011, 10011, 5, 100), (2, 3, 12, 40, 55, 6, 12),
             (2, 2, 31, 60, 64, 7, 20), (1, 2, 300, 2000, 2000, 8, 100)]
    others = [P.Run(1, 8, 31, 60, 120, seed=2, params=P.default_params(t_max=20)),
              P.Run(3, 5, 130, 126, 126, seed=3, params=P.default_params(t_max=20))]
    pairs = [twin(P, pb, m, d, N, K, seed, tm) for pb, m, d, N, K, seed, tm in specs]
    bt = P.Batch(16)
    bt.set_graphs(graphs)
    for a, b in pairs:
        bt.admit(a)
        bt.admit(b)
    for r in others:
        bt.admit(r)
    for t in range(12):  # adaptations at 2, 4, ... for t_max 20; at 10 for t_max 100
        print(f"batched index vs scan, tick {t}", flush=True)
        bt.step()
        for a, b in pairs:
            same_selection(a, b, t)
    bt.synchronize()
    for a, b in pairs:
        sa, sb = a.get_state(), b.get_state()
        for k in ("X", "F", "valid", "V", "gamma"):
            assert np.array_equal(sa[k], sb[k], equal_nan=True), k
        assert a.indexed and not b.indexed
        assert a.counters()["full_rescans"] == 0
    for a, b in pairs:
        bt.retire(a)
        bt.retire(b)
    for r in others:
        bt.retire(r)
    bt.close()
    for a, b in pairs:
        lock(a, b, 3)  # the index is current after the batch
        a.close()
        b.close()
    for r in others:
        r.close()


def test_index_switch_and_rejections(P):
    a = P.Run(1, 3, 20, 105, 105, seed=1)
    a.set_index(False)
    a.set_index(True)
    a.generation()
    p2 = P.Run(1, 5, 20, 10, 15, seed=1)
    with pytest.raises(P.RveaError):
        p2.set_index(True)
    p2.set_index(False)
    p3 = P.Run(1, 2, 20, 10, 10, seed=1)
    assert p3.indexed
    p3.set_index(False)
    p3.set_index(True)
    p3.generation()
    p3.close()
    a.step()
    with pytest.raises(P.RveaError):
        a.set_index(False)  # between step and select
    a.close()
    p2.close()


def test_index_crowded_vectors_fall_back_to_full_scans(P):
    """Vectors crowded far below the grid's resolution (axis ranges
    1 : 1e-3 : 1e-3 set from the host, so the index is unscaled): the crowded
    cells' lists overflow or their boxes pass the staged neighbourhood, their
    rows take the exact full scan (counted), gamma falls back to the full
    pass, and every generation still equals the full-scan run; one generation
    is also checked against the oracle."""
    import oracle as O
    from parity import lockstep, new_stats

    a, b = twin(P, 2, 3, 12, 300, 351, 5, 50)
    st = a.get_state()
    scale = np.array([1.0, 1e-3, 1e-3])
    V = O.unit_vectors(O.lattice_H(351, 3), 3) * scale
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = st["F"] * scale.astype(np.float32)
    for r in (a, b):
        r.set_state(st["X"], F, st["valid"], V=V, t=2)
    assert np.array_equal(a.get_state()["gamma"], b.get_state()["gamma"])
    lock(a, b, 3)
    assert a.counters()["full_rescans"] > 0
    prm = P.default_params(t_max=50)
    stats = lockstep(O, a, prm, 1, new_stats())
    assert stats["near_ties"] <= max(1, 1e-4 * stats["vectors"]), stats
    a.close()
    b.close()
