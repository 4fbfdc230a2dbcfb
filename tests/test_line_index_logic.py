"""The two-objective line index's stopping rule, checked on the host.

The device's row walk (k_grid.hip, two objectives) scans the row's cell and
the cells on either side, then steps outward on a side while the binary64
cosine to that side's next cell boundary (moved outward by 1e-12 in u) plus
1e-12 is not below the best cosine found.  This test restates that walk in
numpy, with the same cell map, constants and binary64 bound, and a cosine
that differs from the device's only in the rounding of its fused
multiply-add (the walk and the brute force here share it), and checks
on random, adapted-looking, crowded and boundary-straddling vector and row
sets that the vector it finds is the brute-force argmax of the same binary64
cosines (largest value, lowest index on ties) for every row, or that the row
is sent to a full scan.  It pins the argument the device code relies on; the
GPU tests compare the device's results with a scan of all vectors.
"""
import numpy as np
import pytest

EPS_U, TAU, WALK = 1e-12, 1e-12, 64


def cell_of(x0, x1, r, G):
    a, b = x0 / r[0], x1 / r[1]
    s = a + b
    with np.errstate(divide="ignore", invalid="ignore"):
        u = b / s
    if not (a >= 0 and b >= 0 and s > 0 and np.isfinite(s) and 0 <= u <= 1):
        return -1
    return min(int(u * G), G - 1)


def cosine(f0, f1, nrm, v0, v1, vn):
    return (f0 * v0 + f1 * v1) / (nrm * vn)


def bound(f0, f1, nrm, u, r):
    b0, b1 = (1.0 - u) * r[0], u * r[1]
    return (f0 * b0 + f1 * b1) / (nrm * np.sqrt(b0 * b0 + b1 * b1))


def build(V, r, G):
    cells = [[] for _ in range(G)]
    for j, (v0, v1) in enumerate(V):
        c = cell_of(v0, v1, r, G)
        assert c >= 0
        cells[c].append(j)
    return cells


def walk(f, V, vn, r, G, cells, skip=None, nrm=None):
    """The row walk; with skip = i it is the gamma walk of vector i (itself
    and vectors at cosine 1 or more skipped, nrm = |v_i|)."""
    f0, f1 = f
    if nrm is None:
        nrm = np.sqrt(f0 * f0 + f1 * f1)
    c = cell_of(f0, f1, r, G)
    best, bj = -np.inf, len(V)

    def scan(cc):
        nonlocal best, bj
        for j in cells[cc]:
            if j == skip:
                continue
            cv = cosine(f0, f1, nrm, V[j, 0], V[j, 1], vn[j])
            if skip is not None and cv >= 1.0:
                continue
            if cv > best or (cv == best and j < bj):
                best, bj = cv, j

    scan(c)
    lo = hi = c
    steps = 0
    while lo > 0:
        if lo < c and bound(f0, f1, nrm, lo / G + EPS_U, r) + TAU < best:
            break
        lo -= 1
        scan(lo)
        steps += 1
        if steps > WALK:
            return None
    steps = 0
    while hi < G - 1:
        if hi > c and bound(f0, f1, nrm, (hi + 1) / G - EPS_U, r) + TAU < best:
            break
        hi += 1
        scan(hi)
        steps += 1
        if steps > WALK:
            return None
    return bj if skip is None else best


def brute(f, V, vn):
    f0, f1 = f
    nrm = np.sqrt(f0 * f0 + f1 * f1)
    cv = np.array([cosine(f0, f1, nrm, V[j, 0], V[j, 1], vn[j]) for j in range(len(V))])
    return int(np.flatnonzero(cv == cv.max())[0])


def lattice(H):
    w = np.stack([1.0 - np.arange(H + 1) / H, np.arange(H + 1) / H], 1)
    return w / np.linalg.norm(w, axis=1, keepdims=True)


def check(V, r, rows):
    G = len(V)
    vn = np.sqrt(V[:, 0] ** 2 + V[:, 1] ** 2)
    cells = build(V, r, G)
    full = 0
    for f in rows:
        got = walk(f, V, vn, r, G, cells)
        if got is None:
            full += 1
            continue
        assert got == brute(f, V, vn), (f, got)
    return full


@pytest.mark.parametrize("scale", [(1.0, 1.0), (30.0, 0.2), (1.0, 1e-6), (1e-3, 1.0)],
                         ids=["unit", "adapted", "extreme", "other-axis"])
def test_walk_finds_the_argmax_on_adapted_lattices(scale):
    rng = np.random.default_rng(0)
    V = lattice(199) * np.array(scale)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    r = np.array(scale) / max(scale)  # the index's scaling after that adaptation
    r = np.maximum(r, 1e-6)
    rows = rng.random((600, 2)) * np.array(scale)
    # rows exactly on vectors, on the cell boundaries and on the axes
    rows = np.concatenate([rows, V[::7] * 3.0, np.array([[1.0, 0.0], [0.0, 1.0]])])
    full = check(V, r, rows)
    if scale[1] >= 1e-3:
        assert full == 0
    # at a 1 : 1e-6 range the neighbouring vectors are ~1e-8 rad apart, so
    # their binary64 cosines are not separable (1 - cos ~ 1e-16): rows
    # near that axis fall back to the full scan, which is exact


def test_walk_with_an_unscaled_line_and_skewed_vectors():
    """Vectors adapted while the line still has unit scaling (a host-set V):
    cells are uneven, rows far from the vectors walk many cells or fall back
    to a full scan, and every row that does not fall back is exact."""
    rng = np.random.default_rng(1)
    V = lattice(300) * np.array([1.0, 1e-3])
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    rows = rng.random((400, 2))
    full = check(V, np.array([1.0, 1.0]), rows)
    assert 0 < full < len(rows)


def test_walk_with_duplicates_and_random_vectors():
    rng = np.random.default_rng(2)
    V = rng.random((150, 2))
    V = np.concatenate([V, V[:20]])  # exact duplicates: ties go to the lower index
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    rows = np.concatenate([rng.random((500, 2)), V[:40] * 2.0])
    assert check(V, np.array([1.0, 1.0]), rows) == 0


def test_walk_with_tiny_lines():
    for H in (1, 2, 3):
        V = lattice(H)
        rows = np.random.default_rng(H).random((100, 2))
        assert check(V, np.array([1.0, 1.0]), rows) == 0


@pytest.mark.parametrize("scale", [(1.0, 1.0), (30.0, 0.2)], ids=["unit", "adapted"])
def test_gamma_walk_finds_the_nearest_other_vector(scale):
    """Eq. 5's gamma on the line: each vector walks as a row, skipping itself
    and exactly parallel vectors; the largest cosine equals the brute-force
    one over all other vectors (duplicates included in the set)."""
    V = lattice(150) * np.array(scale)
    V = np.concatenate([V, V[10:13]])  # exact duplicates
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    r = np.maximum(np.array(scale) / max(scale), 1e-6)
    G = len(V)
    vn = np.sqrt(V[:, 0] ** 2 + V[:, 1] ** 2)
    cells = build(V, r, G)
    for i in range(len(V)):
        got = walk(V[i], V, vn, r, G, cells, skip=i, nrm=vn[i])
        cv = np.array([cosine(V[i, 0], V[i, 1], vn[i], V[j, 0], V[j, 1], vn[j])
                       for j in range(len(V))])
        cv[i] = -np.inf
        cv[cv >= 1.0] = -np.inf
        assert got is not None and got == cv.max(), i
