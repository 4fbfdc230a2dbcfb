"""ctypes + numpy front end of the FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It loads ``oracle/liboracle.so``
(compiled from ``rvea_oracle.c`` with gcc) and never touches the HIP library.
Every function here is argument marshalling; the arithmetic lives in the C
file, whose header cites the passages of the paper each step follows.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class OraParams(C.Structure):
    _fields_ = [
        ("alpha", C.c_double),
        ("fr", C.c_double),
        ("t_max", C.c_int32),
        ("pad_", C.c_int32),
        ("eta_c", C.c_double),
        ("eta_m", C.c_double),
        ("p_c", C.c_double),
        ("p_m", C.c_double),
        ("lb", C.c_double),
        ("ub", C.c_double),
        ("lq", C.c_void_p),
    ]


class OraOp(C.Structure):
    _fields_ = [("op", C.c_int32), ("pad_", C.c_int32), ("a", C.c_double), ("b", C.c_double)]


OP_GA, OP_DE, OP_PSO, OP_CSO, OP_RAND = 0, 1, 2, 3, 4


def op_params(op, a=0.0, b=0.0):
    """ora_op: DE (a = F, b = CR), PSO (a = w, b = c), CSO and random (unused)."""
    return OraOp(int(op), 0, float(a), float(b))


class OraLQ(C.Structure):
    _fields_ = [
        ("A", C.c_void_p),
        ("B", C.c_void_p),
        ("x0", C.c_void_p),
        ("E", C.c_int32),
        ("T", C.c_int32),
        ("sigma", C.c_double),
    ]


POLICY_LQ = 100


DEFAULTS = dict(alpha=2.0, fr=0.1, t_max=100, eta_c=20.0, eta_m=20.0, p_c=1.0, p_m=1.0,
                lb=0.0, ub=1.0)

TAG_INIT, TAG_MATE, TAG_SBX, TAG_SBXPAIR, TAG_MUT = 0, 1, 2, 3, 4


def params(lq=None, **kw):
    """ora_params; ``lq`` = dict(A, B, x0, T, sigma) for the policy problem."""
    d = dict(DEFAULTS)
    d.update(kw)
    p = OraParams(d["alpha"], d["fr"], int(d["t_max"]), 0, d["eta_c"], d["eta_m"],
                  d["p_c"], d["p_m"], d["lb"], d["ub"], None)
    if lq is not None:
        arrs = [_c(lq[k], np.float32) for k in ("A", "B", "x0")]
        sysd = OraLQ(_p(arrs[0]), _p(arrs[1]), _p(arrs[2]), arrs[2].shape[0], int(lq["T"]),
                     float(lq["sigma"]))
        p.lq = C.cast(C.pointer(sysd), C.c_void_p)
        p._keep = (arrs, sysd)  # the C side holds raw pointers into these
    return p


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        P = C.c_void_p
        i64, i32, f64 = C.c_int64, C.c_int, C.c_double
        u64 = C.c_uint64
        sig = {
            "ora_philox4x32_10": (None, [P, P, P]),
            "ora_binomial": (i64, [i64, i64]),
            "ora_lattice_count": (i64, [i32, i32]),
            "ora_lattice": (i64, [i32, i32, P, i64]),
            "ora_normalize_rows": (None, [P, i64, i32, P]),
            "ora_gamma": (None, [i64, i32, P, P]),
            "ora_evaluate_one": (i32, [i32, i32, i32, P, P]),
            "ora_evaluate": (i32, [i32, i32, i32, i64, P, i64, P]),
            "ora_front": (i64, [i32, i32, i32, P, i64]),
            "ora_igd": (f64, [P, i64, P, i64, i32]),
            "ora_init": (None, [u64, i64, i32, f64, f64, P, i64]),
            "ora_bf16": (f64, [f64]),
            "ora_policy_evaluate": (i32, [i64, P, i64, i32, i32, P, P, P, P]),
            "ora_init_gauss_rows": (None, [u64, P, i64, i32, f64, f64, f64, P, P]),
            "ora_init_rows": (None, [u64, P, i64, i32, f64, f64, P]),
            "ora_mate": (i64, [u64, i64, i64, i64, P, P]),
            "ora_sbx_beta": (f64, [f64, f64]),
            "ora_pm_delta": (f64, [f64, f64, f64, f64, f64]),
            "ora_mutation_sites": (i32, [u64, i64, i64, i32, f64, P, P, i32]),
            "ora_mutate_child": (None, [u64, i64, i64, i32, f64, f64, f64, f64, P]),
            "ora_reproduce": (i32, [P, u64, i64, i64, i64, i32, P, i64, P, P, i64, P]),
            "ora_gamma_rows": (None, [i64, i32, P, P, i64, P]),
            "ora_reproduce_pairs": (i32, [P, u64, i64, i64, i32, P, i64, P, P, i64, P, P]),
            "ora_assoc_rows": (None, [i32, i64, i64, i32, f64, P, i64, P, P, P, P, P, P]),
            "ora_select": (i32, [i32, i64, i64, i64, i32, f64, P, P, P, P, P, P, P, P, P]),
            "ora_adapt": (i32, [i64, i32, P, P, P, P]),
            "ora_adapt_period": (i32, [f64, i32]),
            "ora_generation": (i32, [P, i32, i32, i32, i64, i64, u64, i64, P, P, P, P, P, P,
                                     P, P, P, P, P]),
            "ora_run": (i32, [P, i32, i32, i32, i64, i64, u64, i32, P, P, P, P, P, P]),
            "ora_de_draws": (i32, [u64, i64, i64, i32, P, i64, P]),
            "ora_reproduce_op": (i32, [P, P, u64, i64, i64, i64, i32, i32, P, P, P, P, P, P]),
            "ora_generation_op": (i32, [P, P, i32, i32, i32, i64, i64, u64, i64, P, P, P, P, P,
                                        P, P, P, P, P, P, P]),
            "ora_hypervolume": (f64, [i32, i64, P, P, P, P]),
            "ora_expected_utility": (f64, [i32, i64, P, P, P, P, i64, P]),
            "ora_num_threads": (i32, []),
            "ora_set_num_threads": (None, [i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# --------------------------------------------------------------------------
def philox(ctr, key):
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().ora_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def binomial(n, k):
    return int(lib().ora_binomial(n, k))


def lattice_count(H, m):
    return int(lib().ora_lattice_count(H, m))


def lattice(H, m):
    K = lattice_count(H, m)
    W = np.zeros((K, m), np.float64)
    n = lib().ora_lattice(H, m, _p(W), K)
    assert n == K
    return W


def normalize_rows(W):
    W = _c(W, np.float64)
    V = np.zeros_like(W)
    lib().ora_normalize_rows(_p(W), W.shape[0], W.shape[1], _p(V))
    return V


def unit_vectors(H, m):
    return normalize_rows(lattice(H, m))


def lattice_H(K, m):
    """H with C(H+m-1, m-1) == K, or None."""
    h = 1
    while True:
        c = lattice_count(h, m)
        if c == K:
            return h
        if c > K or c <= 0:
            return None
        h += 1


def gamma(V):
    V = _c(V, np.float64)
    g = np.zeros(V.shape[0], np.float64)
    lib().ora_gamma(V.shape[0], V.shape[1], _p(V), _p(g))
    return g


def evaluate(problem, m, X):
    X = _c(X, np.float32)
    n, d = X.shape
    F = np.zeros((n, m), np.float64)
    rc = lib().ora_evaluate(problem, m, d, n, _p(X), d, _p(F))
    if rc != 0:
        raise ValueError("ora_evaluate rejected its arguments")
    return F


def front(problem, m, Hs):
    n = lattice_count(Hs, m)
    Fs = np.zeros((n, m), np.float64)
    assert lib().ora_front(problem, m, Hs, _p(Fs), n) == n
    return Fs


def front_H(m):
    """Lattice divisions for an IGD reference front of at least 5,000 points."""
    h = 1
    while lattice_count(h, m) < 5000:
        h += 1
    return h


def igd(F, Fs):
    F = _c(F, np.float64)
    Fs = _c(Fs, np.float64)
    return float(lib().ora_igd(_p(F), F.shape[0], _p(Fs), Fs.shape[0], F.shape[1]))


def init(seed, N, d, lb=0.0, ub=1.0):
    X = np.zeros((N, d), np.float32)
    lib().ora_init(seed, N, d, lb, ub, _p(X), d)
    return X


def bf16(x):
    return float(lib().ora_bf16(float(x)))


POLICY_D = 6728


def policy_evaluate(X, E, T, A, B, x0):
    """Objectives (n x 2) of policy genes X (n x 6728) on the linear system."""
    X = _c(X, np.float32)
    A = _c(A, np.float32)
    B = _c(B, np.float32)
    x0 = _c(x0, np.float32)
    assert X.shape[1] == POLICY_D and A.shape == (32, 32) and B.shape == (32, 8)
    assert x0.shape == (E, 32)
    F = np.zeros((X.shape[0], 2), np.float64)
    rc = lib().ora_policy_evaluate(X.shape[0], _p(X), X.shape[1], E, T, _p(A), _p(B), _p(x0),
                                   _p(F))
    if rc != 0:
        raise ValueError("ora_policy_evaluate rejected its arguments")
    return F


def init_gauss_rows(seed, rows, d, sigma=0.1, lb=-1.0, ub=1.0, with_pre=False):
    """Gaussian initial genes of individuals ``rows`` (len(rows) x d float32)."""
    rows = _c(rows, np.int64)
    X = np.zeros((len(rows), d), np.float32)
    pre = np.zeros((len(rows), d), np.float64) if with_pre else None
    lib().ora_init_gauss_rows(seed, _p(rows), len(rows), d, sigma, lb, ub, _p(X), _p(pre))
    return (X, pre) if with_pre else X


def init_rows(seed, rows, d, lb=0.0, ub=1.0):
    rows = _c(rows, np.int64)
    X = np.zeros((len(rows), d), np.float32)
    lib().ora_init_rows(seed, _p(rows), len(rows), d, lb, ub, _p(X))
    return X


def mate(seed, t, valid, N):
    valid = _c(valid, np.uint8)
    P = (N + 1) // 2
    parents = np.full((P, 2), -1, np.int32)
    nv = lib().ora_mate(seed, t, valid.shape[0], N, _p(valid), _p(parents))
    return parents, int(nv)


def sbx_beta(mc, eta=20.0):
    return float(lib().ora_sbx_beta(mc, eta))


def pm_delta(x, mm, lb=0.0, ub=1.0, xi=20.0):
    return float(lib().ora_pm_delta(x, lb, ub, mm, xi))


def mutation_sites(seed, t, o, d, p_m, cap=4096):
    sites = np.zeros(cap, np.int32)
    mags = np.zeros(cap, np.float64)
    n = lib().ora_mutation_sites(seed, t, o, d, p_m, _p(sites), _p(mags), cap)
    assert n <= cap
    return sites[:n].copy(), mags[:n].copy()


def mutate_child(seed, t, o, c, p_m=1.0, lb=0.0, ub=1.0, eta_m=20.0):
    c = np.array(c, np.float64)
    lib().ora_mutate_child(seed, t, o, c.shape[0], p_m, lb, ub, eta_m, _p(c))
    return c


def reproduce(prm, seed, t, X, parents, N, with_pre=False):
    """Offspring (N x d, float32) of the slot-ordered parents X (K x d)."""
    X = _c(X, np.float32)
    parents = _c(parents, np.int32)
    K, d = X.shape
    Xoff = np.zeros((N, d), np.float32)
    pre = np.zeros((N, d), np.float64) if with_pre else None
    rc = lib().ora_reproduce(C.byref(prm), seed, t, K, N, d, _p(X), d, _p(parents), _p(Xoff),
                             d, _p(pre))
    if rc != 0:
        raise ValueError("ora_reproduce failed")
    return (Xoff, pre) if with_pre else Xoff


def gamma_rows(V, rows):
    V = _c(V, np.float64)
    rows = _c(rows, np.int64)
    out = np.zeros(len(rows), np.float64)
    lib().ora_gamma_rows(V.shape[0], V.shape[1], _p(V), _p(rows), len(rows), _p(out))
    return out


def reproduce_pairs(prm, seed, t, X, parents, N, pairs):
    """Both children of the listed pair indices: (child1, child2), each n x d."""
    X = _c(X, np.float32)
    parents = _c(parents, np.int32)
    pairs = _c(pairs, np.int64)
    d = X.shape[1]
    o1 = np.zeros((len(pairs), d), np.float32)
    o2 = np.full((len(pairs), d), np.nan, np.float32)
    lib().ora_reproduce_pairs(C.byref(prm), seed, t, N, d, _p(X), d, _p(parents), _p(pairs),
                              len(pairs), _p(o1), _p(o2))
    return o1, o2


def assoc_rows(m, K, t, t_max, alpha, Frows, zstar, V, gam):
    """Association, angle and APD of the given objective rows (ideal point given)."""
    Frows = _c(Frows, np.float64)
    zstar = _c(zstar, np.float64)
    V = _c(V, np.float64)
    gam = _c(gam, np.float64)
    n = Frows.shape[0]
    assoc = np.zeros(n, np.int32)
    theta = np.zeros(n, np.float64)
    apd = np.zeros(n, np.float64)
    lib().ora_assoc_rows(m, K, t, t_max, alpha, _p(Frows), n, _p(zstar), _p(V), _p(gam),
                         _p(assoc), _p(theta), _p(apd))
    return assoc, theta, apd


def select(m, K, N, t, t_max, alpha, Fm, mvalid, V, gam):
    Fm = _c(Fm, np.float64)
    mvalid = _c(mvalid, np.uint8)
    V = _c(V, np.float64)
    gam = _c(gam, np.float64)
    M = K + N
    assert Fm.shape == (M, m) and mvalid.shape == (M,)
    zstar = np.zeros(m, np.float64)
    assoc = np.zeros(M, np.int32)
    theta = np.zeros(M, np.float64)
    apd = np.zeros(M, np.float64)
    surv = np.zeros(K, np.int32)
    rc = lib().ora_select(m, K, N, t, t_max, alpha, _p(Fm), _p(mvalid), _p(V), _p(gam),
                          _p(zstar), _p(assoc), _p(theta), _p(apd), _p(surv))
    if rc != 0:
        raise ValueError("ora_select failed")
    return dict(zstar=zstar, assoc=assoc, theta=theta, apd=apd, surv=surv)


def adapt(V0, F, valid, V):
    V0 = _c(V0, np.float64)
    F = _c(F, np.float64)
    valid = _c(valid, np.uint8)
    Vout = np.array(V, np.float64, copy=True)
    changed = lib().ora_adapt(V0.shape[0], V0.shape[1], _p(V0), _p(F), _p(valid), _p(Vout))
    return Vout, bool(changed)


def adapt_period(fr, t_max):
    return int(lib().ora_adapt_period(fr, t_max))


class State:
    """Slot-ordered run state: X (K x d f32), F (K x m f64), valid, V, V0, gamma."""

    def __init__(self, X, F, valid, V, V0, gamma):
        self.X = _c(X, np.float32).copy()
        self.F = _c(F, np.float64).copy()
        self.valid = _c(valid, np.uint8).copy()
        self.V = _c(V, np.float64).copy()
        self.V0 = _c(V0, np.float64).copy()
        self.gamma = _c(gamma, np.float64).copy()


def initial_state(problem, m, d, N, K, seed, lb=0.0, ub=1.0, lq=None):
    """``lq`` = dict(A, B, x0, T, sigma) for the policy problem."""
    H = lattice_H(K, m)
    if H is None:
        raise ValueError("K is not a Das-Dennis lattice count")
    V0 = unit_vectors(H, m)
    X = np.zeros((K, d), np.float32)
    F = np.full((K, m), np.nan)
    if problem == POLICY_LQ:
        X[:N] = init_gauss_rows(seed, np.arange(N), d, lq["sigma"], lb, ub)
        F[:N] = policy_evaluate(X[:N], lq["x0"].shape[0], lq["T"], lq["A"], lq["B"], lq["x0"])
    else:
        X[:N] = init(seed, N, d, lb, ub)
        F[:N] = evaluate(problem, m, X[:N])
    valid = np.zeros(K, np.uint8)
    valid[:N] = 1
    return State(X, F, valid, V0.copy(), V0, gamma(V0))


def generation(prm, problem, m, d, N, K, seed, t, st):
    """Advance ``st`` in place by generation t (1-based); returns the stage outputs."""
    P = (N + 1) // 2
    Xoff = np.zeros((N, d), np.float32)
    Foff = np.zeros((N, m), np.float64)
    parents = np.zeros((P, 2), np.int32)
    surv = np.zeros(K, np.int32)
    adapted = C.c_int(0)
    rc = lib().ora_generation(C.byref(prm), problem, m, d, N, K, seed, t, _p(st.X), _p(st.F),
                              _p(st.valid), _p(st.V), _p(st.V0), _p(st.gamma), _p(Xoff),
                              _p(Foff), _p(parents), _p(surv), C.byref(adapted))
    if rc != 0:
        raise RuntimeError(f"ora_generation failed ({rc})")
    return dict(Xoff=Xoff, Foff=Foff, parents=parents, surv=surv, adapted=bool(adapted.value))


def run(prm, problem, m, d, N, K, seed, gens):
    X = np.zeros((K, d), np.float32)
    F = np.zeros((K, m), np.float64)
    valid = np.zeros(K, np.uint8)
    V = np.zeros((K, m), np.float64)
    V0 = np.zeros((K, m), np.float64)
    g = np.zeros(K, np.float64)
    rc = lib().ora_run(C.byref(prm), problem, m, d, N, K, seed, gens, _p(X), _p(F), _p(valid),
                       _p(V), _p(V0), _p(g))
    if rc != 0:
        raise RuntimeError(f"ora_run failed ({rc})")
    return State(X, F, valid, V, V0, g)


def de_draws(seed, t, o, d, valid):
    """DE/rand/1/bin draws of child o: (target, r1, r2, r3, j_rand)."""
    P = _c(np.nonzero(_c(valid, np.uint8))[0], np.int32)
    out = np.zeros(5, np.int32)
    if lib().ora_de_draws(seed, t, o, d, _p(P), len(P), _p(out)) != 0:
        raise ValueError("no valid slot")
    return tuple(int(x) for x in out)


def reproduce_op(prm, op, seed, t, X, Vel, valid, F, N):
    """Offspring (N x d) and their velocities by operator ``op`` (op_params)
    from the slot-ordered population X (K x d), velocities Vel (K x d or
    None), valid flags and objectives F (K x m)."""
    X = _c(X, np.float32)
    K, d = X.shape
    F = _c(F, np.float64)
    m = F.shape[1]
    Vel = _c(np.zeros((K, d), np.float32) if Vel is None else Vel, np.float32)
    Xoff = np.zeros((N, d), np.float32)
    Voff = np.zeros((N, d), np.float32)
    rc = lib().ora_reproduce_op(C.byref(prm), C.byref(op), seed, t, K, N, d, m, _p(X), _p(Vel),
                                _p(_c(valid, np.uint8)), _p(F), _p(Xoff), _p(Voff))
    if rc != 0:
        raise ValueError(f"ora_reproduce_op failed ({rc})")
    return Xoff, Voff


def generation_op(prm, op, problem, m, d, N, K, seed, t, st, Vel):
    """Advance ``st`` (and the K x d slot velocities ``Vel``) in place by
    generation t with operator ``op``; returns the stage outputs."""
    Xoff = np.zeros((N, d), np.float32)
    Voff = np.zeros((N, d), np.float32)
    Foff = np.zeros((N, m), np.float64)
    surv = np.zeros(K, np.int32)
    adapted = C.c_int(0)
    rc = lib().ora_generation_op(C.byref(prm), C.byref(op), problem, m, d, N, K, seed, t,
                                 _p(st.X), _p(Vel), _p(st.F), _p(st.valid), _p(st.V), _p(st.V0),
                                 _p(st.gamma), _p(Xoff), _p(Voff), _p(Foff), _p(surv),
                                 C.byref(adapted))
    if rc != 0:
        raise RuntimeError(f"ora_generation_op failed ({rc})")
    return dict(Xoff=Xoff, Voff=Voff, Foff=Foff, surv=surv, adapted=bool(adapted.value))


def hypervolume(F, valid=None, lo=None, hi=None):
    """App. C.2 hypervolume (m = 2, 3) with reference point ones on the
    normalised objectives (F - lo) / (hi - lo); lo = 0, hi = 1 by default."""
    F = _c(F, np.float64)
    n, m = F.shape
    lo = _c(np.zeros(m) if lo is None else lo, np.float64)
    hi = _c(np.ones(m) if hi is None else hi, np.float64)
    v = None if valid is None else _c(valid, np.uint8)
    return float(lib().ora_hypervolume(m, n, _p(F), _p(v), _p(lo), _p(hi)))


def expected_utility(F, W, valid=None, lo=None, hi=None):
    """Mean over the weight rows W of the best utility -w . f' (f' as above)."""
    F = _c(F, np.float64)
    W = _c(W, np.float64)
    n, m = F.shape
    lo = _c(np.zeros(m) if lo is None else lo, np.float64)
    hi = _c(np.ones(m) if hi is None else hi, np.float64)
    v = None if valid is None else _c(valid, np.uint8)
    return float(lib().ora_expected_utility(m, n, _p(F), _p(v), _p(lo), _p(hi), W.shape[0],
                                            _p(W)))


def num_threads():
    return int(lib().ora_num_threads())


def set_num_threads(n):
    lib().ora_set_num_threads(int(n))
