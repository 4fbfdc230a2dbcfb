"""Python binding of librvea.so (include/rvea.h).

Argument marshalling only: every step of a generation runs in the library's
HIP kernels.  PyTorch supplies the device workspace (a uint8 tensor whose
data pointer is handed to rvea_create) and the HIP stream.  There is no
fallback: if the library is missing or fails to load, importing this module
raises.
"""
import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  -- load torch's HIP runtime first: librvea.so binds to it


_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librvea.so")

RVEA_OK, RVEA_EINVAL, RVEA_ENOMEM, RVEA_EDEVICE, RVEA_ESTATE, RVEA_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
LINEAR_MULTIMODAL, SPHERE_UNIMODAL, SPHERE_MULTIMODAL = 1, 2, 3
POLICY_LQ, POLICY_M, POLICY_D, POLICY_E = 100, 2, 6728, 16
KERNEL_OFFSPRING, KERNEL_ASSOC, KERNEL_RERANK, KERNEL_GAMMA, KERNEL_ROLLOUT = 0, 1, 2, 3, 4
OP_GA, OP_DE, OP_PSO, OP_CSO, OP_RAND = 0, 1, 2, 3, 4
OPERATORS = {"ga": OP_GA, "de": OP_DE, "pso": OP_PSO, "cso": OP_CSO, "rand": OP_RAND}

EXPORTS = [
    "rvea_default_params", "rvea_lattice_divisions", "rvea_footprint", "rvea_create",
    "rvea_create_policy",
    "rvea_step", "rvea_select", "rvea_adapt", "rvea_run_generations",
    "rvea_prepare_generations", "rvea_set_graphs", "rvea_set_index",
    "rvea_get_state",
    "rvea_set_state", "rvea_get_offspring", "rvea_get_selection", "rvea_get_rows",
    "rvea_operator_params", "rvea_get_velocities", "rvea_set_velocities",
    "rvea_get_counters",
    "rvea_set_timing", "rvea_kernel_time", "rvea_time_kernels", "rvea_autotune",
    "rvea_synchronize", "rvea_destroy",
    "rvea_status_str", "rvea_last_error",
    "rvea_batch_footprint", "rvea_batch_create", "rvea_batch_admit", "rvea_batch_retire",
    "rvea_batch_step", "rvea_batch_set_graphs", "rvea_batch_size", "rvea_batch_synchronize",
    "rvea_batch_destroy", "rvea_batch_last_error",
    "rvea_indicator_footprint", "rvea_hypervolume", "rvea_expected_utility",
    "rvea_hypervolume_noalloc",
]


class Params(C.Structure):
    _fields_ = [
        ("alpha", C.c_double), ("fr", C.c_double), ("t_max", C.c_int32),
        ("op", C.c_int32), ("eta_c", C.c_double), ("eta_m", C.c_double),
        ("p_c", C.c_double), ("p_m", C.c_double), ("lb", C.c_double), ("ub", C.c_double),
        ("op_a", C.c_double), ("op_b", C.c_double),
    ]


class LQSystem(C.Structure):
    _fields_ = [("A", C.c_void_p), ("B", C.c_void_p), ("x0", C.c_void_p), ("E", C.c_int32),
                ("T", C.c_int32), ("init_sigma", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("rows_per_lane", C.c_int32), ("chunk_vectors", C.c_int32),
                ("rerank_rows", C.c_int32), ("candidates", C.c_int32), ("assoc_us", C.c_double),
                ("default_us", C.c_double), ("rerank_us", C.c_double),
                ("rerank_default_us", C.c_double), ("gamma_rows_per_lane", C.c_int32),
                ("gamma_chunk_vectors", C.c_int32), ("gamma_us", C.c_double),
                ("gamma_default_us", C.c_double)]


class Counters(C.Structure):
    _fields_ = [("nonfinite_rows", C.c_int64), ("full_rescans", C.c_int64),
                ("generations", C.c_int64)]


class RveaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    P, i32, i64, u64, sz = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_size_t
    sig = {
        "rvea_default_params": [P],
        "rvea_lattice_divisions": [i32, i64, P],
        "rvea_footprint": [i32, i32, i32, i64, i64, P, P],
        "rvea_create": [i32, i32, i32, i64, i64, u64, P, P, sz, P, P],
        "rvea_create_policy": [i64, i64, u64, P, P, P, sz, P, P],
        "rvea_step": [P], "rvea_select": [P], "rvea_adapt": [P],
        "rvea_run_generations": [P, i32],
        "rvea_prepare_generations": [P, i32],
        "rvea_set_graphs": [P, i32],
        "rvea_set_index": [P, i32],
        "rvea_get_state": [P, P, P, P, P, P, P, P],
        "rvea_set_state": [P, P, P, P, P, P, i64],
        "rvea_get_offspring": [P, P, P, P],
        "rvea_get_selection": [P, P, P, P, P],
        "rvea_get_rows": [P, i32, P, i64, P, P],
        "rvea_operator_params": [i32, P],
        "rvea_get_velocities": [P, i32, P],
        "rvea_set_velocities": [P, P],
        "rvea_get_counters": [P, P],
        "rvea_set_timing": [P, i32],
        "rvea_kernel_time": [P, i32, P, P],
        "rvea_time_kernels": [P, i32, P],
        "rvea_autotune": [P, P],
        "rvea_synchronize": [P], "rvea_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    for name, args in {
        "rvea_batch_footprint": [i32, P], "rvea_batch_create": [i32, P, sz, P, P],
        "rvea_batch_admit": [P, P], "rvea_batch_retire": [P, P], "rvea_batch_step": [P],
        "rvea_batch_set_graphs": [P, i32], "rvea_batch_size": [P, P],
        "rvea_batch_synchronize": [P], "rvea_batch_destroy": [P],
    }.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    for name, args in {
        "rvea_indicator_footprint": [i32, i64, i64, P],
        "rvea_hypervolume": [i32, i64, P, P, P, P, P, P, sz, P],
        "rvea_expected_utility": [i32, i64, P, P, P, P, i64, P, P, P, sz, P],
        "rvea_hypervolume_noalloc": [i32, i64, P, P, P, P, P, P],
    }.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.rvea_batch_last_error.argtypes = [P]
    L.rvea_batch_last_error.restype = C.c_char_p
    L.rvea_status_str.argtypes = [C.c_int]
    L.rvea_status_str.restype = C.c_char_p
    L.rvea_last_error.argtypes = [P]
    L.rvea_last_error.restype = C.c_char_p
    return L


lib = _load()


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def default_params(op=None, **kw):
    """The defaults of rvea_default_params; ``op`` ("de", "pso", "cso", "rand"
    or an id) selects a reproduction operator with its default parameters,
    which keywords may then override."""
    p = Params()
    lib.rvea_default_params(C.byref(p))
    if op is not None:
        code = OPERATORS[op] if isinstance(op, str) else int(op)
        st = lib.rvea_operator_params(code, C.byref(p))
        if st != RVEA_OK:
            raise RveaError(st, f"unknown operator {op!r}")
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def lattice_divisions(m, K):
    h = C.c_int(0)
    st = lib.rvea_lattice_divisions(m, K, C.byref(h))
    return h.value if st == RVEA_OK else None


def footprint(problem, m, d, N, K, params=None):
    b = C.c_size_t(0)
    st = lib.rvea_footprint(problem, m, d, N, K, C.byref(params) if params else None,
                            C.byref(b))
    if st != RVEA_OK:
        raise RveaError(st, lib.rvea_status_str(st).decode())
    return b.value


class Run:
    """One RVEA run resident on a HIP device.

    ``workspace`` may be a preallocated torch uint8 CUDA tensor of at least
    ``footprint`` bytes; otherwise one is allocated on ``device``.
    """

    def __init__(self, problem, m, d, N, K, seed=0, params=None, device="cuda:0",
                 stream=None, workspace=None, system=None):
        self.problem, self.m, self.d, self.N, self.K = problem, m, d, N, K
        self.M = K + N
        self.seed = seed
        self.indexed = m in (2, 3)  # the library's default association
        self.params = params if params is not None else default_params()
        self.bytes = footprint(problem, m, d, N, K, self.params)
        dev = torch.device(device)
        if workspace is None:
            workspace = torch.empty(self.bytes + 256, dtype=torch.uint8, device=dev)
        self._ws = workspace
        base = workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        avail = workspace.numel() - (aligned - base)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._h = C.c_void_p(0)
        with torch.cuda.device(dev):
            if problem == POLICY_LQ:
                # system: dict(A 32x32, B 32x8, x0 E x 32, T, sigma); None is rejected
                sysp = None
                if system is not None:
                    arrs = [np.ascontiguousarray(system[k], np.float32)
                            for k in ("A", "B", "x0")]
                    if arrs[0].shape != (32, 32) or arrs[1].shape != (32, 8) or \
                            arrs[2].ndim != 2 or arrs[2].shape[1] != 32:
                        raise ValueError("system: A 32x32, B 32x8, x0 E x 32")
                    sysd = LQSystem(_p(arrs[0]), _p(arrs[1]), _p(arrs[2]), arrs[2].shape[0],
                                    int(system["T"]), float(system.get("sigma", 0.1)))
                    sysp = C.byref(sysd)
                st = lib.rvea_create_policy(N, K, C.c_uint64(seed), C.byref(self.params),
                                            sysp, C.c_void_p(aligned), avail,
                                            C.c_void_p(self.stream.cuda_stream),
                                            C.byref(self._h))
            else:
                st = lib.rvea_create(problem, m, d, N, K, C.c_uint64(seed), C.byref(self.params),
                                     C.c_void_p(aligned), avail,
                                     C.c_void_p(self.stream.cuda_stream), C.byref(self._h))
        if st != RVEA_OK:
            raise RveaError(st, "rvea_create: " + lib.rvea_status_str(st).decode() + ": "
                            + lib.rvea_last_error(None).decode())

    # ------------------------------------------------------------------
    def _chk(self, st, what):
        if st != RVEA_OK:
            msg = lib.rvea_last_error(self._h).decode() if self._h else ""
            raise RveaError(st, f"{what}: {lib.rvea_status_str(st).decode()} {msg}")

    def step(self):
        self._chk(lib.rvea_step(self._h), "rvea_step")

    def select(self):
        self._chk(lib.rvea_select(self._h), "rvea_select")

    def adapt(self):
        self._chk(lib.rvea_adapt(self._h), "rvea_adapt")

    def generation(self):
        self.step()
        self.select()
        self.adapt()

    def run(self, n):
        self._chk(lib.rvea_run_generations(self._h, n), "rvea_run_generations")

    def prepare(self, n):
        """Capture the graphs run(n) would launch, without running them."""
        self._chk(lib.rvea_prepare_generations(self._h, n), "rvea_prepare_generations")

    def set_graphs(self, on):
        self._chk(lib.rvea_set_graphs(self._h, 1 if on else 0), "rvea_set_graphs")

    def set_index(self, on):
        """Association through the vector index (True, the default for m = 3)
        or by full scans (False); the results are the same."""
        self._chk(lib.rvea_set_index(self._h, 1 if on else 0), "rvea_set_index")
        self.indexed = bool(on)

    def synchronize(self):
        self._chk(lib.rvea_synchronize(self._h), "rvea_synchronize")

    def get_state(self, genes=True):
        K, d, m = self.K, self.d, self.m
        X = np.zeros((K, d), np.float32) if genes else None
        F = np.zeros((K, m), np.float32)
        valid = np.zeros(K, np.uint8)
        V = np.zeros((K, m), np.float64)
        V0 = np.zeros((K, m), np.float64)
        g = np.zeros(K, np.float64)
        t = C.c_int64(0)
        self._chk(lib.rvea_get_state(self._h, _p(X), _p(F), _p(valid), _p(V), _p(V0), _p(g),
                                     C.byref(t)), "rvea_get_state")
        return dict(X=X, F=F, valid=valid, V=V, V0=V0, gamma=g, t=t.value)

    def set_state(self, X, F, valid, V=None, gamma=None, t=0):
        X = np.ascontiguousarray(X, np.float32)
        F = np.ascontiguousarray(F, np.float32)
        valid = np.ascontiguousarray(valid, np.uint8)
        assert X.shape == (self.K, self.d) and F.shape == (self.K, self.m)
        V = None if V is None else np.ascontiguousarray(V, np.float64)
        gamma = None if gamma is None else np.ascontiguousarray(gamma, np.float64)
        self._chk(lib.rvea_set_state(self._h, _p(X), _p(F), _p(valid), _p(V), _p(gamma),
                                     int(t)), "rvea_set_state")

    def get_offspring(self, genes=True):
        N, d, m = self.N, self.d, self.m
        X = np.zeros((N, d), np.float32) if genes else None
        F = np.zeros((N, m), np.float32)
        parents = np.zeros(((N + 1) // 2, 2), np.int32)
        self._chk(lib.rvea_get_offspring(self._h, _p(X), _p(F), _p(parents)),
                  "rvea_get_offspring")
        return dict(X=X, F=F, parents=parents)

    def get_velocities(self, offspring=False):
        """Velocities of a PSO or CSO run: the slots' (K x d) or the last
        offspring's (N x d)."""
        V = np.zeros((self.N if offspring else self.K, self.d), np.float32)
        self._chk(lib.rvea_get_velocities(self._h, 1 if offspring else 0, _p(V)),
                  "rvea_get_velocities")
        return V

    def set_velocities(self, V):
        V = np.ascontiguousarray(V, np.float32)
        assert V.shape == (self.K, self.d)
        self._chk(lib.rvea_set_velocities(self._h, _p(V)), "rvea_set_velocities")

    def get_selection(self):
        z = np.zeros(self.m, np.float32)
        assoc = np.zeros(self.M, np.int32)
        apd = np.zeros(self.M, np.float64)
        surv = np.zeros(self.K, np.int32)
        self._chk(lib.rvea_get_selection(self._h, _p(z), _p(assoc), _p(apd), _p(surv)),
                  "rvea_get_selection")
        return dict(zstar=z, assoc=assoc, apd=apd, surv=surv)

    def get_rows(self, idx, offspring=False, genes=True):
        idx = np.ascontiguousarray(idx, np.int64)
        X = np.zeros((len(idx), self.d), np.float32) if genes else None
        F = np.zeros((len(idx), self.m), np.float32)
        self._chk(lib.rvea_get_rows(self._h, 1 if offspring else 0, _p(idx), len(idx), _p(X),
                                    _p(F)), "rvea_get_rows")
        return X, F

    def counters(self):
        c = Counters()
        self._chk(lib.rvea_get_counters(self._h, C.byref(c)), "rvea_get_counters")
        return dict(nonfinite_rows=c.nonfinite_rows, full_rescans=c.full_rescans,
                    generations=c.generations)

    def set_timing(self, kernels):
        """kernels: iterable of kernel ids to bracket with events (empty = off)."""
        mask = 0
        for k in kernels:
            mask |= 1 << int(k)
        self._chk(lib.rvea_set_timing(self._h, mask), "rvea_set_timing")

    def autotune(self):
        """Time the association tile candidates and keep the fastest (state unchanged)."""
        t = Tuning()
        self._chk(lib.rvea_autotune(self._h, C.byref(t)), "rvea_autotune")
        return dict(rows_per_lane=t.rows_per_lane, chunk_vectors=t.chunk_vectors,
                    rerank_rows=t.rerank_rows, candidates=t.candidates, assoc_us=t.assoc_us,
                    default_us=t.default_us, rerank_us=t.rerank_us,
                    rerank_default_us=t.rerank_default_us,
                    gamma_rows_per_lane=t.gamma_rows_per_lane,
                    gamma_chunk_vectors=t.gamma_chunk_vectors, gamma_us=t.gamma_us,
                    gamma_default_us=t.gamma_default_us)

    def kernel_time(self, kernel):
        ms = C.c_double(0)
        n = C.c_int64(0)
        self._chk(lib.rvea_kernel_time(self._h, kernel, C.byref(ms), C.byref(n)),
                  "rvea_kernel_time")
        return ms.value, n.value

    def time_kernels(self, reps=20):
        """Per-launch ms of reproduce+evaluate, association and re-rank, each
        launched reps times back to back on the current state (call between
        step() and select(); state unchanged)."""
        ms = (C.c_double * 3)()
        self._chk(lib.rvea_time_kernels(self._h, reps, ms), "rvea_time_kernels")
        return dict(offspring=ms[0], assoc=ms[1], rerank=ms[2])

    def close(self):
        if self._h:
            lib.rvea_destroy(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_footprint(max_runs):
    b = C.c_size_t(0)
    st = lib.rvea_batch_footprint(max_runs, C.byref(b))
    if st != RVEA_OK:
        raise RveaError(st, "rvea_batch_footprint")
    return b.value


class Batch:
    """Many runs advanced together, one generation per step()."""

    def __init__(self, max_runs, device="cuda:0", stream=None):
        dev = torch.device(device)
        nbytes = batch_footprint(max_runs)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self._ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._h = C.c_void_p(0)
        self.runs = []
        st = lib.rvea_batch_create(max_runs, C.c_void_p(aligned), nbytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(self._h))
        if st != RVEA_OK:
            raise RveaError(st, "rvea_batch_create: " + lib.rvea_status_str(st).decode())

    def _chk(self, st, what):
        if st != RVEA_OK:
            raise RveaError(st, f"{what}: {lib.rvea_status_str(st).decode()} "
                                f"{lib.rvea_batch_last_error(self._h).decode()}")

    def admit(self, run):
        self._chk(lib.rvea_batch_admit(self._h, run._h), "rvea_batch_admit")
        self.runs.append(run)

    def retire(self, run):
        self._chk(lib.rvea_batch_retire(self._h, run._h), "rvea_batch_retire")
        self.runs.remove(run)

    def step(self, n=1):
        for _ in range(n):
            self._chk(lib.rvea_batch_step(self._h), "rvea_batch_step")

    def set_graphs(self, on):
        self._chk(lib.rvea_batch_set_graphs(self._h, 1 if on else 0), "rvea_batch_set_graphs")

    def size(self):
        n = C.c_int(0)
        self._chk(lib.rvea_batch_size(self._h, C.byref(n)), "rvea_batch_size")
        return n.value

    def synchronize(self):
        self._chk(lib.rvea_batch_synchronize(self._h), "rvea_batch_synchronize")

    def close(self):
        if self._h:
            lib.rvea_batch_destroy(self._h)
            self._h = C.c_void_p(0)
            self.runs = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ indicators
def indicator_footprint(m, n, nw=0):
    b = C.c_size_t(0)
    st = lib.rvea_indicator_footprint(m, n, nw, C.byref(b))
    if st != RVEA_OK:
        raise RveaError(st, "rvea_indicator_footprint: " + lib.rvea_status_str(st).decode())
    return b.value


def _device_rows(F, valid, device):
    """F (n x m) and the optional valid mask as contiguous device tensors."""
    F = torch.as_tensor(F, dtype=torch.float32, device=device).contiguous()
    if F.ndim != 2:
        raise ValueError("F must be n x m")
    if valid is not None:
        valid = torch.as_tensor(valid, dtype=torch.uint8, device=device).contiguous()
        if valid.shape != (F.shape[0],):
            raise ValueError("valid must have one entry per row")
    return F, valid


def _bounds(m, lo, hi):
    lo = np.ascontiguousarray(np.zeros(m) if lo is None else lo, np.float64)
    hi = np.ascontiguousarray(np.ones(m) if hi is None else hi, np.float64)
    if lo.shape != (m,) or hi.shape != (m,):
        raise ValueError("lo and hi need one value per objective")
    return lo, hi


def _indicator_call(fn, name, args, device, stream):
    dev = torch.device(device)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    with torch.cuda.device(dev):
        st = fn(*args(out, s))
    if st != RVEA_OK:
        raise RveaError(st, f"{name}: {lib.rvea_status_str(st).decode()} "
                            f"{lib.rvea_last_error(None).decode()}")
    s.synchronize()
    return float(out.item())


def hypervolume(F, valid=None, lo=None, hi=None, device="cuda:0", stream=None):
    """Hypervolume of the rows of F (m = 2, 3) on normalised objectives
    (F - lo) / (hi - lo), reference point ones (rvea_hypervolume)."""
    F, valid = _device_rows(F, valid, device)
    n, m = F.shape
    lo, hi = _bounds(m, lo, hi)
    ws = torch.empty(indicator_footprint(m, n) + 256, dtype=torch.uint8, device=F.device)
    wsp = (ws.data_ptr() + 255) // 256 * 256
    return _indicator_call(lib.rvea_hypervolume, "rvea_hypervolume", lambda out, s: (
        m, n, C.c_void_p(F.data_ptr()), C.c_void_p(valid.data_ptr()) if valid is not None
        else None, _p(lo), _p(hi), C.c_void_p(out.data_ptr()), C.c_void_p(wsp),
        ws.numel() - (wsp - ws.data_ptr()), C.c_void_p(s.cuda_stream)), device, stream)


def expected_utility(F, W, valid=None, lo=None, hi=None, device="cuda:0", stream=None):
    """Mean over the weight rows W of the best utility -w . f' over the rows of
    F (rvea_expected_utility)."""
    F, valid = _device_rows(F, valid, device)
    n, m = F.shape
    W = torch.as_tensor(W, dtype=torch.float64, device=F.device).contiguous()
    if W.ndim != 2 or W.shape[1] != m:
        raise ValueError("W must be nw x m")
    nw = W.shape[0]
    lo, hi = _bounds(m, lo, hi)
    ws = torch.empty(indicator_footprint(m, n, nw) + 256, dtype=torch.uint8, device=F.device)
    wsp = (ws.data_ptr() + 255) // 256 * 256
    return _indicator_call(lib.rvea_expected_utility, "rvea_expected_utility", lambda out, s: (
        m, n, C.c_void_p(F.data_ptr()), C.c_void_p(valid.data_ptr()) if valid is not None
        else None, _p(lo), _p(hi), nw, C.c_void_p(W.data_ptr()), C.c_void_p(out.data_ptr()),
        C.c_void_p(wsp), ws.numel() - (wsp - ws.data_ptr()), C.c_void_p(s.cuda_stream)),
        device, stream)
