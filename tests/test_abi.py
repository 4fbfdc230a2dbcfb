"""The C-ABI library loads and exports every entry point include/rvea.h
declares; host-side argument checks and status codes (no device needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rvea.h")


def declared():
    text = open(HEADER).read()
    return set(re.findall(r"^(?:rvea_status|const char \*)\s*(rvea_\w+)\s*\(", text, re.M))


@pytest.fixture(scope="module")
def P():
    import paper_2404_01159_amd as P

    return P


def test_header_declarations_are_exported(P):
    names = declared()
    assert len(names) >= 20
    L = C.CDLL(P.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert names == set(P.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (rvea_\w+)", out))
    assert names <= exported


def test_default_params(P):
    p = P.default_params()
    assert (p.alpha, p.fr, p.t_max, p.eta_c, p.eta_m, p.p_c, p.p_m, p.lb, p.ub) == (
        2.0, 0.1, 100, 20.0, 20.0, 1.0, 1.0, 0.0, 1.0)


def test_lattice_divisions(P):
    assert P.lattice_divisions(3, 105) == 13
    assert P.lattice_divisions(3, 10011) == 140
    assert P.lattice_divisions(3, 100128) == 446
    assert P.lattice_divisions(2, 4096) == 4095
    assert P.lattice_divisions(3, 106) is None


def test_footprint_and_argument_checks(P):
    b1 = P.footprint(1, 3, 500, 10011, 10011)
    b3 = P.footprint(3, 3, 5000, 100128, 100128)
    # the gene pool (K+N rows of round_up(d,32) floats) dominates; the
    # association's chunk partials and the vector index come next
    assert b1 >= 2 * 10011 * 512 * 4 and b1 < 2 * 10011 * 512 * 4 * 2.0
    assert b3 >= 2 * 100128 * 5024 * 4 and b3 < 5e9
    bad = [
        (0, 3, 12, 105, 105), (4, 3, 12, 105, 105), (1, 1, 12, 1, 1), (1, 9, 12, 9, 9),
        (1, 3, 2, 105, 105), (1, 3, 12, 106, 105), (1, 3, 12, 0, 105), (1, 3, 12, 100, 106),
    ]
    for args in bad:
        with pytest.raises(P.RveaError):
            P.footprint(*args)
    for kw in [dict(p_m=4.5), dict(p_m=-1.0), dict(lb=1.0, ub=1.0), dict(t_max=0),
               dict(p_c=1.5), dict(fr=0.0), dict(op=5), dict(op=-1), dict(op_a=0.5),
               dict(eta_c=-1.0)]:
        with pytest.raises(P.RveaError):
            P.footprint(1, 3, 12, 105, 105, P.default_params(**kw))
    # operator parameters: ranges per operator, unused ones 0
    for op, kw in [("de", dict(op_a=2.5)), ("de", dict(op_b=1.5)), ("pso", dict(op_a=1.5)),
                   ("pso", dict(op_b=-0.1)), ("cso", dict(op_a=0.1)), ("rand", dict(op_b=1.0))]:
        with pytest.raises(P.RveaError):
            P.footprint(1, 3, 12, 105, 105, P.default_params(op, **kw))
    with pytest.raises(P.RveaError):
        P.default_params(7)
    # the swarm operators add a velocity pool the size of the gene pool
    ga = P.footprint(1, 3, 500, 105, 105)
    for op in ("de", "rand"):
        assert P.footprint(1, 3, 500, 105, 105, P.default_params(op)) <= ga
    for op in ("pso", "cso"):
        assert P.footprint(1, 3, 500, 105, 105, P.default_params(op)) >= ga + 210 * 512 * 4 - 256
    de = P.default_params("de")
    assert (de.op, de.op_a, de.op_b) == (1, 0.5, 0.9)


def test_create_rejects_bad_workspace_before_touching_a_device(P):
    from paper_2404_01159_amd import rvea as R

    h = C.c_void_p(0)
    prm = P.default_params()
    need = P.footprint(2, 3, 12, 105, 105, prm)
    assert R.lib.rvea_create(2, 3, 12, 105, 105, 0, C.byref(prm), None, need, None,
                             C.byref(h)) == R.RVEA_EINVAL
    assert R.lib.rvea_create(2, 3, 12, 105, 105, 0, C.byref(prm), C.c_void_p(4096 + 8), need,
                             None, C.byref(h)) == R.RVEA_EINVAL
    assert R.lib.rvea_create(2, 3, 12, 105, 105, 0, C.byref(prm), C.c_void_p(4096), need - 1,
                             None, C.byref(h)) == R.RVEA_ENOMEM
    assert h.value is None


def test_null_handles_and_status_strings(P):
    from paper_2404_01159_amd import rvea as R

    for fn in ("rvea_step", "rvea_select", "rvea_adapt", "rvea_synchronize", "rvea_destroy"):
        assert getattr(R.lib, fn)(None) == R.RVEA_EINVAL
    assert R.lib.rvea_run_generations(None, 1) == R.RVEA_EINVAL
    assert R.lib.rvea_prepare_generations(None, 1) == R.RVEA_EINVAL
    assert R.lib.rvea_time_kernels(None, 1, None) == R.RVEA_EINVAL
    assert R.lib.rvea_status_str(0) == b"ok"
    assert R.lib.rvea_status_str(-4) == b"call out of order"
    assert R.lib.rvea_last_error(None) == b"no run"


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2404_01159_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "rvea_oracle" not in text, f
                assert "liboracle" not in text, f
