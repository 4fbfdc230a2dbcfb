"""The paper's scaling sweeps (Tables 3 and 4) against the oracle at both
ends of each: Series 1 (m = 3, d = 100) at n = 32 and n = 16,384, Series 2
(m = 3, n = 100) at d = 512 and d = 262,144.  N = n individuals and K = the
smallest lattice count >= n (so some slots start empty).  Each case runs two
generations from initialization and one adapting generation, stage by stage
from identical state."""
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


def ends():
    from workloads import SERIES1, SERIES2

    return [SERIES1[0], SERIES1[-1], SERIES2[0], SERIES2[-1]]


@pytest.mark.parametrize("c", ends(), ids=lambda c: c["name"])
def test_sweep_ends_match_oracle(P, O, c):
    prm = P.default_params(t_max=c["gens"])
    run = P.Run(c["problem"], c["m"], c["d"], c["N"], c["K"], seed=c["seed"], params=prm)
    st = run.get_state()
    assert st["valid"].sum() == c["N"] and c["K"] >= c["N"]
    stats = lockstep(O, run, prm, 2, new_stats())
    st = run.get_state()
    run.set_state(st["X"], st["F"], st["valid"], V=st["V"], gamma=st["gamma"], t=9)
    stats = lockstep(O, run, prm, 1, stats)
    assert stats["adaptations"] == 1
    assert stats["straddles"] <= max(2, 1e-6 * stats["genes"]), stats
    assert stats["near_ties"] <= max(1, 1e-4 * stats["vectors"]), stats
    print(f"{c['name']}: {stats}")
    run.close()
