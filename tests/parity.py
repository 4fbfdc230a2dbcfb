"""Comparison rules shared by the GPU parity tests (HIP path vs oracle).

- Genes: bit-exact.  The only tolerated difference is a 1-ulp binary32
  disagreement where the oracle's binary64 child lies within a few binary64
  ulps of the binary32 rounding midpoint (the two sides' pow() may differ in
  the last binary64 bit), and such cases must be rare.
- Objectives: within 1e-5 relative (absolute floor 1e-30); for the policy
  rollouts (bfloat16 weights and layer inputs on the matrix cores against a
  binary64 oracle that rounds the same operands), within 1e-3 relative.
- Selection from identical merged objectives: ideal point and association
  exact, APD within 1e-12 relative (both sides finish in binary64),
  survivors exact except near-ties: a vector whose two survivors are both
  associated with it by the oracle and whose oracle APDs differ by at most
  1e-6 relative.  Near-ties must stay below 1e-4 of the vectors.
"""
import numpy as np

OBJ_RTOL = 1e-5
# policy rollouts: bfloat16 operands on both sides, binary32 accumulation on
# the matrix cores against binary64 in the oracle.  Where the two sums of a
# layer differ in their last bits, the next layer's input can round to the
# neighbouring bfloat16 value (2^-8 relative), and such flips carry through
# the 200 steps: measured worst 7.7e-4 (the 64-individual initial
# population), against which the split-bfloat16 dynamics (2^-17 per
# product) are negligible
POLICY_RTOL = 1e-3
APD_RTOL = 1e-12
NEAR_TIE_RTOL = 1e-6


def gene_mismatches(got, want, pre=None):
    """Indices where got != want; asserts each is a rounding straddle of pre."""
    got = np.asarray(got, np.float32)
    want = np.asarray(want, np.float32)
    bad = np.nonzero(got.view(np.uint32) != want.view(np.uint32))
    if len(bad[0]) == 0:
        return 0
    if pre is None:
        raise AssertionError(f"{len(bad[0])} genes differ; first at {tuple(b[0] for b in bad)}")
    g = got[bad].astype(np.float64)
    w = want[bad].astype(np.float64)
    p = np.asarray(pre)[bad]
    one_ulp = np.nextafter(want[bad], got[bad]).astype(np.float64) == g
    mid = 0.5 * (g + w)
    near = np.abs(p - mid) <= 8 * np.spacing(np.abs(p))
    assert np.all(one_ulp & near), f"genes differ beyond rounding straddles at {bad}"
    return len(bad[0])


def objectives_close(got, want, rtol=OBJ_RTOL):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    err = np.abs(got - want)
    lim = rtol * np.abs(want) + 1e-30
    ok = err <= lim
    assert np.all(ok), (f"objectives differ: worst rel {np.max(err / (np.abs(want) + 1e-30)):.3g}"
                        f" at {np.argwhere(~ok)[:5].tolist()}")
    return float(np.max(err / (np.abs(want) + 1e-30)))


def compare_selection(sel, ref, K):
    z_gpu = np.asarray(sel["zstar"], np.float64)
    assert np.array_equal(z_gpu, ref["zstar"]), (z_gpu, ref["zstar"])
    assert np.array_equal(sel["assoc"], ref["assoc"]), (
        f"association differs at {np.nonzero(sel['assoc'] != ref['assoc'])[0][:10]}")
    fin = np.isfinite(ref["apd"])
    assert np.array_equal(np.isfinite(sel["apd"]), fin)
    a, b = sel["apd"][fin], ref["apd"][fin]
    assert np.all(np.abs(a - b) <= APD_RTOL * np.abs(b) + 1e-300), "APD differs"
    return survivor_near_ties(sel["surv"], ref["surv"], ref["apd"], ref["assoc"], K)


def survivor_near_ties(sg, so, apd_o, assoc_o, K):
    mism = np.nonzero(sg != so)[0]
    for j in mism:
        a, b = int(sg[j]), int(so[j])
        assert a >= 0 and b >= 0, f"vector {j}: survivor {a} vs {b}"
        assert assoc_o[a] == j, f"vector {j}: GPU survivor {a} not in the subpopulation"
        assert abs(apd_o[a] - apd_o[b]) <= NEAR_TIE_RTOL * apd_o[b], f"vector {j} not a near-tie"
    return len(mism)


def ora_params(O, prm):
    """The oracle's parameter record for the binding's Params."""
    return O.params(alpha=prm.alpha, fr=prm.fr, t_max=prm.t_max, eta_c=prm.eta_c,
                    eta_m=prm.eta_m, p_c=prm.p_c, p_m=prm.p_m, lb=prm.lb, ub=prm.ub)


def new_stats():
    return dict(straddles=0, genes=0, near_ties=0, vectors=0, adaptations=0, generations=0)


def check_generation(O, run, prm, st, off, sel, st2, stats, exact_survivors=False):
    """One completed generation of `run` against the oracle, stage by stage
    from identical state (Alg. 2): st is the run's state before it, off its
    offspring (X, F, mating pairs), sel its selection, st2 its state after.

    Mating draws exact; offspring genes bit-exact but for counted rounding
    straddles (App. B); objectives at OBJ_RTOL; selection from the GPU's
    merged objectives (Alg. 1): ideal point and association exact, APD at
    APD_RTOL, survivors exact but for counted near-ties (none allowed with
    exact_survivors); the new population is the survivors' rows; at an
    adapting generation V exact and gamma at 1e-13."""
    problem, m, d, N, K, seed = run.problem, run.m, run.d, run.N, run.K, run.seed
    op = ora_params(O, prm)
    t = st["t"] + 1
    assert st2["t"] == t
    parents, nv = O.mate(seed, t, st["valid"], N)
    assert nv == st["valid"].sum()
    assert np.array_equal(off["parents"], parents), f"mating differs at t={t}"
    Xo, pre = O.reproduce(op, seed, t, st["X"], parents, N, with_pre=True)
    stats["straddles"] += gene_mismatches(off["X"], Xo, pre)
    stats["genes"] += Xo.size
    objectives_close(off["F"], O.evaluate(problem, m, off["X"]))
    return check_after_offspring(O, run, prm, st, off, sel, st2, stats, exact_survivors)


def check_after_offspring(O, run, prm, st, off, sel, st2, stats, exact_survivors=False):
    """The rest of a generation once its offspring are checked: selection
    from the GPU's merged objectives (Alg. 1), the new population, and the
    adaptation (Alg. 2), as check_generation states."""
    m, N, K = run.m, run.N, run.K
    period = O.adapt_period(prm.fr, prm.t_max)
    t = st["t"] + 1
    Fm = np.vstack([st["F"], off["F"]]).astype(np.float64)
    mv = np.concatenate([st["valid"], np.ones(N, np.uint8)])
    ref = O.select(m, K, N, t, prm.t_max, prm.alpha, Fm, mv, st["V"], st["gamma"])
    nt = compare_selection(sel, ref, K)
    if exact_survivors:
        assert nt == 0 and np.array_equal(sel["surv"], ref["surv"]), "survivors differ"
    stats["near_ties"] += nt
    stats["vectors"] += K
    # the new population is the survivors' rows (Alg. 1)
    Xm = np.vstack([st["X"], off["X"]])
    s = sel["surv"]
    assert np.array_equal(st2["valid"], (s >= 0).astype(np.uint8))
    ok = s >= 0
    assert np.array_equal(st2["X"][ok], Xm[s[ok]])
    assert np.array_equal(st2["F"][ok], Fm[s[ok]].astype(np.float32))
    if t % period == 0:
        Vo, changed = O.adapt(st2["V0"], st2["F"].astype(np.float64), st2["valid"], st["V"])
        assert np.array_equal(st2["V"], Vo), f"adapted vectors differ at t={t}"
        if changed:
            assert np.allclose(st2["gamma"], O.gamma(Vo), rtol=1e-13, atol=0)
            stats["adaptations"] += 1
    else:
        assert np.array_equal(st2["V"], st["V"]) and np.array_equal(st2["gamma"], st["gamma"])
    stats["generations"] += 1
    return ref


def lockstep(O, run, prm, gens, stats, exact_survivors=False):
    """gens generations of a single run, each checked by check_generation;
    the offspring are read between rvea_step and rvea_select."""
    for _ in range(gens):
        st = run.get_state()
        run.step()
        off = run.get_offspring()
        run.select()
        sel = run.get_selection()
        run.adapt()
        check_generation(O, run, prm, st, off, sel, run.get_state(), stats, exact_survivors)
    return stats
