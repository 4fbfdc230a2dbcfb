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
