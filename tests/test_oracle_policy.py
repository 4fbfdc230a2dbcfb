"""Pins of the oracle's policy-rollout problem (the neuroevolution setting of
Sec. 4.3, with a synthetic linear system in place of the physics engine).

Each test checks the oracle against something other than itself: closed
forms of the linear recurrence, a bit-level bfloat16 rounding of binary32,
hand-traced single-path networks, the rollout average, and the normal
distribution of the initial genes.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O
import workloads as W

D = O.POLICY_D
W1, B1, W2, W3, B3 = 0, 2048, 2112, 6208, 6720


def bf16_bits(x):
    """float32 -> bfloat16 (round to nearest even) by integer arithmetic on the bits."""
    u = np.asarray(x, np.float32).reshape(-1).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def system(seed=0, E=16):
    S = W.lq_system(seed, E=E)
    return S["A"].astype(np.float64), S["B"].astype(np.float64), S["x0"].astype(np.float64), S


def test_bf16_rounding_matches_bit_level_rne():
    r = np.random.default_rng(0)
    x = (r.standard_normal(20000) * np.exp(r.uniform(-20, 20, 20000))).astype(np.float32)
    # exact ties: low 16 bits 0x8000, both parities of the kept part
    ties = (r.integers(0x3F000000, 0x40800000, 2000, dtype=np.uint64) & ~np.uint64(0xFFFF)) | 0x8000
    x = np.concatenate([x, ties.astype(np.uint32).view(np.float32), [0.0, -0.0, 1.0, -2.5]])
    want = bf16_bits(x)
    got = np.array([O.bf16(float(v)) for v in x])
    assert np.array_equal(got, want)
    assert O.bf16(1.0 + 2.0**-8) == 1.0               # tie to even (down)
    assert O.bf16(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6  # tie to even (up)


def closed_form_f1(A, B, x0, u, T):
    """sum_{t=1..T} |x_t|^2 for x_{t+1} = A x_t + B u with constant u, from
    x_t = A^t x0 + (I - A)^{-1} (I - A^t) B u, averaged over the rows of x0."""
    n = A.shape[0]
    c = np.linalg.solve(np.eye(n) - A, B @ u)
    tot = 0.0
    At = np.eye(n)
    for _ in range(T):
        At = At @ A
        xt = x0 @ At.T + (c - At @ c)[None, :]
        tot += np.sum(xt * xt)
    return tot / x0.shape[0]


def test_zero_policy_is_the_free_response():
    A, B, x0, S = system(1)
    T = 37
    F = O.policy_evaluate(np.zeros((1, D), np.float32), 16, T, S["A"], S["B"], S["x0"])
    want = np.mean([sum(np.sum((np.linalg.matrix_power(A, t) @ x0[e]) ** 2)
                        for t in range(1, T + 1)) for e in range(16)])
    assert F[0, 1] == 0.0
    assert abs(F[0, 0] - want) <= 1e-12 * want


def test_output_bias_only_policy_is_a_constant_input():
    A, B, x0, S = system(2)
    T = 50
    w = np.zeros(D, np.float32)
    w[B1:B1 + 64] = np.linspace(-0.5, 0.5, 64)  # blocked by W2 = 0
    w[B3:B3 + 8] = np.linspace(-0.7, 0.9, 8)
    F = O.policy_evaluate(w[None], 16, T, S["A"], S["B"], S["x0"])
    u = np.tanh(w[B3:B3 + 8].astype(np.float64))
    assert abs(F[0, 1] - T * np.sum(u * u)) <= 1e-12 * F[0, 1]
    want = closed_form_f1(A, B, x0, u, T)
    assert abs(F[0, 0] - want) <= 1e-10 * want


def test_hidden_bias_path_pins_b1_w2_w3_offsets():
    # W1 = 0: h1 = tanh(b1); one path b1[j1] -> W2[j2, j1] -> W3[q, j2]
    A, B, x0, S = system(3)
    T = 20
    j1, j2, q = 37, 5, 6
    w = np.zeros(D, np.float32)
    w[B1 + j1] = 0.8
    w[W2 + j2 * 64 + j1] = 1.25
    w[W3 + q * 64 + j2] = -2.0
    h1 = np.tanh(0.8)
    h2 = np.tanh(1.25 * bf16_bits(h1)[0])
    uq = np.tanh(-2.0 * bf16_bits(h2)[0])
    u = np.zeros(8)
    u[q] = uq
    F = O.policy_evaluate(w[None], 16, T, S["A"], S["B"], S["x0"])
    assert abs(F[0, 1] - T * uq * uq) <= 1e-12 * F[0, 1]
    want = closed_form_f1(A, B, x0, u, T)
    assert abs(F[0, 0] - want) <= 1e-10 * want


def test_input_path_traced_by_hand():
    # A = 0: x_{t+1} = B u_t; one path x[k1] -> W1[j1, k1] -> W2[j2, j1] -> W3[q, j2]
    _, B, x0, S = system(4)
    Az = np.zeros((32, 32), np.float32)
    T = 3
    k1, j1, j2, q = 29, 50, 11, 3
    w = np.zeros(D, np.float32)
    w[W1 + j1 * 32 + k1] = 1.5
    w[W2 + j2 * 64 + j1] = -0.75
    w[W3 + q * 64 + j2] = 2.5
    f1 = f2 = 0.0
    for e in range(16):
        x = x0[e].copy()
        for _ in range(T):
            h1 = np.tanh(1.5 * bf16_bits(np.float32(x[k1]))[0])
            h2 = np.tanh(-0.75 * bf16_bits(h1)[0])
            uq = np.tanh(2.5 * bf16_bits(h2)[0])
            f2 += uq * uq
            x = B[:, q] * uq
            f1 += np.sum(x * x)
    F = O.policy_evaluate(w[None], 16, T, Az, S["B"], S["x0"])
    assert abs(F[0, 0] - f1 / 16) <= 1e-12 * F[0, 0]
    assert abs(F[0, 1] - f2 / 16) <= 1e-12 * F[0, 1]


def test_objectives_average_the_rollouts():
    _, _, _, S = system(5)
    X = W.policy_population(6, 3)
    F = O.policy_evaluate(X, 16, 30, S["A"], S["B"], S["x0"])
    per = np.stack([O.policy_evaluate(X, 1, 30, S["A"], S["B"], S["x0"][e:e + 1])
                    for e in range(16)])
    assert np.allclose(F, per.mean(axis=0), rtol=1e-13, atol=0)


def test_gaussian_init_is_normal_and_clipped():
    X = O.init_gauss_rows(7, np.arange(48), D, sigma=0.1, lb=-1.0, ub=1.0)
    z = X.reshape(-1).astype(np.float64) / 0.1
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    # the two members of each Box-Muller pair are uncorrelated
    pairs = X.reshape(48, -1, 2)
    assert abs(np.corrcoef(pairs[..., 0].ravel(), pairs[..., 1].ravel())[0, 1]) < 0.01
    # other individuals draw other numbers; clipping to tight bounds
    assert not np.array_equal(X[0], X[1])
    Xc = O.init_gauss_rows(7, np.arange(4), D, sigma=0.1, lb=-0.05, ub=0.05)
    assert Xc.min() >= np.float32(-0.05) and Xc.max() <= np.float32(0.05)
    frac = np.mean(np.abs(Xc) == np.float32(0.05))
    assert abs(frac - 2 * stats.norm.sf(0.5)) < 0.02
    # same individuals, same genes regardless of the row set
    assert np.array_equal(O.init_gauss_rows(7, [3, 9], D), X[[3, 9]])


def test_linear_system_generator():
    S = W.lq_system(0)
    assert S["A"].shape == (32, 32) and S["B"].shape == (32, 8) and S["x0"].shape == (16, 32)
    rho = np.max(np.abs(np.linalg.eigvals(S["A"].astype(np.float64))))
    assert abs(rho - 0.95) < 1e-6
    assert abs(S["B"].std() - 0.1) < 0.02


@pytest.mark.parametrize("gens", [3])
def test_policy_run_keeps_selection_invariants(gens):
    S = dict(W.lq_system(0), T=8, sigma=0.1)
    K = N = 12  # m = 2, H = 11
    prm = O.params(lq=S, lb=-1.0, ub=1.0, t_max=gens)
    st = O.run(prm, O.POLICY_LQ, 2, D, N, K, 0, gens)
    assert 1 <= st.valid.sum() <= K
    assert np.all(np.isfinite(st.F[st.valid == 1]))
    assert np.all(np.abs(st.X) <= 1.0)
    assert np.all(st.F[st.valid == 1] >= 0)
