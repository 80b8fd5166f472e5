"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks retypes the oracle's formula: each compares it with a
brute-force search, a library routine of another kind, a separately written
centralised solver, a hand-worked example, an identity between two different
expressions, or an invariant the paper proves.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle.reference as O
from rpca_inputs import equal_widths, gaussian_init, planted_instance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------
# S-subproblem (eq. "optS")
# --------------------------------------------------------------------------

def test_soft_threshold_matches_bruteforce_grid():
    """1-D brute force: argmin_s 1/2 (s - x)^2 + lambda |s| on a 1e-5 grid."""
    lam = 0.7
    xs = np.concatenate([_rng(0).uniform(-3.0, 3.0, 40),
                         [0.0, lam, -lam, 2 * lam, -2 * lam, 1e-9, -2.99]])
    grid = np.linspace(-4.0, 4.0, 800001)
    for x in xs:
        f = 0.5 * (grid - x) ** 2 + lam * np.abs(grid)
        s_bf = grid[int(np.argmin(f))]
        s = O.soft_threshold(np.array([x]), lam)[0]
        assert abs(s - s_bf) <= 2e-5, (x, s, s_bf)


def test_soft_threshold_subgradient_optimality():
    """0 in (s - x) + lambda * d|s|: |x - s| <= lambda, and x - s = lambda sign(s)
    where s != 0 (the optimality condition, not the formula)."""
    X = _rng(1).normal(scale=2.0, size=(40, 30))
    lam = 0.5
    S = O.soft_threshold(X, lam)
    resid = X - S
    assert np.all(np.abs(resid) <= lam * (1 + 1e-15))
    nz = S != 0
    assert nz.any() and (~nz).any()
    np.testing.assert_allclose(resid[nz], lam * np.sign(S[nz]), rtol=0, atol=1e-14)
    assert np.all(np.abs(X[~nz]) <= lam)


def test_huber_is_the_infimal_convolution_bruteforce():
    """H_lambda(x) = min_s 1/2 (x - s)^2 + lambda |s| (eq. "cancelV"), by grid."""
    lam = 0.6
    grid = np.linspace(-6.0, 6.0, 1200001)
    for x in [-4.0, -0.61, -0.6, -0.2, 0.0, 0.3, 0.6, 1.7, 5.0]:
        bf = float(np.min(0.5 * (x - grid) ** 2 + lam * np.abs(grid)))
        assert abs(O.huber(np.array([x]), lam) - bf) <= 1e-9


def test_huber_identity_with_soft_threshold():
    """min_S 1/2||X - S||^2 + lambda||S||_1 = H_lambda(X): the value at the
    soft-threshold equals the piecewise Huber sum, and no perturbation beats it."""
    X = _rng(2).normal(scale=1.5, size=(25, 17))
    lam = 0.4
    S = O.soft_threshold(X, lam)
    val = 0.5 * np.sum((X - S) ** 2) + lam * np.sum(np.abs(S))
    assert abs(val - O.huber(X, lam)) <= 1e-12 * abs(val)
    rng = _rng(3)
    for _ in range(20):
        P = S + rng.normal(scale=1e-3, size=S.shape)
        assert 0.5 * np.sum((X - P) ** 2) + lam * np.sum(np.abs(P)) >= val


# --------------------------------------------------------------------------
# V-subproblem (eq. "condition1") and the closed-form U step
# --------------------------------------------------------------------------

def test_ridge_V_matches_augmented_least_squares():
    """min_V 1/2||U V^T - D||^2 + rho/2||V||^2 solved by lstsq (SVD) on the
    stacked system [U; sqrt(rho) I] V^T = [D; 0]."""
    rng = _rng(4)
    U = rng.normal(size=(30, 4))
    D = rng.normal(size=(30, 11))
    rho = 0.3
    V = O.ridge_V(U, D, rho)
    A = np.vstack([U, math.sqrt(rho) * np.eye(4)])
    B = np.vstack([D, np.zeros((4, 11))])
    Vt = np.linalg.lstsq(A, B, rcond=None)[0]
    np.testing.assert_allclose(V, Vt.T, rtol=1e-10, atol=1e-12)


def test_closed_U_matches_augmented_least_squares():
    """argmin_U L_i(U, V, S) by lstsq on [V; sqrt(c) I] U^T = [(M - S)^T; 0],
    c = rho n_i / n."""
    rng = _rng(5)
    V = rng.normal(size=(9, 3))
    S = rng.normal(size=(20, 9))
    M = rng.normal(size=(20, 9))
    rho, n_i, n = 0.5, 9, 27
    U = O.closed_U(V, S, M, rho, n_i, n)
    c = rho * n_i / n
    A = np.vstack([V, math.sqrt(c) * np.eye(3)])
    B = np.vstack([(M - S).T, np.zeros((3, 20))])
    Ut = np.linalg.lstsq(A, B, rcond=None)[0]
    np.testing.assert_allclose(U, Ut.T, rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------
# U gradient (Lemma 2) and the exact inner solution (Lemmas 1 and 4)
# --------------------------------------------------------------------------

def _small_problem(seed=6, m=7, n_i=5, r=2):
    rng = _rng(seed)
    U = rng.normal(size=(m, r))
    V = rng.normal(size=(n_i, r))
    S = rng.normal(size=(m, n_i)) * (rng.random((m, n_i)) < 0.3)
    M = rng.normal(size=(m, n_i)) * 2
    return U, V, S, M


def test_grad_U_central_differences():
    U, V, S, M = _small_problem()
    rho, lam, n_i, n = 0.4, 0.3, 5, 13
    G = O.grad_U(U, V, S, M, rho, n_i, n)
    h = 1e-6
    FD = np.zeros_like(U)
    for a in range(U.shape[0]):
        for b in range(U.shape[1]):
            E = np.zeros_like(U)
            E[a, b] = h
            FD[a, b] = (O.local_objective(U + E, V, S, M, rho, lam, n_i, n)
                        - O.local_objective(U - E, V, S, M, rho, lam, n_i, n)) / (2 * h)
    np.testing.assert_allclose(G, FD, rtol=1e-6, atol=1e-7)


def test_local_objectives_sum_to_global_under_consensus():
    """Section 2.2: with U_i = U, sum_i L_i = the objective of eq.
    "noncovex_problem" (the rho n_i / n weights sum to one)."""
    rng = _rng(7)
    widths = [3, 5, 2]
    m, r = 6, 2
    U = rng.normal(size=(m, r))
    Vs = [rng.normal(size=(w, r)) for w in widths]
    Ss = [rng.normal(size=(m, w)) for w in widths]
    Ms = [rng.normal(size=(m, w)) for w in widths]
    rho, lam, n = 0.7, 0.2, sum(widths)
    tot = sum(O.local_objective(U, V, S, M, rho, lam, w, n)
              for V, S, M, w in zip(Vs, Ss, Ms, widths))
    assert abs(tot - O.objective(U, Vs, Ss, Ms, rho, lam)) <= 1e-12 * abs(tot)


def _exact_inner(U, M, rho, lam, iters=4000):
    S0 = np.zeros_like(M)
    return O.inner_solve(U, M, S0, rho, lam, inner=iters)


def test_exact_inner_solution_satisfies_lemma4_identities():
    """At the exact (V*, S*): Lambda = M - U V*^T - S* has |Lambda|_inf <= lambda
    and rho V* = Lambda^T U (Lemma 4 proof); the objective equals the Huber form
    rho/2||V||^2 + H_lambda(M - U V^T) of eq. "cancelV"."""
    rng = _rng(8)
    U = rng.normal(size=(10, 3))
    M = rng.normal(size=(10, 6)) * 3
    rho, lam = 0.5, 0.4
    V, S, _ = _exact_inner(U, M, rho, lam)
    Lam = M - U @ V.T - S
    assert np.max(np.abs(Lam)) <= lam * (1 + 1e-12)
    np.testing.assert_allclose(rho * V, Lam.T @ U, rtol=0, atol=1e-10)
    val = 0.5 * np.sum(Lam * Lam) + 0.5 * rho * np.sum(V * V) + lam * np.sum(np.abs(S))
    hub = 0.5 * rho * np.sum(V * V) + O.huber(M - U @ V.T, lam)
    assert abs(val - hub) <= 1e-11 * abs(val)


def test_inner_solution_is_unique_from_any_start():
    """Lemma 1: h is strongly convex, so alternations from different S starts
    reach the same (V*, S*)."""
    rng = _rng(9)
    U = rng.normal(size=(9, 2))
    M = rng.normal(size=(9, 5)) * 2
    rho, lam = 0.6, 0.3
    V1, S1, _ = O.inner_solve(U, M, np.zeros_like(M), rho, lam, inner=4000)
    V2, S2, _ = O.inner_solve(U, M, rng.normal(size=M.shape) * 5, rho, lam, inner=4000)
    np.testing.assert_allclose(V1, V2, atol=1e-11)
    np.testing.assert_allclose(S1, S2, atol=1e-11)


def test_danskin_gradient_of_g():
    """Lemma 2: grad g_i(U) = grad_U L_i(U, V*, S*), checked against central
    differences of g_i(U) = inf_{V,S} L_i(U, V, S)."""
    rng = _rng(10)
    m, n_i, r, n = 6, 4, 2, 10
    U = rng.normal(size=(m, r))
    M = rng.normal(size=(m, n_i)) * 2
    rho, lam = 0.5, 0.3

    def g(Ux):
        V, S, _ = _exact_inner(Ux, M, rho, lam)
        return O.local_objective(Ux, V, S, M, rho, lam, n_i, n)

    V, S, _ = _exact_inner(U, M, rho, lam)
    G = O.grad_U(U, V, S, M, rho, n_i, n)
    h = 1e-6
    FD = np.zeros_like(U)
    for a in range(m):
        for b in range(r):
            E = np.zeros_like(U)
            E[a, b] = h
            FD[a, b] = (g(U + E) - g(U - E)) / (2 * h)
    np.testing.assert_allclose(G, FD, rtol=1e-5, atol=1e-6)


# --------------------------------------------------------------------------
# Whole rounds of Algorithm 1
# --------------------------------------------------------------------------

def test_hand_worked_round_golden():
    with open(os.path.join(GOLDEN, "hand_2x2_one_round.json")) as f:
        gold = json.load(f)
    inp, exp = gold["inputs"], gold["expected"]
    M = np.array(inp["M"])
    Ms = [M[:, :1], M[:, 1:]]
    U0 = np.array(inp["U0"])
    for mode in ("grad", "closed"):
        res = O.dcfpca(Ms, inp["r"], inp["rho"], inp["lambda"], 1, U0, K=1, inner=1,
                       u_mode=mode, eta0=inp["eta"])
        np.testing.assert_allclose(np.vstack(res.V), np.array(exp["V"]), atol=1e-15)
        np.testing.assert_allclose(res.S_full(), np.array(exp["S"]), atol=1e-15)
        np.testing.assert_allclose(res.U, np.array(exp[mode]["U"]), atol=1e-15)
        np.testing.assert_allclose(res.L_full(), np.array(exp[mode]["L"]), atol=1e-15)
        h = res.history[0]
        assert abs(h["objective"] - exp["objective"]) <= 1e-14
        assert abs(h["lambda_fro_sq"] - exp["lambda_fro_sq"]) <= 1e-15
        assert h["nnz"] == exp["nnz"]


def test_hand_worked_decaying_step_golden():
    """Two GRAD rounds with eta_t = eta0 / sqrt(t + 1) (Section 4.2's decaying
    rate, rounds indexed from 0), worked by hand: pins the schedule's index
    (a constant step or a schedule indexed from 1 gives other values)."""
    with open(os.path.join(GOLDEN, "hand_2x2_eta_sqrt_two_rounds.json")) as f:
        gold = json.load(f)
    inp, exp = gold["inputs"], gold["expected"]
    M = np.array(inp["M"])
    Ms = [M[:, :1], M[:, 1:]]
    U0 = np.array(inp["U0"])
    res = O.dcfpca(Ms, inp["r"], inp["rho"], inp["lambda"], inp["T"], U0, K=1, inner=1,
                   u_mode="grad", eta0=inp["eta0"], eta_sched="sqrt")
    np.testing.assert_allclose(res.U, np.array(exp["U"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.vstack(res.V), np.array(exp["V"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(res.S_full(), np.array(exp["S"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(res.L_full(), np.array(exp["L"]), rtol=0, atol=1e-15)
    h = res.history[1]
    assert abs(h["objective"] - exp["objective_round1"]) <= 1e-14
    assert abs(h["lambda_fro_sq"] - exp["lambda_fro_sq_round1"]) <= 1e-15
    assert h["nnz"] == exp["nnz_round1"]
    # The same rounds with a constant step differ.
    res_c = O.dcfpca(Ms, inp["r"], inp["rho"], inp["lambda"], inp["T"], U0, u_mode="grad",
                     eta0=inp["eta0"], eta_sched="const")
    assert np.max(np.abs(res_c.U - np.array(exp["U"]))) > 1e-3


def test_hand_worked_lambda_schedule_golden():
    """A lambda schedule (0.5, then 0.25), worked by hand: round 1's V update
    consumes S re-solved at lambda_1 for the factors that produced the last
    residual, not the stored S of round 0 (whose V would differ)."""
    with open(os.path.join(GOLDEN, "hand_2x2_lambda_schedule.json")) as f:
        gold = json.load(f)
    inp, exp = gold["inputs"], gold["expected"]
    M = np.array(inp["M"])
    Ms = [M[:, :1], M[:, 1:]]
    U0 = np.array(inp["U0"])
    res = O.dcfpca(Ms, inp["r"], inp["rho"], inp["lambda"], inp["T"], U0, K=1, inner=1,
                   u_mode="grad", eta0=inp["eta0"], lam_schedule=inp["lam_schedule"])
    np.testing.assert_allclose(res.U, np.array(exp["U"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.vstack(res.V), np.array(exp["V"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(res.S_full(), np.array(exp["S"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(res.L_full(), np.array(exp["L"]), rtol=0, atol=1e-15)
    h = res.history[1]
    assert abs(h["objective"] - exp["objective_round1"]) <= 1e-14
    assert abs(h["lambda_fro_sq"] - exp["lambda_fro_sq_round1"]) <= 1e-15
    assert h["nnz"] == exp["nnz_round1"]
    assert np.max(np.abs(np.vstack(res.V) - np.array(exp["stored_reading_V"]))) > 1e-2
    # The objective at the target lambda: round 0 ran at lambda_0, round 1 at the target.
    assert abs(res.history[0]["objective_target"] - exp["objective_target_round0"]) <= 1e-14
    assert res.history[1]["objective_target"] == pytest.approx(exp["objective_round1"], abs=1e-14)


def test_hand_worked_step_multiplier_golden():
    """The consensus step relaxed by omega = 3/2, worked by hand for both U
    steps; for the gradient step it equals one round with step omega eta."""
    with open(os.path.join(GOLDEN, "hand_2x2_step_multiplier.json")) as f:
        gold = json.load(f)
    inp, exp = gold["inputs"], gold["expected"]
    M = np.array(inp["M"])
    Ms = [M[:, :1], M[:, 1:]]
    U0 = np.array(inp["U0"])
    for mode in ("closed", "grad"):
        res = O.dcfpca(Ms, inp["r"], inp["rho"], inp["lambda"], 1, U0, u_mode=mode,
                       eta0=inp["eta"], omega_schedule=[inp["omega"]])
        np.testing.assert_allclose(res.U, np.array(exp[mode]["U"]), rtol=0, atol=1e-15)
        np.testing.assert_allclose(res.L_full(), np.array(exp[mode]["L"]), rtol=0, atol=1e-15)
    g = O.dcfpca(Ms, inp["r"], inp["rho"], inp["lambda"], 1, U0, u_mode="grad",
                 eta0=inp["eta"] * inp["omega"])
    np.testing.assert_allclose(g.U, np.array(exp["grad"]["U"]), rtol=0, atol=1e-15)


def test_target_objective_is_the_objective_at_the_target_lambda():
    """Rounds at the problem's lambda: the Huber form of the objective (S at
    its optimum, Appendix A.2's identity) equals the recorded objective with
    S = soft(R), also in the rounds of a continuation that have reached
    lambda. A multiplier of one is the plain step (to rounding: U + 1 (x - U)
    is x up to an ulp)."""
    inst = planted_instance(60, [20, 25], 3, 0.1, values="signed", lo=5.0, hi=20.0, seed=4)
    lam = 1.0 / math.sqrt(inst.n)
    U0 = gaussian_init(inst.m, 3, 1)
    a = O.dcfpca(inst.blocks(), 3, 0.1, lam, 8, U0)
    for h in a.history:
        assert h["objective_target"] == pytest.approx(h["objective"], rel=1e-12)
    mx = float(np.abs(inst.M).max())
    sched = [max(lam, mx * 0.5 ** t) for t in range(12)]
    b = O.dcfpca(inst.blocks(), 3, 0.1, lam, 12, U0, lam_schedule=sched)
    for lt, h in zip(sched, b.history):
        if lt == lam:
            assert h["objective_target"] == pytest.approx(h["objective"], rel=1e-12)
    c = O.dcfpca(inst.blocks(), 3, 0.1, lam, 8, U0, omega_schedule=[1.0] * 8)
    assert O.relative_error(c.L_full(), a.L_full()) <= 1e-12
    assert O.relative_error(c.S_full(), a.S_full()) <= 1e-12


def _tiny_instance(seed=11, m=40, widths=(7, 13, 5, 15), r=3, s=0.08):
    inst = planted_instance(m, list(widths), r, s, values="uniform", hi=10.0, seed=seed)
    return inst, gaussian_init(m, r, seed + 100)


def test_split_invariance_grad_K1():
    """Section 2.2: with K = 1 the mean of the client steps is one global
    gradient step, so E clients with step eta equal one client with eta / E."""
    inst, U0 = _tiny_instance()
    E = inst.E
    lam, rho, eta = 1 / math.sqrt(inst.n), 0.1, 2e-3
    a = O.dcfpca(inst.blocks(), 3, rho, lam, 25, U0, u_mode="grad", eta0=eta)
    b = O.dcfpca([inst.M], 3, rho, lam, 25, U0, u_mode="grad", eta0=eta / E)
    assert O.relative_error(a.L_full(), b.L_full()) <= 1e-12
    assert O.relative_error(a.S_full(), b.S_full()) <= 1e-12


def _bcd_reference(M, U0, rho, lam, T):
    """Centralised block-coordinate descent on (V, S, U), written separately:
    V and U by lstsq on stacked ridge systems, S by X - clip(X, -lam, lam)."""
    U = U0.copy()
    r = U.shape[1]
    S = np.zeros_like(M)
    V = None
    for _ in range(T):
        A = np.vstack([U, math.sqrt(rho) * np.eye(r)])
        V = np.linalg.lstsq(A, np.vstack([M - S, np.zeros((r, M.shape[1]))]), rcond=None)[0].T
        X = M - U @ V.T
        S = X - np.clip(X, -lam, lam)
        B = np.vstack([V, math.sqrt(rho) * np.eye(r)])
        U = np.linalg.lstsq(B, np.vstack([(M - S).T, np.zeros((r, M.shape[0]))]), rcond=None)[0].T
    return U @ V.T, S


def test_single_client_closed_equals_centralised_bcd():
    """E = 1 (CF-PCA, Section 4.2) with the closed-form U step is plain
    alternating minimisation of eq. "noncovex_problem"."""
    inst, U0 = _tiny_instance(seed=12)
    lam, rho = 1 / math.sqrt(inst.n), 0.1
    res = O.dcfpca([inst.M], 3, rho, lam, 30, U0, u_mode="closed")
    L_ref, S_ref = _bcd_reference(inst.M, U0, rho, lam, 30)
    assert O.relative_error(res.L_full(), L_ref) <= 1e-10
    assert O.relative_error(res.S_full(), S_ref) <= 1e-10


@pytest.mark.parametrize("mode,eta", [("closed", 0.0), ("grad", 1e-3)])
def test_K_local_steps_with_one_client_unroll(mode, eta):
    """With E = 1 the mean is the identity, so K local steps per round for T
    rounds equal K*T rounds of one step (constant eta)."""
    inst, U0 = _tiny_instance(seed=13, m=30, widths=(24,))
    lam, rho = 1 / math.sqrt(inst.n), 0.1
    a = O.dcfpca([inst.M], 3, rho, lam, 4, U0, K=3, u_mode=mode, eta0=eta)
    b = O.dcfpca([inst.M], 3, rho, lam, 12, U0, K=1, u_mode=mode, eta0=eta)
    assert O.relative_error(a.L_full(), b.L_full()) <= 1e-12
    assert O.relative_error(a.S_full(), b.S_full()) <= 1e-12


def test_objective_monotone_single_client():
    """Block-coordinate descent never increases the objective: E = 1 with the
    closed U step, and E = 1 with a gradient step below 1/(||V^T V|| + rho)."""
    inst, U0 = _tiny_instance(seed=14, m=40, widths=(40,))
    lam, rho = 1 / math.sqrt(inst.n), 0.1
    for mode, eta in (("closed", 0.0), ("grad", 2e-3)):
        res = O.dcfpca([inst.M], 3, rho, lam, 60, U0, u_mode=mode, eta0=eta)
        F = np.array([h["objective"] for h in res.history])
        assert np.all(np.diff(F) <= 1e-12 * np.abs(F[:-1])), mode


def test_each_substep_descends_local_objective_many_clients():
    """For any E, each V, S and closed U sub-step minimises its block, so the
    client's local objective L_i never rises within a local step."""
    inst, U0 = _tiny_instance(seed=15)
    lam, rho = 1 / math.sqrt(inst.n), 0.1
    n = inst.n
    U = U0.copy()
    Ms = inst.blocks()
    Ss = [np.zeros_like(Mi) for Mi in Ms]
    Vs = [np.zeros((Mi.shape[1], 3)) for Mi in Ms]
    for _t in range(8):
        new_U = []
        for i, Mi in enumerate(Ms):
            w = Mi.shape[1]
            f0 = O.local_objective(U, Vs[i], Ss[i], Mi, rho, lam, w, n)
            V = O.ridge_V(U, Mi - Ss[i], rho)
            f1 = O.local_objective(U, V, Ss[i], Mi, rho, lam, w, n)
            S = O.soft_threshold(Mi - U @ V.T, lam)
            f2 = O.local_objective(U, V, S, Mi, rho, lam, w, n)
            Ui = O.closed_U(V, S, Mi, rho, w, n)
            f3 = O.local_objective(Ui, V, S, Mi, rho, lam, w, n)
            tol = 1e-12 * abs(f0)
            assert f1 <= f0 + tol and f2 <= f1 + tol and f3 <= f2 + tol
            Vs[i], Ss[i] = V, S
            new_U.append(Ui)
        U = sum(new_U) / len(new_U)


def test_lambda_to_infinity_is_rank_r_singular_value_thresholding():
    """With lambda above max|M| the S-step returns zero, and eq.
    "noncovex_problem" becomes the factored nuclear-norm problem (Section 1):
    its minimiser is sum_{k<=r} max(sigma_k - rho, 0) u_k v_k^T."""
    rng = _rng(16)
    m, n, r = 30, 24, 3
    qu, _ = np.linalg.qr(rng.normal(size=(m, r)))
    qv, _ = np.linalg.qr(rng.normal(size=(n, r)))
    M = qu @ np.diag([10.0, 7.0, 5.0]) @ qv.T + 1e-3 * rng.normal(size=(m, n))
    rho = 0.5
    lam = 10.0 * np.max(np.abs(M))
    U0 = rng.normal(size=(m, r))
    res = O.dcfpca([M], r, rho, lam, 400, U0, u_mode="closed")
    assert np.all(res.S_full() == 0)
    Us, sv, Vt = np.linalg.svd(M)
    L_svt = (Us[:, :r] * np.maximum(sv[:r] - rho, 0.0)) @ Vt[:r]
    assert O.relative_error(res.L_full(), L_svt) <= 1e-8


def test_theorem2_regime_drives_U_to_zero():
    """Theorem 2: when rho^2 > lambda^2 m n the gradient vanishes only at
    U = 0; gradient rounds shrink ||U|| monotonically to zero."""
    inst, U0 = _tiny_instance(seed=17, m=20, widths=(10, 10), r=2)
    lam, rho = 0.01, 1.0
    assert rho ** 2 > lam ** 2 * inst.m * inst.n
    res = O.dcfpca(inst.blocks(), 2, rho, lam, 300, U0, u_mode="grad", eta0=0.5)
    u = np.sqrt([h["u_sq"] for h in res.history])
    assert np.all(np.diff(u) <= 0)
    assert u[-1] <= 1e-6 * np.linalg.norm(U0)


def test_planted_recovery_small_instance():
    """A small planted instance is recovered to the order of the penalty's
    bias (lambda per corrupted entry, rho per singular value)."""
    m = 100
    inst = planted_instance(m, equal_widths(100, 4), 3, 0.05, values="uniform", hi=10.0,
                            seed=18)
    U0 = gaussian_init(m, 3, 118)
    lam, rho = 1 / math.sqrt(inst.n), 0.1
    res = O.dcfpca(inst.blocks(), 3, rho, lam, 800, U0, u_mode="closed")
    err = O.relative_error(res.L_full(), inst.Lstar)
    s, r = 0.05, 3
    floor = math.sqrt(lam ** 2 * s * r * (inst.m + inst.n) + rho ** 2 * r) / np.linalg.norm(inst.Lstar)
    assert err <= 3.0 * floor, (err, floor)


def test_constant_lambda_schedule_is_the_plain_method():
    """A schedule that holds lambda re-evaluates S^(t) as the soft-threshold of
    the residual that produced it, which is the stored S itself: the iterates
    are exactly those of the plain method."""
    inst = planted_instance(60, [20, 25], 3, 0.1, values="signed", lo=5.0, hi=20.0, seed=4)
    lam = 1.0 / math.sqrt(inst.n)
    U0 = gaussian_init(inst.m, 3, 1)
    a = O.dcfpca(inst.blocks(), 3, 0.1, lam, 12, U0)
    b = O.dcfpca(inst.blocks(), 3, 0.1, lam, 12, U0, lam_schedule=[lam] * 12)
    assert np.array_equal(a.L_full(), b.L_full()) and np.array_equal(a.S_full(), b.S_full())
    assert [h["objective"] for h in a.history] == [h["objective"] for h in b.history]


def test_lambda_continuation_shortens_the_early_phase():
    """lambda_t = max(lambda, max|M| 0.8^t): starting with every entry below
    the threshold, L absorbs the bulk of M before S takes the outliers, so the
    planted L* is approached to 1e-2 within 30 rounds, where the plain method
    (S absorbing almost all of the residual from the start, so that L moves
    by about lambda per round) is still far away."""
    inst = planted_instance(300, [100, 100, 100], 5, 0.10, values="signed", lo=5.0, hi=20.0,
                            seed=3)
    lam = 1.0 / math.sqrt(inst.n)
    U0 = gaussian_init(inst.m, 5, 7)
    Ls = inst.Ustar @ inst.Vstar.T
    mx = float(np.abs(inst.M).max())
    sched = [max(lam, mx * 0.8 ** t) for t in range(30)]
    cont = O.dcfpca(inst.blocks(), 5, 0.1, lam, 30, U0, lam_schedule=sched, record=False)
    plain = O.dcfpca(inst.blocks(), 5, 0.1, lam, 30, U0, record=False)
    assert O.relative_error(cont.L_full(), Ls) < 1e-2
    assert O.relative_error(plain.L_full(), Ls) > 0.5


def _mlp_case(seed=0, n=12):
    import oracle.controller as C
    rng = np.random.default_rng(seed)
    p = 0.3 * rng.standard_normal(C.N_PARAMS)
    X = rng.standard_normal((n, C.N_IN))
    T = np.stack([rng.uniform(C.G_MIN, 1.0, n), rng.uniform(C.W_MIN, C.W_MAX, n)], axis=1)
    return C, p, X, T


def test_mlp_gradient_matches_finite_differences():
    """The chain-rule gradient of the controller MLP's mean loss agrees with
    central differences of the loss in every parameter block."""
    C, p, X, T = _mlp_case()
    g = C.grad(p, X, T)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(C.N_PARAMS - 1, 60, replace=False), [C.N_PARAMS - 1]])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (C.loss(p + e, X, T) - C.loss(p - e, X, T)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(fd), (k, fd, g[k])


def test_mlp_special_cases_and_descent():
    """Zero weights give y_k = lo_k + (hi_k - lo_k) sigmoid(b3_k) for every
    input; the outputs stay in [g_min, 1] and [w_min, w_max]; small gradient
    steps decrease the loss."""
    C, p, X, T = _mlp_case(seed=2)
    z = np.zeros(C.N_PARAMS)
    z[-2], z[-1] = 0.7, -1.3
    y, _ = C.forward(z, X)
    assert np.allclose(y[:, 0], C.G_MIN + (1 - C.G_MIN) / (1 + math.exp(-0.7)), rtol=0, atol=1e-15)
    assert np.allclose(y[:, 1], C.W_MIN + (C.W_MAX - C.W_MIN) / (1 + math.exp(1.3)), rtol=0,
                       atol=1e-15)
    y, _ = C.forward(p * 20, X)
    assert np.all(y[:, 0] >= C.G_MIN) and np.all(y[:, 0] <= 1.0)
    assert np.all(y[:, 1] >= C.W_MIN) and np.all(y[:, 1] <= C.W_MAX)
    losses = [C.loss(p, X, T)]
    for _ in range(20):
        p = C.sgd_step(p, X, T, 0.5)
        losses.append(C.loss(p, X, T))
    assert all(b < a for a, b in zip(losses, losses[1:]))
