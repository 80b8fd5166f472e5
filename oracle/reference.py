"""Plain FP64 CPU oracle for DCF-PCA (arXiv 2207.11669).

TEST INFRASTRUCTURE. Only the test suite, the package's smoke check and the
benchmark's CPU-baseline leg may import or run anything in this directory. The
GPU library never calls it and shares no code with it; the two meet only on
inputs drawn by `rpca_inputs`.

What it computes: Algorithm 1 (Section 2.2) for the nonconvex objective

    1/2 ||U V^T + S - M||_F^2 + rho/2 (||U||_F^2 + ||V||_F^2) + lambda ||S||_1

(Section 1, eq. "noncovex_problem"), with M split column-wise over E clients
(Section 2.1). Everything is float64 numpy; library primitives (matmul, solve,
Cholesky) serve as steps, and nothing is fused, blocked or reordered beyond the
paper's own order. Clients run one after another, as the paper's experiments
do (Section 4.1, "Implementation").

Readings taken where the paper is silent, garbled or ambiguous:

* The local (V, S) argmin of eq. "VS_arg" is reached by `inner` Gauss-Seidel
  alternations of the two closed forms: V from the ridge normal equations of
  the Lemma 4 proof (eq. "condition1"), then S by the soft-threshold of
  eq. "optS". One alternation is the default; the exact argmin is the limit.
  The displayed form just before eq. "optS" carries a stray factor V on both
  sides; eq. "condition1" is used instead.
* The local U step (eq. "U_local") has garbled indices; it is taken at the
  local iterate with the fresh (V, S): U <- U - eta * grad_U L_i(U, V_new, S_new),
  which is the gradient step on g_i that Lemma 2 describes.
* The U-gradient regulariser is rho * n_i / n * U, as follows from the
  definition of L_i (Section 2.2); the Lemma 4 proof drops rho.
* Besides that literal gradient step ("grad"), a closed-form U step
  ("closed") is offered: U <- argmin_U L_i(U, V, S) = (M_i - S_i) V (V^T V +
  rho n_i / n I)^{-1}. It has no step size; with E = 1 it is centralised
  alternating minimisation (the CF-PCA baseline of Section 4.2).
* Consensus is the unweighted mean of the client factors (eq. "U_agg").
* S_i^(0) = 0 (a random dense start contradicts the sparsity prior); V_i^(0) is
  never used because every local step computes V first. U^(0) is an input.
* eta_sched "const" uses eta0 every round; "sqrt" uses eta0 / sqrt(t + 1) with
  t the round index, a concrete form of the decaying rate of Section 4.2 that
  is defined at t = 0.
* The recorded round objective is sum_i L_i(U_i, V_i, S_i) at the last local
  (V, S) update of the round, with U_i the client's factor before its U step.
* A lambda schedule (lambda_t per round; the paper fixes lambda, so this is
  the caller's choice, e.g. a continuation down to the target) is read as:
  round t minimises the objective at lambda_t, so its alternation starts with
  the S-subproblem (eq. "optS") at lambda_t solved exactly for the factors
  that produced the last residual, S^(t) = soft(M_i - U^(t-1) V_i^(t)T,
  lambda_t), the S that objective prescribes for those factors; every later
  soft-threshold of the round uses lambda_t too. With one alternation and
  K = 1 the stored S of the previous round is exactly that soft-threshold
  when lambda does not change, so a constant schedule is the plain method.
  (Keeping the stored S instead would start round t from an S that is optimal
  for lambda_{t-1}, not for the objective the round descends.)

Parity pins live in the test suite; every function here is pinned by at least
one check that does not retype its formula (closed forms, library routines of
another kind, brute force, invariants, hand-derived values).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "soft_threshold",
    "huber",
    "ridge_V",
    "inner_solve",
    "grad_U",
    "closed_U",
    "local_objective",
    "objective",
    "eta_at",
    "Result",
    "dcfpca",
    "relative_error",
]


def soft_threshold(X: np.ndarray, lam: float) -> np.ndarray:
    """S-subproblem solution, eq. "optS": sign(X) * max(|X| - lambda, 0)."""
    return np.sign(X) * np.maximum(np.abs(X) - lam, 0.0)


def huber(X: np.ndarray, lam: float) -> float:
    """Huber loss H_lambda summed over entries (Appendix A.2, piecewise form)."""
    X = np.asarray(X, dtype=np.float64)
    a = np.abs(X)
    inner = a <= lam
    return float(np.sum(np.where(inner, 0.5 * X * X, lam * a - 0.5 * lam * lam)))


def ridge_V(U: np.ndarray, D: np.ndarray, rho: float) -> np.ndarray:
    """V-subproblem solution for fixed S, eq. "condition1" (Lemma 4 proof):
    (U^T U + rho I) V^T = U^T D with D = M_i - S_i. Returns V (n_i x r)."""
    r = U.shape[1]
    G = U.T @ U + rho * np.eye(r)
    return np.linalg.solve(G, U.T @ D).T


def inner_solve(U: np.ndarray, M: np.ndarray, S: np.ndarray, rho: float, lam: float,
                inner: int = 1):
    """Local (V, S) step of eq. "VS_arg" by `inner` alternations (V first,
    then S from the new V). Returns (V, S, R) with R = M - U V^T of the last
    alternation."""
    V = None
    R = None
    for _ in range(int(inner)):
        V = ridge_V(U, M - S, rho)
        R = M - U @ V.T
        S = soft_threshold(R, lam)
    return V, S, R


def grad_U(U: np.ndarray, V: np.ndarray, S: np.ndarray, M: np.ndarray, rho: float,
           n_i: int, n: int) -> np.ndarray:
    """grad_U L_i(U, V, S) = (U V^T + S - M) V + rho n_i / n U (Lemma 2 proof)."""
    return (U @ V.T + S - M) @ V + (rho * n_i / n) * U


def closed_U(V: np.ndarray, S: np.ndarray, M: np.ndarray, rho: float, n_i: int,
             n: int) -> np.ndarray:
    """argmin_U L_i(U, V, S) = (M - S) V (V^T V + rho n_i / n I)^{-1}."""
    r = V.shape[1]
    A = V.T @ V + (rho * n_i / n) * np.eye(r)
    return np.linalg.solve(A, ((M - S) @ V).T).T


def local_objective(U: np.ndarray, V: np.ndarray, S: np.ndarray, M: np.ndarray,
                    rho: float, lam: float, n_i: int, n: int) -> float:
    """L_i(U, V_i, S_i) of Section 2.2 (local objective under consensus)."""
    resid = U @ V.T + S - M
    return float(0.5 * np.sum(resid * resid) + 0.5 * rho * np.sum(V * V)
                 + lam * np.sum(np.abs(S)) + 0.5 * rho * (n_i / n) * np.sum(U * U))


def objective(U: np.ndarray, Vs: Sequence[np.ndarray], Ss: Sequence[np.ndarray],
              Ms: Sequence[np.ndarray], rho: float, lam: float) -> float:
    """Global objective, eq. "noncovex_problem", with V and S split by client."""
    total = 0.5 * rho * float(np.sum(U * U))
    for V, S, M in zip(Vs, Ss, Ms):
        resid = U @ V.T + S - M
        total += float(0.5 * np.sum(resid * resid) + 0.5 * rho * np.sum(V * V)
                       + lam * np.sum(np.abs(S)))
    return total


def eta_at(eta0: float, sched: str, t: int) -> float:
    if sched == "const":
        return float(eta0)
    if sched == "sqrt":
        return float(eta0) / math.sqrt(t + 1.0)
    raise ValueError(f"unknown eta schedule {sched!r}")


@dataclasses.dataclass
class Result:
    U: np.ndarray
    V: List[np.ndarray]
    S: List[np.ndarray]
    history: List[dict]

    @property
    def L(self) -> List[np.ndarray]:
        """Algorithm 1's output L_i = U^(T) V_i^T."""
        return [self.U @ V.T for V in self.V]

    def L_full(self) -> np.ndarray:
        return np.concatenate(self.L, axis=1)

    def S_full(self) -> np.ndarray:
        return np.concatenate(self.S, axis=1)


def dcfpca(Ms: Sequence[np.ndarray], r: int, rho: float, lam: float, T: int,
           U0: np.ndarray, K: int = 1, inner: int = 1, u_mode: str = "closed",
           eta0: float = 0.0, eta_sched: str = "const",
           S0: Optional[Sequence[np.ndarray]] = None, t0: int = 0,
           record: bool = True, lam_schedule: Optional[Sequence[float]] = None,
           omega_schedule: Optional[Sequence[float]] = None) -> Result:
    """Algorithm 1 (Section 2.2): T rounds of broadcast, K local steps per
    client, and the mean of the client factors.

    Ms: the client blocks M_i (m x n_i). U0: U^(0) (m x r). S0: optional
    starting S_i (default zeros). t0: index of the first round (for the eta
    schedule when resuming). lam_schedule: optional lambda_t for each of the T
    rounds (K = 1 and inner = 1 only; see the module's readings).
    omega_schedule: optional multiplier omega_t of each round's consensus
    step, U^(t+1) = U^(t) + omega_t (mean_i U_i - U^(t)) (a relaxation of eq.
    "U_agg"; for the gradient step, the step size omega_t eta). The recorded
    objective_target is the objective at lambda (the problem's, not lambda_t)
    with S at its optimum for the round's factors: by the Huber identity of
    Appendix A.2, sum_i H_lambda(M_i - U_i V_i^T) plus the penalties.
    """
    Ms = [np.asarray(Mi, dtype=np.float64) for Mi in Ms]
    E = len(Ms)
    widths = [Mi.shape[1] for Mi in Ms]
    n = int(sum(widths))
    U = np.array(U0, dtype=np.float64, copy=True)
    if U.shape[1] != r:
        raise ValueError("U0 must have r columns")
    S = [np.zeros_like(Mi) if S0 is None else np.array(S0[i], dtype=np.float64, copy=True)
         for i, Mi in enumerate(Ms)]
    V: List[Optional[np.ndarray]] = [None] * E
    if lam_schedule is not None:
        if K != 1 or inner != 1:
            raise ValueError("a lambda schedule needs K = 1 and inner = 1")
        if len(lam_schedule) < T:
            raise ValueError("lam_schedule needs one lambda per round")
    if omega_schedule is not None and len(omega_schedule) < T:
        raise ValueError("omega_schedule needs one multiplier per round")
    R_last: List[Optional[np.ndarray]] = [None] * E
    history = []
    for t in range(int(t0), int(t0) + int(T)):
        lam_t = lam if lam_schedule is None else float(lam_schedule[t - int(t0)])
        eta = eta_at(eta0, eta_sched, t) if u_mode == "grad" else 0.0
        client_U = []
        F = 0.0
        F_target = 0.0
        lam_sq = 0.0
        nnz = 0
        for i in range(E):  # clients one after another (Section 4.1)
            Ui = U.copy()  # broadcast of U^(t) (eq. "U_agg" of the previous round)
            if lam_schedule is not None and R_last[i] is not None:
                S[i] = soft_threshold(R_last[i], lam_t)  # S^(t) at lambda_t
            for _k in range(int(K)):
                Vi, Si, Ri = inner_solve(Ui, Ms[i], S[i], rho, lam_t, inner)
                R_last[i] = Ri
                if record and _k == K - 1:
                    F += local_objective(Ui, Vi, Si, Ms[i], rho, lam_t, widths[i], n)
                    F_target += (huber(Ri, lam) + 0.5 * rho * float(np.sum(Vi * Vi))
                                 + 0.5 * rho * (widths[i] / n) * float(np.sum(Ui * Ui)))
                    Lam = Ri - Si
                    lam_sq += float(np.sum(Lam * Lam))
                    nnz += int(np.count_nonzero(Si))
                if u_mode == "grad":
                    Ui = Ui - eta * grad_U(Ui, Vi, Si, Ms[i], rho, widths[i], n)
                elif u_mode == "closed":
                    Ui = closed_U(Vi, Si, Ms[i], rho, widths[i], n)
                else:
                    raise ValueError(f"unknown u_mode {u_mode!r}")
                V[i] = Vi
                S[i] = Si
            client_U.append(Ui)
        U_new = sum(client_U) / E  # eq. "U_agg"
        if omega_schedule is not None:
            U_new = U + float(omega_schedule[t - int(t0)]) * (U_new - U)
        if record:
            du = U_new - U
            history.append(dict(t=t, objective=F, lambda_fro_sq=lam_sq, nnz=nnz,
                                du_sq=float(np.sum(du * du)), u_sq=float(np.sum(U_new * U_new)),
                                objective_target=F_target))
        U = U_new
    return Result(U=U, V=[v for v in V], S=S, history=history)


def relative_error(A: np.ndarray, B: np.ndarray) -> float:
    """||A - B||_F / ||B||_F."""
    den = float(np.linalg.norm(B))
    return float(np.linalg.norm(A - B)) / (den if den > 0 else 1.0)
