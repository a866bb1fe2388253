"""Plain FP64 oracle of the local feedback policy (Sec. IV-B of Gupta et al.,
arXiv 2509.16079): least-squares Jacobians from rollouts, then TVLQR.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this module. It never imports the GPU
package, and the GPU package never imports it.

State order x_g = (x, z, theta, phi, x_dot, z_dot, theta_dot), control
u = phi_dot (Sec. III-B). Readings taken where the text is garbled:

* State rates. The rollouts step every state by explicit Euler, so the rate
  of a state at step k is exactly (x_{k+1} - x_k) / dt.
* Eq. 28. Of the continuous-time Jacobians only the three acceleration rows
  are regressed, on the five columns theta, phi, x_dot, z_dot, theta_dot
  (the 3 x 5 block A_hat) and on u (the 3 x 1 block B_hat). The other rows
  are kinematic and known: the rates of x, z, theta are the states x_dot,
  z_dot, theta_dot, and the rate of phi is u. The printed identity block of
  the first three rows reads as this kinematic coupling.
* The TVLQR of Eqs. 29-30 runs on the explicit-Euler discretisation that
  the rollouts integrate, A_k = I + dt dF/dx and B_k = dt dF/du, and pairs
  A_k, B_k with the cost-to-go of the next step in the recursion as the
  gain equation does: S_k = A_k' S_{k+1} A_k - A_k' S_{k+1} B_k
  (R + B_k' S_{k+1} B_k)^-1 B_k' S_{k+1} A_k + Q from S_N = Q_f. S is
  symmetric; each step keeps it so by averaging with its transpose, since
  rounding would otherwise seed an antisymmetric part that the recursion
  multiplies by A_k' ... A_k, which grows when the open loop is unstable.
* A time step whose regression matrix [dX dU] (K x 6) is rank-deficient
  (fewer than 6 samples, a zero column, or a smallest singular value at most
  1e-7 times the largest after scaling each column to unit norm) gets
  A_hat = 0, B_hat = 0 and a status flag.
"""
from __future__ import annotations

import numpy as np

N_X = 7
ACC = (4, 5, 6)            # rows of the accelerations (A_hat, B_hat rows)
REG = (2, 3, 4, 5, 6)      # state columns of A_hat
RANK_TOL = 1e-7


def state_rates(traj: np.ndarray, dt: float) -> np.ndarray:
    """Rates of the states along trajectories [..., H + 1, 7]: exact for an
    explicit Euler integration. Returns [..., H, 7]."""
    traj = np.asarray(traj, dtype=np.float64)
    return (traj[..., 1:, :] - traj[..., :-1, :]) / dt


def regress_step(dx: np.ndarray, du: np.ndarray, dxdot: np.ndarray):
    """Eq. 27 at one time step with the sparsity of Eq. 28.

    dx [K, 7] state deviations from the nominal, du [K] control deviations,
    dxdot [K, 7] rate deviations. Returns (A_hat [3, 5], B_hat [3], ok)."""
    Z = np.concatenate([dx[:, REG], du[:, None]], axis=1)     # K x 6 regressors
    Y = dxdot[:, ACC]                                          # K x 3 targets
    norms = np.linalg.norm(Z, axis=0)
    if np.any(norms == 0.0):
        return np.zeros((3, 5)), np.zeros(3), False
    sv = np.linalg.svd(Z / norms, compute_uv=False)   # min(K, 6) values
    if sv.size < Z.shape[1] or sv[-1] <= RANK_TOL * sv[0]:
        return np.zeros((3, 5)), np.zeros(3), False
    W, *_ = np.linalg.lstsq(Z, Y, rcond=None)                  # 6 x 3: [A_hat'; B_hat']
    return W[:5].T.copy(), W[5].copy(), True


def continuous_jacobians(a_hat: np.ndarray, b_hat: np.ndarray):
    """Eq. 28: the full 7 x 7 and 7 x 1 continuous-time Jacobians from the
    regressed blocks and the known kinematic rows."""
    A = np.zeros((N_X, N_X))
    B = np.zeros(N_X)
    A[0, 4] = A[1, 5] = A[2, 6] = 1.0
    B[3] = 1.0
    A[np.ix_(ACC, REG)] = a_hat
    B[list(ACC)] = b_hat
    return A, B


def synthesize(traj_nom, traj, du, dt):
    """Least-squares Jacobians at every step (Eqs. 26-28).

    traj_nom [H + 1, 7] the nominal trajectory, traj [K, H + 1, 7] the
    perturbed rollouts, du [K, H] their control deviations from the nominal.
    Returns dict with a_hat [H, 3, 5], b_hat [H, 3], A [H, 7, 7] and
    B [H, 7] (discrete, explicit Euler), status [H] (1 = rank-deficient)."""
    traj_nom = np.asarray(traj_nom, dtype=np.float64)
    traj = np.asarray(traj, dtype=np.float64)
    du = np.asarray(du, dtype=np.float64)
    K, H1, _ = traj.shape
    H = H1 - 1
    rate_nom = state_rates(traj_nom, dt)
    rate = state_rates(traj, dt)
    out = dict(a_hat=np.zeros((H, 3, 5)), b_hat=np.zeros((H, 3)),
               A=np.zeros((H, N_X, N_X)), B=np.zeros((H, N_X)),
               status=np.zeros(H, dtype=np.int32))
    for k in range(H):
        a_hat, b_hat, ok = regress_step(traj[:, k] - traj_nom[k], du[:, k],
                                        rate[:, k] - rate_nom[k])
        Ac, Bc = continuous_jacobians(a_hat, b_hat)
        out["a_hat"][k], out["b_hat"][k] = a_hat, b_hat
        out["A"][k] = np.eye(N_X) + dt * Ac
        out["B"][k] = dt * Bc
        out["status"][k] = 0 if ok else 1
    return out


def tvlqr(A, B, q_f, q_c, r_c):
    """Eqs. 29-30 backwards from S_N = Q_f (diagonal weights q_f, q_c; scalar
    r_c for the one control). A [H, 7, 7], B [H, 7]. Returns S [H + 1, 7, 7]
    and the gains [H, 7] (u_k = u_k^d - gain_k . (x_k - x_k^d))."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    H = A.shape[0]
    Q = np.diag(np.asarray(q_c, dtype=np.float64))
    S = np.zeros((H + 1, N_X, N_X))
    gain = np.zeros((H, N_X))
    S[H] = np.diag(np.asarray(q_f, dtype=np.float64))
    for k in range(H - 1, -1, -1):
        Sn, Ak, Bk = S[k + 1], A[k], B[k]
        inv = 1.0 / (r_c + Bk @ Sn @ Bk)          # (R + B'SB)^-1, one control
        BSA = Bk @ Sn @ Ak                          # B'SA, a row of 7
        Sk = Ak.T @ Sn @ Ak - np.outer(BSA, BSA) * inv + Q     # Eq. 29
        S[k] = 0.5 * (Sk + Sk.T)
        gain[k] = inv * BSA                         # Eq. 30
    return S, gain


def policy(traj_nom, traj, du, dt, q_f, q_c, r_c):
    """Sec. IV-B end to end: synthesis, then TVLQR."""
    syn = synthesize(traj_nom, traj, du, dt)
    S, gain = tvlqr(syn["A"], syn["B"], q_f, q_c, r_c)
    syn["S"], syn["gain"] = S, gain
    return syn


# TVLQR weights of the paper's experiments (Sec. V-A)
Q_F = np.array([400.0, 400.0, 10.0, 1.0, 1.0, 1.0, 1.0])
Q_C = np.array([0.1, 0.1, 5.0, 0.1, 0.1, 0.1, 5.0])
R_C = 0.01
