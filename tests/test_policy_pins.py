"""CPU pins of the policy oracle (Sec. IV-B): least-squares Jacobians and
TVLQR, each checked against something other than the oracle itself —
exact recovery of a linear system that generated the data, the analytic
Jacobian of a smooth nonlinear system, the discrete algebraic Riccati
equation (SciPy), and a brute-force quadratic program over the whole
control sequence."""
import numpy as np
import pytest
import scipy.linalg

from oracle import policy as P
from tests.policy_data import euler_linear_data as _euler_data


def test_p18_recovers_the_linear_system_that_made_the_data():
    rng = np.random.default_rng(0)
    K, H, dt = 64, 12, 0.01
    a_hats = rng.normal(size=(H, 3, 5))
    b_hats = rng.normal(size=(H, 3))
    nom, traj, du = _euler_data(rng, K, H, dt, a_hats, b_hats)
    syn = P.synthesize(nom, traj, du, dt)
    assert np.all(syn["status"] == 0)
    np.testing.assert_allclose(syn["a_hat"], a_hats, rtol=0, atol=1e-8)
    np.testing.assert_allclose(syn["b_hat"], b_hats, rtol=0, atol=1e-8)
    # the discrete map reproduces every perturbed step of the data
    for k in range(H):
        pred = (traj[:, k] - nom[k]) @ syn["A"][k].T + np.outer(du[:, k], syn["B"][k])
        np.testing.assert_allclose(pred, traj[:, k + 1] - nom[k + 1], rtol=0, atol=1e-10)


def _pendulum_glider(x, u):
    """A smooth nonlinear test system with the glider's state layout:
    accelerations depend on theta, phi, x_dot, z_dot, theta_dot and u."""
    th, ph, xd, zd, q = x[..., 2], x[..., 3], x[..., 4], x[..., 5], x[..., 6]
    f = np.zeros(x.shape)
    f[..., 0], f[..., 1], f[..., 2], f[..., 3] = xd, zd, q, u
    f[..., 4] = -0.3 * xd * np.abs(xd) * 0.1 + np.sin(th + ph) + 0.2 * u
    f[..., 5] = -9.81 + 0.5 * xd * np.sin(th) - 0.1 * zd * zd
    f[..., 6] = -4.0 * np.sin(th) - 0.5 * q + 1.5 * np.cos(ph) * u
    return f


def _pendulum_jacobian(x, u):
    th, ph, xd, zd, q = x[2], x[3], x[4], x[5], x[6]
    a = np.zeros((3, 5))          # columns theta, phi, x_dot, z_dot, theta_dot
    a[0] = [np.cos(th + ph), np.cos(th + ph), -0.06 * np.abs(xd), 0, 0]
    a[1] = [0.5 * xd * np.cos(th), 0, 0.5 * np.sin(th), -0.2 * zd, 0]
    a[2] = [-4.0 * np.cos(th), -1.5 * np.sin(ph) * u, 0, 0, -0.5]
    b = np.array([0.2, 0.0, 1.5 * np.cos(ph)])
    return a, b


def test_p18_small_perturbations_give_the_analytic_jacobian():
    # Eq. 26: with perturbations of size s the regression returns the
    # Jacobian at the nominal up to O(s)
    rng = np.random.default_rng(1)
    K, H, dt, s = 200, 6, 0.01, 1e-5
    x0 = np.array([0.0, 0.0, 0.3, -0.2, 6.0, -0.4, 0.5])
    u_nom = 0.3 * np.sin(np.arange(H))
    nom = np.zeros((H + 1, 7))
    nom[0] = x0
    for k in range(H):
        nom[k + 1] = nom[k] + dt * _pendulum_glider(nom[k], u_nom[k])
    traj = np.zeros((K, H + 1, 7))
    traj[:, 0] = x0 + rng.normal(scale=s, size=(K, 7))
    du = rng.normal(scale=s, size=(K, H))
    for k in range(H):
        traj[:, k + 1] = traj[:, k] + dt * _pendulum_glider(traj[:, k], u_nom[k] + du[:, k])
    syn = P.synthesize(nom, traj, du, dt)
    for k in range(H):
        a, b = _pendulum_jacobian(nom[k], u_nom[k])
        np.testing.assert_allclose(syn["a_hat"][k], a, rtol=0, atol=2e-4)
        np.testing.assert_allclose(syn["b_hat"][k], b, rtol=0, atol=2e-4)


def test_p18_rank_deficient_steps_are_flagged():
    rng = np.random.default_rng(2)
    K, H, dt = 32, 4, 0.01
    nom, traj, du = _euler_data(rng, K, H, dt, rng.normal(size=(H, 3, 5)),
                                rng.normal(size=(H, 3)))
    du[:, 1] = 0.0                       # no control excitation at step 1
    syn = P.synthesize(nom, traj, du, dt)
    assert list(syn["status"]) == [0, 1, 0, 0]
    assert np.all(syn["a_hat"][1] == 0) and np.all(syn["b_hat"][1] == 0)
    few = P.synthesize(nom, traj[:5], du[:5], dt)   # 5 samples, 6 unknowns per row
    assert np.all(few["status"] == 1)


def _glider_like_system(rng, dt):
    Ac = np.zeros((7, 7))
    Ac[0, 4] = Ac[1, 5] = Ac[2, 6] = 1.0
    Ac[4:7, 2:7] = rng.normal(scale=0.5, size=(3, 5))
    Bc = np.zeros(7)
    Bc[3] = 1.0
    Bc[4:7] = rng.normal(size=3)
    return np.eye(7) + dt * Ac, dt * Bc


def test_p19_long_horizon_converges_to_the_algebraic_riccati_solution():
    # a generic controllable pair (slightly unstable open loop)
    rng = np.random.default_rng(3)
    A = np.eye(7) + 0.05 * rng.normal(size=(7, 7))
    B = rng.normal(size=7)
    ctrb = np.column_stack([np.linalg.matrix_power(A, i) @ B for i in range(7)])
    assert np.linalg.matrix_rank(ctrb) == 7
    H = 4000
    q_f, q_c, r_c = P.Q_F, P.Q_C, P.R_C
    S, gain = P.tvlqr(np.repeat(A[None], H, 0), np.repeat(B[None], H, 0), q_f, q_c, r_c)
    X = scipy.linalg.solve_discrete_are(A, B[:, None], np.diag(q_c), np.array([[r_c]]))
    np.testing.assert_allclose(S[0], X, rtol=1e-8, atol=1e-8 * np.abs(X).max())
    K_are = np.linalg.solve(np.array([[r_c]]) + B[None] @ X @ B[:, None], B[None] @ X @ A)
    np.testing.assert_allclose(gain[0], K_are[0], rtol=1e-8, atol=1e-10)


def test_p19_cost_to_go_is_the_minimum_of_the_quadratic_program():
    # brute force: the finite-horizon cost is a quadratic in the H controls;
    # its minimum over all control sequences is x0' S_0 x0, and the minimiser
    # is the TVLQR feedback
    rng = np.random.default_rng(4)
    H, dt = 10, 0.05
    As, Bs = zip(*[_glider_like_system(rng, dt) for _ in range(H)])
    A, B = np.array(As), np.array(Bs)
    q_f, q_c, r_c = P.Q_F, P.Q_C, P.R_C
    S, gain = P.tvlqr(A, B, q_f, q_c, r_c)
    x0 = rng.normal(size=7)
    # lifted states x_k = Phi_k x0 + G_k u (u = all H controls)
    Phi = [np.eye(7)]
    G = [np.zeros((7, H))]
    for k in range(H):
        Phi.append(A[k] @ Phi[-1])
        Gk = A[k] @ G[-1]
        Gk[:, k] += B[k]
        G.append(Gk)
    Qs = [np.diag(q_c)] * H + [np.diag(q_f)]
    M = r_c * np.eye(H)
    v = np.zeros(H)
    c = 0.0
    for k in range(H + 1):
        M += G[k].T @ Qs[k] @ G[k]
        v += G[k].T @ Qs[k] @ Phi[k] @ x0
        c += x0 @ Phi[k].T @ Qs[k] @ Phi[k] @ x0
    u_star = -np.linalg.solve(M, v)
    j_star = u_star @ M @ u_star + 2 * v @ u_star + c
    assert abs(j_star - x0 @ S[0] @ x0) <= 1e-9 * abs(j_star)
    # closed loop under the gains reproduces the minimiser
    x = x0.copy()
    u_loop = []
    for k in range(H):
        u_loop.append(-gain[k] @ x)
        x = A[k] @ x + B[k] * u_loop[-1]
    np.testing.assert_allclose(u_loop, u_star, rtol=1e-9, atol=1e-9 * np.abs(u_star).max())


@pytest.mark.parametrize("k", [0, 3])
def test_p19_cost_to_go_matrices_are_symmetric_positive_definite(k):
    rng = np.random.default_rng(5)
    H = 8
    As, Bs = zip(*[_glider_like_system(rng, 0.02) for _ in range(H)])
    S, _ = P.tvlqr(np.array(As), np.array(Bs), P.Q_F, P.Q_C, P.R_C)
    np.testing.assert_allclose(S[k], S[k].T, rtol=0, atol=1e-12 * np.abs(S[k]).max())
    assert np.linalg.eigvalsh(S[k]).min() > 0


# ---------------------- P21 finite-difference Jacobians through the model

def _fd_case(**over):
    from paper_2509_16079_amd import workloads as W
    c = W.replan_case(K=8, H=10, P=0, iterations=1, Kp=8, n_bound=16)
    c["params"] = dict(c["params"], **over)
    return c


def test_p21_fd_nominal_is_the_uninterrupted_rollout():
    from oracle import fd as F
    from oracle import oracle as O
    c = _fd_case()
    A, B, x_nom = F.fd_jacobians(c["params"], c["dt"], c["g"], c["gb"], c["wx"], c["wz"], c["wg"],
                                 c["pairs"], c["u_plan"][:10], [1e-4] * 5, 1e-4)
    ref = O.rollout_batch(c["params"], 1, 10, c["dt"], c["g"][None], c["gb"][None],
                          np.array([0, 2], dtype=np.int64), None, c["wx"], c["wz"], c["wg"],
                          c["pairs"][None], c["u_plan"][None, :10], np.zeros(7), np.zeros(7),
                          traj=True)
    np.testing.assert_allclose(x_nom, ref["traj"][0], rtol=1e-12, atol=1e-14)


def test_p21_no_elevator_area_means_no_control_derivative():
    # u enters the accelerations only through the elevator force
    from oracle import fd as F
    c = _fd_case(s_elev=0.0)
    _, B, _ = F.fd_jacobians(c["params"], c["dt"], c["g"], c["gb"], c["wx"], c["wz"], c["wg"],
                             c["pairs"], c["u_plan"][:10], [1e-4] * 5, 1e-4)
    assert np.all(B[:, 4:7] == 0.0)
    assert np.all(B[:, 3] == c["dt"])


def test_p21_first_step_agrees_with_the_least_squares_synthesis():
    # at step 0 both methods perturb the same state and wake: with 1e-6
    # perturbations of the regressors only (x and z are not regressors, and
    # the wake makes the accelerations depend on them) the regression and
    # the central differences agree to O(h)
    from oracle import fd as F
    from oracle import oracle as O
    c = _fd_case()
    A, B, _ = F.fd_jacobians(c["params"], c["dt"], c["g"], c["gb"], c["wx"], c["wz"], c["wg"],
                             c["pairs"], c["u_plan"][:1], [1e-6] * 5, 1e-6)
    rng = np.random.default_rng(0)
    K = 64
    g0 = np.repeat(c["g"][None], K + 1, 0)
    g0[1:, 2:] += rng.normal(scale=1e-6, size=(K, 5))
    du = np.zeros((K + 1, 1))
    du[1:, 0] = rng.normal(scale=1e-6, size=K)
    tr = O.rollout_batch(c["params"], K + 1, 1, c["dt"], g0, np.zeros((K + 1, 16)),
                         np.array([0, 2], dtype=np.int64), np.zeros(K + 1, dtype=np.int32),
                         c["wx"], c["wz"], c["wg"], None, c["u_plan"][None, :1] + du,
                         np.zeros(7), np.zeros(7), traj=True)["traj"]
    syn = P.synthesize(tr[0], tr[1:], du[1:], c["dt"])
    np.testing.assert_allclose(syn["A"][0], A[0], rtol=0, atol=1e-4 * np.abs(A[0]).max())
    np.testing.assert_allclose(syn["B"][0], B[0], rtol=0, atol=1e-4 * np.abs(B[0]).max())
