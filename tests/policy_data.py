"""Seeded inputs of the policy tests (shared by the oracle pins and the GPU
parity tests; no step of the method is computed here).

euler_linear_data: a nominal trajectory and K perturbed trajectories whose
deviations follow a given linear system with the glider's kinematic rows,
stepped by explicit Euler."""
import numpy as np


def euler_linear_data(rng, K, H, dt, a_hats, b_hats, sx=0.02, su=0.1):
    """Deviations obey d(dx)/dt = A_c,k dx + B_c,k du with the acceleration
    rows of A_c,k, B_c,k given by a_hats [H, 3, 5] (columns theta, phi,
    x_dot, z_dot, theta_dot) and b_hats [H, 3]; the rates of x, z, theta are
    x_dot, z_dot, theta_dot and the rate of phi is du. Returns (nominal
    [H+1, 7], trajectories [K, H+1, 7], du [K, H])."""
    nom = np.cumsum(rng.normal(size=(H + 1, 7)), axis=0)
    dx = np.zeros((K, H + 1, 7))
    dx[:, 0] = rng.normal(scale=sx, size=(K, 7))
    du = rng.normal(scale=su, size=(K, H))
    for k in range(H):
        d = dx[:, k]
        rate = np.zeros((K, 7))
        rate[:, 0], rate[:, 1], rate[:, 2] = d[:, 4], d[:, 5], d[:, 6]
        rate[:, 3] = du[:, k]
        rate[:, 4:7] = d[:, 2:7] @ a_hats[k].T + np.outer(du[:, k], b_hats[k])
        dx[:, k + 1] = d + dt * rate
    return nom, nom[None] + dx, du
