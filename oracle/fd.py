"""Plain FP64 oracle of the finite-difference Jacobians that Sec. IV-B of
Gupta et al. (arXiv 2509.16079) compares its least-squares synthesis with.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this module. It never imports the GPU
package, and the GPU package never imports it.

Reading (the paper names the method, not its steps): along the nominal
trajectory, at every step k the one-step accelerations (x_{k+1} - x_k)/dt of
the velocity rows are differenced centrally in each of theta, phi, x_dot,
z_dot, theta_dot and in u, every perturbed step starting from the nominal's
full state at step k (glider, previous bound circulations, wake); the
Jacobians then take the same form as the least-squares ones (Eq. 28, explicit
Euler).
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from oracle import policy as P

X_OX = (2, 3, 4, 5, 6)     # theta, phi, x_dot, z_dot, theta_dot


def _one_step(params, dt, g0s, gb, wx, wz, wg, pairs, u):
    """One step of len(g0s) rollouts from one shared wake; returns the
    oracle outputs with final wake and bound circulations."""
    K = len(g0s)
    pr = None if pairs is None else np.repeat(np.asarray(pairs, dtype=np.int32)[None], K, 0)
    return O.rollout_batch(params, K, 1, dt, np.asarray(g0s), np.repeat(gb[None], K, 0),
                           np.array([0, len(wx)], dtype=np.int64), np.zeros(K, dtype=np.int32),
                           wx, wz, wg, pr, np.asarray(u, dtype=np.float64)[:, None],
                           np.zeros(7), np.zeros(7), final_wake=True, gb_final=True)


def fd_jacobians(params, dt, g, gb, wx, wz, wg, pairs, u_nom, h_x, h_u):
    """Returns A [H, 7, 7], B [H, 7] (explicit Euler form) and the nominal
    trajectory [H + 1, 7]."""
    g = np.asarray(g, dtype=np.float64)
    gb = np.asarray(gb, dtype=np.float64)
    wx, wz, wg = (np.asarray(a, dtype=np.float64) for a in (wx, wz, wg))
    u_nom = np.asarray(u_nom, dtype=np.float64)
    H = len(u_nom)
    A = np.zeros((H, 7, 7))
    B = np.zeros((H, 7))
    x_nom = np.zeros((H + 1, 7))
    for k in range(H):
        x_nom[k] = g
        g0s = [g.copy()]
        for j, c in enumerate(X_OX):
            for sgn in (1.0, -1.0):
                x = g.copy()
                x[c] += sgn * h_x[j]
                g0s.append(x)
        g0s += [g.copy(), g.copy()]
        u = [u_nom[k]] * 11 + [u_nom[k] + h_u, u_nom[k] - h_u]
        out = _one_step(params, dt, g0s, gb, wx, wz, wg, pairs, u)
        acc = (out["g_final"][:, 4:7] - np.asarray(g0s)[:, 4:7]) / dt
        a_hat = np.zeros((3, 5))
        for j in range(5):
            a_hat[:, j] = (acc[1 + 2 * j] - acc[2 + 2 * j]) / (2.0 * h_x[j])
        b_hat = (acc[11] - acc[12]) / (2.0 * h_u)
        Ac, Bc = P.continuous_jacobians(a_hat, b_hat)
        A[k] = np.eye(7) + dt * Ac
        B[k] = dt * Bc
        # the nominal advances by row 0's step
        n = int(out["n_final"][0])
        o0 = out["out_off"][0]
        g, gb = out["g_final"][0].copy(), out["gb_final"][0].copy()
        wx, wz, wg = (out[key][o0:o0 + n].copy() for key in ("wx", "wz", "wg"))
    x_nom[H] = g
    return A, B, x_nom
