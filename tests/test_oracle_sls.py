"""Pins of the output-feedback SLS oracle (Sec. 4.2) against facts that do
not reuse its formulas: Gaussian conditioning of the stacked linear system
(the covariance and the innovation gain the Kalman recursion must produce),
the discrete algebraic Riccati equation (scipy) in the time-invariant limit,
the composition meaning of the scan elements, the observer error and the
closed loop simulated step by step, the affine SLS constraints of eq.
phi_equation, and the worst-case disturbance that attains each tube width."""
import numpy as np
import pytest
import scipy.linalg

from oracle import sls


def _system(seed, N=6, n=3, p=2, m=2):
    rng = np.random.default_rng(seed)
    A = [np.eye(n) + 0.3 * rng.normal(size=(n, n)) for _ in range(N)]
    Bm = [rng.normal(size=(n, m)) for _ in range(N)]
    C = [rng.normal(size=(p, n)) for _ in range(N)]
    E = [0.2 * rng.normal(size=(n, n)) for _ in range(N)]
    F = [0.1 * np.eye(p) + 0.05 * rng.normal(size=(p, p)) for _ in range(N)]
    Xi = 0.5 * rng.normal(size=(n, n))
    return A, Bm, C, E, F, Xi


def _stacked(A, C, E, F, Xi):
    """Each x_j and y_{j+1} as a linear map of z = [xi, w_0.., e_0..] (all
    independent standard normal): x_0 = Xi xi, x_{j+1} = A_j x_j + E_j w_j,
    y_{j+1} = C_j x_j + F_j e_j."""
    N, n, p = len(A), A[0].shape[0], C[0].shape[0]
    dz = n + N * n + N * p
    X = [np.zeros((n, dz))]
    X[0][:, :n] = Xi
    Y = []
    for j in range(N):
        w = np.zeros((n, dz))
        w[:, n + j * n:n + (j + 1) * n] = E[j]
        e = np.zeros((p, dz))
        e[:, n + N * n + j * p:n + N * n + (j + 1) * p] = F[j]
        Y.append(C[j] @ X[j] + e)
        X.append(A[j] @ X[j] + w)
    return X, Y


def test_kalman_is_gaussian_conditioning():
    A, _, C, E, F, Xi = _system(1)
    Pi, L = sls.kalman_serial(A, C, E, F, Xi)
    X, Y = _stacked(A, C, E, F, Xi)
    for j in range(len(A) + 1):
        Sxx = X[j] @ X[j].T
        if j == 0:
            cond = Sxx
        else:
            Ys = np.vstack(Y[:j])
            G = X[j] @ Ys.T @ np.linalg.inv(Ys @ Ys.T)
            cond = Sxx - G @ Ys @ X[j].T
            # the coefficient of the newest measurement y_j is -L_j^T
            np.testing.assert_allclose(G[:, -C[0].shape[0]:], -L[j - 1].T, rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(Pi[j], cond, rtol=1e-9, atol=1e-11)


def test_kalman_reaches_the_riccati_fixed_point():
    rng = np.random.default_rng(2)
    n, p, N = 4, 2, 400
    A0 = 0.9 * np.linalg.qr(rng.normal(size=(n, n)))[0] + 0.05 * rng.normal(size=(n, n))
    C0 = rng.normal(size=(p, n))
    E0 = 0.3 * rng.normal(size=(n, n))
    F0 = 0.2 * np.eye(p)
    Pi, L = sls.kalman_serial([A0] * N, [C0] * N, [E0] * N, [F0] * N, np.eye(n))
    X = scipy.linalg.solve_discrete_are(A0.T, C0.T, E0 @ E0.T, F0 @ F0.T)
    np.testing.assert_allclose(Pi[-1], X, rtol=1e-10, atol=1e-12)
    K = A0 @ X @ C0.T @ np.linalg.inv(F0 @ F0.T + C0 @ X @ C0.T)      # predictor gain
    np.testing.assert_allclose(-L[-1].T, K, rtol=1e-9, atol=1e-12)


def _random_element(rng, n):
    G = rng.normal(size=(n, n))
    H = rng.normal(size=(n, n))
    return (rng.normal(size=(n, n)), G @ G.T / n, H @ H.T / n)


def test_combination_is_composition_and_associative():
    rng = np.random.default_rng(3)
    n = 4
    for _ in range(5):
        a, b, c = (_random_element(rng, n) for _ in range(3))
        H = rng.normal(size=(n, n))
        Pi = H @ H.T
        np.testing.assert_allclose(sls.apply(sls.combine(a, b), Pi), sls.apply(b, sls.apply(a, Pi)),
                                   rtol=1e-9, atol=1e-10)
        left = sls.combine(sls.combine(a, b), c)
        right = sls.combine(a, sls.combine(b, c))
        for u, v in zip(left, right):
            np.testing.assert_allclose(u, v, rtol=1e-9, atol=1e-10)


def test_scans_reproduce_the_recursion():
    A, _, C, E, F, Xi = _system(4, N=11)
    Pi, L = sls.kalman_serial(A, C, E, F, Xi)
    el = sls.elements(A, C, E, F, Xi)
    np.testing.assert_allclose(sls.kalman_scan_sequential(el), Pi, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(sls.kalman_scan_tree(el), Pi, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(sls.gains(A, C, F, Pi), L, rtol=1e-9, atol=1e-11)


def test_observer_error_superposition_and_constraint():
    A, _, C, E, F, Xi = _system(5)
    N, n, p = len(A), A[0].shape[0], C[0].shape[0]
    _, L = sls.kalman_serial(A, C, E, F, Xi)
    Phx, Phy = sls.observer(A, C, L)
    # affine constraint of eq. phi_equation restricted to the observer response
    M = np.eye((N + 1) * n) - sls.downshift(A, N)
    ZC = sls.downshift(C, N)
    np.testing.assert_allclose(sls.dense(Phx) @ M - sls.dense(Phy) @ ZC, np.eye((N + 1) * n), atol=1e-11)
    # the observer run step by step: the error is the superposition
    rng = np.random.default_rng(6)
    x = rng.normal(size=n)
    xh = np.zeros(n)
    w = rng.normal(size=(N, n))
    e = rng.normal(size=(N, p))
    err = [x - xh]
    for j in range(N):
        y = C[j] @ x + F[j] @ e[j]
        xh = A[j] @ xh - L[j].T @ (y - C[j] @ xh)
        x = A[j] @ x + E[j] @ w[j]
        err.append(x - xh)
    for k in range(N + 1):
        s = Phx[k, 0] @ err[0]
        for j in range(k):
            s = s + Phx[k, j + 1] @ E[j] @ w[j] + Phy[k, j + 1] @ F[j] @ e[j]
        np.testing.assert_allclose(s, err[k], rtol=1e-9, atol=1e-11)


def _closed_loop(A, Bm, C, E, F, K, L, x0, w, e):
    """u_j = K_j xhat_j with the Kalman observer, run step by step."""
    N = len(A)
    x, xh = x0.copy(), np.zeros_like(x0)
    xs, us = [x.copy()], []
    for j in range(N):
        u = K[j] @ xh
        y = C[j] @ x + F[j] @ e[j]
        xh = A[j] @ xh + Bm[j] @ u - L[j].T @ (y - C[j] @ xh)
        x = A[j] @ x + Bm[j] @ u + E[j] @ w[j]
        xs.append(x.copy())
        us.append(u)
    us.append(K[N] @ xh)
    return np.concatenate(xs), np.concatenate(us)


def test_assembly_is_the_observer_based_closed_loop():
    A, Bm, C, E, F, Xi = _system(7)
    N, n, p, m = len(A), A[0].shape[0], C[0].shape[0], Bm[0].shape[1]
    rng = np.random.default_rng(8)
    K = [0.3 * rng.normal(size=(m, n)) for _ in range(N + 1)]
    _, L = sls.kalman_serial(A, C, E, F, Xi)
    Phx, Phy = sls.observer(A, C, L)
    Pbx, Pbu = sls.state_feedback(A, Bm, K)
    ZA, ZB, ZC = sls.downshift(A, N), sls.downshift(Bm, N), sls.downshift(C, N)
    M = np.eye((N + 1) * n) - ZA
    xw, uw, xe, ue = sls.assemble(Pbx, Pbu, sls.dense(Phx), sls.dense(Phy), M)
    Phi = np.block([[xw, xe], [uw, ue]])
    # both affine constraints of eq. phi_equation
    D = (N + 1) * n
    lhs = np.hstack([M, -ZB]) @ Phi
    np.testing.assert_allclose(lhs, np.hstack([np.eye(D), np.zeros((D, (N + 1) * p))]), atol=1e-10)
    rhs = Phi @ np.vstack([M, -ZC])
    np.testing.assert_allclose(rhs, np.vstack([np.eye(D), np.zeros(((N + 1) * m, D))]), atol=1e-10)
    # the responses of the observer-based controller to x0, w, e
    x0 = rng.normal(size=n)
    w = rng.normal(size=(N, n))
    e = rng.normal(size=(N, p))
    xs, us = _closed_loop(A, Bm, C, E, F, K, L, x0, w, e)
    wt = np.concatenate([x0] + [E[j] @ w[j] for j in range(N)])
    et = np.concatenate([np.zeros(p)] + [F[j] @ e[j] for j in range(N)])
    np.testing.assert_allclose(xw @ wt + xe @ et, xs, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(uw @ wt + ue @ et, us, rtol=1e-9, atol=1e-10)


def test_tube_width_is_attained_by_the_worst_disturbance():
    A, Bm, C, E, F, Xi = _system(9)
    N, n, p, m = len(A), A[0].shape[0], C[0].shape[0], Bm[0].shape[1]
    rng = np.random.default_rng(10)
    K = [0.3 * rng.normal(size=(m, n)) for _ in range(N + 1)]
    _, L = sls.kalman_serial(A, C, E, F, Xi)
    Phx, Phy = sls.observer(A, C, L)
    Pbx, Pbu = sls.state_feedback(A, Bm, K)
    M = np.eye((N + 1) * n) - sls.downshift(A, N)
    xw, uw, xe, ue = sls.assemble(Pbx, Pbu, sls.dense(Phx), sls.dense(Phy), M)
    tau = sls.tubes(xw, xe, E, F, n, p)
    assert np.all(tau[0] == 0)
    for k, r in [(N, 0), (N, n - 1), (3, 1), (1, 2)]:
        w = np.zeros((N, n))
        e = np.zeros((N, p))
        for j in range(k):
            # the unit vector aligned with this state's row of each block
            rw = xw[k * n + r, (j + 1) * n:(j + 2) * n] @ E[j]
            re = xe[k * n + r, (j + 1) * p:(j + 2) * p] @ F[j]
            # (the last measurement noise cannot reach x_k yet: its block is 0)
            w[j] = rw / max(np.linalg.norm(rw), 1e-300)
            e[j] = re / max(np.linalg.norm(re), 1e-300)
        xs, _ = _closed_loop(A, Bm, C, E, F, K, L, np.zeros(n), w, e)
        assert xs[k * n + r] == pytest.approx(tau[k, r], rel=1e-9)
    # random disturbances in the unit balls stay inside the tubes
    for _ in range(20):
        w = rng.normal(size=(N, n))
        w /= np.maximum(1.0, np.linalg.norm(w, axis=1))[:, None]
        e = rng.normal(size=(N, p))
        e /= np.maximum(1.0, np.linalg.norm(e, axis=1))[:, None]
        xs, _ = _closed_loop(A, Bm, C, E, F, K, L, np.zeros(n), w, e)
        assert np.all(np.abs(xs.reshape(N + 1, n)) <= tau + 1e-12)


def test_transitions_of_identity_and_nilpotent_steps():
    n, N = 3, 5
    T = sls.transitions([np.eye(n)] * N)
    for k in range(N + 1):
        for j in range(k + 1):
            np.testing.assert_array_equal(T[k, j], np.eye(n))
    S = np.diag([1.0, 1.0], k=1)          # shift: S^3 = 0
    T = sls.transitions([S] * N)
    np.testing.assert_array_equal(T[4, 1], np.zeros((n, n)))
    np.testing.assert_array_equal(T[3, 1], S @ S)
