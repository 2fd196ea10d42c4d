"""Output-feedback SLS, stage 3 (Sec. 4.2, "Simulator-Informed GPU-Parallel
Output Feedback SLS"): the Kalman recursion, its associative-scan form, the
observer propagations, the assembly of the closed-loop responses and the
tube widths, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions.  A nominal trajectory of N steps; per step j = 0 .. N-1 the
linearization A_j (n x n), the output matrix C_j (p x n), the disturbance
scalings E_j (n x n) and F_j (p x p); the initial uncertainty Xi (n x n).
The system is x_{j+1} = A_j x_j + B_j u_j + E_j w_j with the measurement
y_{j+1} = C_j x_j + F_j e_j: the measurement of x_j arrives with index j+1,
as in the paper's perception model y_{k+1} = h(q_k) + e_k (Sec. 4.4).
Block matrices over the horizon have N+1 block rows and columns (times
0 .. N); Z is the block downshift, so (ZA)_{j+1,j} = A_j, (ZC)_{j+1,j} = C_j,
and M = I - ZA.  Block arrays below are (N+1, N+1, rows, cols) with the
block (k, j) at [k, j]; `dense` flattens them.

Kalman recursion (eq. kalman_recursions), j = 0 .. N-1:
    Pi_0 = Xi Xi^T
    L_{j+1} = -(F_j F_j^T + C_j Pi_j C_j^T)^{-1} C_j Pi_j A_j^T        (p x n)
    Pi_{j+1} = E_j E_j^T + A_j Pi_j A_j^T + A_j Pi_j C_j^T L_{j+1}
Pi_j is the covariance of x_j given y_1 .. y_j, and -L_{j+1}^T the gain on
the innovation of y_{j+1}.  The paper also indexes Pi and L by the injection
time k; the recursion does not depend on k, so one sequence serves every k.

Observer propagations (eq. backward_propagations), read with the gain of
the measurement each step consumes: the observer update of step j uses
y_{j+1}, hence L_{j+1}, and its error map is Ahat_j = A_j + L_{j+1}^T C_j.
For every k, Phi^x_{k,k} = I, and for j < k
    Phi^x_{k,j} = Phi^x_{k,j+1} Ahat_j,      Phi^y_{k,j+1} = Phi^x_{k,j+1} L_{j+1}^T
(Phi^y_{k,j} for 1 <= j <= k is the printed Phi^x_{k,j} L_{k,j}^T; column 0
of Phi^y is zero since no measurement has index 0).  The printed Phi^x
recursion multiplies by A_j + L_{k,j}^T C_j, whose gain index is one lower;
the reading here is the one for which [Phi^x, Phi^y] satisfies the paper's
affine constraint Phi^x (I - ZA) - Phi^y ZC = I (eq. phi_equation) and is
the response of the observer error to the disturbances, which the pins
check.

Associative form (eqs. combination_rules, initialization).  An element
(At, Dt, Pt) stands for the map Pi -> Pt + At^T (I + Pi Dt)^{-1} Pi At; the
step j element is (A_j^T, C_j^T (F_j F_j^T)^{-1} C_j, E_j E_j^T) and the
initial one (0, 0, Xi Xi^T).  Combining a (applied first) with b:
    P  = At_b^T (I + P_a Dt_b)^{-1} P_a At_b + P_b
    At = At_a (I + Dt_b P_a)^{-1} At_b
    Dt = At_a (I + Dt_b P_a)^{-1} Dt_b At_a^T + Dt_a
The printed rules name the operands by index pairs (i, m) and (m, l) whose
order is garbled between the rules, the initialization and the stated
product; in this reading the pair (m, l) is the element applied first.  Pi_j
is the P of the initial element combined with step elements 0 .. j-1.

Assembly (the equation following eq. backward_propagations), for a
state-feedback response (Phibar^x, Phibar^u) of stage 2 and the observer
response (Phihat^x, Phihat^y):
    Phi^xw = Phibar^x + Phihat^x - Phibar^x M Phihat^x
    Phi^uw = Phibar^u (I - M Phihat^x)
    Phi^xe = Phihat^y - Phibar^x M Phihat^y
    Phi^ue = -Phibar^u M Phihat^y

Tube widths (eq. of_optimization, the tightening constraints): the
disturbance w_j (scaled by E_j) enters block j+1 of the state and e_j
(scaled by F_j) block j+1 of the measurement, so with unit-ball w_j, e_j
    tau_k = sum_{j<k} ||Phi^xw_{k,j+1} E_j||_{2,r} + ||Phi^xe_{k,j+1} F_j||_{2,r}
with ||.||_{2,r} the vector of row two-norms (one width per state).
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- Kalman recursion
def kalman_serial(A, C, E, F, Xi):
    """Pi (N+1, n, n) and L (N, p, n) with L[j] = L_{j+1}."""
    N = len(A)
    Pi = [Xi @ Xi.T]
    L = []
    for j in range(N):
        S = F[j] @ F[j].T + C[j] @ Pi[j] @ C[j].T
        Lj = -np.linalg.solve(S, C[j] @ Pi[j] @ A[j].T)
        L.append(Lj)
        Pi.append(E[j] @ E[j].T + A[j] @ Pi[j] @ A[j].T + A[j] @ Pi[j] @ C[j].T @ Lj)
    return np.array(Pi), np.array(L)


def gains(A, C, F, Pi):
    """L (N, p, n), L[j] = L_{j+1}, from Pi_0 .. Pi_{N-1} (eq. kalman_recursions)."""
    return np.array([-np.linalg.solve(F[j] @ F[j].T + C[j] @ Pi[j] @ C[j].T, C[j] @ Pi[j] @ A[j].T)
                     for j in range(len(A))])


# ---------------------------------------------------------------- associative form
def elements(A, C, E, F, Xi):
    """The initial element followed by the N step elements (eq. initialization)."""
    n = A[0].shape[0]
    out = [(np.zeros((n, n)), np.zeros((n, n)), Xi @ Xi.T)]
    for j in range(len(A)):
        out.append((A[j].T.copy(), C[j].T @ np.linalg.solve(F[j] @ F[j].T, C[j]), E[j] @ E[j].T))
    return out


def combine(a, b):
    """Element `a` followed by element `b` (eq. combination_rules)."""
    Aa, Da, Pa = a
    Ab, Db, Pb = b
    I = np.eye(Pa.shape[0])
    P = Ab.T @ np.linalg.inv(I + Pa @ Db) @ Pa @ Ab + Pb
    Wi = np.linalg.inv(I + Db @ Pa)
    At = Aa @ Wi @ Ab
    Dt = Aa @ Wi @ Db @ Aa.T + Da
    return At, Dt, P


def apply(e, Pi):
    """The map an element stands for, evaluated at Pi."""
    At, Dt, Pt = e
    return Pt + At.T @ np.linalg.inv(np.eye(Pt.shape[0]) + Pi @ Dt) @ Pi @ At


def kalman_scan_sequential(elems):
    """Pi_0 .. Pi_N as the prefix combinations folded left to right."""
    acc = elems[0]
    out = [acc[2]]
    for e in elems[1:]:
        acc = combine(acc, e)
        out.append(acc[2])
    return np.array(out)


def kalman_scan_tree(elems):
    """The same prefixes by an inclusive Hillis-Steele scan (in round r every
    element i >= 2^r is combined with the prefix ending 2^r earlier): another
    association of the same products, the one a parallel scan evaluates."""
    cur = list(elems)
    off = 1
    while off < len(cur):
        cur = [cur[i] if i < off else combine(cur[i - off], cur[i]) for i in range(len(cur))]
        off *= 2
    return np.array([e[2] for e in cur])


# ---------------------------------------------------------------- block operators
def transitions(Ahat):
    """Block array T (N+1, N+1, n, n) with T[k, k] = I and, for j < k,
    T[k, j] = Ahat_{k-1} ... Ahat_j (Ahat given for j = 0 .. N-1)."""
    N, n = len(Ahat), Ahat[0].shape[0]
    T = np.zeros((N + 1, N + 1, n, n))
    for k in range(N + 1):
        T[k, k] = np.eye(n)
        for j in range(k - 1, -1, -1):
            T[k, j] = T[k, j + 1] @ Ahat[j]
    return T


def observer(A, C, L):
    """Phihat^x (N+1, N+1, n, n) and Phihat^y (N+1, N+1, n, p) by eq.
    backward_propagations (with the gain reading above)."""
    N = len(A)
    p = C[0].shape[0]
    Phx = transitions([A[j] + L[j].T @ C[j] for j in range(N)])
    n = Phx.shape[2]
    Phy = np.zeros((N + 1, N + 1, n, p))
    for k in range(N + 1):
        for j in range(1, k + 1):
            Phy[k, j] = Phx[k, j] @ L[j - 1].T
    return Phx, Phy


def dense(Bk):
    """Block array (R, S, r, s) -> matrix (R r, S s)."""
    R, S, r, s = Bk.shape
    return Bk.transpose(0, 2, 1, 3).reshape(R * r, S * s)


def downshift(Ms, N):
    """Z blkdiag(Ms_0 .. Ms_{N-1}, 0): block (j+1, j) = Ms[j]."""
    r, s = Ms[0].shape
    out = np.zeros(((N + 1) * r, (N + 1) * s))
    for j in range(N):
        out[(j + 1) * r:(j + 2) * r, j * s:(j + 1) * s] = Ms[j]
    return out


def state_feedback(A, Bm, K):
    """(Phibar^x, Phibar^u) of the static-per-step state feedback u_j = K_j x_j
    (K given for j = 0 .. N), dense: Phibar^x = (I - Z(A + B K))^{-1},
    Phibar^u = blkdiag(K) Phibar^x.  Stage 2 of the decomposition (GPU-SLS) is
    prior work that the paper cites; any state-feedback response satisfying
    [I - ZA, -ZB] [Phibar^x; Phibar^u] = I can stand in for its output."""
    N = len(A)
    Phx = dense(transitions([A[j] + Bm[j] @ K[j] for j in range(N)]))
    n, m = A[0].shape[0], K[0].shape[0]
    Kb = np.zeros(((N + 1) * m, (N + 1) * n))
    for j in range(N + 1):
        Kb[j * m:(j + 1) * m, j * n:(j + 1) * n] = K[j]
    return Phx, Kb @ Phx


def assemble(Pbx, Pbu, Phx, Phy, M):
    """Phi^xw, Phi^uw, Phi^xe, Phi^ue (dense) from the stage-2 and stage-3
    responses (dense) and M = I - ZA."""
    MPhx = M @ Phx
    MPhy = M @ Phy
    return (Pbx + Phx - Pbx @ MPhx, Pbu - Pbu @ MPhx, Phy - Pbx @ MPhy, -Pbu @ MPhy)


def tubes(Phi_w, Phi_e, E, F, n, p):
    """tau (N+1, rows per block) from the dense Phi^{.w} ((N+1) r, (N+1) n) and
    Phi^{.e} ((N+1) r, (N+1) p); tau_0 = 0."""
    N = len(E)
    r = Phi_w.shape[0] // (N + 1)
    tau = np.zeros((N + 1, r))
    for k in range(N + 1):
        rows = slice(k * r, (k + 1) * r)
        for j in range(k):
            bw = Phi_w[rows, (j + 1) * n:(j + 2) * n] @ E[j]
            be = Phi_e[rows, (j + 1) * p:(j + 2) * p] @ F[j]
            tau[k] += np.linalg.norm(bw, axis=1) + np.linalg.norm(be, axis=1)
    return tau
