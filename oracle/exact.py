"""Exact two-point function of the boundary-driven free-fermion chain.

Oracle (test infrastructure).  Sec. 2.1: C_ij = <c_i^+ c_j> obeys the closed
linear equation (eqCorr) dC/dt = -i K C + i C K^+ + Gamma with
K = J A - (i gamma/2)(P_1 + P_N) (A: nearest-neighbour adjacency, P_k the
projector on site k; the paper's delta_{N,1} delta_{j,N} is read as
delta_{i,N} delta_{j,N}, the only reading consistent with eq. LindbladEff) and Gamma = gamma e_1 e_1^T.  Its solution is
eq. (SoleqCorr).
"""
import numpy as np
import scipy.linalg as sla


def k_matrix(L, J=1.0, gamma=0.5):
    """K of eq. (eqCorr): hopping part J*A and the loss terms of source and sink."""
    K = np.zeros((L, L), dtype=np.complex128)
    for i in range(L - 1):
        K[i, i + 1] = J
        K[i + 1, i] = J
    K[0, 0] += -0.5j * gamma
    K[L - 1, L - 1] += -0.5j * gamma
    return K


def gamma_matrix(L, gamma=0.5):
    G = np.zeros((L, L), dtype=np.complex128)
    G[0, 0] = gamma
    return G


def c_initial(occ):
    """C(0) = diag(occ) for an occupation-number product state (vacuum: all zero)."""
    return np.diag(np.asarray(occ, dtype=np.complex128))


def c_exact(t, occ, J=1.0, gamma=0.5):
    """eq. (SoleqCorr): C(t) = e^{-iKt} C0 e^{iK^+ t} + int_0^t e^{-iK s} Gamma e^{iK^+ s} ds.

    The integral is evaluated in closed form through the stationary solution C_ss of
    -i K C_ss + i C_ss K^+ + Gamma = 0 (a Sylvester equation):
    C(t) = C_ss + e^{-iKt}(C0 - C_ss)e^{iK^+ t}.  For gamma = 0 the integral vanishes.
    """
    L = len(occ)
    K = k_matrix(L, J, gamma)
    C0 = c_initial(occ)
    U = sla.expm(-1j * K * t)
    if gamma == 0.0:
        return U @ C0 @ U.conj().T
    Css = stationary(L, J, gamma)
    return Css + U @ (C0 - Css) @ U.conj().T


def stationary(L, J=1.0, gamma=0.5):
    K = k_matrix(L, J, gamma)
    # (-iK) X + X (iK^+) = -Gamma
    return sla.solve_sylvester(-1j * K, 1j * K.conj().T, -gamma_matrix(L, gamma))


def c_rk4(t, occ, nsteps, J=1.0, gamma=0.5):
    """Fourth-order Runge-Kutta integration of eq. (eqCorr) (the paper's own procedure, Sec. 2.1)."""
    L = len(occ)
    K = k_matrix(L, J, gamma)
    Gm = gamma_matrix(L, gamma)
    Kd = K.conj().T

    def f(C):
        return -1j * (K @ C) + 1j * (C @ Kd) + Gm

    C = c_initial(occ)
    h = t / nsteps
    for _ in range(nsteps):
        k1 = f(C)
        k2 = f(C + 0.5 * h * k1)
        k3 = f(C + 0.5 * h * k2)
        k4 = f(C + h * k3)
        C = C + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return C


def density_current(C):
    """Density <n_i> = C_ii and current <j_i> = i (C_{i,i-1} - C_{i-1,i}) (Sec. 2.1)."""
    n = np.real(np.diag(C)).copy()
    j = np.array([np.real(1j * (C[i, i - 1] - C[i - 1, i])) for i in range(1, C.shape[0])])
    return n, j


def c_exact_channels(t, occ, channels, J=1.0):
    """C(t) for linear sources c_k^+, linear sinks c_k and dephasing n_k at arbitrary sites.

    The channels extend eq. (eqCorr) term by term.
    - Sources and sinks: each adds -(i/2) gamma_k P_k to K. A source also adds gamma_k e_k e_k^T to
      Gamma. This is eq. (eqCorr) with the channel list of Sec. 2.1.
    - Dephasing n_k: this is quadratic, so the equation stays closed.
      -(gamma/2) [n_k, [n_k, c_i^+ c_j]] = -(gamma/2)(delta_ki - delta_kj)^2 c_i^+ c_j.
      Off-diagonal entries therefore decay at (gamma_i + gamma_j)/2.

        dC/dt = -i K C + i C K^+ + Gamma - D o C,   D_ij = (g_i + g_j)/2 (1 - delta_ij)

    With row-major vec(C) this is a linear ODE dv/dt = M v + vec(Gamma). Here
    M = -i (K (x) 1) + i (1 (x) K^*) - diag(vec D). It is integrated exactly by the exponential
    of the augmented generator [[M, vec Gamma], [0, 0]].
    """
    L = len(occ)
    K = np.zeros((L, L), dtype=np.complex128)
    for i in range(L - 1):
        K[i, i + 1] = J
        K[i + 1, i] = J
    G = np.zeros((L, L), dtype=np.complex128)
    gph = np.zeros(L)
    for kind, k, g in channels:
        if kind in ("source", "sink"):
            K[k, k] += -0.5j * g
            if kind == "source":
                G[k, k] += g
        elif kind == "dephasing":
            gph[k] += g
        else:
            raise ValueError(kind)
    Dm = 0.5 * (gph[:, None] + gph[None, :]) * (1.0 - np.eye(L))
    I = np.eye(L)
    M = -1j * np.kron(K, I) + 1j * np.kron(I, K.conj()) - np.diag(Dm.reshape(-1))
    n2 = L * L
    aug = np.zeros((n2 + 1, n2 + 1), dtype=np.complex128)
    aug[:n2, :n2] = M
    aug[:n2, n2] = G.reshape(-1)
    E = sla.expm(aug * t)
    v0 = c_initial(occ).reshape(-1)
    v = E[:n2, :n2] @ v0 + E[:n2, n2]
    return v.reshape(L, L)
