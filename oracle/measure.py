"""Correlation measurement C_ij = <c_i^+ c_j> by exact contraction.

Oracle (test infrastructure).  Sec. 2.1 defines C_ij; with the Jordan-Wigner
map c_i = (prod_{k<i} F_k) s-_i one has, for i < j,
    c_i^+ c_j = s+_i (prod_{i<k<j} F_k) s-_j ,   C_ii = <n_i>,   C_ji = conj(C_ij).
Expectations are full contractions of the network (the gauge-independent form
of Sec. 2.2 Fig. 3, without assuming any canonical gauge):
  * pure state / purified X: <psi|O|psi> with O acting on the ket index and the
    identity on the Kraus index (Sec. 3.2 eq. Purified2: Tr(XX^+ O) = <X|O (x) 1|X>);
  * MPDO: Tr(rho O) = sum_m t_O[m] ... with the local trace vector
    t_O[m = n*2 + n'] = O[n', n] (Sec. 3.1).
"""
import numpy as np

from .model import SP, SM, NUM, JWF, ID2


def _embed(O, d):
    """O (x) 1_{dk} on the index p = n*dk + k (d = 2*dk)."""
    dk = d // 2
    return np.kron(O, np.eye(dk, dtype=np.complex128))


def transfer_left(X, B, O):
    """X[a',a] -> sum_{p',p} O[p',p] B[:,p',:]^+ X B[:,p,:]  (bra index first)."""
    d = B.shape[1]
    out = np.zeros((B.shape[2], B.shape[2]), dtype=np.complex128)
    for pp in range(d):
        for p in range(d):
            if O[pp, p] != 0:
                out += O[pp, p] * (B[:, pp, :].conj().T @ X @ B[:, p, :])
    return out


def transfer_right(Y, B, O):
    """Y[c',c] -> sum_{p',p} O[p',p] conj(B[:,p',:]) Y B[:,p,:]^T."""
    d = B.shape[1]
    out = np.zeros((B.shape[0], B.shape[0]), dtype=np.complex128)
    for pp in range(d):
        for p in range(d):
            if O[pp, p] != 0:
                out += O[pp, p] * (B[:, pp, :].conj() @ Y @ B[:, p, :].T)
    return out


def _envs(state):
    L = state.L
    E = [np.ones((1, 1), dtype=np.complex128)]
    for i in range(L):
        d = state.tensors[i].shape[1]
        E.append(transfer_left(E[-1], state.tensors[i], _embed(ID2, d)))
    R = [None] * (L + 1)
    R[L] = np.ones((1, 1), dtype=np.complex128)
    for i in range(L - 1, -1, -1):
        d = state.tensors[i].shape[1]
        R[i] = transfer_right(R[i + 1], state.tensors[i], _embed(ID2, d))
    return E, R


def norm2(state):
    """<psi|psi> including exp(2 lognorm)."""
    E, _ = _envs(state)
    return float(np.real(E[-1][0, 0])) * np.exp(2 * state.lognorm)


def corr_mps(state, normalize=True):
    """C_ij for a pure MPS or a purified X.

    normalize=True: <psi|O|psi>/<psi|psi> (quantum trajectories, purified: Tr(rho O)/Tr rho).
    normalize=False: <psi|O|psi> with the true scale exp(2 lognorm) (linear QSD, Sec. 4.2).
    Returns (C, norm2) where norm2 = <psi|psi> including the scale.
    """
    L = state.L
    E, R = _envs(state)
    raw_norm = np.real(E[L][0, 0])
    C = np.zeros((L, L), dtype=np.complex128)
    for i in range(L):
        Bi = state.tensors[i]
        di = Bi.shape[1]
        C[i, i] = np.sum(transfer_left(E[i], Bi, _embed(NUM, di)) * R[i + 1])
        X = transfer_left(E[i], Bi, _embed(SP, di))
        for j in range(i + 1, L):
            Bj = state.tensors[j]
            dj = Bj.shape[1]
            C[i, j] = np.sum(transfer_left(X, Bj, _embed(SM, dj)) * R[j + 1])
            X = transfer_left(X, Bj, _embed(JWF, dj))
            C[j, i] = np.conj(C[i, j])
    scale = np.exp(2 * state.lognorm)
    if normalize:
        C = C / raw_norm
    else:
        C = C * scale
    return C, raw_norm * scale


def _tvec(O):
    """Local trace vector t_O[m = n*2 + n'] = O[n', n]."""
    t = np.zeros(4, dtype=np.complex128)
    for n in range(2):
        for nn in range(2):
            t[n * 2 + nn] = O[nn, n]
    return t


def _mat(B, O):
    return np.einsum("m,amc->ac", _tvec(O), B)


def corr_mpdo(state):
    """C_ij = Tr(rho c_i^+ c_j) / Tr(rho) for the vectorized density matrix.  Returns (C, Tr rho).

    Both triangles are evaluated directly (a truncated rho need not be exactly hermitian):
    for a < b, C_ab uses s+_a (prod F) s-_b and C_ba uses s-_a (prod F) s+_b, since
    c_b^+ c_a = s-_a (prod_{a<k<b} F_k) s+_b (the string factors left of a square to one,
    and F s- = s-).
    """
    L = state.L
    e = [np.ones(1, dtype=np.complex128)]
    for i in range(L):
        e.append(e[-1] @ _mat(state.tensors[i], ID2))
    r = [None] * (L + 1)
    r[L] = np.ones(1, dtype=np.complex128)
    for i in range(L - 1, -1, -1):
        r[i] = _mat(state.tensors[i], ID2) @ r[i + 1]
    tr = e[L][0]
    C = np.zeros((L, L), dtype=np.complex128)
    for a in range(L):
        C[a, a] = e[a] @ _mat(state.tensors[a], NUM) @ r[a + 1]
        xu = e[a] @ _mat(state.tensors[a], SP)
        xl = e[a] @ _mat(state.tensors[a], SM)
        for b in range(a + 1, L):
            C[a, b] = xu @ _mat(state.tensors[b], SM) @ r[b + 1]
            C[b, a] = xl @ _mat(state.tensors[b], SP) @ r[b + 1]
            xu = xu @ _mat(state.tensors[b], JWF)
            xl = xl @ _mat(state.tensors[b], JWF)
    return C / tr, tr * np.exp(state.lognorm)


def jump_expectations(state, ops):
    """(<psi|psi>_stored, [<psi|L_k^+ L_k|psi>_stored]) for local jump operators ops=[(site, L)].

    Stored-tensor values (without exp(2 lognorm)); ratios give the normalized rates of
    Sec. 4.1 eq. (TransitionRate).
    """
    E, R = _envs(state)
    nrm = float(np.real(E[state.L][0, 0]))
    vals = []
    for site, Lop in ops:
        B = state.tensors[site]
        O = _embed(Lop.conj().T @ Lop, B.shape[1])
        vals.append(float(np.real(np.sum(transfer_left(E[site], B, O) * R[site + 1]))))
    return nrm, vals


def local_expectations(state, ops):
    """(<psi|psi>_stored, [<psi|O_k|psi>_stored]) for single-site operators ops=[(site, O)], complex.

    The shifted jump operators of Sec. 4.1 and 4.2 need <L_k> itself (not only <L_k^+ L_k>);
    ratios to the norm give the expectation in the normalized state.
    """
    E, R = _envs(state)
    nrm = float(np.real(E[state.L][0, 0]))
    vals = []
    for site, O in ops:
        B = state.tensors[site]
        vals.append(complex(np.sum(transfer_left(E[site], B, _embed(O, B.shape[1])) * R[site + 1])))
    return nrm, vals
