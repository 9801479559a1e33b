"""Kraus-index compression of the locally purified density matrix.

Oracle (test infrastructure).  Sec. 3.2: the jump part of the first-order
splitting acts on rho = X X^+ as rho -> rho + gamma dt L rho L^+ (the
factor (1 + gamma_i dt L_i (x) L_i^+)), i.e. on the site tensor through
    R = sum_k [A^k (A^k)^+ + gamma dt (L A^k)(L A^k)^+]     (eq. MatrixR, with the
                                                            gamma dt factor, which the printed
                                                            eq. MatrixR lacks)
followed by the diagonalization R = sum lambda |phi><phi| and
A^{k} <- sqrt(lambda_k) phi_k for the chi_k largest lambda (eq. NewPurified).

The paper's local R assumes the rest of the network acts as the identity on
the site's bond indices (the site is the orthogonality centre).  In the
Hastings form used here every tensor right of a bond is a right isometry and
the left environment of site s is diag(Lambda_{s-1}^2), so the eigenproblem is
posed for Lambda_{s-1} A (the site tensor weighted by its environment); the new tensor is then taken as M W
(no Lambda^{-1}), exactly like the Hastings two-site split.

Two routes are implemented:
  kraus_full   : builds R ((d chi_l chi_r)^2) and diagonalizes it, as written;
  kraus_thin   : R = M M^+ with M = [A | sqrt(gamma dt) L A] ((d chi_l chi_r) x 2 chi_k),
                 so its nonzero eigenpairs come from the 2chi_k x 2chi_k matrix M^+ M = W diag W^+:
                 A_new = M W[:, :chi_k].  Same result (up to a unitary on k) at far lower cost.
Tensor layout: A[a, p, c] with p = n*dk + k.
"""
import numpy as np


def _split(A, dk):
    chil, d, chir = A.shape
    return A.reshape(chil, d // dk, dk, chir)  # [a, n, k, c]


def _m_matrix(A, dk, Lop, gamma, dt):
    A4 = _split(A, dk)
    LA = np.einsum("nm,amkc->ankc", Lop, A4)
    M = np.concatenate([A4, np.sqrt(gamma * dt) * LA], axis=2)  # [a, n, 2dk, c]
    chil, n, kk, chir = M.shape
    return M.transpose(0, 1, 3, 2).reshape(chil * n * chir, kk), (chil, n, chir)


def kraus_thin(A, dk, Lop, gamma, dt, chi_k, lam_left=None):
    """Thin route: eigen-decomposition of Mw^+ Mw (2dk x 2dk), Mw = Lambda_left M;
    returns M W[:, :chi_k], the new tensor with chi_k Kraus columns."""
    M, (chil, n, chir) = _m_matrix(A, dk, Lop, gamma, dt)
    lw = np.ones(chil) if lam_left is None else np.asarray(lam_left, dtype=np.float64)
    Mw = (lw[:, None, None] * M.reshape(chil, n * chir, -1)).reshape(M.shape)
    G = Mw.conj().T @ Mw
    w, W = np.linalg.eigh(G)
    order = np.argsort(w)[::-1][:chi_k]
    Anew = np.zeros((M.shape[0], chi_k), dtype=np.complex128)
    Anew[:, :order.size] = M @ W[:, order]       # [(a n c), chi_k]; zero columns if 2dk < chi_k
    Anew = Anew.reshape(chil, n, chir, chi_k).transpose(0, 1, 3, 2)
    return Anew.reshape(chil, n * chi_k, chir)


def kraus_full(A, dk, Lop, gamma, dt, chi_k, lam_left=None):
    """Route as written in the paper: diagonalize R = Mw Mw^+ directly (Mw = Lambda_left M),
    A^{k} = sqrt(lambda_k) phi_k, returned in the unweighted gauge (divided by Lambda_left > 0)."""
    M, (chil, n, chir) = _m_matrix(A, dk, Lop, gamma, dt)
    lw = np.ones(chil) if lam_left is None else np.asarray(lam_left, dtype=np.float64)
    Mw = (lw[:, None, None] * M.reshape(chil, n * chir, -1)).reshape(M.shape)
    R = Mw @ Mw.conj().T
    lam, phi = np.linalg.eigh(R)
    order = np.argsort(lam)[::-1][:chi_k]
    Anew = phi[:, order] * np.sqrt(np.maximum(lam[order], 0.0))[None, :]
    Anew = (Anew.reshape(chil, n * chir, chi_k) / lw[:, None, None]).reshape(-1, chi_k)
    Anew = Anew.reshape(chil, n, chir, chi_k).transpose(0, 1, 3, 2)
    return Anew.reshape(chil, n * chi_k, chir)


def local_rho_block(A, dk, lam_left=None):
    """sum_k A^{n,k}_{ab} (A^{n',k}_{a'b'})^*  as a matrix over (n,a,b) -- invariant under unitaries on k.
    With lam_left the left index is weighted by Lambda (the site's left environment)."""
    if lam_left is not None:
        A = np.asarray(lam_left)[:, None, None] * A
    A4 = _split(A, dk)
    chil, n, kk, chir = A4.shape
    Mm = A4.transpose(0, 1, 3, 2).reshape(chil * n * chir, kk)
    return Mm @ Mm.conj().T


def kraus_step(state, jumps, dt, chi_k, route="thin"):
    """Apply the Kraus compression at every jump site (Sec. 3.2, after the h^eff sweep)."""
    fn = kraus_thin if route == "thin" else kraus_full
    for site, op, g in jumps:
        A = state.tensors[site]
        dk = A.shape[1] // 2
        lam = state.lams[site - 1] if site > 0 else None
        state.tensors[site] = fn(A, dk, op, g, dt, chi_k, lam)
