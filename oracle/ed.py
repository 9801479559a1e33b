"""Exact integration of the full Lindblad equation for short chains.

Oracle (test infrastructure).  Sec. 1 eq. (Lindblad) written with genuine
fermionic operators built by the Jordan-Wigner map of Sec. 2.1 (so the sink
L2 = c_N carries its string here, which pins dropping it in the local model), vectorized
with the row-major map of eq. (Choi): A rho B -> A (x) B^T.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .model import SP, SM, JWF, ID2


def _site_op(op, k, L, string=False):
    """Operator acting with `op` on site k (0-based) and, if `string`, F on all sites < k."""
    mats = []
    for j in range(L):
        if j == k:
            mats.append(sp.csr_matrix(op))
        elif string and j < k:
            mats.append(sp.csr_matrix(JWF))
        else:
            mats.append(sp.identity(2, dtype=np.complex128, format="csr"))
    out = mats[0]
    for m in mats[1:]:
        out = sp.kron(out, m, format="csr")
    return out


def fermion_ops(L):
    """c_k = (prod_{j<k} F_j) s-_k  (Jordan-Wigner, Sec. 2.1)."""
    c = [_site_op(SM, k, L, string=True) for k in range(L)]
    cd = [ck.conj().T.tocsr() for ck in c]
    return c, cd


def hamiltonian(L, J=1.0):
    """eq. (Hamiltonian): H = -J sum (c_{i+1}^+ c_i + c_i^+ c_{i+1})."""
    c, cd = fermion_ops(L)
    H = sp.csr_matrix((2 ** L, 2 ** L), dtype=np.complex128)
    for i in range(L - 1):
        H = H - J * (cd[i + 1] @ c[i] + cd[i] @ c[i + 1])
    return H.tocsr()


def jump_ops(L, gamma=0.5, sink_string=True):
    """L1 = c_1^+ (source) and L2 = c_N (sink), both at rate gamma (Sec. 2.1)."""
    c, cd = fermion_ops(L)
    sink = c[L - 1] if sink_string else _site_op(SM, L - 1, L, string=False)
    return [(cd[0], gamma), (sink, gamma)]


def liouvillian(L, J=1.0, gamma=0.5, sink_string=True):
    """Vectorized generator of eq. (Lindblad) with rho_ij -> index i*D + j (eq. Choi)."""
    D = 2 ** L
    H = hamiltonian(L, J)
    I = sp.identity(D, dtype=np.complex128, format="csr")
    Lv = -1j * (sp.kron(H, I) - sp.kron(I, H.T))
    for Lk, g in jump_ops(L, gamma, sink_string):
        LdL = (Lk.conj().T @ Lk).tocsr()
        Lv = Lv + g * (sp.kron(Lk, Lk.conj()) - 0.5 * sp.kron(LdL, I) - 0.5 * sp.kron(I, LdL.T))
    return Lv.tocsr()


def jump_ops_general(L, channels):
    """Fermionic jump operators for a list of (kind, site, rate) channels (Sec. 2.1 mentions
    these alternatives): kind "source" -> c_k^+, "sink" -> c_k (each with its Jordan-Wigner
    string), "dephasing" -> n_k = c_k^+ c_k."""
    c, cd = fermion_ops(L)
    out = []
    for kind, k, g in channels:
        if kind == "source":
            op = cd[k]
        elif kind == "sink":
            op = c[k]
        elif kind == "dephasing":
            op = (cd[k] @ c[k]).tocsr()
        else:
            raise ValueError(kind)
        out.append((op, float(g)))
    return out


def liouvillian_general(L, channels, J=1.0):
    """Vectorized generator of eq. (Lindblad) for an arbitrary list of channels (row-major vec)."""
    D = 2 ** L
    H = hamiltonian(L, J)
    I = sp.identity(D, dtype=np.complex128, format="csr")
    Lv = -1j * (sp.kron(H, I) - sp.kron(I, H.T))
    for Lk, g in jump_ops_general(L, channels):
        LdL = (Lk.conj().T @ Lk).tocsr()
        Lv = Lv + g * (sp.kron(Lk, Lk.conj()) - 0.5 * sp.kron(LdL, I) - 0.5 * sp.kron(I, LdL.T))
    return Lv.tocsr()


def evolve_rho_general(occ, t, channels, J=1.0):
    L = len(occ)
    D = 2 ** L
    v = product_rho(occ).reshape(-1)
    v = spla.expm_multiply(liouvillian_general(L, channels, J) * t, v)
    return v.reshape(D, D)


def product_rho(occ):
    """rho(0) = |occ><occ| for an occupation-number product state."""
    L = len(occ)
    idx = 0
    for n in occ:
        idx = idx * 2 + int(n)
    D = 2 ** L
    rho = np.zeros((D, D), dtype=np.complex128)
    rho[idx, idx] = 1.0
    return rho


def evolve_rho(occ, t, J=1.0, gamma=0.5, sink_string=True):
    """rho(t) = e^{Lt} rho(0) (eq. SolLindbladChoi), via scipy's expm_multiply."""
    L = len(occ)
    D = 2 ** L
    Lv = liouvillian(L, J, gamma, sink_string)
    v = product_rho(occ).reshape(-1)
    v = spla.expm_multiply(Lv * t, v)
    return v.reshape(D, D)


def corr_from_rho(rho, L):
    """C_ij = Tr(rho c_i^+ c_j) with explicit fermionic operators."""
    c, cd = fermion_ops(L)
    C = np.zeros((L, L), dtype=np.complex128)
    for i in range(L):
        for j in range(L):
            O = (cd[i] @ c[j]).toarray()
            C[i, j] = np.trace(rho @ O)
    return C


def corr_from_psi(psi, L):
    """C_ij = <psi| c_i^+ c_j |psi> / <psi|psi> for a dense state vector."""
    c, cd = fermion_ops(L)
    nrm = np.vdot(psi, psi)
    C = np.zeros((L, L), dtype=np.complex128)
    for i in range(L):
        for j in range(L):
            C[i, j] = np.vdot(psi, cd[i] @ (c[j] @ psi)) / nrm
    return C
