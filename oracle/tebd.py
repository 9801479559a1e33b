"""Hastings-form TEBD: two-site update, truncation and Trotter layer schedule.

Oracle (test infrastructure).

The state is psi = exp(lognorm) * B_0 B_1 ... B_{L-1} with site tensors
B_i[a, p, c] (left bond, physical, right bond), bond weights Lambda_b on the
bond between sites b and b+1, and an accumulated discarded weight.  The
physical index p is n (pure state, d=2), m = n*d + n' (MPDO, Sec. 3.1 eq. MPDO)
or n*dk + k (locally purified, Sec. 3.2 eq. Purified1).

Two-site update (Sec. 2.3 eq. Theta and the SVD that follows it; Sec. 3.2 eq.
ThetaPurified):
    Theta~[a,p',q',c] = sum_{p,q} G[p'q',pq] sum_b B_i[a,p,b] B_{i+1}[b,q,c]
    Theta = Lambda_{i-1}[a] Theta~           (Lambda_{-1} = 1)
    Theta(n_L = (a,p'), n_R = (q',c)) = U S V^+          (SVD)
    keep k = min(chi_max, #{S_a > cutoff * S_0}) singular values
    discarded weight = sum_{a>=k} S_a^2 / sum_a S_a^2       (eq. HilbertSchmidtNorm,
                                                          eq. TruncationErr without its typos)
    s = (sum_{a<k} S_a^2)^{1/2}
    B_{i+1} <- V^+[:k]                   (right isometry)
    B_i     <- Theta~ V[:, :k] / s       (Hastings: no Lambda^{-1})
    Lambda_i <- S[:k] / s,  lognorm += log s
The state is never renormalized (the scale goes to lognorm), which is what the
non-hermitian and Liouvillian evolutions of Sec. 3 and 4 require: for a vectorized
density matrix sum Lambda^2 is Tr rho^2, not Tr rho.
"""
import numpy as np

from .model import trotter_layers, layer_bonds


class TNState:
    """One MPS / MPDO / purified-MPO instance in Hastings form."""

    def __init__(self, tensors, lams, lognorm=0.0):
        self.tensors = [np.array(t, dtype=np.complex128) for t in tensors]
        self.lams = [np.array(l, dtype=np.float64) for l in lams]
        self.lognorm = float(lognorm)
        self.trunc = 0.0

    @property
    def L(self):
        return len(self.tensors)

    def copy(self):
        s = TNState(self.tensors, self.lams, self.lognorm)
        s.trunc = self.trunc
        return s

    def bond_dims(self):
        return [1] + [t.shape[2] for t in self.tensors]


def product_state(occ, kind="mps", dk=None):
    """Occupation-number product state (bond dimension 1 everywhere).

    kind 'mps': p = n.  'mpdo': rho = |occ><occ|, p = m = n*2 + n' = 3n.
    'purified': X with a single Kraus column, p = n*dk_i + 0 (dk: per-site Kraus
    dimension, default 1).
    """
    L = len(occ)
    tensors = []
    for i, n in enumerate(occ):
        n = int(n)
        if kind == "mps":
            t = np.zeros((1, 2, 1), dtype=np.complex128)
            t[0, n, 0] = 1.0
        elif kind == "mpdo":
            t = np.zeros((1, 4, 1), dtype=np.complex128)
            t[0, 3 * n, 0] = 1.0
        elif kind == "purified":
            k = 1 if dk is None else dk[i]
            t = np.zeros((1, 2 * k, 1), dtype=np.complex128)
            t[0, n * k, 0] = 1.0
        else:
            raise ValueError(kind)
        tensors.append(t)
    lams = [np.ones(1) for _ in range(L - 1)]
    return TNState(tensors, lams)


def theta_tilde(Bl, Br, G):
    """Theta~ = gate applied to the contraction of two neighbour tensors (eq. Theta), no Lambda."""
    dl, dr = Bl.shape[1], Br.shape[1]
    M = np.tensordot(Bl, Br, axes=([2], [0]))  # [a, p, q, c]
    G4 = G.reshape(dl, dr, dl, dr)
    return np.einsum("PQpq,apqc->aPQc", G4, M)


def truncation_rank(S, chi_max, cutoff):
    """k = min(chi_max, #{S_a > cutoff*S_0}), at least 1 (descending order, no multiplet protection)."""
    if S.size == 0 or S[0] <= 0.0:
        return 1
    k = int(np.count_nonzero(S > cutoff * S[0]))
    return max(1, min(chi_max, k))


def two_site_update(state, b, G, chi_max, cutoff, driver="gesdd"):
    """Update bond b (sites b, b+1) with gate G in place; return the discarded weight.

    driver selects the LAPACK SVD routine ("gesdd", numpy's default, or "gesvd").  Both are
    exact to rounding; at a binding chi their results differ by the sensitivity of the
    truncation itself, which is the scale at which truncated runs can be compared."""
    Bl, Br = state.tensors[b], state.tensors[b + 1]
    chil, dl = Bl.shape[0], Bl.shape[1]
    dr, chir = Br.shape[1], Br.shape[2]
    Tt = theta_tilde(Bl, Br, G)
    lam_left = state.lams[b - 1] if b > 0 else np.ones(1)
    Th = lam_left[:, None, None, None] * Tt
    X = Th.reshape(chil * dl, dr * chir)
    if driver == "gesdd":
        U, S, Vh = np.linalg.svd(X, full_matrices=False)
    else:
        import scipy.linalg
        U, S, Vh = scipy.linalg.svd(X, full_matrices=False, lapack_driver=driver)
    k = truncation_rank(S, chi_max, cutoff)
    tot = float(np.sum(S ** 2))
    kept = float(np.sum(S[:k] ** 2))
    w = (tot - kept) / tot if tot > 0 else 0.0
    s = np.sqrt(kept) if kept > 0 else 1.0
    Vk = Vh[:k]                                  # k x (dr chir)
    state.tensors[b + 1] = Vk.reshape(k, dr, chir).copy()
    Bn = Tt.reshape(chil * dl, dr * chir) @ Vk.conj().T / s
    state.tensors[b] = Bn.reshape(chil, dl, k)
    state.lams[b] = S[:k] / s
    state.lognorm += float(np.log(s))
    state.trunc += w
    return w


def apply_layer(state, gates, parity, chi_max, cutoff, driver="gesdd"):
    """One Trotter layer: all bonds of one parity (they commute, Sec. 2.3)."""
    for b in layer_bonds(state.L, parity):
        two_site_update(state, b, gates[b], chi_max, cutoff, driver=driver)


def trotter_step(state, gate_fn, order, dt, chi_max, cutoff, driver="gesdd"):
    """One Trotter step; gate_fn(b, tau) returns the bond gate for time tau (Sec. 2.3).
    driver: the LAPACK SVD routine of every two-site update (see two_site_update)."""
    for parity, tau in trotter_layers(order, dt):
        gates = {b: gate_fn(b, tau) for b in layer_bonds(state.L, parity)}
        apply_layer(state, gates, parity, chi_max, cutoff, driver=driver)


def to_dense(state):
    """Contract the chain into a dense vector psi (index ordering: site 0 most significant)."""
    v = state.tensors[0][0]  # [p, c]
    for t in state.tensors[1:]:
        v = np.tensordot(v, t, axes=([v.ndim - 1], [0]))
        v = v.reshape(-1, t.shape[2])
    return v[:, 0] * np.exp(state.lognorm)
