"""Model and local gates of the boundary-driven free-fermion chain.

Oracle (test infrastructure).  Sec. 2.1 eq. (Hamiltonian): H = -J sum_i
(c_{i+1}^+ c_i + c_i^+ c_{i+1}); jump operators L1 = c_1^+ (source on the first
site) and L2 = c_N (sink on the last site), both with rate gamma.  Under the
Jordan-Wigner map the bond term is -J (s+ s- + s- s+) and L1 = s+_1; the string
carried by L2 is dropped, so L2 = s-_N: for states block-diagonal in the particle
number (the dynamics keep them so) the string only changes a sign that cancels in
L rho L^+ (the exact integration in ed.py keeps the string and pins this).

Local basis |0> (empty), |1> (occupied); matrices are [out, in].
Two-site index: n_i * d + n_{i+1}.  Sites are 0-based here.
"""
import numpy as np
import scipy.linalg as sla

SP = np.array([[0, 0], [1, 0]], dtype=np.complex128)   # s+ = |1><0| = c^+ locally
SM = np.array([[0, 1], [0, 0]], dtype=np.complex128)   # s- = |0><1|
NUM = np.array([[0, 0], [0, 1]], dtype=np.complex128)  # n = s+ s-
JWF = np.array([[1, 0], [0, -1]], dtype=np.complex128)  # (-1)^n, the Jordan-Wigner string factor
ID2 = np.eye(2, dtype=np.complex128)


class Model:
    """Chain of L sites, hopping J, source at site 0 and sink at site L-1 (Sec. 2.1).

    jumps: list of (site, 2x2 operator, rate).  Default: [(0, s+, gamma), (L-1, s-, gamma)].
    """

    def __init__(self, L, J=1.0, gamma=0.5, jumps=None):
        assert L >= 2
        self.L = L
        self.J = float(J)
        self.gamma = float(gamma)
        if jumps is None:
            jumps = [(0, SP.copy(), gamma), (L - 1, SM.copy(), gamma)]
        self.jumps = [(int(s), np.asarray(op, dtype=np.complex128), float(g)) for s, op, g in jumps]

    def h_bond(self, b):
        """Bond term h_{b,b+1} = -J (s+ (x) s- + s- (x) s+), Sec. 2.3 (the sum H_S = sum_i h_{i,i+1})."""
        return -self.J * (np.kron(SP, SM) + np.kron(SM, SP))

    def _bond_share(self, site, b):
        """Weight with which the on-site term of `site` goes to bond b.

        Sec. 3.2 eq. (LindbladLocal): a site shared by two bonds gives each a quarter
        (i.e. half of its -i/2 gamma L^+L term); an edge site gives its single bond the
        full half.
        """
        L = self.L
        bonds = [bb for bb in (site - 1, site) if 0 <= bb <= L - 2]
        return (1.0 / len(bonds)) if b in bonds else 0.0

    def h_eff_bond(self, b):
        """Non-hermitian bond Hamiltonian h^eff_{b,b+1} = h - (i/2) sum_k w_k gamma_k L_k^+ L_k.

        Sec. 3.2 eq. (LindbladLocal) and the effective Hamiltonian of eq. (EffHamiltonian);
        the same local operators drive the quantum-trajectory and diffusion evolutions of Sec. 4.
        """
        h = self.h_bond(b).copy()
        for site, op, g in self.jumps:
            w = self._bond_share(site, b)
            if w == 0.0:
                continue
            LdL = op.conj().T @ op
            term = np.kron(LdL, ID2) if site == b else np.kron(ID2, LdL)
            h = h - 0.5j * w * g * term
        return h

    def liouvillian_bond(self, b):
        """Two-site Liouvillian on the vectorized density matrix, local index m = n*d + n'.

        Sec. 3.1 eq. (Liouvillian) with the row-major map rho_ij -> |i>(x)|j> of eq. (Choi):
        A rho B -> A (x) B^T, hence L rho L^+ -> L (x) L^*, 1 (x) H^T and 1 (x) (L^+L)^T
        (the paper prints L (x) L^+ and 1 (x) H, which break the trace).  Dissipators are split over bonds like the effective Hamiltonian.
        Returned as a 16x16 matrix in the basis (m_b, m_{b+1}) = ((n_b, n'_b), (n_{b+1}, n'_{b+1})).
        """
        h = self.h_bond(b)
        I4 = np.eye(4, dtype=np.complex128)
        # basis ((n_b n_{b+1}), (n'_b n'_{b+1}))
        ell = -1j * (np.kron(h, I4) - np.kron(I4, h.T))
        for site, op, g in self.jumps:
            w = self._bond_share(site, b)
            if w == 0.0:
                continue
            Lop = np.kron(op, ID2) if site == b else np.kron(ID2, op)
            LdL = Lop.conj().T @ Lop
            ell = ell + w * g * (np.kron(Lop, Lop.conj()) - 0.5 * np.kron(LdL, I4) - 0.5 * np.kron(I4, LdL.T))
        # permute (n_b, n_{b+1}, n'_b, n'_{b+1}) -> (n_b, n'_b, n_{b+1}, n'_{b+1})
        T = ell.reshape(2, 2, 2, 2, 2, 2, 2, 2)
        T = T.transpose(0, 2, 1, 3, 4, 6, 5, 7)
        return T.reshape(16, 16)


def gate_unitary(model, b, tau):
    """exp(-i h_{b,b+1} tau), Sec. 2.3 (bond evolution operator)."""
    return sla.expm(-1j * model.h_bond(b) * tau)


def gate_heff(model, b, tau):
    """exp(-i h^eff_{b,b+1} tau): quantum trajectories, diffusion and purified evolution (Sec. 3.2, 4)."""
    return sla.expm(-1j * model.h_eff_bond(b) * tau)


def gate_liouville(model, b, tau):
    """exp(l_{b,b+1} tau) on the MPDO local indices (Sec. 3.1)."""
    return sla.expm(model.liouvillian_bond(b) * tau)


def purified_gate(g4, dk_left, dk_right):
    """Embed a 4x4 gate on (n_b, n_{b+1}) into the purified index p = n*dk + k (eq. ThetaPurified).

    The gate does not touch the Kraus indices k_b, k_{b+1}.
    Returned matrix is [(p'_b p'_{b+1}), (p_b p_{b+1})], size (2 dk_l 2 dk_r)^2.
    """
    G = g4.reshape(2, 2, 2, 2)  # [n'_b, n'_{b+1}, n_b, n_{b+1}]
    dl, dr = 2 * dk_left, 2 * dk_right
    out = np.zeros((dl, dr, dl, dr), dtype=np.complex128)
    for k1 in range(dk_left):
        for k2 in range(dk_right):
            for a in range(2):
                for bb in range(2):
                    for c in range(2):
                        for e in range(2):
                            out[a * dk_left + k1, bb * dk_right + k2, c * dk_left + k1, e * dk_right + k2] = G[a, bb, c, e]
    return out.reshape(dl * dr, dl * dr)


def layer_bonds(L, parity):
    """Bonds of one Trotter layer, named by their left site (0-based).

    parity 0: bonds (0,1),(2,3),... = the paper's odd bonds (1-based left site odd).
    parity 1: bonds (1,2),(3,4),... = the paper's even bonds.  Sec. 2.3.
    """
    return list(range(parity, L - 1, 2))


def trotter_layers(order, dt):
    """Sequence of (parity, time fraction) applied to the state, first element first.

    Sec. 2.3: first order e^{-iH_e dt} e^{-iH_o dt} acts with the odd bonds first;
    second order e^{-iH_e dt/2} e^{-iH_o dt} e^{-iH_e dt/2}.  Parity 0 holds the bonds
    (0,1), (2,3), ... (0-based), the paper's odd bonds.
    """
    if order == 1:
        return [(0, dt), (1, dt)]
    if order == 2:
        return [(1, dt / 2), (0, dt), (1, dt / 2)]
    raise ValueError("order must be 1 or 2")


def channel_jumps(channels):
    """Local jump list (site, 2x2 operator, rate) of a channel list (kind, site, rate).

    kind "source" -> s+, "sink" -> s- (Jordan-Wigner strings dropped; they cancel in L rho L^+
    for states block-diagonal in the particle number), "dephasing" -> n = s+ s-.
    """
    ops = {"source": SP, "sink": SM, "dephasing": SP @ SM}
    return [(int(k), ops[kind].copy(), float(g)) for kind, k, g in channels]


def two_sources(L, gamma=0.5):
    """Alternative driving of Sec. 2.1: sources c_1^+ and c_N^+."""
    return [("source", 0, gamma), ("source", L - 1, gamma)]


def source_sink_dephasing(L, gamma=0.5, gamma_phi=0.2):
    """Source c_1^+, sink c_N and dephasing c_i^+ c_i on every site (Sec. 2.1)."""
    return [("source", 0, gamma), ("sink", L - 1, gamma)] + [("dephasing", i, gamma_phi) for i in range(L)]
