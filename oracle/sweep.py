"""The paper's sequential sweep in the mixed decomposition (Sec. 2.3 with eq. MPSMixte,
eq. ShiftCenter and Fig. 4): the orthogonality centre travels along the chain, so every
two-site SVD is taken on a block that contains the centre and is exact for any gate,
unitary or not.

Oracle (test infrastructure).

State convention between steps: the TNState of the layer-parallel form with every tensor
right-canonical (eq. GaugeR) except site 0, which holds the centre.  During a pass the
tensors left of the centre c are left-canonical (eq. GaugeL), those right of it
right-canonical.

Update of bond b (sites b, b+1) when the centre is on one of the two sites:
    Theta(n_L = (a, p'), n_R = (q', c)) = [G applied to T_b T_{b+1}] = U S V^+
    truncation, discarded weight and s = norm of the kept S as in the layer-parallel form;
    Lambda_b <- S[:k] / s,  lognorm += log s;
    centre moving right:  T_b <- U[:, :k],            T_{b+1} <- diag(S/s) V^+[:k]
    centre moving left:   T_b <- U[:, :k] diag(S/s),  T_{b+1} <- V^+[:k]
No Lambda weights enter Theta: the centre tensor carries them.  A centre shift
(eq. ShiftCenter) is this update with the identity gate; the paper allows a QR there, an
SVD is used here.

Order of the updates in one Trotter step (the product of layers of Sec. 2.3, layers taken
in the order model.trotter_layers gives): passes alternate direction, the first going from
left to right; inside a pass the bonds of the layer's parity are visited in the pass's
direction, and before each gate the centre is shifted (one bond at a time, in the
direction of travel) until it sits on one of the bond's two sites.  After the last pass
the centre is shifted back to site 0.  For first order this is the paper's scheme:
parity-0 (the paper's odd) bonds left to right, parity-1 bonds right to left.
"""
import numpy as np

from .model import trotter_layers, layer_bonds
from .tebd import theta_tilde, truncation_rank


def center_update(state, b, G, chi_max, cutoff, right):
    """Update bond b with gate G (None: identity) with the centre on site b or b+1; the
    centre leaves on site b+1 (right=True) or site b.  Returns the discarded weight."""
    Tl, Tr = state.tensors[b], state.tensors[b + 1]
    chil, dl = Tl.shape[0], Tl.shape[1]
    dr, chir = Tr.shape[1], Tr.shape[2]
    if G is None:
        G = np.eye(dl * dr, dtype=np.complex128)
    X = theta_tilde(Tl, Tr, G).reshape(chil * dl, dr * chir)
    U, S, Vh = np.linalg.svd(X, full_matrices=False)
    k = truncation_rank(S, chi_max, cutoff)
    tot = float(np.sum(S ** 2))
    kept = float(np.sum(S[:k] ** 2))
    w = (tot - kept) / tot if tot > 0 else 0.0
    s = np.sqrt(kept) if kept > 0 else 1.0
    lam = S[:k] / s
    if right:
        state.tensors[b] = U[:, :k].reshape(chil, dl, k).copy()
        state.tensors[b + 1] = (lam[:, None] * Vh[:k]).reshape(k, dr, chir)
    else:
        state.tensors[b] = (U[:, :k] * lam[None, :]).reshape(chil, dl, k)
        state.tensors[b + 1] = Vh[:k].reshape(k, dr, chir).copy()
    state.lams[b] = lam
    state.lognorm += float(np.log(s))
    state.trunc += w
    return w


def sweep_schedule(L, order):
    """List of (bond, layer index or -1 for a centre shift, centre moves right) for one step."""
    ops = []
    c, right = 0, True
    for li, (parity, _) in enumerate(trotter_layers(order, 1.0)):
        bonds = list(layer_bonds(L, parity))
        for b in (bonds if right else bonds[::-1]):
            while c < b:
                ops.append((c, -1, True))
                c += 1
            while c > b + 1:
                ops.append((c - 1, -1, False))
                c -= 1
            ops.append((b, li, right))
            c = b + 1 if right else b
        right = not right
    while c > 0:
        ops.append((c - 1, -1, False))
        c -= 1
    return ops


def sweep_trotter_step(state, gate_fn, order, dt, chi_max, cutoff):
    """One Trotter step by the sequential sweep; gate_fn(b, tau) as in tebd.trotter_step."""
    layers = trotter_layers(order, dt)
    for b, li, right in sweep_schedule(state.L, order):
        G = None if li < 0 else gate_fn(b, layers[li][1])
        center_update(state, b, G, chi_max, cutoff, right)
