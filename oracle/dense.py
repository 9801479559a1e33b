"""Exact Trotter products on the full state (no MPS, no truncation).

Oracle (test infrastructure).  Applies the same bond gates, in the same order
as the TEBD schedule (Sec. 2.3), to the dense vector psi[n_0..n_{L-1}] (pure
state) or to the dense vectorized density matrix R[m_0..m_{L-1}],
m = n*2 + n' (Sec. 3.1).  With chi large enough TEBD must reproduce these
products to rounding.
"""
import numpy as np

from .model import trotter_layers, layer_bonds


def product_vector(occ, local_dim=2, kind="mps"):
    L = len(occ)
    v = np.zeros((local_dim,) * L, dtype=np.complex128)
    idx = tuple((3 * int(n) if kind == "mpdo" else int(n)) for n in occ)
    v[idx] = 1.0
    return v


def apply_gate(v, G, b):
    """Apply a two-site gate G [(p'q'),(pq)] to sites b, b+1 of the dense tensor v."""
    d = v.shape[b]
    G4 = G.reshape(d, d, d, d)
    w = np.tensordot(G4, v, axes=([2, 3], [b, b + 1]))  # [p', q', rest...]
    return np.moveaxis(w, [0, 1], [b, b + 1])


def trotter_dense(v, gate_fn, order, dt, nsteps):
    L = v.ndim
    for _ in range(nsteps):
        for parity, tau in trotter_layers(order, dt):
            for b in layer_bonds(L, parity):
                v = apply_gate(v, gate_fn(b, tau), b)
    return v


def rho_from_vec(R):
    """R[m_0..m_{L-1}] with m = n*2 + n'  ->  rho[(n_0..), (n'_0..)]."""
    L = R.ndim
    T = R.reshape((2, 2) * L)
    perm = [2 * k for k in range(L)] + [2 * k + 1 for k in range(L)]
    T = T.transpose(perm)
    D = 2 ** L
    return T.reshape(D, D)
