"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side tests/bench.

Holds none of the method's arithmetic: only random streams (PCG64) and the
construction of random right-isometric site tensors with prescribed bond
weights, used as pre-evolved stand-ins for saturated trajectory states.
"""
import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniforms(seed, shape):
    """FP64 uniforms in [0, 1): quantum-jump draws, one per trajectory per step."""
    return rng(seed).random(shape)


def normals(seed, shape):
    """FP64 standard normals: real and imaginary parts of Wiener increments."""
    return rng(seed).standard_normal(shape)


def neel(L):
    """Neel occupation pattern, first site occupied: 1,0,1,0,..."""
    return [1 - (i % 2) for i in range(L)]


def bond_dims(L, chi, d=2):
    """Largest bond dimensions an open chain of L sites with local dimension d allows, capped at chi."""
    dims = [1]
    for b in range(1, L):
        dims.append(int(min(chi, d ** min(b, L - b))))
    dims.append(1)
    return dims


def random_isometric_mps(seed, L, chi, d=2, decay=8.0):
    """Random MPS in right-isometric (Hastings) form with geometric bond weights.

    Site tensors B_i[a, p, c] with sum_{p,c} B B^+ = 1 on the left index; bond weights
    Lambda_b[a] proportional to exp(-a/decay), normalized to sum Lambda^2 = 1.
    Returns (tensors, lams, dims).
    """
    g = rng(seed)
    dims = bond_dims(L, chi, d)
    tensors = []
    for i in range(L):
        cl, cr = dims[i], dims[i + 1]
        X = g.standard_normal((d * cr, cl)) + 1j * g.standard_normal((d * cr, cl))
        Q, _ = np.linalg.qr(X)           # (d cr) x cl with orthonormal columns
        B = Q.conj().T.reshape(cl, d, cr)
        tensors.append(B)
    lams = []
    for b in range(L - 1):
        lam = np.exp(-np.arange(dims[b + 1]) / decay)
        lams.append(lam / np.sqrt(np.sum(lam ** 2)))
    return tensors, lams, dims


def rainbow_mps(L):
    """The rainbow state of an even chain: site i and site L-1-i share one particle in
    (|01> + |10>)/sqrt(2), for every i < L/2.  Its Schmidt spectrum at bond b is flat, of rank
    2^min(b+1, L-1-b), so every two-site block has exactly tied singular values.  Right-isometric
    (Hastings) form with the bond index holding the occupations of the open pairs' left sites,
    the newest in the lowest bit: site i < L/2 opens pair i, B[a, p, 2a + p] = 1/sqrt(2); site
    j >= L/2 closes the newest pair, B[a, 1 - (a mod 2), a div 2] = 1.  Returns (tensors, lams, dims)."""
    assert L % 2 == 0 and L >= 2
    h = L // 2
    dims = [1] + [2 ** min(b + 1, L - 1 - b) for b in range(L - 1)] + [1]
    tensors = []
    for i in range(L):
        cl, cr = dims[i], dims[i + 1]
        B = np.zeros((cl, 2, cr), dtype=np.complex128)
        for a in range(cl):
            if i < h:
                for p in range(2):
                    B[a, p, 2 * a + p] = 1.0 / np.sqrt(2.0)
            else:
                B[a, 1 - (a % 2), a // 2] = 1.0
        tensors.append(B)
    lams = [np.full(dims[b + 1], 1.0 / np.sqrt(dims[b + 1])) for b in range(L - 1)]
    return tensors, lams, dims
