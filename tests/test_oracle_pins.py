"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: exact
integration of the Lindblad equation (ED), the closed-form two-point function,
special cases with elementary solutions, invariants, Trotter convergence
orders, and library routines.  CPU only.
"""
import numpy as np
import pytest

from oracle import model as M
from oracle import exact, ed, dense, tebd, measure, stochastic, kraus

NEEL4 = [1, 0, 1, 0]


@pytest.mark.parametrize("occ", [[0, 0, 0, 0], NEEL4, [1, 0, 1, 0, 1]])
@pytest.mark.parametrize("t", [0.7, 1.3])
def test_closed_form_matches_exact_lindblad(occ, t):
    """eq. (SoleqCorr), with the second edge term of K read as delta_iN delta_jN, equals exact
    integration of eq. (Lindblad)."""
    L = len(occ)
    rho = ed.evolve_rho(occ, t, J=1.0, gamma=0.5, sink_string=True)
    C_ed = ed.corr_from_rho(rho, L)
    C_cf = exact.c_exact(t, occ, J=1.0, gamma=0.5)
    assert np.max(np.abs(C_ed - C_cf)) < 1e-11
    assert abs(np.trace(rho) - 1) < 1e-12


def test_sink_string_does_not_change_correlations():
    """Dropping the Jordan-Wigner string of L2 = c_N in the jump leaves C(t) unchanged."""
    occ = [1, 0, 1, 0]
    a = ed.corr_from_rho(ed.evolve_rho(occ, 1.1, sink_string=True), 4)
    b = ed.corr_from_rho(ed.evolve_rho(occ, 1.1, sink_string=False), 4)
    assert np.max(np.abs(a - b)) < 1e-12


def test_closed_form_matches_rk4():
    """Sec. 2.1: the paper integrates eq. (eqCorr) numerically; RK4 converges to the closed form."""
    occ = [1, 0] * 4
    C1 = exact.c_exact(2.0, occ)
    C2 = exact.c_rk4(2.0, occ, 4000)
    assert np.max(np.abs(C1 - C2)) < 1e-12


def test_special_case_no_dissipation():
    """gamma=0: C(t) = e^{-iJAt} C0 e^{iJAt} (unitary free fermions), checked against ED."""
    occ = [1, 0, 0, 1]
    C_ed = ed.corr_from_rho(ed.evolve_rho(occ, 0.9, gamma=0.0), 4)
    A = np.zeros((4, 4))
    for i in range(3):
        A[i, i + 1] = A[i + 1, i] = 1
    import scipy.linalg as sla
    U = sla.expm(-1j * A * 0.9)
    C = U @ np.diag(occ).astype(complex) @ U.conj().T
    assert np.max(np.abs(C_ed - C)) < 1e-12
    assert np.max(np.abs(exact.c_exact(0.9, occ, gamma=0.0) - C)) < 1e-12


def test_special_case_no_hopping():
    """J=0: n_1(t) = 1 - (1-n_1(0)) e^{-gamma t}, n_N(t) = n_N(0) e^{-gamma t} (source fills, sink empties)."""
    g, t = 0.5, 1.7
    for occ in ([0, 1, 0, 1], [1, 0, 1, 1]):
        C = exact.c_exact(t, occ, J=0.0, gamma=g)
        assert abs(C[0, 0].real - (1 - (1 - occ[0]) * np.exp(-g * t))) < 1e-13
        assert abs(C[3, 3].real - occ[3] * np.exp(-g * t)) < 1e-13
        C_ed = ed.corr_from_rho(ed.evolve_rho(occ, t, J=0.0, gamma=g), 4)
        assert np.max(np.abs(C - C_ed)) < 1e-12


def test_bond_liouvillians_sum_to_full_generator():
    """With row-major vectorization (A rho B -> A (x) B^T), sum_b of the two-site Liouvillians (local index m = n*2+n') is the
    vectorized generator of eq. (Lindblad), built independently from operator matrices."""
    for L in (2, 3):
        mdl = M.Model(L, J=1.0, gamma=0.5)
        D = 4 ** L
        tot = np.zeros((D, D), dtype=complex)
        for b in range(L - 1):
            lb = mdl.liouvillian_bond(b)
            left = np.eye(4 ** b)
            right = np.eye(4 ** (L - b - 2))
            tot += np.kron(np.kron(left, lb), right)
        full = ed.liouvillian(L, 1.0, 0.5, sink_string=False).toarray()
        # full acts on rho_{I,J} -> index I*2^L + J; reorder to sites (n_k n'_k)
        perm = np.arange(D).reshape((2,) * (2 * L))
        order = []
        for k in range(L):
            order += [k, L + k]
        perm = perm.transpose(order).reshape(-1)
        full_sites = full[np.ix_(perm, perm)]
        assert np.max(np.abs(tot - full_sites)) < 1e-13


def test_gate_invariants():
    mdl = M.Model(6, gamma=0.5)
    for b in range(5):
        U = M.gate_unitary(mdl, b, 0.05)
        assert np.max(np.abs(U.conj().T @ U - np.eye(4))) < 1e-14
        G = M.gate_liouville(mdl, b, 0.05)
        # trace preservation: <<1| G = <<1| with <<1|m = delta_{n n'} on both sites
        t1 = np.zeros(4)
        t1[0] = t1[3] = 1
        one = np.kron(t1, t1)
        assert np.max(np.abs(one @ G - one)) < 1e-14
        # hermiticity preservation: G maps vec(rho) of a hermitian two-site rho to a hermitian one
        rng = np.random.default_rng(b)
        X = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        rho = X @ X.conj().T
        v = rho.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(16)
        w = (G @ v).reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)
        assert np.max(np.abs(w - w.conj().T)) < 1e-13
    # the non-unitary edge gates shrink norms (contraction), bulk ones don't
    He = M.gate_heff(mdl, 0, 0.05)
    assert np.linalg.norm(He, 2) <= 1 + 1e-14
    assert np.linalg.norm(M.gate_heff(mdl, 2, 0.05) - M.gate_unitary(mdl, 2, 0.05)) < 1e-15


def _mpdo_gate_fn(mdl):
    cache = {}

    def fn(b, tau):
        key = (b, tau)
        if key not in cache:
            cache[key] = M.gate_liouville(mdl, b, tau)
        return cache[key]
    return fn


def test_tebd_mpdo_equals_dense_trotter_without_truncation():
    """TEBD machinery (Theta, SVD split, Hastings form, layer schedule) reproduces the exact
    Trotter product when chi does not bind."""
    L = 6
    occ = [1, 0] * 3
    mdl = M.Model(L)
    fn = _mpdo_gate_fn(mdl)
    st = tebd.product_state(occ, "mpdo")
    for _ in range(6):
        tebd.trotter_step(st, fn, 2, 0.05, chi_max=4 ** 3, cutoff=0.0)
    v = dense.trotter_dense(dense.product_vector(occ, 4, "mpdo"), fn, 2, 0.05, 6)
    vt = tebd.to_dense(st).reshape((4,) * L)
    assert np.max(np.abs(vt - v)) < 1e-12
    C, tr = measure.corr_mpdo(st)
    rho = dense.rho_from_vec(v)
    C2 = ed.corr_from_rho(rho, L) / np.trace(rho)
    assert np.max(np.abs(C - C2)) < 1e-12
    assert abs(tr - 1) < 1e-12


def test_tebd_mps_equals_dense_trotter_heff():
    L = 7
    occ = [1, 0, 1, 0, 1, 0, 1]
    mdl = M.Model(L)
    fn = lambda b, tau: M.gate_heff(mdl, b, tau)
    st = tebd.product_state(occ, "mps")
    for _ in range(5):
        tebd.trotter_step(st, fn, 1, 0.1, chi_max=64, cutoff=0.0)
    v = dense.trotter_dense(dense.product_vector(occ, 2), fn, 1, 0.1, 5)
    assert np.max(np.abs(tebd.to_dense(st).reshape((2,) * L) - v)) < 1e-12
    C, n2 = measure.corr_mps(st, normalize=True)
    psi = v.reshape(-1)
    assert np.max(np.abs(C - ed.corr_from_psi(psi, L))) < 1e-12
    assert abs(n2 - np.vdot(psi, psi).real) < 1e-12


def test_trotter_orders():
    """Second-order splitting error falls by ~4 when dt halves, first order by ~2 (Sec. 2.3);
    the Liouvillian gates keep Tr rho = 1 exactly."""
    L = 6
    occ = [1, 0] * 3
    mdl = M.Model(L)
    fn = _mpdo_gate_fn(mdl)
    Cex = exact.c_exact(1.0, occ)
    errs = {}
    for order in (1, 2):
        for dt in (0.1, 0.05):
            n = int(round(1.0 / dt))
            v = dense.trotter_dense(dense.product_vector(occ, 4, "mpdo"), fn, order, dt, n)
            rho = dense.rho_from_vec(v)
            assert abs(np.trace(rho) - 1) < 1e-13
            errs[(order, dt)] = np.max(np.abs(ed.corr_from_rho(rho, L) - Cex))
    r1 = errs[(1, 0.1)] / errs[(1, 0.05)]
    r2 = errs[(2, 0.1)] / errs[(2, 0.05)]
    assert 1.7 < r1 < 2.3
    assert 3.5 < r2 < 4.5


def test_discarded_weight_is_hilbert_schmidt_error():
    """eq. (HilbertSchmidtNorm): the discarded weight equals ||psi - psi_chi||^2 / ||psi||^2."""
    L = 8
    occ = [1, 0] * 4
    mdl = M.Model(L, gamma=0.0)
    fn = lambda b, tau: M.gate_unitary(mdl, b, tau)
    st = tebd.product_state(occ, "mps")
    for _ in range(8):
        tebd.trotter_step(st, fn, 1, 0.3, chi_max=256, cutoff=0.0)
    before = tebd.to_dense(st)
    s2 = st.copy()
    # centre bond 0 has Lambda_{-1} = 1: truncate it to 1 state
    w = tebd.two_site_update(s2, 0, np.eye(4, dtype=complex), chi_max=1, cutoff=0.0)
    after = tebd.to_dense(s2)
    err = np.vdot(before - after, before - after).real / np.vdot(before, before).real
    assert w > 1e-4
    assert abs(err - w) < 1e-12


def test_corr_mps_and_mpdo_match_dense_operators():
    rng = np.random.default_rng(3)
    L = 5
    tensors = []
    dims = [1, 2, 4, 4, 2, 1]
    for i in range(L):
        tensors.append(rng.normal(size=(dims[i], 2, dims[i + 1])) + 1j * rng.normal(size=(dims[i], 2, dims[i + 1])))
    st = tebd.TNState(tensors, [np.ones(d) for d in dims[1:-1]], lognorm=0.3)
    psi = tebd.to_dense(st)
    C, n2 = measure.corr_mps(st, normalize=True)
    assert np.max(np.abs(C - ed.corr_from_psi(psi, L))) < 1e-12
    Cu, n2u = measure.corr_mps(st, normalize=False)
    assert np.max(np.abs(Cu - ed.corr_from_psi(psi, L) * np.vdot(psi, psi))) < 1e-10
    # MPDO of a random (non-hermitian) operator
    tensors = [rng.normal(size=(dims[i], 4, dims[i + 1])) + 1j * rng.normal(size=(dims[i], 4, dims[i + 1])) for i in range(L)]
    st = tebd.TNState(tensors, [np.ones(d) for d in dims[1:-1]])
    v = tebd.to_dense(st).reshape((4,) * L)
    rho = dense.rho_from_vec(v)
    C, tr = measure.corr_mpdo(st)
    assert np.max(np.abs(C - ed.corr_from_rho(rho, L) / np.trace(rho))) < 1e-11


def test_purified_measurement_matches_dense():
    rng = np.random.default_rng(5)
    L = 4
    dk = [2, 1, 1, 3]
    dims = [1, 2, 3, 2, 1]
    tensors = [rng.normal(size=(dims[i], 2 * dk[i], dims[i + 1])) + 1j * rng.normal(size=(dims[i], 2 * dk[i], dims[i + 1])) for i in range(L)]
    st = tebd.TNState(tensors, [np.ones(d) for d in dims[1:-1]])
    # dense X[(n...),(k...)]
    v = tebd.to_dense(st)  # index (p_0 p_1 ...), p = n*dk + k
    X = v.reshape([2 * x for x in dk]).reshape(*sum([[2, x] for x in dk], []))
    perm = [2 * i for i in range(L)] + [2 * i + 1 for i in range(L)]
    X = X.transpose(perm).reshape(2 ** L, -1)
    rho = X @ X.conj().T
    C, n2 = measure.corr_mps(st, normalize=True)
    assert np.max(np.abs(C - ed.corr_from_rho(rho, L) / np.trace(rho))) < 1e-12
    assert np.min(np.linalg.eigvalsh(rho)) > -1e-12


def test_qt_norm_loss_equals_jump_probability():
    """eq. (DecroisPsiLindblad): one h^eff step loses norm dt * sum gamma <L^+L> + O(dt^2)."""
    L = 6
    mdl = M.Model(L)
    occ = [1, 0] * 3
    st = tebd.product_state(occ, "mps")
    fn = lambda b, tau: M.gate_heff(mdl, b, tau)
    for _ in range(10):
        tebd.trotter_step(st, fn, 1, 0.05, 64, 0.0)
    ops = [(s, op) for s, op, g in mdl.jumps]
    for dt in (0.01, 0.005):
        s = st.copy()
        n0 = measure.norm2(s)
        nrm, vals = measure.jump_expectations(s, ops)
        p = dt * sum(g * v for (site, op, g), v in zip(mdl.jumps, vals)) / nrm
        tebd.trotter_step(s, fn, 1, dt, 64, 0.0)
        loss = 1 - measure.norm2(s) / n0
        assert abs(loss - p) < 3 * dt ** 2


def _traj_average(kind, ntraj, L, T, dt, seed):
    mdl = M.Model(L)
    occ = [1, 0] * (L // 2)
    fn_cache = {}

    def fn(b, tau):
        if (b, tau) not in fn_cache:
            fn_cache[(b, tau)] = M.gate_heff(mdl, b, tau)
        return fn_cache[(b, tau)]
    nsteps = int(round(T / dt))
    rng = np.random.default_rng(seed)
    Cs, norms = [], []
    for _ in range(ntraj):
        st = tebd.product_state(occ, "mps")
        if kind == "qt":
            us = rng.random(nsteps)
            for k in range(nsteps):
                stochastic.qt_step(st, mdl, mdl.jumps, dt, us[k], fn, 32, 1e-12)
            C, n2 = measure.corr_mps(st, normalize=True)
        else:
            if kind == "qsd":
                rn, nk = rng.standard_normal((nsteps, 4)), "gauss"
            else:
                rn, nk = rng.random((nsteps, 2)), "binary"
            for k in range(nsteps):
                stochastic.qsd_step(st, mdl.jumps, dt, rn[k], fn, 32, 1e-12, noise_kind=nk)
            C, n2 = measure.corr_mps(st, normalize=False)
            norms.append(n2)
        Cs.append(C)
    return np.array(Cs), np.array(norms)


@pytest.mark.parametrize("kind", ["qt", "qsd", "qsd_binary"])
def test_trajectory_average_matches_exact_within_clt(kind):
    """Sec. 4: the trajectory average reproduces the Lindblad dynamics; error bar eq. (ErrorCLT).
    qsd_binary uses the paper's noise eta = +-1 (Sec. 4.2), qsd complex Gaussian increments."""
    L, T, dt, ntraj = 4, 1.0, 0.01, 200
    Cs, norms = _traj_average(kind, ntraj, L, T, dt, seed=11)
    Cex = exact.c_exact(T, [1, 0] * (L // 2))
    n = np.real(np.einsum("tii->ti", Cs))
    mean = n.mean(0)
    err = n.std(0, ddof=1) / np.sqrt(ntraj)
    ne = np.real(np.diag(Cex))
    # 4 sigma plus the O(dt) splitting bias
    assert np.all(np.abs(mean - ne) < 4 * err + 0.02)
    if kind != "qt":
        # mean norm is conserved (Sec. 4.2)
        assert abs(norms.mean() - 1) < 4 * norms.std(ddof=1) / np.sqrt(ntraj) + 0.02


def test_qsd_ratio_estimator_is_the_norm_weighted_average():
    """Sec. 4.2 (linear unravelling, histories not renormalized): the ratio estimator
    sum <psi|O|psi> / sum <psi|psi> is the average of the normalized expectations weighted by
    each history's norm; for one history it is that history's normalized C, and the mean norm
    is the plain contraction <psi|psi> with the carried scale."""
    L, chi, dt, nsteps, B = 6, 8, 0.02, 12, 5
    mdl = M.Model(L)
    fn = lambda b, tau: M.gate_heff(mdl, b, tau)  # noqa: E731
    rng = np.random.default_rng(5)
    states = []
    for _ in range(B):
        st = tebd.product_state([1, 0] * (L // 2), "mps")
        rn = rng.standard_normal((nsteps, 4))
        for k in range(nsteps):
            stochastic.qsd_step(st, mdl.jumps, dt, rn[k], fn, chi, 1e-12)
        states.append(st)
    mean, ratio, mnorm = stochastic.qsd_estimators(states)
    norms = np.array([measure.norm2(st) for st in states])
    assert np.std(norms) > 1e-3  # the histories' norms differ, so the two estimators differ
    Cn = [measure.corr_mps(st, normalize=True)[0] for st in states]
    weighted = sum(n * C for n, C in zip(norms, Cn)) / norms.sum()
    assert np.max(np.abs(ratio - weighted)) < 1e-12
    assert abs(mnorm - norms.mean()) < 1e-12
    assert np.max(np.abs(mean - sum(n * C for n, C in zip(norms, Cn)) / B)) < 1e-12
    assert np.max(np.abs(mean - ratio)) > 1e-6
    m1, r1, n1 = stochastic.qsd_estimators(states[:1])
    assert np.max(np.abs(r1 - Cn[0])) < 1e-12
    assert np.max(np.abs(m1 - norms[0] * Cn[0])) < 1e-12 and abs(n1 - norms[0]) < 1e-12


def test_kraus_thin_route_equals_full_diagonalization():
    """Sec. 3.2, eq. MatrixR / eq. NewPurified with the gamma dt factor: the 2chi_k x 2chi_k Gram
    route gives the same sum_k A A^+ as diagonalizing the full R."""
    rng = np.random.default_rng(7)
    for dk in (1, 2, 4):
        A = rng.normal(size=(3, 2 * dk, 5)) + 1j * rng.normal(size=(3, 2 * dk, 5))
        lam = np.array([0.8, 0.5, 0.33])
        for Lop in (M.SP, M.SM):
            a = kraus.kraus_thin(A, dk, Lop, 0.5, 0.02, 4, lam)
            b = kraus.kraus_full(A, dk, Lop, 0.5, 0.02, 4, lam)
            ra, rb = kraus.local_rho_block(a, 4, lam), kraus.local_rho_block(b, 4, lam)
            assert np.max(np.abs(ra - rb)) < 1e-12
            a = kraus.kraus_thin(A, dk, Lop, 0.5, 0.02, 4)
            ra = kraus.local_rho_block(a, 4)
            # with chi_k >= 2 dk nothing is discarded: the block equals A A^+ + gamma dt (LA)(LA)^+
            if 2 * dk <= 4:
                A4 = A.reshape(3, 2, dk, 5)
                LA = np.einsum("nm,amkc->ankc", Lop, A4)
                def blk(T):
                    return T.transpose(0, 1, 3, 2).reshape(3 * 2 * 5, dk)
                want = blk(A4) @ blk(A4).conj().T + 0.5 * 0.02 * blk(LA) @ blk(LA).conj().T
                assert np.max(np.abs(ra - want)) < 1e-12


def test_purified_evolution_is_positive_and_close_to_exact():
    """Sec. 3.2: rho = XX^+ stays positive; first-order splitting converges to the exact C(t)."""
    L = 4
    occ = [1, 0, 1, 0]
    mdl = M.Model(L)
    chik = 4
    dks = [chik if i in (0, L - 1) else 1 for i in range(L)]
    T = 1.0
    errs = []
    for dt in (0.02, 0.01):
        st = tebd.product_state(occ, "purified", dk=dks)
        g4 = {}
        for _ in range(int(round(T / dt))):
            for parity, tau in M.trotter_layers(1, dt):
                for b in M.layer_bonds(L, parity):
                    G = M.purified_gate(M.gate_heff(mdl, b, tau), dks[b], dks[b + 1])
                    tebd.two_site_update(st, b, G, 64, 0.0)
            kraus.kraus_step(st, mdl.jumps, dt, chik)
        C, tr = measure.corr_mps(st, normalize=True)
        errs.append(np.max(np.abs(C - exact.c_exact(T, occ))))
    assert errs[1] < 0.6 * errs[0]
    assert errs[1] < 0.05


@pytest.mark.parametrize("which", ["default", "two_sources", "dephasing"])
def test_closed_form_for_other_channel_sets_matches_exact_lindblad(which):
    """Sec. 2.1 alternative jump sets: the channel-generalized closed form (sources, sinks,
    dephasing) equals exact integration of eq. (Lindblad) with fermionic operators and strings."""
    L, t = 4, 0.9
    occ = [1, 0, 1, 0]
    if which == "default":
        ch = [("source", 0, 0.5), ("sink", L - 1, 0.5)]
    elif which == "two_sources":
        ch = M.two_sources(L, 0.5)
    else:
        ch = M.source_sink_dephasing(L, 0.5, 0.3)
    rho = ed.evolve_rho_general(occ, t, ch)
    C_ed = ed.corr_from_rho(rho, L)
    C_cf = exact.c_exact_channels(t, occ, ch)
    assert np.max(np.abs(C_ed - C_cf)) < 1e-11
    if which == "default":
        assert np.max(np.abs(C_cf - exact.c_exact(t, occ))) < 1e-12


def test_pure_dephasing_closed_form():
    """No hopping, dephasing only: populations are frozen and coherences decay as exp(-gamma t)."""
    L, t, gphi = 3, 0.8, 0.4
    C0 = np.array([[0.5, 0.2 + 0.1j, 0.0], [0.2 - 0.1j, 0.3, 0.1], [0.0, 0.1, 0.6]])
    # build the same ODE from a product start is not possible for coherences; check the generator
    ch = [("dephasing", i, gphi) for i in range(L)]
    occ = [1, 0, 1]
    C = exact.c_exact_channels(t, occ, ch, J=0.0)
    assert np.max(np.abs(C - np.diag(occ))) < 1e-14
    # generator action on a matrix with coherences: off-diagonals scale by exp(-gphi t)
    Dm = gphi * (1 - np.eye(L))
    assert np.allclose(C0 * np.exp(-Dm * t), np.where(np.eye(L) > 0, C0, C0 * np.exp(-gphi * t)))


def test_tebd_with_dephasing_matches_dense_trotter_and_exact():
    """The TEBD machinery with the dephasing channel set equals the dense Trotter product (L=5,
    chi not binding), and that product approaches exact integration of eq. (Lindblad) at 2nd order."""
    L = 5
    occ = [1, 0, 1, 0, 1]
    ch = M.source_sink_dephasing(L, 0.5, 0.3)
    mdl = M.Model(L, jumps=M.channel_jumps(ch))
    fn = _mpdo_gate_fn(mdl)
    T = 0.4
    errs = []
    for nsteps in (4, 8):
        dt = T / nsteps
        st = tebd.product_state(occ, "mpdo")
        for _ in range(nsteps):
            tebd.trotter_step(st, fn, 2, dt, chi_max=4 ** 3, cutoff=0.0)
        v = dense.trotter_dense(dense.product_vector(occ, 4, "mpdo"), fn, 2, dt, nsteps)
        assert np.max(np.abs(tebd.to_dense(st).reshape((4,) * L) - v)) < 1e-12
        C, tr = measure.corr_mpdo(st)
        assert abs(tr - 1) < 1e-12
        errs.append(np.max(np.abs(C - exact.c_exact_channels(T, occ, ch))))
    assert 3.0 < errs[0] / errs[1] < 5.0


# ------------------------------------------------------------------ shifted jump operators
def _site_op_dense(O, site, L):
    return np.kron(np.kron(np.eye(2 ** site), O), np.eye(2 ** (L - site - 1)))


def _random_state(L, seed=5):
    import tn_inputs
    tensors, lams, _ = tn_inputs.random_isometric_mps(seed, L, 8)
    return tebd.TNState(tensors, lams)


def _dense_shift_terms(psi, jumps, L):
    """Normalized <L_k> and shifted rates <L^+L> - |<L>|^2, from dense operators."""
    psi = psi / np.linalg.norm(psi)
    ls, rates = [], []
    for site, op, g in jumps:
        Ld = _site_op_dense(op, site, L)
        l = np.vdot(psi, Ld @ psi)
        ls.append(l)
        rates.append(g * (np.vdot(Ld @ psi, Ld @ psi).real - abs(l) ** 2))
    return ls, rates


def test_shifted_qt_jump_is_orthogonal_to_the_state():
    """Sec. 4.1: with Delta_k = -<L_k> the jumped state (L_k - <L_k>) psi is orthogonal to psi,
    and jump k is chosen with probability dt gamma_k (<L_k^+ L_k> - |<L_k>|^2)."""
    L, dt = 6, 0.05
    ch = M.source_sink_dephasing(L, 0.5, 0.3)
    mdl = M.Model(L, jumps=M.channel_jumps(ch))
    st0 = _random_state(L)
    psi0 = tebd.to_dense(st0)
    ls, rates = _dense_shift_terms(psi0, mdl.jumps, L)
    assert min(abs(l) for l in ls) > 1e-3  # every shift is non-trivial on this state
    edges = np.concatenate([[0.0], np.cumsum(rates) * dt])
    for k in range(len(mdl.jumps)):
        st = st0.copy()
        u = 0.5 * (edges[k] + edges[k + 1])
        assert stochastic.qt_jump_shifted(st, mdl.jumps, dt, u) == k
        psi1 = tebd.to_dense(st)
        assert abs(np.linalg.norm(psi1) - 1) < 1e-12
        assert abs(np.vdot(psi0, psi1)) / np.linalg.norm(psi0) < 1e-12
        site, op, g = mdl.jumps[k]
        ref = _site_op_dense(op, site, L) @ psi0 - ls[k] * psi0
        ref /= np.linalg.norm(ref)
        assert abs(abs(np.vdot(ref, psi1)) - 1) < 1e-12
    st = st0.copy()
    assert stochastic.qt_jump_shifted(st, mdl.jumps, dt, edges[-1] + 1e-9) == -1


def test_shifted_qt_norm_loss_equals_shifted_rates():
    """Sec. 4.1: the no-jump evolution with the shifted h^eff loses norm
    dt sum_k gamma_k (<L_k^+ L_k> - |<L_k>|^2) + O(dt^2); the unshifted loss differs by
    dt sum_k gamma_k |<L_k>|^2, so a wrong drift factor fails this."""
    L = 6
    ch = M.source_sink_dephasing(L, 0.5, 0.3)
    mdl = M.Model(L, jumps=M.channel_jumps(ch))
    fn = lambda b, tau: M.gate_heff(mdl, b, tau)
    st0 = _random_state(L)
    ls, rates = _dense_shift_terms(tebd.to_dense(st0), mdl.jumps, L)
    res = []
    for dt in (0.01, 0.005):
        st = st0.copy()
        assert stochastic.qt_step_shifted(st, mdl.jumps, dt, 0.999999, fn, 64, 0.0) == -1
        loss = 1 - np.linalg.norm(tebd.to_dense(st)) ** 2
        res.append(loss - dt * sum(rates))
        shift_part = dt * sum(g * abs(l) ** 2 for (s, o, g), l in zip(mdl.jumps, ls))
        assert abs(res[-1]) < 0.1 * shift_part
    assert abs(res[1]) < 0.35 * abs(res[0])  # O(dt^2)


@pytest.mark.parametrize("shifted", [True, False])
def test_shifted_qsd_norm_change_has_no_sqrt_dt_term(shifted):
    """Sec. 4.2: with A_k = sqrt(gamma_k)(L_k - <L_k>) and binary noise the one-step change of
    <psi|psi> is sum_{k != k'} eta_k eta_k' <A_k^+ A_k'> dt up to O(dt^{3/2}) for the linear step
    psi + (sum eta_k A_k sqrt(dt) + B dt) psi.  The product form applied here, one factor per
    channel in order, adds sum_{k<k'} eta_k eta_k' 2 Re<A_k' A_k> dt (zero on average).  Without
    the shift a term ~ sqrt(dt) remains (checked as the contrast)."""
    L = 6
    ch = M.source_sink_dephasing(L, 0.5, 0.3)
    mdl = M.Model(L, jumps=M.channel_jumps(ch))
    fn = lambda b, tau: M.gate_heff(mdl, b, tau)
    st0 = _random_state(L)
    psi0 = tebd.to_dense(st0)
    n0 = np.vdot(psi0, psi0).real
    ls, _ = _dense_shift_terms(psi0, mdl.jumps, L)
    u = np.random.default_rng(3).random(len(mdl.jumps))
    eta = np.where(u < 0.5, -1.0, 1.0)
    ph = psi0 / np.sqrt(n0)
    Aop = [np.sqrt(g) * (_site_op_dense(op, s, L) - l * np.eye(2 ** L)) for (s, op, g), l in zip(mdl.jumps, ls)]
    A = [a @ ph for a in Aop]
    K = len(A)
    cross = sum(eta[k] * eta[q] * np.vdot(A[k], A[q]) for k in range(K) for q in range(K) if k != q).real
    cross += sum(2 * eta[k] * eta[q] * np.vdot(ph, Aop[q] @ A[k]).real for k in range(K) for q in range(k + 1, K))
    res = []
    for dt in (4e-4, 1e-4):
        st = st0.copy()
        step = stochastic.qsd_step_shifted if shifted else stochastic.qsd_step
        step(st, mdl.jumps, dt, u, fn, 64, 0.0, noise_kind="binary")
        n1 = np.linalg.norm(tebd.to_dense(st)) ** 2
        res.append(n1 / n0 - 1 - cross * dt)
    if shifted:
        assert abs(res[1]) < 0.2 * abs(res[0])  # dt^{3/2} or faster: ratio <= 1/8
        assert abs(res[0]) < 0.1 * abs(cross) * 4e-4
    else:
        assert 0.4 < abs(res[1]) / abs(res[0]) < 0.6  # the sqrt(dt) term


def _traj_channels(kind, ntraj, L, T, dt, seed, ch, shifted):
    mdl = M.Model(L, jumps=M.channel_jumps(ch))
    occ = [1, 0] * (L // 2)
    cache = {}

    def fn(b, tau):
        if (b, tau) not in cache:
            cache[(b, tau)] = M.gate_heff(mdl, b, tau)
        return cache[(b, tau)]
    nsteps = int(round(T / dt))
    rng = np.random.default_rng(seed)
    Cs, norms = [], []
    for _ in range(ntraj):
        st = tebd.product_state(occ, "mps")
        if kind == "qt":
            us = rng.random(nsteps)
            step = stochastic.qt_step_shifted if shifted else (
                lambda s, j, d, uu, f, c, e: stochastic.qt_step(s, mdl, j, d, uu, f, c, e))
            for k in range(nsteps):
                step(st, mdl.jumps, dt, us[k], fn, 32, 1e-12)
            C, n2 = measure.corr_mps(st, normalize=True)
        else:
            rn = rng.standard_normal((nsteps, 2 * len(mdl.jumps)))
            step = stochastic.qsd_step_shifted if shifted else stochastic.qsd_step
            for k in range(nsteps):
                step(st, mdl.jumps, dt, rn[k], fn, 32, 1e-12)
            C, n2 = measure.corr_mps(st, normalize=False)
            norms.append(n2)
        Cs.append(C)
    return np.array(Cs), np.array(norms)


@pytest.mark.parametrize("kind", ["qt", "qsd"])
def test_shifted_trajectory_average_matches_exact(kind):
    """Any shift leaves the average dynamics equal to eq. (Lindblad): shifted QT and QSD
    ensembles with dephasing (where <L_k> = <n_k> is not zero) match the exact C(t) within
    eq. (ErrorCLT); the shifted QSD norm fluctuates less than the unshifted one (Sec. 4.2)."""
    L, T, dt, ntraj = 4, 0.6, 0.01, 120
    ch = M.source_sink_dephasing(L, 0.5, 0.3)
    Cs, norms = _traj_channels(kind, ntraj, L, T, dt, 21, ch, True)
    Cex = exact.c_exact_channels(T, [1, 0] * (L // 2), ch)
    for part in (np.real, np.imag):
        v = part(Cs[:, np.arange(L - 1), np.arange(1, L)])
        mean, err = v.mean(0), v.std(0, ddof=1) / np.sqrt(ntraj)
        assert np.all(np.abs(mean - part(Cex[np.arange(L - 1), np.arange(1, L)])) < 4 * err + 0.02)
    n = np.real(np.einsum("tii->ti", Cs))
    mean, err = n.mean(0), n.std(0, ddof=1) / np.sqrt(ntraj)
    assert np.all(np.abs(mean - np.real(np.diag(Cex))) < 4 * err + 0.02)
    if kind == "qsd":
        _, norms_u = _traj_channels(kind, ntraj, L, T, dt, 21, ch, False)
        assert abs(norms.mean() - 1) < 4 * norms.std(ddof=1) / np.sqrt(ntraj) + 0.02
        assert norms.std() < 0.5 * norms_u.std()


# ------------------------------------------------------------------ sequential sweep (Sec. 2.3)
from oracle import sweep  # noqa: E402


@pytest.mark.parametrize("kind,order", [("mps", 1), ("mps", 2), ("mpdo", 1), ("mpdo", 2)])
def test_sweep_equals_dense_trotter_without_truncation(kind, order):
    """The sequential sweep applies exactly the Trotter product of Sec. 2.3 (chi not binding),
    with the dephasing channel set, so every gate of the chain is non-unitary."""
    L = 6 if kind == "mps" else 5
    occ = [1, 0, 1, 0, 1, 0][:L]
    ch = M.source_sink_dephasing(L, 0.5, 0.3)
    mdl = M.Model(L, jumps=M.channel_jumps(ch))
    fn = (lambda b, tau: M.gate_heff(mdl, b, tau)) if kind == "mps" else _mpdo_gate_fn(mdl)
    d = 2 if kind == "mps" else 4
    st = tebd.product_state(occ, kind)
    for _ in range(4):
        sweep.sweep_trotter_step(st, fn, order, 0.1, chi_max=d ** L, cutoff=0.0)
    v = dense.trotter_dense(dense.product_vector(occ, d, kind), fn, order, 0.1, 4)
    assert np.max(np.abs(tebd.to_dense(st).reshape((d,) * L) - v)) < 1e-12


def _gauge_r_defect(T):
    """max |sum_p T^p T^p+ - 1| (eq. GaugeR) for T[a, p, c]."""
    M2 = np.einsum("apc,bpc->ab", T, T.conj())
    return np.max(np.abs(M2 - np.eye(T.shape[0])))


def test_sweep_keeps_right_canonical_form_with_nonunitary_gates():
    """After each step of the sweep every tensor but the centre (site 0) satisfies eq. GaugeR,
    although the gates are not unitary; the layer-parallel form loses it on the same run."""
    L = 6
    ch = M.source_sink_dephasing(L, 0.5, 0.3)
    mdl = M.Model(L, jumps=M.channel_jumps(ch))
    fn = lambda b, tau: M.gate_heff(mdl, b, tau)
    s1 = tebd.product_state([1, 0] * 3, "mps")
    s2 = s1.copy()
    for _ in range(6):
        sweep.sweep_trotter_step(s1, fn, 1, 0.1, 64, 0.0)
        tebd.trotter_step(s2, fn, 1, 0.1, 64, 0.0)
        assert max(_gauge_r_defect(T) for T in s1.tensors[1:]) < 1e-12
    assert max(_gauge_r_defect(T) for T in s2.tensors[1:]) > 1e-3


def test_sweep_discarded_weight_is_hilbert_schmidt_error_at_binding_chi():
    """With the centre inside the updated block, the SVD truncation of every update (gate or
    centre shift) removes exactly its discarded weight from the whole state:
    ||psi_full - psi_kept||^2 / ||psi_full||^2 = sum_{a>=k} S_a^2 / sum S_a^2 (eq.
    HilbertSchmidtNorm), with non-unitary gates and chi binding."""
    import tn_inputs
    L, chi = 6, 3
    tensors, lams, _ = tn_inputs.random_isometric_mps(9, L, 8)
    st = tebd.TNState(tensors, lams)
    ch = M.source_sink_dephasing(L, 0.5, 0.3)
    mdl = M.Model(L, jumps=M.channel_jumps(ch))
    layers = M.trotter_layers(1, 0.2)
    nontrivial = 0
    for b, li, right in sweep.sweep_schedule(L, 1):
        G = None if li < 0 else M.gate_heff(mdl, b, layers[li][1])
        psi = tebd.to_dense(st)
        if G is not None:
            psi = dense.apply_gate(psi.reshape((2,) * L), G, b).reshape(-1)
        w = sweep.center_update(st, b, G, chi, 0.0, right)
        err = np.linalg.norm(psi - tebd.to_dense(st)) ** 2 / np.linalg.norm(psi) ** 2
        assert abs(err - w) < 1e-12 * max(1.0, w)
        nontrivial += w > 1e-6
    assert nontrivial >= 3


def test_sweep_schedule_follows_the_paper_for_first_order():
    """Sec. 2.3, written out for N = 6 from the paper's description: gate (1,2), shift the centre,
    gate (3,4), shift, gate (5,6) -- the centre reaches the right edge -- then the even bonds in
    reverse order, (4,5) then (2,3), each preceded by a centre shift to the left, and a last
    shift back to the first site.  0-based bonds; -1 marks a centre shift."""
    R, Lf = True, False
    expect = [(0, 0, R), (1, -1, R), (2, 0, R), (3, -1, R), (4, 0, R),
              (4, -1, Lf), (3, 1, Lf), (2, -1, Lf), (1, 1, Lf), (0, -1, Lf)]
    assert sweep.sweep_schedule(6, 1) == expect


# ---- eq. ErrorCLT: batch statistics (oracle/stats.py) and the current of Sec. 2.1

def test_density_current_obeys_the_continuity_equation():
    """Sec. 2.1: d<n_i>/dt = <j_i> - <j_{i+1}> in the bulk, with the source and sink adding
    gamma (1 - n_1) and -gamma n_N at the ends; d<n_i>/dt by central differences of the closed
    form, so a wrong sign or index in the current fails."""
    from oracle import exact
    occ, t, h, g = [1, 0, 1, 0, 1, 0], 0.8, 1e-4, 0.5
    n_m, _ = exact.density_current(exact.c_exact(t - h, occ, gamma=g))
    n_p, _ = exact.density_current(exact.c_exact(t + h, occ, gamma=g))
    n, j = exact.density_current(exact.c_exact(t, occ, gamma=g))
    dn = (n_p - n_m) / (2 * h)
    assert np.max(np.abs(dn[1:-1] - (j[:-1] - j[1:]))) < 1e-6
    assert abs(dn[0] - (g * (1 - n[0]) - j[0])) < 1e-6
    assert abs(dn[-1] - (j[-1] - g * n[-1])) < 1e-6
    assert np.max(np.abs(j)) > 0.05  # a current flows at this time


def test_batch_variance_special_cases():
    """Identical histories: variance and CLT error 0.  Two histories: the sample variance with
    divisor B - 1 is |X_1 - X_2|^2 / 2, entry by entry, for complex entries."""
    from oracle import stats
    g = np.random.default_rng(11)
    X = g.standard_normal((3, 4)) + 1j * g.standard_normal((3, 4))
    same = np.stack([X] * 5)
    assert np.max(np.abs(stats.batch_mean(same) - X)) < 1e-15 * np.max(np.abs(X))
    assert np.max(stats.batch_variance(same)) < 1e-30
    assert np.max(stats.clt_error(same)) < 1e-15
    Y = g.standard_normal((3, 4)) + 1j * g.standard_normal((3, 4))
    two = np.stack([X, Y])
    assert np.max(np.abs(stats.batch_variance(two) - np.abs(X - Y) ** 2 / 2)) < 1e-14
    assert np.max(np.abs(stats.clt_error(two) - np.abs(X - Y) / 2)) < 1e-14
    assert np.array_equal(stats.batch_variance(X[None]), np.zeros((3, 4)))


def test_batch_variance_of_a_known_distribution():
    """Complex Gaussian draws with E|z - mu|^2 = s2: the sample variance is s2 within five of its
    standard deviations (|z - mu|^2 is exponential, so that deviation is s2 / sqrt(B))."""
    from oracle import stats
    g = np.random.default_rng(12)
    B, s2, mu = 4000, 2.5, 0.3 - 0.7j
    z = mu + np.sqrt(s2 / 2) * (g.standard_normal((B, 3)) + 1j * g.standard_normal((B, 3)))
    v = stats.batch_variance(z)
    assert np.all(np.abs(v - s2) < 5 * s2 / np.sqrt(B))
    assert np.all(np.abs(stats.batch_mean(z) - mu) < 5 * np.sqrt(s2 / B))


def test_clt_error_covers_the_mean_at_its_confidence():
    """eq. ErrorCLT: over many batches of 50 normal draws, |mean - mu| < 2 sqrt(var/B) holds for
    about 95 % of them (Student t with 49 degrees of freedom: 94.9 %)."""
    from oracle import stats
    g = np.random.default_rng(13)
    hits = 0
    trials = 2000
    for _ in range(trials):
        x = 1.7 + 0.4 * g.standard_normal(50)
        hits += abs(stats.batch_mean(x) - 1.7) < 2 * stats.clt_error(x)
    assert 0.93 < hits / trials < 0.965


def test_ratio_mean_divides_out_the_norms():
    """Sec. 4.2 ratio estimator: when every history's normalized expectation is the same c,
    sum_b <psi_b|O|psi_b> / sum_b <psi_b|psi_b> is c exactly, while the plain mean is not."""
    from oracle import stats
    g = np.random.default_rng(14)
    norms = 0.5 + g.random(7)
    c = np.array([[0.25, 0.1 - 0.2j], [0.1 + 0.2j, 0.6]])
    X = norms[:, None, None] * c[None]
    assert np.max(np.abs(stats.ratio_mean(X, norms) - c)) < 1e-15
    assert np.max(np.abs(stats.batch_mean(X) - c)) > 1e-3
