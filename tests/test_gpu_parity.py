"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

FP64 mode: <= 1e-10 on gauge-invariant results (correlations, norms, traces, jump choices)
with chi not binding.  SPLIT mode (complex64 MFMA contractions, FP64 SVD): <= 1e-5
normwise relative on the correlation matrix (max|dC| / max|C|).
"""
import numpy as np
import pytest

import tn_inputs
from oracle import model as M, tebd, measure, stochastic, kraus, exact, stats

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_18841_amd import api  # noqa: E402


def _oracle_gate_fn(mdl, kind, dks=None):
    cache = {}

    def fn(b, tau):
        key = (b, tau)
        if key not in cache:
            if kind == "mpdo":
                cache[key] = M.gate_liouville(mdl, b, tau)
            elif kind == "purified":
                cache[key] = M.purified_gate(M.gate_heff(mdl, b, tau), dks[b], dks[b + 1])
            else:
                cache[key] = M.gate_heff(mdl, b, tau)
        return cache[key]
    return fn


def _normwise(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# (precision, tolerance, bits of the Theta contraction in split mode)
PRECS = [(api.FP64, 1e-10, None), (api.SPLIT, 1e-5, 32), (api.SPLIT, 1e-5, 64)]


@pytest.mark.parametrize("prec,tol,bits", PRECS)
def test_mps_heff_trotter_matches_oracle(prec, tol, bits):
    L, chi, dt, nsteps = 8, 16, 0.1, 5
    occ = tn_inputs.neel(L)
    mdl = M.Model(L)
    st = tebd.product_state(occ, "mps")
    fn = _oracle_gate_fn(mdl, "mps")
    for _ in range(nsteps):
        tebd.trotter_step(st, fn, 1, dt, chi, 1e-12)
    C_o, n_o = measure.corr_mps(st, normalize=True)
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), 2, chi, occ, precision=prec,
                  sv_cutoff=1e-12 if prec == api.FP64 else 1e-6)
    if bits:
        g.theta_precision(bits)
    for _ in range(nsteps):
        g.tebd_step(dt, order=1)
    C_g, var, _, nrm = g.measure_corr(normalize=1)
    assert _normwise(C_g, C_o) < tol
    assert abs(nrm[0] - n_o) / n_o < tol
    g.close()


@pytest.mark.parametrize("prec,tol,bits", PRECS)
def test_mpdo_second_order_matches_oracle(prec, tol, bits):
    L, chi, dt, nsteps = 6, 64, 0.05, 6
    occ = tn_inputs.neel(L)
    mdl = M.Model(L)
    st = tebd.product_state(occ, "mpdo")
    fn = _oracle_gate_fn(mdl, "mpdo")
    for _ in range(nsteps):
        tebd.trotter_step(st, fn, 2, dt, chi, 1e-12)
    C_o, tr_o = measure.corr_mpdo(st)
    g = api.State(api.KIND_MPDO, api.Model.free_fermion(L), 1, chi, occ, precision=prec,
                  sv_cutoff=1e-12 if prec == api.FP64 else 1e-6)
    if bits:
        g.theta_precision(bits)
    g.tebd_step(dt, order=2, n_steps=nsteps)
    C_g, _, _, tr = g.measure_corr()
    assert _normwise(C_g, C_o) < tol
    assert abs(tr[0] - tr_o.real) < tol
    # the exact Trotter product keeps Tr rho = 1 (Liouvillian gates are trace preserving)
    assert abs(tr[0] - 1.0) < 10 * tol
    g.close()


def test_qsd_batch_matches_oracle_per_trajectory():
    L, chi, dt, nsteps, B = 6, 8, 0.02, 10, 4
    occ = tn_inputs.neel(L)
    mdl = M.Model(L)
    noise = tn_inputs.normals(123, (nsteps, B, 2, 2))
    fn = _oracle_gate_fn(mdl, "mps")
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, occ)
    for k in range(nsteps):
        g.tebd_step(dt, order=1)
        g.apply_jumps(api.MODE_QSD, dt, noise[k].reshape(-1), api.NOISE_GAUSS)
    _, _, C_each, nrm = g.measure_corr(normalize=0, each=True)
    for b in range(B):
        st = tebd.product_state(occ, "mps")
        for k in range(nsteps):
            stochastic.qsd_step(st, mdl.jumps, dt, noise[k, b].reshape(-1), fn, chi, 1e-12)
        C_o, n_o = measure.corr_mps(st, normalize=False)
        assert _normwise(C_each[b], C_o) < 1e-10
        assert abs(nrm[b] - n_o) / n_o < 1e-10
    g.close()


@pytest.mark.parametrize("prec,tol", [(api.FP64, 1e-10), (api.SPLIT, 1e-5)])
def test_qsd_batch_estimators_match_oracle(prec, tol):
    """Sec. 4.2, linear unravelling: the batch mean of <psi|O|psi>, the ratio estimator
    sum <psi|O|psi> / sum <psi|psi> (normalize 2) and the mean norm against the oracle's."""
    L, chi, dt, nsteps, B = 6, 8, 0.05, 20, 6  # the histories' norms spread over 0.9 .. 1.8
    occ = tn_inputs.neel(L)
    mdl = M.Model(L)
    noise = tn_inputs.normals(321, (nsteps, B, 2, 2))
    fn = _oracle_gate_fn(mdl, "mps")
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, occ, precision=prec)
    for k in range(nsteps):
        g.tebd_step(dt, order=1)
        g.apply_jumps(api.MODE_QSD, dt, noise[k].reshape(-1), api.NOISE_GAUSS)
    C_lin, var0, each0, n0 = g.measure_corr(normalize=0, each=True)
    C_rat, var2, each2, n2 = g.measure_corr(normalize=2, each=True)
    g.close()
    states = []
    for b in range(B):
        st = tebd.product_state(occ, "mps")
        for k in range(nsteps):
            stochastic.qsd_step(st, mdl.jumps, dt, noise[k, b].reshape(-1), fn, chi, 1e-12)
        states.append(st)
    mean_o, ratio_o, mnorm_o = stochastic.qsd_estimators(states)
    assert _normwise(C_lin, mean_o) < tol
    assert _normwise(C_rat, ratio_o) < tol
    assert abs(n2.mean() - mnorm_o) / mnorm_o < tol
    # per instance, mode 2 returns the linear values of mode 0
    assert np.array_equal(each0, each2) and np.array_equal(n0, n2) and np.array_equal(var0, var2)
    assert _normwise(C_rat, C_lin) > 0.1  # the two estimators differ by 17 % at this sample


def _variance_within(var, var_o, vals, tol):
    """Per-history errors delta_b with |delta_b| <= dC = tol max|C| move the sample variance
    (1/(B-1)) sum_b |C_b - mean|^2 of an entry by at most
        (1/(B-1)) sum_b (2 |C_b - mean| |delta_b - mean(delta)| + |delta_b - mean(delta)|^2)
        <= 4 sqrt(B/(B-1)) std dC + 4 dC^2 B/(B-1)
    (|delta_b - mean(delta)| <= 2 dC; Cauchy-Schwarz for the first sum; std = sqrt(variance)):
    the bound the variance is held to, entry by entry, for the correlation tolerance tol
    (normwise max|dC| / max|C|)."""
    B = len(vals)
    dC = tol * np.max(np.abs(np.stack(vals)))
    bound = 4.0 * np.sqrt(B / (B - 1)) * np.sqrt(var_o) * dC + 4.0 * dC ** 2 * B / (B - 1)
    assert np.all(np.abs(var - var_o) <= bound), np.max(np.abs(var - var_o) / bound)


@pytest.mark.parametrize("normalize", [0, 1, 2])
@pytest.mark.parametrize("prec,tol", [(api.FP64, 1e-10), (api.SPLIT, 1e-5)])
def test_batch_variance_matches_oracle_mps(normalize, prec, tol):
    """eq. ErrorCLT: C_var is the sample variance (divisor B - 1) of the per-history values
    around their arithmetic mean, E|C_b - mean|^2 per entry; the per-history values are
    <psi|O|psi> (normalize 0 and 2) or <psi|O|psi>/<psi|psi> (normalize 1)."""
    L, chi, dt, nsteps, B = 6, 8, 0.05, 12, 5
    occ = tn_inputs.neel(L)
    mdl = M.Model(L)
    noise = tn_inputs.normals(4321, (nsteps, B, 2, 2))
    fn = _oracle_gate_fn(mdl, "mps")
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, occ, precision=prec,
                  sv_cutoff=1e-12 if prec == api.FP64 else 1e-6)
    for k in range(nsteps):
        g.tebd_step(dt, order=1)
        g.apply_jumps(api.MODE_QSD, dt, noise[k].reshape(-1), api.NOISE_GAUSS)
    _, var, _, _ = g.measure_corr(normalize=normalize)
    g.close()
    vals = []
    for b in range(B):
        st = tebd.product_state(occ, "mps")
        for k in range(nsteps):
            stochastic.qsd_step(st, mdl.jumps, dt, noise[k, b].reshape(-1), fn, chi, 1e-12)
        vals.append(measure.corr_mps(st, normalize=(normalize == 1))[0])
    var_o = stats.batch_variance(np.stack(vals))
    assert np.max(var_o) > 1e-4  # the histories differ
    _variance_within(var, var_o, vals, tol)


@pytest.mark.parametrize("prec,tol", [(api.FP64, 1e-10), (api.SPLIT, 1e-5)])
def test_batch_variance_matches_oracle_mpdo(prec, tol):
    """The same statistic over a batch of density matrices started from different occupations
    (Tr(rho O)/Tr rho per instance)."""
    L, chi, dt, nsteps = 6, 64, 0.05, 6
    occs = [tn_inputs.neel(L), [0] * L, [1, 1, 0, 0, 1, 0], [0, 1, 1, 0, 0, 1]]
    mdl = M.Model(L)
    fn = _oracle_gate_fn(mdl, "mpdo")
    g = api.State(api.KIND_MPDO, api.Model.free_fermion(L), len(occs), chi, occs[0], precision=prec,
                  sv_cutoff=1e-12 if prec == api.FP64 else 1e-6)
    vals = []
    for b, occ in enumerate(occs):
        st = tebd.product_state(occ, "mpdo")
        g.set_instance(b, st.tensors, st.lams, 0.0)
        for _ in range(nsteps):
            tebd.trotter_step(st, fn, 2, dt, chi, 1e-12)
        vals.append(measure.corr_mpdo(st)[0])
    g.tebd_step(dt, order=2, n_steps=nsteps)
    _, var, _, _ = g.measure_corr()
    g.close()
    var_o = stats.batch_variance(np.stack(vals))
    assert np.max(var_o) > 1e-3
    _variance_within(var, var_o, vals, tol)


def test_qt_batch_matches_oracle_jump_by_jump():
    L, chi, dt, nsteps, B = 6, 8, 0.05, 12, 6
    occ = tn_inputs.neel(L)
    mdl = M.Model(L)
    us = tn_inputs.uniforms(77, (nsteps, B))
    us[:, 0] = 0.001  # force early jumps on trajectory 0
    fn = _oracle_gate_fn(mdl, "mps")
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, occ)
    gj = []
    for k in range(nsteps):
        jumped, mask = g.apply_jumps(api.MODE_QT, dt, us[k])
        gj.append(jumped.copy())
        g.tebd_step(dt, order=1, mask=mask)
    _, _, C_each, _ = g.measure_corr(normalize=1, each=True)
    for b in range(B):
        st = tebd.product_state(occ, "mps")
        oj = []
        for k in range(nsteps):
            oj.append(stochastic.qt_step(st, mdl, mdl.jumps, dt, us[k, b], fn, chi, 1e-12))
        assert oj == [int(x[b]) for x in gj]
        C_o, _ = measure.corr_mps(st, normalize=True)
        assert _normwise(C_each[b], C_o) < 1e-10
    assert any(x[0] >= 0 for x in gj)
    g.close()


def test_purified_kraus_matches_oracle():
    L, chi, chik, dt, nsteps = 4, 32, 4, 0.05, 6
    occ = tn_inputs.neel(L)
    mdl = M.Model(L)
    dks = [chik if i in (0, L - 1) else 1 for i in range(L)]
    fn = _oracle_gate_fn(mdl, "purified", dks)
    st = tebd.product_state(occ, "purified", dk=dks)
    g = api.State(api.KIND_PURIFIED, api.Model.free_fermion(L), 1, chi, occ, chi_k_max=chik)
    for _ in range(nsteps):
        tebd.trotter_step(st, fn, 1, dt, chi, 1e-12)
        kraus.kraus_step(st, mdl.jumps, dt, chik)
        g.tebd_step(dt, order=1)
        g.apply_jumps(api.MODE_KRAUS, dt)
    C_o, tr_o = measure.corr_mps(st, normalize=True)
    C_g, _, _, tr = g.measure_corr()
    assert _normwise(C_g, C_o) < 1e-10
    assert abs(tr[0] - tr_o) / tr_o < 1e-10
    # eig(C) in [0, 1] (rho = XX^+ is a state)
    ev = np.linalg.eigvalsh((C_g + C_g.conj().T) / 2)
    assert ev.min() > -1e-10 and ev.max() < 1 + 1e-10
    g.close()


def test_state_roundtrip_and_single_layer_on_random_state():
    """A random right-isometric state with geometric bond weights (a pre-evolved stand-in):
    set it, read it back bit-exactly, run one layer, compare the updated bond weights
    (singular values) and correlations with the oracle on the same input."""
    L, chi = 10, 16
    tensors, lams, dims = tn_inputs.random_isometric_mps(5, L, chi)
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), 3, chi, tn_inputs.neel(L), sv_cutoff=0.0)
    g.set_instance(1, tensors, lams, 0.0)
    t2, l2, ln, _ = g.get_instance(1)
    for a, b in zip(tensors, t2):
        assert np.array_equal(a, b)
    for a, b in zip(lams, l2):
        assert np.array_equal(a, b)
    mdl = M.Model(L)
    st = tebd.TNState(tensors, lams)
    fn = _oracle_gate_fn(mdl, "mps")
    gates = {b: fn(b, 0.05) for b in M.layer_bonds(L, 0)}
    tebd.apply_layer(st, gates, 0, chi, 0.0)
    # GPU: run a first-order step = layer 0 then layer 1; compare after the full step instead
    tebd.apply_layer(st, {b: fn(b, 0.05) for b in M.layer_bonds(L, 1)}, 1, chi, 0.0)
    g.tebd_step(0.05, order=1)
    t3, l3, ln3, _ = g.get_instance(1)
    for b in range(L - 1):
        k = min(len(l3[b]), len(st.lams[b]))
        assert np.max(np.abs(l3[b][:k] - st.lams[b][:k])) < 1e-10
    s3 = tebd.TNState(t3, l3, ln3)
    C_g, _ = measure.corr_mps(s3, normalize=True)
    C_o, _ = measure.corr_mps(st, normalize=True)
    assert _normwise(C_g, C_o) < 1e-10
    g.close()


@pytest.mark.parametrize("chi", [40, 60])
@pytest.mark.parametrize("prec,tol,bits", PRECS)
def test_uneven_orders_match_oracle(chi, prec, tol, bits):
    """Bond dimensions 40 and 60 at L = 14, so the Hermitian eigenproblems reach orders
    n = 2 chi_r = 80 and 120 next to smaller ones: the two-stage Householder reduction hands
    trailing blocks of order 64 on from orders that are not multiples of 32, and the blocked
    back-transformation ends on a partial block of reflectors.  One first-order step on a random
    right-isometric state; bond weights and correlations against the oracle."""
    L = 14
    tensors, lams, dims = tn_inputs.random_isometric_mps(11 + chi, L, chi)
    assert max(dims) == chi
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), 2, chi, tn_inputs.neel(L), precision=prec,
                  sv_cutoff=0.0)
    if bits:
        g.theta_precision(bits)
    g.set_instance(0, tensors, lams, 0.0)
    g.replicate(0)
    mdl = M.Model(L)
    st = tebd.TNState(tensors, lams)
    fn = _oracle_gate_fn(mdl, "mps")
    for parity in (0, 1):
        tebd.apply_layer(st, {b: fn(b, 0.05) for b in M.layer_bonds(L, parity)}, parity, chi, 0.0)
    g.tebd_step(0.05, order=1)
    for inst in (0, 1):
        t3, l3, ln3, _ = g.get_instance(inst)
        err = 0.0
        for b in range(L - 1):
            k = min(len(l3[b]), len(st.lams[b]))
            err = max(err, np.max(np.abs(l3[b][:k] - st.lams[b][:k])))
        assert err < tol, (inst, err)
        C_g, _ = measure.corr_mps(tebd.TNState(t3, l3, ln3), normalize=True)
        C_o, _ = measure.corr_mps(st, normalize=True)
        assert _normwise(C_g, C_o) < tol
    g.close()


@pytest.mark.parametrize("prec,tol,bits", PRECS)
def test_mpdo_orders_match_oracle(prec, tol, bits):
    """Local dimension 4 (vectorized density matrix) at chi = 32: the Gram orders n = 4 chi_r reach
    128, so the split path's two-stage Householder reduction, the matrix-core Gram (row weights
    over d_l = 4) and the blocked back-transformation run behind the 16 x 16 Liouvillian gate.
    One first-order step on a random right-isometric tensor train; bond weights against the
    oracle."""
    L, chi = 8, 32
    tensors, lams, dims = tn_inputs.random_isometric_mps(77, L, chi, d=4)
    assert max(dims) == chi
    g = api.State(api.KIND_MPDO, api.Model.free_fermion(L), 2, chi, tn_inputs.neel(L), precision=prec,
                  sv_cutoff=0.0)
    if bits:
        g.theta_precision(bits)
    g.set_instance(0, tensors, lams, 0.0)
    g.replicate(0)
    mdl = M.Model(L)
    st = tebd.TNState(tensors, lams)
    fn = _oracle_gate_fn(mdl, "mpdo")
    for parity in (0, 1):
        tebd.apply_layer(st, {b: fn(b, 0.05) for b in M.layer_bonds(L, parity)}, parity, chi, 0.0)
    g.tebd_step(0.05, order=1)
    for inst in (0, 1):
        _, l3, _, _ = g.get_instance(inst)
        err = 0.0
        for b in range(L - 1):
            k = min(len(l3[b]), len(st.lams[b]))
            err = max(err, np.max(np.abs(l3[b][:k] - st.lams[b][:k])))
        assert err < tol, (inst, err)
    g.close()
