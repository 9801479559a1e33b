"""Edge cases of the two-site update through the C ABI, against the oracle: the largest problem
the library accepts (chi = 256, so the Hermitian eigenproblem has n = d chi_r = 512 and takes
the global-memory Householder / QL / eigenvector kernels), the shortest chain (L = 2, one
bond), chi = 1 (every update truncates to a product state), exactly tied singular values (the
rainbow state, which sends split mode to its degenerate-cluster route), and independence of an
instance's result from the batch it sits in."""
import numpy as np
import pytest

import tn_inputs
from oracle import model as M, tebd, measure

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_18841_amd import api  # noqa: E402


def _normwise(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _heff(mdl):
    cache = {}

    def fn(b, tau):
        if (b, tau) not in cache:
            cache[(b, tau)] = M.gate_heff(mdl, b, tau)
        return cache[(b, tau)]
    return fn


@pytest.mark.parametrize("prec,tol", [(api.FP64, 1e-10), (api.SPLIT, 1e-5)])
def test_largest_problem_chi256(prec, tol):
    """L = 18 random right-isometric state with bond dimensions up to 256 and geometric weights
    (a saturated stand-in): one first-order step gives 512 x 512 items at the middle bonds, chi
    binds there at a well-separated cut."""
    L, chi, dt = 18, 256, 0.05
    tensors, lams, dims = tn_inputs.random_isometric_mps(11, L, chi)
    assert max(dims) == 256
    mdl = M.Model(L)
    st = tebd.TNState(tensors, lams)
    tebd.trotter_step(st, _heff(mdl), 1, dt, chi, 0.0 if prec == api.FP64 else 1e-6)
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), 1, chi, tn_inputs.neel(L), precision=prec,
                  sv_cutoff=0.0 if prec == api.FP64 else 1e-6)
    g.set_instance(0, tensors, lams, 0.0)
    g.tebd_step(dt, order=1)
    t1, l1, ln1, _ = g.get_instance(0)
    C_g, _, _, _ = g.measure_corr(normalize=1)
    g.close()
    assert [t.shape[2] for t in t1] == [t.shape[2] for t in st.tensors]
    for b in range(L - 1):
        assert np.max(np.abs(l1[b] - st.lams[b])) < (1e-10 if prec == api.FP64 else 1e-5)
    C_o, _ = measure.corr_mps(st, normalize=True)
    assert _normwise(C_g, C_o) < tol


@pytest.mark.parametrize("kind", ["mps", "mpdo"])
def test_two_site_chain(kind):
    L, chi, dt, nsteps = 2, 16, 0.1, 6
    occ = [1, 0]
    mdl = M.Model(L)
    fn = (lambda b, tau: M.gate_heff(mdl, b, tau)) if kind == "mps" else (lambda b, tau: M.gate_liouville(mdl, b, tau))
    o = tebd.product_state(occ, kind)
    for _ in range(nsteps):
        tebd.trotter_step(o, fn, 2, dt, chi, 1e-12)
    g = api.State(api.KIND_MPDO if kind == "mpdo" else api.KIND_MPS, api.Model.free_fermion(L), 1, chi, occ,
                  precision=api.FP64)
    g.tebd_step(dt, order=2, n_steps=nsteps)
    if kind == "mpdo":
        C_o, tr_o = measure.corr_mpdo(o)
        C_g, _, _, tr = g.measure_corr()
        assert abs(tr[0] - tr_o.real) < 1e-10
    else:
        C_o, _ = measure.corr_mps(o, normalize=True)
        C_g, _, _, _ = g.measure_corr(normalize=1)
    g.close()
    assert _normwise(C_g, C_o) < 1e-10


def test_chi_one_keeps_a_product_state():
    """chi = 1: each update keeps the leading Schmidt vector only (discarded weight > 0), so the
    state stays a product state; GPU and oracle agree on it and on the discarded weight."""
    L, dt, nsteps = 6, 0.1, 4
    occ = tn_inputs.neel(L)
    mdl = M.Model(L)
    o = tebd.product_state(occ, "mps")
    for _ in range(nsteps):
        tebd.trotter_step(o, _heff(mdl), 1, dt, 1, 1e-12)
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), 1, 1, occ, precision=api.FP64)
    tw = g.tebd_step(dt, order=1, n_steps=nsteps)
    t1, _, _, _ = g.get_instance(0)
    C_g, _, _, _ = g.measure_corr(normalize=1)
    g.close()
    assert all(t.shape[0] == 1 and t.shape[2] == 1 for t in t1)
    assert o.trunc > 1e-4
    assert abs(tw[0] - o.trunc) < 1e-10
    C_o, _ = measure.corr_mps(o, normalize=True)
    assert _normwise(C_g, C_o) < 1e-10


@pytest.mark.parametrize("prec", [api.FP64, api.SPLIT])
def test_result_does_not_depend_on_the_batch(prec):
    """The same instance alone (B = 1) and at position 2 of a batch of 5 other states gives
    bit-identical tensors: items are independent work units."""
    L, chi, dt = 10, 16, 0.05
    tensors, lams, _ = tn_inputs.random_isometric_mps(21, L, chi)
    out = []
    for B, pos in ((1, 0), (5, 2)):
        g = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, tn_inputs.neel(L), precision=prec)
        g.tuning(set_variant=0)
        for b in range(B):
            if b != pos:
                t2, l2, _ = tn_inputs.random_isometric_mps(100 + b, L, chi)
                g.set_instance(b, t2, l2, 0.0)
        g.set_instance(pos, tensors, lams, 0.0)
        g.tebd_step(dt, order=2, n_steps=3)
        out.append(g.get_instance(pos))
        g.close()
    for ta, tb in zip(out[0][0], out[1][0]):
        assert np.array_equal(ta, tb)
    for la, lb in zip(out[0][1], out[1][1]):
        assert np.array_equal(la, lb)
    assert out[0][2] == out[1][2]


@pytest.mark.parametrize("prec", [api.FP64, api.SPLIT])
def test_exactly_degenerate_spectrum(prec):
    """The rainbow state (site i shares a particle with site L-1-i) has flat Schmidt spectra; with
    the identity gate (dt = 0) every kept singular value of every bond ties exactly, in complex64
    too.  Split mode then takes every item's vectors from inverse iteration with separated shifts
    and re-orthogonalization (the route for degenerate multiplets), and FP64 mode meets exact
    ties in its Jacobi refinement.  Nothing is truncated (rank <= chi),
    so bond weights and correlations must match the oracle run on the same input with the same
    truncation (and the state must come back unchanged)."""
    L, chi, cut = 8, 16, 1e-6
    tol = 1e-10 if prec == api.FP64 else 1e-5
    tensors, lams, dims = tn_inputs.rainbow_mps(L)
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), 3, chi, tn_inputs.neel(L), precision=prec,
                  sv_cutoff=cut)
    g.set_instance(0, tensors, lams, 0.0)
    g.replicate(0)
    mdl = M.Model(L)
    st = tebd.TNState(tensors, lams)
    for parity in (0, 1):
        tebd.apply_layer(st, {b: M.gate_heff(mdl, b, 0.0) for b in M.layer_bonds(L, parity)}, parity, chi, cut)
    g.tebd_step(0.0, order=1)
    # the bulk updates hold tied multiplets: split mode counts them on the cluster route, each also
    # re-orthogonalized; FP64 mode has no such route
    fb, mgs = g.stats(reset=True)
    if prec == api.SPLIT:
        assert fb >= 3 * (L - 3) and mgs >= fb, (fb, mgs)
    else:
        assert (fb, mgs) == (0, 0)
    assert g.stats() == (0, 0)
    C_o, _ = measure.corr_mps(st, normalize=True)
    for inst in range(3):
        t3, l3, ln3, _ = g.get_instance(inst)
        for b in range(L - 1):
            assert len(l3[b]) == len(st.lams[b]), (b, len(l3[b]), len(st.lams[b]))
            assert np.max(np.abs(l3[b] - st.lams[b])) < tol
        C_g, _ = measure.corr_mps(tebd.TNState(t3, l3, ln3), normalize=True)
        assert np.max(np.abs(C_g - C_o)) / np.max(np.abs(C_o)) < tol
    g.close()


def test_host_rejects_non_finite_and_out_of_range_inputs():
    """Inputs that would put NaN or Inf into the kernels are refused on the host with TN_EINVAL
    before anything is launched, and the state stays usable."""
    L, chi = 6, 8
    bad = api.Model.free_fermion(L)
    bad.h[2, 1, 1] = np.nan
    with pytest.raises(api.TnError) as e:
        api.State(api.KIND_MPS, bad, 2, chi, tn_inputs.neel(L))
    assert e.value.code == api.TN_EINVAL
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), 2, chi, tn_inputs.neel(L))
    tensors, lams, _ = tn_inputs.random_isometric_mps(3, L, chi)
    t_nan = [t.copy() for t in tensors]
    t_nan[2][0, 0, 0] = np.inf
    l_neg = [x.copy() for x in lams]
    l_neg[1][0] = -0.5
    for args in ((t_nan, lams, 0.0), (tensors, l_neg, 0.0), (tensors, lams, np.nan)):
        with pytest.raises(api.TnError) as e:
            g.set_instance(0, *args)
        assert e.value.code == api.TN_EINVAL
    for mode, rnd, kind in ((api.MODE_QT, np.array([0.5, 1.5]), api.NOISE_GAUSS),
                            (api.MODE_QSD, np.full(2 * 2 * 2, np.nan), api.NOISE_GAUSS),
                            (api.MODE_QSD, np.full(2 * 2, -0.1), api.NOISE_BINARY)):
        with pytest.raises(api.TnError) as e:
            g.apply_jumps(mode, 0.01, rnd, kind)
        assert e.value.code == api.TN_EINVAL
    with pytest.raises(api.TnError):
        g.apply_jumps(api.MODE_QSD, -0.01, np.zeros(2 * 2 * 2), api.NOISE_GAUSS)
    # the state is untouched and still steps
    g.set_instance(0, tensors, lams, 0.0)
    g.tebd_step(0.01)
    C, _, _, _ = g.measure_corr()
    assert np.all(np.isfinite(C))
    g.close()
