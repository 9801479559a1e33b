"""Bond-size buckets: the bucket table follows the chain's largest bond dimensions, the autotuner
makes one choice per size class, and the results do not depend on the bucketing (Sec. 2.3:
the items of a layer are independent, so how they are grouped into launches changes nothing)."""
import numpy as np
import pytest

import tn_inputs
from oracle import model as M, tebd, measure

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_18841_amd import api  # noqa: E402


def _size_class(n):
    return 0 if n <= 64 else (1 if n <= 128 else (2 if n <= 256 else 3))


def _expected_buckets(L, chi, d, parity):
    """(largest Gram order, number of bond positions) per bucket, largest class first.  The Gram
    order of bond b is d_{b+1} D_{b+2}, D the largest bond dimension min(chi, d^b, d^(L-b))."""
    D = tn_inputs.bond_dims(L, chi, d)
    out = []
    for c in (3, 2, 1, 0):
        ns = [d * D[b + 2] for b in range(parity, L - 1, 2) if _size_class(d * D[b + 2]) == c]
        if ns:
            out.append((max(ns), len(ns)))
    return out


@pytest.mark.parametrize("kind,L,chi", [(api.KIND_MPS, 64, 64), (api.KIND_MPS, 16, 32), (api.KIND_MPDO, 10, 64),
                                        (api.KIND_MPS, 24, 256)])
def test_bucket_table_follows_the_structural_dims(kind, L, chi):
    d = 4 if kind == api.KIND_MPDO else 2
    st = api.State(kind, api.Model.free_fermion(L), 2, chi, [0] * L, precision=api.SPLIT if chi <= 128 else api.FP64)
    for p in (0, 1):
        got = [(n, nb) for n, nb, _ in st.buckets(parity=p)]
        assert got == _expected_buckets(L, chi, d, p), (p, got)
        assert sum(nb for _, nb in got) == len(range(p, L - 1, 2))
    st.close()


def test_small_layers_go_out_whole_unless_forced():
    """Default bucketing leaves a layer of fewer items than compute units whole; on = 2 buckets it.
    Both give the unbucketed result up to rounding (this checks the switch, the next test the
    results)."""
    L, chi = 16, 64
    out = []
    for on in (1, 2, 0):
        st = api.State(api.KIND_MPS, api.Model.free_fermion(L), 3, chi, [0] * L, precision=api.FP64)
        st.tuning(set_variant=0)
        st.buckets(on=on)
        for b in range(3):
            t, lam, _ = tn_inputs.random_isometric_mps(40 + b, L, chi)
            st.set_instance(b, t, lam, 0.0)
        st.tebd_step(0.05, order=2, n_steps=2)
        out.append([st.get_instance(b) for b in range(3)])
        st.close()
    # on = 1 with a 24-item layer is the unbucketed launch: bit for bit
    for a, b in zip(out[0], out[2]):
        for ta, tb in zip(a[0], b[0]):
            assert np.array_equal(ta, tb)
    for a, b in zip(out[1], out[2]):
        for la, lb in zip(a[1], b[1]):
            assert np.max(np.abs(la - lb)) < 1e-12


def test_autotuner_times_each_size_class():
    """L = 64, chi = 64, B = 1024: the middle bonds (order 128) and the edge bonds (order <= 64)
    form two classes whose first chunks are both large enough to time."""
    L, chi, B = 64, 64, 1024
    st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, tn_inputs.neel(L), precision=api.SPLIT,
                   sv_cutoff=1e-6)
    tensors, lams, _ = tn_inputs.random_isometric_mps(5, L, chi)
    st.set_instance(0, tensors, lams)
    st.replicate(0)
    st.tebd_step(0.01)
    v, ms = st.tuning()
    assert v in (0, 1) and ms[0] > 0 and ms[1] > 0
    for p in (0, 1):
        bk = st.buckets(parity=p)
        assert [n for n, _, _ in bk] == [128, 32 if p == 0 else 64]
        assert all(h in (0, 1) for _, _, h in bk)
    # the largest class's choice is the state-wide one
    assert st.buckets(parity=0)[0][2] == v
    st.tuning(set_variant=1)
    assert all(h == 1 for p in (0, 1) for _, _, h in st.buckets(parity=p))
    st.close()


def _run(kind, prec, L, chi, B, on, nsteps, seed):
    d = 4 if kind == api.KIND_MPDO else 2
    st = api.State(kind, api.Model.free_fermion(L), B, chi, [0] * L, precision=prec,
                   sv_cutoff=1e-12 if prec == api.FP64 else 1e-6)
    st.tuning(set_variant=0)
    st.buckets(on=on)  # 2: bucket these one-chunk layers too
    for b in range(B):
        t, lam, _ = tn_inputs.random_isometric_mps(seed + b, L, chi, d=d)
        st.set_instance(b, t, lam, 0.0)
    st.tebd_step(0.05, order=2, n_steps=nsteps)
    inst = [st.get_instance(b) for b in range(B)]
    _, _, C_each, nrm = st.measure_corr(normalize=0, each=True)
    st.close()
    return inst, C_each, nrm


@pytest.mark.parametrize("kind,prec,L,chi,tol", [(api.KIND_MPS, api.SPLIT, 16, 64, 2e-6),
                                                 (api.KIND_MPS, api.FP64, 16, 64, 1e-12),
                                                 (api.KIND_MPDO, api.SPLIT, 8, 32, 2e-6),
                                                 (api.KIND_MPDO, api.FP64, 6, 64, 1e-12)])
def test_results_do_not_depend_on_the_bucketing(kind, prec, L, chi, tol):
    """Mixed bucket sizes (orders 4 .. 256; the FP64 MPDO chain puts its order-256 bond through
    the general eigen path and Jacobi refinement), every layer bucketed.  With the bucketing on, a small bond's workspace
    strides and kernel tiles follow its bucket instead of the largest bond, which changes the
    order of some roundings (and with it the gauge of nearly sign-free eigenvector columns), not
    the result: Schmidt values, bond dimensions, log-norms and correlation matrices agree to
    rounding.  Tolerances: 1e-12 in FP64; in split precision a few units of complex64 storage
    rounding (6e-8) times the 3 x 2 layers and the chain's accumulation."""
    B = 5
    on, C_on, n_on = _run(kind, prec, L, chi, B, 2, 3, 300)
    off, C_off, n_off = _run(kind, prec, L, chi, B, 0, 3, 300)
    for a, b in zip(on, off):
        assert len(a[1]) == len(b[1])
        for la, lb in zip(a[1], b[1]):
            assert la.shape == lb.shape and np.max(np.abs(la - lb)) < tol
        assert abs(a[2] - b[2]) < tol
    assert np.max(np.abs(n_on - n_off) / n_off) < tol
    assert np.max(np.abs(C_on - C_off)) < tol


def test_bucketed_mpdo_across_the_order_128_boundary_matches_oracle():
    """An MPDO chain (L = 6, d = 4) whose middle bond reaches Gram order 256 (the general eigen
    path) and whose other bonds stay at order <= 64 (the bisection path once they sit in buckets
    of their own): the split-precision result stays within the split tolerance of the oracle."""
    L, chi, dt, nsteps = 6, 64, 0.05, 4
    occ = [1, 0, 1, 0, 0, 1]
    mdl = M.Model(L)
    g = api.State(api.KIND_MPDO, api.Model.free_fermion(L), 1, chi, occ, precision=api.SPLIT, sv_cutoff=1e-6)
    g.buckets(on=2)  # one instance: every layer fits one chunk
    assert [n for n, _, _ in g.buckets(parity=0)] == [64]
    assert [n for n, _, _ in g.buckets(parity=1)] == [256, 16]
    st = tebd.product_state(occ, "mpdo")
    for _ in range(nsteps):
        g.tebd_step(dt, order=2)
        tebd.trotter_step(st, lambda b, tau: M.gate_liouville(mdl, b, tau), 2, dt, chi, 1e-12)
    C_g, _, _, _ = g.measure_corr()
    C_o = measure.corr_mpdo(st)[0]
    assert np.max(np.abs(C_g - C_o)) < 1e-5
    g.close()


def test_bucket_switch_rejects_bad_arguments():
    st = api.State(api.KIND_MPS, api.Model.free_fermion(8), 2, 16, [0] * 8)
    for on, parity in ((3, 0), (-2, 0), (1, 2), (1, -1)):
        with pytest.raises(api.TnError) as e:
            st.buckets(on=on, parity=parity)
        assert e.value.code == api.TN_EINVAL
    assert st.buckets(parity=1) == st.buckets(on=-1, parity=1)
    st.close()
