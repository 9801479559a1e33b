"""The Householder autotuner: it reports a choice with timings, an override switches the
kernel, and both kernels meet the FP64 parity bar against the oracle."""
import numpy as np
import pytest

import tn_inputs
from oracle import model as M, tebd, measure, stochastic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_18841_amd import api  # noqa: E402


def test_autotuner_reports_a_timed_choice():
    """A first chunk of 2048 items (B = 256, 8 bonds per layer) is timed; the wave-tile kernel
    is taken only when it is more than 5 % faster."""
    L, chi, B = 16, 32, 256
    st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, tn_inputs.neel(L), precision=api.SPLIT,
                   sv_cutoff=1e-6)
    tensors, lams, _ = tn_inputs.random_isometric_mps(5, L, chi)
    st.set_instance(0, tensors, lams)
    st.replicate(0)
    v0, ms0 = st.tuning()
    assert ms0 == [0.0, 0.0]
    st.tebd_step(0.01)
    v, ms = st.tuning()
    assert v in (0, 1) and ms[0] > 0 and ms[1] > 0
    assert (v == 1) == (ms[1] < 0.95 * ms[0])
    st.close()


def test_small_states_keep_the_default_kernel_without_timing():
    """Chunks too small to time against launch overhead keep the MFMA kernel, so repeated runs
    make the same choice (and give bit-identical results)."""
    L, chi, B = 10, 16, 8
    st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, tn_inputs.neel(L))
    st.tebd_step(0.01)
    v, ms = st.tuning()
    assert v == 0 and ms == [0.0, 0.0]
    st.close()


@pytest.mark.parametrize("variant", [0, 1])
def test_both_householder_kernels_match_oracle(variant):
    L, chi, dt, nsteps, B = 10, 16, 0.02, 6, 3
    occ = tn_inputs.neel(L)
    mdl = M.Model(L)
    noise = tn_inputs.normals(77, (nsteps, B, 2, 2))
    g = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, occ, precision=api.FP64)
    g.tuning(variant)
    for k in range(nsteps):
        g.tebd_step(dt, order=1)
        g.apply_jumps(api.MODE_QSD, dt, noise[k].reshape(-1), api.NOISE_GAUSS)
    assert g.tuning()[0] == variant
    _, _, C_each, nrm = g.measure_corr(normalize=0, each=True)
    fn = lambda b, tau: M.gate_heff(mdl, b, tau)  # noqa: E731
    for b in range(B):
        o = tebd.product_state(occ, "mps")
        for k in range(nsteps):
            stochastic.qsd_step(o, mdl.jumps, dt, noise[k, b].reshape(-1), fn, chi, 1e-12)
        C, n2 = measure.corr_mps(o, normalize=False)
        assert np.max(np.abs(C_each[b] - C)) / np.max(np.abs(C)) < 1e-10
        assert abs(nrm[b] - n2) / n2 < 1e-10
    g.close()
