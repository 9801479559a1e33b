"""Scaled-down versions of the paper's N = 24 comparisons with the exact solution (Sec. 3.1,
3.2, 4.1, 4.2 figures; the paper prints no values, so the tests check the trends the method
fixes): the paper's vacuum initial state, L1 = c_1^+, L2 = c_N, gamma = 0.5, J = 1.  The
deviation is the RMS over sites of <n_i>(t) against eq. (SoleqCorr)."""
import numpy as np
import pytest

import tn_inputs
from oracle import exact

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_18841_amd import api  # noqa: E402

N, GAMMA = 24, 0.5
VAC = [0] * N


def _rms(C, T):
    ne = np.real(np.diag(exact.c_exact(T, VAC, 1.0, GAMMA)))
    return float(np.sqrt(np.mean((np.real(np.diag(C)) - ne) ** 2)))


def _mpdo(chi, dt, T, prec):
    st = api.State(api.KIND_MPDO, api.Model.free_fermion(N, 1.0, GAMMA), 1, chi, VAC, precision=prec,
                   sv_cutoff=1e-12 if prec == api.FP64 else 1e-6)
    st.tebd_step(dt, order=2, n_steps=int(round(T / dt)))
    C, _, _, tr = st.measure_corr()
    st.close()
    return _rms(C, T), tr[0]


def test_study_mpdo_second_order_convergence():
    """Vectorized Lindblad (Sec. 3.1): the deviation falls as dt^2 (2nd-order splitting) and is
    converged in chi at this time.  The gates preserve Tr rho; truncation moves it at the scale of
    the discarded weight (~1e-8 here)."""
    T = 2.0
    r16, t16 = _mpdo(16, 0.02, T, api.FP64)
    r32, t32 = _mpdo(32, 0.02, T, api.FP64)
    r32h, t32h = _mpdo(32, 0.01, T, api.FP64)
    assert r32h < 1e-6
    assert 3.0 < r32 / r32h < 5.0
    assert abs(r16 - r32) < 0.2 * r32
    assert max(abs(t16 - 1), abs(t32 - 1), abs(t32h - 1)) < 1e-6
    # split precision: FP32 tensor storage adds ~1e-5 at this length, still far below the
    # trajectory methods' statistical error
    rs, ts = _mpdo(64, 0.01, T, api.SPLIT)
    assert rs < 3e-5 and abs(ts - 1) < 1e-4


def test_study_purified_is_positive():
    """Locally purified form (Sec. 3.2): rho = X X^+ keeps C Hermitian with eigenvalues in [0, 1]
    and follows the exact solution at the first-order splitting error."""
    st = api.State(api.KIND_PURIFIED, api.Model.free_fermion(N, 1.0, GAMMA), 1, 32, VAC, precision=api.FP64,
                   chi_k_max=4)
    dt, T = 0.01, 1.0
    for _ in range(int(round(T / dt))):
        st.tebd_step(dt, order=1)
        st.apply_jumps(api.MODE_KRAUS, dt)
    C, _, _, _ = st.measure_corr()
    st.close()
    assert np.max(np.abs(C - C.conj().T)) < 1e-12
    ev = np.linalg.eigvalsh((C + C.conj().T) / 2)
    assert ev.min() > -1e-12 and ev.max() < 1 + 1e-12
    assert _rms(C, T) < 1e-3


def _trajectories(kind, B, chi, dt, T):
    n = int(round(T / dt))
    st = api.State(api.KIND_MPS, api.Model.free_fermion(N, 1.0, GAMMA), B, chi, VAC, precision=api.SPLIT,
                   sv_cutoff=1e-6)
    if kind == "qt":
        us = tn_inputs.uniforms(21, (n, B))
        for k in range(n):
            _, mask = st.apply_jumps(api.MODE_QT, dt, us[k])
            st.tebd_step(dt, order=1, mask=mask)
        _, _, Ce, _ = st.measure_corr(normalize=1, each=True)
    else:
        nz = tn_inputs.normals(22, (n, B * 4))
        for k in range(n):
            st.tebd_step(dt, order=1)
            st.apply_jumps(api.MODE_QSD, dt, nz[k], api.NOISE_GAUSS)
        _, _, Ce, _ = st.measure_corr(normalize=0, each=True)
    st.close()
    return np.real(np.einsum("bii->bi", Ce))


@pytest.mark.parametrize("kind", ["qt", "qsd"])
def test_study_trajectory_error_vs_number_of_histories(kind):
    """Quantum trajectories (Sec. 4.1) and state diffusion (Sec. 4.2), chi = 16: the deviation of
    the average over n_conf histories falls with n_conf (eq. ErrorCLT) down to the splitting bias."""
    T = 2.0
    dens = _trajectories(kind, 1024, 16, 0.01, T)
    ne = np.real(np.diag(exact.c_exact(T, VAC, 1.0, GAMMA)))
    rms = {nc: float(np.sqrt(np.mean((dens[:nc].mean(0) - ne) ** 2))) for nc in (16, 64, 1024)}
    assert rms[1024] < rms[16] / 3
    assert rms[1024] < 5e-3
    err = dens.std(0, ddof=1) / np.sqrt(dens.shape[0])
    assert np.all(np.abs(dens.mean(0) - ne) < 4 * err + 0.01)
