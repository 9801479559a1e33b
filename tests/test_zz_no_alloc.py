"""measure_corr_noalloc through the C ABI: the measurement with its workspace in the library's
static scratch equals measure_corr bit for bit, on consecutive calls of different sizes, and an
instance whose workspace exceeds the scratch is refused."""
import ctypes

import numpy as np
import pytest

import tn_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_18841_amd import api, _lib  # noqa: E402


def _noalloc(st, normalize):
    """Direct C-ABI call of measure_corr_noalloc (every output requested)."""
    L, B = st.L, st.B
    mean = np.zeros((L, L), dtype=np.complex128)
    var = np.zeros((L, L))
    each = np.zeros((B, L, L), dtype=np.complex128)
    nrm = np.zeros(B)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    rc = _lib.load().measure_corr_noalloc(st.h, normalize, dp(mean.view(np.float64)), dp(var),
                                          dp(each.view(np.float64)), dp(nrm))
    assert rc == 0, _lib.load().mps_last_error().decode()
    return mean, var, each, nrm


def _qsd(prec, B, L, chi, nsteps, seed):
    st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, tn_inputs.neel(L), precision=prec,
                   sv_cutoff=1e-12 if prec == api.FP64 else 1e-6)
    if chi >= 16:
        tensors, lams, _ = tn_inputs.random_isometric_mps(seed, L, chi)
        st.set_instance(0, tensors, lams, 0.0)
        st.replicate(0)
    noise = tn_inputs.normals(seed, (nsteps, B * 4))
    for k in range(nsteps):
        st.tebd_step(0.01, order=1)
        st.apply_jumps(api.MODE_QSD, 0.01, noise[k], api.NOISE_GAUSS)
    return st


def _same(got, ref):
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_noalloc_measurement_equals_measure_corr_on_consecutive_calls():
    # 1: L = 64, chi = 64 in split precision needs ~8.5 MB per instance, so the 40 instances
    #    are measured in three groups of the static scratch
    big = _qsd(api.SPLIT, 40, 64, 64, 3, 5)
    for normalize in (0, 2):
        ref = big.measure_corr(normalize=normalize, each=True)
        print(f"noalloc: B=40 L=64 chi=64 split normalize={normalize}", flush=True)
        _same(_noalloc(big, normalize), ref)
    big.close()
    # 2: a smaller input right after, FP64, one group
    small = _qsd(api.FP64, 3, 8, 8, 5, 6)
    ref = small.measure_corr(normalize=1, each=True)
    print("noalloc: B=3 L=8 chi=8 fp64", flush=True)
    _same(_noalloc(small, 1), ref)
    # the arena path after the static one still agrees (neither disturbs the other)
    _same(small.measure_corr(normalize=1, each=True), ref)
    small.close()
    # 3: a density matrix (trace-vector sweep)
    mp = api.State(api.KIND_MPDO, api.Model.free_fermion(6), 2, 16, tn_inputs.neel(6))
    mp.tebd_step(0.05, order=2, n_steps=4)
    ref = mp.measure_corr(each=True)
    print("noalloc: MPDO B=2 L=6", flush=True)
    _same(_noalloc(mp, 1), ref)
    mp.close()


def test_noalloc_refuses_an_instance_above_the_scratch():
    # MPS, FP64, L = 64, chi = 256: one instance's sweep workspace is 272 MB > 128 MiB
    st = api.State(api.KIND_MPS, api.Model.free_fermion(64), 1, 256, tn_inputs.neel(64), precision=api.FP64)
    lib = _lib.load()
    L = 64
    mean = np.zeros((L, L), dtype=np.complex128)
    rc = lib.measure_corr_noalloc(st.h, 1, mean.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  None, None, None)
    assert rc == -2  # TN_ENOMEM
    assert "TN_SCRATCH_BYTES" in lib.mps_last_error().decode()
    # the arena path measures the same state
    C, _, _, _ = st.measure_corr()
    assert abs(np.trace(C).real - 32) < 1e-10  # Neel product state: 32 particles
    st.close()
