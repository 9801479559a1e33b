"""Asynchronous measurement through the C ABI (measure_corr_start / measure_corr_finish): the
measurement of a snapshot taken in stream order, overlapped with the steps that follow it, returns
what measure_corr returns at the time of the snapshot, bit for bit; and its misuse is refused."""
import numpy as np
import pytest

import tn_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_18841_amd import api  # noqa: E402


def _qsd_state(prec, B=6, L=10, chi=16, seed=3):
    st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, tn_inputs.neel(L), precision=prec,
                   sv_cutoff=1e-12 if prec == api.FP64 else 1e-6)
    noise = tn_inputs.normals(seed, (40, B * 4))
    return st, noise


def _evolve(st, noise, k0, n, dt=0.05):
    for k in range(k0, k0 + n):
        st.tebd_step(dt, order=1)
        st.apply_jumps(api.MODE_QSD, dt, noise[k], api.NOISE_GAUSS)


@pytest.mark.parametrize("prec", [api.FP64, api.SPLIT])
@pytest.mark.parametrize("normalize", [0, 1, 2])
def test_async_measurement_is_the_snapshot_measurement(prec, normalize):
    st, noise = _qsd_state(prec)
    _evolve(st, noise, 0, 12)
    ref = st.measure_corr(normalize=normalize, each=True)
    st.measure_async_enable()
    st.measure_start(normalize)
    _evolve(st, noise, 12, 6)  # the live state moves on while the snapshot is measured
    got = st.measure_finish(each=True)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    now = st.measure_corr(normalize=normalize, each=True)
    assert not np.array_equal(now[2], ref[2])
    # a second round on the same buffer
    st.measure_start(normalize)
    got2 = st.measure_finish(each=True)
    for a, b in zip(got2, now):
        assert np.array_equal(a, b)
    st.close()


def test_async_measurement_mpdo():
    L, chi = 6, 16
    st = api.State(api.KIND_MPDO, api.Model.free_fermion(L), 3, chi, tn_inputs.neel(L), precision=api.FP64)
    st.tebd_step(0.05, order=2, n_steps=4)
    ref = st.measure_corr(each=True)
    st.measure_async_enable()
    st.measure_start()
    st.tebd_step(0.05, order=2, n_steps=2)
    got = st.measure_finish(each=True)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    st.close()


def test_async_measurement_refuses_misuse():
    st, noise = _qsd_state(api.FP64, B=2, L=6, chi=8)
    with pytest.raises(api.TnError):
        st.measure_start(0)  # no buffer yet
    st.measure_async_enable()
    with pytest.raises(api.TnError):
        st.measure_finish()  # nothing outstanding
    snap = st.measure_corr(normalize=0, each=True)
    st.measure_start(0)
    with pytest.raises(api.TnError):
        st.measure_start(0)  # one outstanding at a time
    held = st._abuf
    with pytest.raises(api.TnError):
        st.measure_async_enable()  # refused while a measurement is outstanding ...
    assert st._abuf is held  # ... and the buffer that measurement writes stays alive
    _evolve(st, noise, 0, 2)
    got = st.measure_finish(each=True)
    for a, b in zip(got, snap):
        assert np.array_equal(a, b)
    lib = st.lib
    assert lib.tn_measure_async_enable(st.h, None, 1 << 20) == -1  # TN_EINVAL
    nb = int(lib.tn_measure_async_bytes(st.h))
    assert lib.tn_measure_async_enable(st.h, st._abuf.data_ptr() + (-st._abuf.data_ptr()) % 256, nb - 256) \
        == -2  # TN_ENOMEM
    st.close()


def test_async_measurement_over_several_instance_groups():
    # more instances than one measurement group holds (1024), so the sweep runs group by group
    st, noise = _qsd_state(api.FP64, B=1030, L=4, chi=4, seed=9)
    _evolve(st, noise, 0, 5)
    ref = st.measure_corr(normalize=2, each=True)
    st.measure_async_enable()
    st.measure_start(2)
    _evolve(st, noise, 5, 2)
    got = st.measure_finish(each=True)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    st.close()


def test_async_measurement_purified():
    # a Kraus index on the jump sites: the snapshot holds the wider site tensors as they are
    L, chi, chik = 6, 16, 4
    st = api.State(api.KIND_PURIFIED, api.Model.free_fermion(L), 3, chi, tn_inputs.neel(L), chi_k_max=chik)
    for _ in range(4):
        st.tebd_step(0.05, order=1)
        st.apply_jumps(api.MODE_KRAUS, 0.05)
    ref = st.measure_corr(each=True)
    st.measure_async_enable()
    st.measure_start()
    for _ in range(2):
        st.tebd_step(0.05, order=1)
        st.apply_jumps(api.MODE_KRAUS, 0.05)
    got = st.measure_finish(each=True)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    st.close()
