"""HIP-graph replay of Trotter steps gives the same results as eager launches, replay after
replay, with eager work (noise, jumps, measurements) between the replays."""
import numpy as np
import pytest

import tn_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2609_18841_amd import api  # noqa: E402


@pytest.mark.parametrize("prec,order", [(api.SPLIT, 1), (api.FP64, 2)])
def test_graph_replay_equals_eager(prec, order):
    L, chi, B, dt = 12, 16, 6, 0.02
    occ = tn_inputs.neel(L)
    nz = tn_inputs.normals(12, (6, B * 4))
    outs = []
    for graph in (True, False):
        st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, occ, precision=prec,
                       sv_cutoff=1e-6 if prec == api.SPLIT else 1e-12)
        st.graph_enable(graph)
        rec = []
        for k in range(6):
            st.tebd_step(dt, order=order, n_steps=2)
            st.apply_jumps(api.MODE_QSD, dt, nz[k], api.NOISE_GAUSS)
            _, _, C_each, nrm = st.measure_corr(normalize=0, each=True)
            rec.append((C_each.copy(), nrm.copy()))
        outs.append(rec)
        st.close()
    for (Ca, na), (Cb, nb) in zip(*outs):
        assert np.array_equal(Ca, Cb) and np.array_equal(na, nb)


def test_graph_replay_with_changing_dt_and_masked_steps():
    """A new dt only rewrites the gate slots the graph reads; masked steps replay a graph of their
    own that reads the mask from its arena slot, with a different mask at every replay."""
    L, chi, B = 10, 16, 4
    occ = tn_inputs.neel(L)
    us = tn_inputs.uniforms(13, (6, B))
    outs = []
    for graph in (True, False):
        st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, occ)
        st.graph_enable(graph)
        for k in range(6):
            dt = 0.01 * (1 + k % 3)
            _, mask = st.apply_jumps(api.MODE_QT, dt, us[k])
            st.tebd_step(dt, order=1, mask=mask if k % 2 else None)
        _, _, C_each, nrm = st.measure_corr(normalize=1, each=True)
        outs.append((C_each, nrm))
        st.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_two_stream_overlap_is_bit_identical():
    """Layers with more items than one workspace chunk run their chunks on two streams; every
    item is computed the same way, so the state equals the one-stream run bit for bit (eager and
    graph replay)."""
    L, chi, B, dt = 64, 16, 320, 0.01   # 320 * 32 = 10240 items per layer > one chunk
    occ = tn_inputs.neel(L)
    nz = tn_inputs.normals(5, (3, B * 2 * 2))
    res = []
    for overlap, graph in ((False, False), (True, False), (True, True)):
        st = api.State(api.KIND_MPS, api.Model.free_fermion(L), B, chi, occ, precision=api.SPLIT, sv_cutoff=1e-6)
        st.overlap(overlap)
        st.graph_enable(graph)
        for k in range(3):
            st.tebd_step(dt, order=1)
            st.apply_jumps(api.MODE_QSD, dt, nz[k], api.NOISE_GAUSS)
        res.append([st.get_instance(b) for b in (0, 161, B - 1)])
        st.close()
    for other in res[1:]:
        for a, b in zip(res[0], other):
            for ta, tb in zip(a[0], b[0]):
                assert np.array_equal(ta, tb)
            for la, lb in zip(a[1], b[1]):
                assert np.array_equal(la, lb)
            assert a[2] == b[2]
