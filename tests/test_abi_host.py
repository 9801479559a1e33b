"""CPU tests of the C-ABI library: it loads, exports every symbol of include/tebd.h, and its
host-side FP64 gate builder (Pade scaling-and-squaring) matches the oracle's gates."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2609_18841_amd import _lib, api
from oracle import model as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "tebd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "for", "while", "sizeof")))


def test_library_exports_every_header_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    syms = _header_symbols()
    assert set(syms) == set(_lib.EXPORTS)
    for name in syms:
        assert hasattr(lib, name), name


def test_arena_size_and_invalid_shapes():
    assert api.mps_arena_bytes(api.KIND_MPS, 16, 4, 32) > 0
    assert api.mps_arena_bytes(api.KIND_MPS, 1, 4, 32) == 0
    assert api.mps_arena_bytes(api.KIND_MPS, 16, 0, 32) == 0
    assert api.mps_arena_bytes(7, 16, 4, 32) == 0


@pytest.mark.parametrize("L", [2, 5, 8])
@pytest.mark.parametrize("tau", [0.05, 0.01, 0.3])
def test_host_gates_match_oracle(L, tau):
    mdl = M.Model(L, J=1.0, gamma=0.5)
    m = api.Model.free_fermion(L, 1.0, 0.5)
    for b in range(L - 1):
        g = api.tn_gate(api.KIND_MPS, m, b, tau)
        assert np.max(np.abs(g - M.gate_heff(mdl, b, tau))) < 1e-14
        G = api.tn_gate(api.KIND_MPDO, m, b, tau)
        assert np.max(np.abs(G - M.gate_liouville(mdl, b, tau))) < 1e-14


def test_host_gate_rejects_bad_bond():
    m = api.Model.free_fermion(4)
    with pytest.raises(api.TnError):
        api.tn_gate(api.KIND_MPS, m, 3, 0.1)


@pytest.mark.parametrize("which", ["two_sources", "dephasing"])
def test_host_gates_match_oracle_for_other_channel_sets(which):
    """Alternative jump sets of Sec. 2.1 (two sources; dephasing on every site with source and
    sink): the host gate builder agrees with the oracle's gates."""
    L, tau = 6, 0.05
    ch = M.two_sources(L, 0.5) if which == "two_sources" else M.source_sink_dephasing(L, 0.5, 0.3)
    mdl = M.Model(L, jumps=M.channel_jumps(ch))
    m = api.Model.channels(L, ch)
    for b in range(L - 1):
        g = api.tn_gate(api.KIND_MPS, m, b, tau)
        assert np.max(np.abs(g - M.gate_heff(mdl, b, tau))) < 1e-14
        G = api.tn_gate(api.KIND_MPDO, m, b, tau)
        assert np.max(np.abs(G - M.gate_liouville(mdl, b, tau))) < 1e-14


def test_binding_constants_match_header():
    """Every #define of include/tebd.h that the binding mirrors has the header's value."""
    import re
    from paper_2609_18841_amd import api
    hdr = open(os.path.join(ROOT, "include", "tebd.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (TN_\w+)\s+(-?\d+)", hdr)}
    pairs = {"TN_KIND_MPS": api.KIND_MPS, "TN_KIND_MPDO": api.KIND_MPDO, "TN_KIND_PURIFIED": api.KIND_PURIFIED,
             "TN_FP64": api.FP64, "TN_SPLIT": api.SPLIT, "TN_MODE_QT": api.MODE_QT, "TN_MODE_QSD": api.MODE_QSD,
             "TN_MODE_KRAUS": api.MODE_KRAUS, "TN_MODE_QT_SHIFT": api.MODE_QT_SHIFT,
             "TN_MODE_QSD_SHIFT": api.MODE_QSD_SHIFT, "TN_NOISE_GAUSS": api.NOISE_GAUSS,
             "TN_NOISE_BINARY": api.NOISE_BINARY,
             "TN_SCHED_LAYER": api.SCHED_LAYER, "TN_SCHED_SWEEP": api.SCHED_SWEEP}
    for name, val in pairs.items():
        assert defs[name] == val, name
    for i, k in enumerate(api.K_NAMES):
        assert defs["TN_K_" + k.upper()] == i
