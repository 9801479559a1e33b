"""Python binding of the C ABI (argument marshalling only; every step runs in the HIP library).

Names follow include/tebd.h.  PyTorch supplies the device arena (a uint8 tensor)
and the HIP stream; all arithmetic happens in libtebd.so.
"""
import ctypes

import numpy as np

from . import _lib

KIND_MPS, KIND_MPDO, KIND_PURIFIED = 0, 1, 2
FP64, SPLIT = 0, 1
MODE_QT, MODE_QSD, MODE_KRAUS, MODE_QT_SHIFT, MODE_QSD_SHIFT = 0, 1, 2, 3, 4
NOISE_GAUSS, NOISE_BINARY = 0, 1
TN_OK, TN_EINVAL, TN_ENOMEM, TN_EHIP, TN_ENOCONV, TN_ENUMERIC = 0, -1, -2, -3, -4, -5
SCHED_LAYER, SCHED_SWEEP = 0, 1
K_THETA, K_GRAM, K_HETRD, K_STEQR, K_VECS, K_SPLIT, K_MEASURE, K_JUMPS = range(8)
K_NAMES = ["theta", "gram", "hetrd", "steqr", "vecs", "split", "measure", "jumps"]

_ERR = {0: "TN_OK", -1: "TN_EINVAL", -2: "TN_ENOMEM", -3: "TN_EHIP", -4: "TN_ENOCONV", -5: "TN_ENUMERIC"}


class TnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERR.get(code, code)}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise TnError(rc, _lib.load().mps_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if a is not None else None


def _ubp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)) if a is not None else None


class Model:
    """tn_model: two-site terms h_bond[(L-1), 4, 4] and local jump operators (site, 2x2, rate)."""

    def __init__(self, L, h_bond, jumps):
        self.L = int(L)
        self.h = np.ascontiguousarray(np.asarray(h_bond, dtype=np.complex128).reshape(L - 1, 4, 4))
        self.sites = np.ascontiguousarray(np.array([j[0] for j in jumps], dtype=np.int32))
        self.ops = np.ascontiguousarray(np.array([np.asarray(j[1], dtype=np.complex128) for j in jumps]).reshape(-1, 2, 2)) \
            if jumps else np.zeros((0, 2, 2), dtype=np.complex128)
        self.gam = np.ascontiguousarray(np.array([j[2] for j in jumps], dtype=np.float64))
        self._hv = self.h.view(np.float64)
        self._ov = self.ops.view(np.float64)

    @staticmethod
    def free_fermion(L, J=1.0, gamma=0.5):
        """Sec. 2.1 chain: h = -J (s+ s- + s- s+), source s+ on site 0, sink s- on site L-1, rate gamma."""
        sp = np.array([[0, 0], [1, 0]], dtype=np.complex128)
        sm = sp.T.copy()
        h = -J * (np.kron(sp, sm) + np.kron(sm, sp))
        return Model(L, [h] * (L - 1), [(0, sp, gamma), (L - 1, sm, gamma)])

    @staticmethod
    def channels(L, channels, J=1.0):
        """Hopping chain of Sec. 2.1 with a list of (kind, site, rate) channels: kind "source"
        (s+), "sink" (s-) or "dephasing" (n = s+ s-), e.g. the alternative drives the section
        mentions (two sources; dephasing on every site)."""
        sp = np.array([[0, 0], [1, 0]], dtype=np.complex128)
        sm = sp.T.copy()
        ops = {"source": sp, "sink": sm, "dephasing": sp @ sm}
        h = -J * (np.kron(sp, sm) + np.kron(sm, sp))
        return Model(L, [h] * (L - 1), [(int(k), ops[kind], float(g)) for kind, k, g in channels])

    def struct(self):
        m = _lib.TnModel()
        m.L = self.L
        m.d = 2
        m.h_bond = self._hv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        m.n_jumps = len(self.gam)
        m.jump_site = self.sites.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        m.jump_op = self._ov.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(self.gam) else None
        m.gamma = self.gam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(self.gam) else None
        return m


def tn_gate(kind, model, bond, tau):
    D = 16 if kind == KIND_MPDO else 4
    out = np.zeros((D, D), dtype=np.complex128)
    st = model.struct()
    _check(_lib.load().tn_gate(kind, ctypes.byref(st), bond, tau, out.view(np.float64).ctypes.data_as(
        ctypes.POINTER(ctypes.c_double))))
    return out


def mps_arena_bytes(kind, L, batch, chi_max, chi_k_max=1, precision=FP64, chunk_items=0):
    return int(_lib.load().mps_arena_bytes(kind, L, batch, chi_max, chi_k_max, precision, chunk_items))


class State:
    """A batch of tensor-network instances living in a torch-owned device arena."""

    def __init__(self, kind, model, batch, chi_max, init_occ, precision=FP64, chi_k_max=1, sv_cutoff=1e-12,
                 device="cuda:0", stream=None):
        import torch
        lib = _lib.load()
        self.lib = lib
        self.kind, self.model, self.B, self.chi, self.L = kind, model, batch, chi_max, model.L
        self.precision = precision
        self._chik = chi_k_max
        nbytes = mps_arena_bytes(kind, model.L, batch, chi_max, chi_k_max, precision)
        if nbytes == 0:
            raise TnError(-1, "invalid shape for mps_arena_bytes")
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        # a created stream (default priority) of its own: tebd_step can then capture and replay
        # HIP graphs; every entry point synchronizes it before returning host outputs
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        occ = np.ascontiguousarray(np.asarray(init_occ, dtype=np.int32))
        self._mstruct = model.struct()
        h = ctypes.c_void_p()
        _check(lib.mps_alloc(ctypes.byref(h), kind, ctypes.byref(self._mstruct), batch, chi_max, chi_k_max, precision,
                             _ip(occ), float(sv_cutoff), ctypes.c_void_p(self.arena.data_ptr()), nbytes,
                             ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h
        self.tcap = int(lib.mps_instance_tensor_capacity(h))
        self.lcap = int(lib.mps_instance_lambda_capacity(h))

    def close(self):
        if self.h:
            _check(self.lib.mps_free(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- hot path
    def tebd_step(self, dt, order=1, n_steps=1, mask=None):
        tw = np.zeros(self.B)
        m = None if mask is None else np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
        _check(self.lib.tebd_step(self.h, float(dt), order, n_steps, _ubp(m), _dp(tw)))
        return tw

    def apply_jumps(self, mode, dt, rnd=None, noise_kind=NOISE_GAUSS):
        r = None if rnd is None else np.ascontiguousarray(np.asarray(rnd, dtype=np.float64))
        need = {MODE_QT: self.B, MODE_QT_SHIFT: self.B}.get(mode)
        if mode in (MODE_QSD, MODE_QSD_SHIFT):
            need = self.B * len(self.model.gam) * (2 if noise_kind == NOISE_GAUSS else 1)
        if need is not None and r is not None and r.size < need:
            raise ValueError(f"rnd holds {r.size} numbers, mode {mode} reads {need}")
        jumped = np.zeros(self.B, dtype=np.int32)
        mask = np.zeros(self.B, dtype=np.uint8)
        _check(self.lib.apply_jumps(self.h, mode, float(dt), _dp(r), noise_kind, _ip(jumped), _ubp(mask)))
        return jumped, mask

    def measure_corr(self, normalize=1, each=False):
        """(C_mean, C_var, C_each or None, norms).  normalize on an MPS: 1 normalized per
        instance, 0 the linear QSD values <psi|O|psi>, 2 the same per instance with C_mean the
        ratio sum <psi|O|psi> / sum <psi|psi>."""
        L = self.L
        mean = np.zeros((L, L), dtype=np.complex128)
        var = np.zeros((L, L))
        ce = np.zeros((self.B, L, L), dtype=np.complex128) if each else None
        nrm = np.zeros(self.B)
        _check(self.lib.measure_corr(self.h, normalize, _dp(mean.view(np.float64)), _dp(var),
                                     _dp(ce.view(np.float64)) if each else None, _dp(nrm)))
        return mean, var, ce, nrm

    def measure_corr_noalloc(self, normalize=1, each=False):
        """measure_corr with the sweep's workspace in the library's static scratch (allocates no
        device memory); same results."""
        L = self.L
        mean = np.zeros((L, L), dtype=np.complex128)
        var = np.zeros((L, L))
        ce = np.zeros((self.B, L, L), dtype=np.complex128) if each else None
        nrm = np.zeros(self.B)
        _check(self.lib.measure_corr_noalloc(self.h, normalize, _dp(mean.view(np.float64)), _dp(var),
                                             _dp(ce.view(np.float64)) if each else None, _dp(nrm)))
        return mean, var, ce, nrm

    def measure_async_enable(self):
        """Give the state the second device buffer that measure_start / measure_finish use."""
        import torch
        nb = int(self.lib.tn_measure_async_bytes(self.h))
        buf = torch.empty(nb + 256, dtype=torch.uint8, device=self.arena.device)
        base = buf.data_ptr()
        _check(self.lib.tn_measure_async_enable(self.h, ctypes.c_void_p(base + (-base) % 256), nb))
        # the library now holds the new buffer; only then may the one it held before be released
        # (a refused call leaves the old buffer in use by an outstanding measurement)
        self._abuf = buf

    def measure_start(self, normalize=1):
        """Snapshot the state and start measuring it; later steps overlap with the measurement."""
        _check(self.lib.measure_corr_start(self.h, normalize))

    def measure_finish(self, each=False):
        """Results of the outstanding measure_start, as measure_corr returns them."""
        L = self.L
        mean = np.zeros((L, L), dtype=np.complex128)
        var = np.zeros((L, L))
        ce = np.zeros((self.B, L, L), dtype=np.complex128) if each else None
        nrm = np.zeros(self.B)
        _check(self.lib.measure_corr_finish(self.h, _dp(mean.view(np.float64)), _dp(var),
                                            _dp(ce.view(np.float64)) if each else None, _dp(nrm)))
        return mean, var, ce, nrm

    # ---- state I/O
    def get_instance(self, inst):
        dims = np.zeros(self.L + 1, dtype=np.int32)
        t = np.zeros(2 * self.tcap)
        lam = np.zeros(self.lcap)
        ln = np.zeros(1)
        tr = np.zeros(1)
        _check(self.lib.mps_get_instance(self.h, inst, _ip(dims), _dp(t), _dp(lam), _dp(ln), _dp(tr)))
        tz = t.view(np.complex128)
        tensors, lams = [], []
        off, lo = 0, 0
        for i in range(self.L):
            d = self._dsite(i)
            n = dims[i] * d * dims[i + 1]
            tensors.append(tz[off:off + n].reshape(dims[i], d, dims[i + 1]).copy())
            off += n
        for b in range(self.L - 1):
            lams.append(lam[lo:lo + dims[b + 1]].copy())
            lo += dims[b + 1]
        return tensors, lams, float(ln[0]), float(tr[0])

    def dims(self, inst):
        """Bond dimensions of instance inst (L + 1 ints, dims[0] = dims[L] = 1)."""
        d = np.zeros(self.L + 1, dtype=np.int32)
        _check(self.lib.mps_get_instance(self.h, inst, _ip(d), None, None, None, None))
        return d

    def lams(self, inst):
        """Bond weights of instance inst: a list of L - 1 arrays (bond b holds dims[b + 1] values)."""
        d = np.zeros(self.L + 1, dtype=np.int32)
        lam = np.zeros(self.lcap)
        _check(self.lib.mps_get_instance(self.h, inst, _ip(d), None, _dp(lam), None, None))
        out, lo = [], 0
        for b in range(self.L - 1):
            out.append(lam[lo:lo + d[b + 1]].copy())
            lo += d[b + 1]
        return out

    def set_instance(self, inst, tensors, lams, lognorm=0.0):
        dims = np.array([1] + [t.shape[2] for t in tensors], dtype=np.int32)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.complex128).reshape(-1) for t in tensors]))
        lflat = np.ascontiguousarray(np.concatenate([np.asarray(l, dtype=np.float64).reshape(-1) for l in lams])) \
            if lams else np.zeros(1)
        _check(self.lib.mps_set_instance(self.h, inst, _ip(dims), _dp(flat.view(np.float64)), _dp(lflat),
                                         float(lognorm)))

    def replicate(self, src=0):
        _check(self.lib.mps_replicate(self.h, src))

    def _dsite(self, i):
        if self.kind == KIND_MPDO:
            return 4
        if self.kind == KIND_PURIFIED and i in set(int(x) for x in self.model.sites):
            return 2 * self._chik
        return 2

    # ---- timing
    def stats(self, reset=False):
        """(items whose vectors came from the degenerate-cluster route (inverse iteration, or QL
        for a broken tridiagonal), items re-orthogonalized) since mps_alloc or the last reset
        (split precision, n <= 128, chi <= 64)."""
        a, b = ctypes.c_longlong(), ctypes.c_longlong()
        _check(self.lib.tn_stats(self.h, 1 if reset else 0, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def prof_enable(self, on=True):
        _check(self.lib.tn_prof_enable(self.h, 1 if on else 0))

    def tuning(self, set_variant=-1):
        """(variant, [ms_mfma, ms_tiles]) of the Householder autotuner; set_variant 0/1 overrides."""
        v = ctypes.c_int()
        ms = (ctypes.c_float * 2)()
        _check(self.lib.tn_tuning(self.h, int(set_variant), ctypes.byref(v), ms))
        return v.value, [ms[0], ms[1]]

    def graph_enable(self, on=True):
        """Allow (default) or forbid HIP-graph replay of unmasked Trotter steps."""
        _check(self.lib.tn_graph_enable(self.h, 1 if on else 0))

    def overlap(self, on=True):
        """Allow (default) or forbid running the chunks of a layer on two streams."""
        _check(self.lib.tn_overlap(self.h, 1 if on else 0))

    def buckets(self, on=-1, parity=0):
        """[(largest Gram order, bond positions, Householder variant)] of the parity's bond-size
        buckets; on = 1 (layers of at least one item per compute unit), 2 (every layer) or 0 (off) switches the
        bucketing first, -1 only reports."""
        cnt = ctypes.c_int()
        nmax, nb, hv = (ctypes.c_int * 4)(), (ctypes.c_int * 4)(), (ctypes.c_int * 4)()
        _check(self.lib.tn_buckets(self.h, int(on), int(parity), ctypes.byref(cnt), nmax, nb, hv))
        return [(nmax[i], nb[i], hv[i]) for i in range(cnt.value)]

    def theta_precision(self, bits):
        """Split mode: form Theta on the FP32 (32, default) or the FP64 (64) matrix cores."""
        _check(self.lib.tn_theta_precision(self.h, int(bits)))

    def schedule(self, sched):
        """SCHED_LAYER (layer-parallel Hastings form) or SCHED_SWEEP (sequential sweep with the
        orthogonality centre, Sec. 2.3) for the following tebd_step calls."""
        _check(self.lib.tn_schedule(self.h, int(sched)))

    def prof_query(self, kid):
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        _check(self.lib.tn_prof_query(self.h, kid, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def prof_busy(self, kid):
        """Wall ms during which some launch of kernel id `kid` was running (both streams)."""
        ms = ctypes.c_double()
        _check(self.lib.tn_prof_busy(self.h, kid, ctypes.byref(ms)))
        return ms.value
