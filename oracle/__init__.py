"""Plain CPU complex128 oracle for the TEBD-Lindblad hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (``paper_2609_18841_amd``) and imports nothing from it.

Everything here is written from the paper (C. Chatelain, "A first introduction
to Matrix Product State algorithms for the integration of Lindblad equation"):
plain loops, numpy/scipy library primitives (matmul, SVD, eigh, expm,
Sylvester solver), complex128 throughout, no blocking or fusion beyond what the
paper's definitions state.  Each function cites the section/equation it
follows, and states how it reads a passage where the paper is ambiguous or garbled.

Modules
-------
model      local operators, bond Hamiltonians, jump operators, gates (Sec. 2.1,
           2.3, 3.1, 3.2)
exact      closed-form correlation matrix, eq. (eqCorr)/(SoleqCorr) (Sec. 2.1)
ed         exact integration of the full Lindblad equation for small chains
dense      exact Trotter products on the full state vector / density vector
tebd       Hastings-form TEBD two-site update + layer schedule (Sec. 2.3, 3.1,
           3.2, 4)
sweep      the paper's sequential mixed-canonical sweep (Sec. 2.3, eq. ShiftCenter)
stochastic quantum-trajectory and quantum-state-diffusion steps, and the batch estimators
           of the linear unravelling (Sec. 4.1, 4.2)
kraus      Kraus-index compression of the locally purified form (Sec. 3.2)
measure    <c_i^+ c_j> by exact (gauge-independent) contraction
"""
