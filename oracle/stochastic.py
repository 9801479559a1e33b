"""Quantum trajectories and quantum state diffusion on an MPS.

Oracle (test infrastructure).  Random numbers are inputs (FP64), so the HIP
path can be compared draw for draw.

Quantum trajectories, Sec. 4.1: per time step, with the current
state normalized, the jump probabilities are p_k = gamma_k dt <L_k^+ L_k>
(eq. TransitionRate times dt).  One uniform u in [0,1) picks jump k if
sum_{k'<k} p_k' <= u < sum_{k'<=k} p_k'; the jumped state is L_k psi, renormalized.
If no jump occurs the state is evolved by one Trotter step of exp(-i h^eff dt)
gates.  Jump XOR evolution, as stated in the paper.

Quantum state diffusion, Sec. 4.2 eqs. (EqMvtStochPsi), (DefAB) and the
product form that follows them: after the h^eff Trotter
step, apply prod_k (1 + dW_k sqrt(gamma_k) L_k) on the jump sites; no
renormalization (linear unravelling).  dW_k = sqrt(dt) (x + i y)/sqrt(2) with
x, y standard normals (complex Gaussian, E|dW|^2 = dt, E dW^2 = 0), or
dW_k = eta sqrt(dt) with eta = +-1 (the paper's binary noise).

Shifted jump operators (Sec. 4.1, the shift L_k -> L_k + Delta_k with Delta_k = -<L_k>,
and Sec. 4.2, A_k = sqrt(gamma_k)(L_k - <L_k>) with the matching B).  With l_k = <L_k> in the
normalized state just before the dissipative part of the step:
  - QT: rates gamma_k dt (<L_k^+ L_k> - |l_k|^2) (eq. for W with the shifted operator); a
    jump applies L_k - l_k; without a jump the state-dependent single-site part of the
    shifted h^eff, -(i/2) gamma_k (|Delta_k|^2 + 2 Delta_k^* L_k), is applied as its
    first-order factor 1 + dt gamma_k (l_k^* L_k - |l_k|^2/2) before the h^eff Trotter step;
  - QSD: after the h^eff Trotter step, per channel in channel order, the same drift factor
    (the extra part of B times dt) and then 1 + dW_k sqrt(gamma_k)(L_k - l_k).
All l_k of a step are taken from the same state, before any of the step's factors.
"""
import numpy as np

from .measure import corr_mps, jump_expectations, local_expectations
from .tebd import trotter_step


def apply_site_op(state, site, O):
    """B[a,p,c] -> sum_q O[p,q] B[a,q,c] (operator on the physical index of one site)."""
    B = state.tensors[site]
    state.tensors[site] = np.einsum("pq,aqc->apc", O, B)


def qt_decide(state, jumps, dt, u):
    """Return (k or -1, nrm, expectations) for one trajectory, Sec. 4.1."""
    ops = [(site, op) for site, op, g in jumps]
    nrm, vals = jump_expectations(state, ops)
    cum = 0.0
    for k, (site, op, g) in enumerate(jumps):
        cum += g * dt * vals[k] / nrm
        if u < cum:
            return k, nrm, vals
    return -1, nrm, vals


def qt_jump(state, jumps, dt, u):
    """Dissipative half of a quantum-trajectory step.  Returns the jump index or -1.

    On a jump the operator is applied and lognorm set so that the state is normalized;
    otherwise lognorm is set so that the current state is normalized (the evolution
    that follows starts from a normalized state).
    """
    k, nrm, vals = qt_decide(state, jumps, dt, u)
    if k >= 0:
        site, op, g = jumps[k]
        apply_site_op(state, site, op)
        state.lognorm = -0.5 * np.log(vals[k])
    else:
        state.lognorm = -0.5 * np.log(nrm)
    return k


def qt_step(state, model, jumps, dt, u, gate_fn, chi_max, cutoff):
    k = qt_jump(state, jumps, dt, u)
    if k < 0:
        trotter_step(state, gate_fn, 1, dt, chi_max, cutoff)
    return k


def qsd_increments(jumps, dt, rnd_row, noise_kind="gauss"):
    """dW_k for one trajectory and one step (complex Gaussian or the paper's binary eta)."""
    out = []
    for k in range(len(jumps)):
        if noise_kind == "gauss":
            x, y = rnd_row[2 * k], rnd_row[2 * k + 1]
            out.append(np.sqrt(dt) * (x + 1j * y) / np.sqrt(2.0))
        else:
            eta = -1.0 if rnd_row[k] < 0.5 else 1.0
            out.append(eta * np.sqrt(dt))
    return out


def qsd_noise_ops(jumps, dt, rnd_row, noise_kind="gauss"):
    """Local operators 1 + dW_k sqrt(gamma_k) L_k for one trajectory and one step."""
    dWs = qsd_increments(jumps, dt, rnd_row, noise_kind)
    return [(site, np.eye(op.shape[0], dtype=np.complex128) + dW * np.sqrt(g) * op)
            for (site, op, g), dW in zip(jumps, dWs)]


def qsd_noise(state, jumps, dt, rnd_row, noise_kind="gauss"):
    for site, O in qsd_noise_ops(jumps, dt, rnd_row, noise_kind):
        apply_site_op(state, site, O)


def qsd_step(state, jumps, dt, rnd_row, gate_fn, chi_max, cutoff, noise_kind="gauss", driver="gesdd"):
    trotter_step(state, gate_fn, 1, dt, chi_max, cutoff, driver=driver)
    qsd_noise(state, jumps, dt, rnd_row, noise_kind)


def _shift_means(state, jumps):
    """(nrm, <L_k^+L_k>/nrm, <L_k>/nrm) for every channel, from the current state."""
    ops = [(site, op) for site, op, g in jumps]
    nrm, m = jump_expectations(state, ops)
    _, l = local_expectations(state, ops)
    return nrm, [v / nrm for v in m], [v / nrm for v in l]


def drift_factor(op, g, dt, lk):
    """1 + dt gamma (l^* L - |l|^2/2): the single-site part of the shifted generator, first order."""
    one = np.eye(op.shape[0], dtype=np.complex128)
    return one + dt * g * (np.conj(lk) * op - 0.5 * abs(lk) ** 2 * one)


def qt_jump_shifted(state, jumps, dt, u):
    """Dissipative half of a quantum-trajectory step with shifted jump operators.

    Returns the jump index or -1; lognorm is set as in qt_jump (normalized after a jump,
    normalized before the no-jump factors otherwise).
    """
    nrm, mh, lh = _shift_means(state, jumps)
    cum, k = 0.0, -1
    for q, (site, op, g) in enumerate(jumps):
        cum += g * dt * (mh[q] - abs(lh[q]) ** 2)
        if u < cum:
            k = q
            break
    if k >= 0:
        site, op, g = jumps[k]
        apply_site_op(state, site, op - lh[k] * np.eye(op.shape[0], dtype=np.complex128))
        state.lognorm = -0.5 * np.log(nrm * (mh[k] - abs(lh[k]) ** 2))
    else:
        state.lognorm = -0.5 * np.log(nrm)
        for q, (site, op, g) in enumerate(jumps):
            apply_site_op(state, site, drift_factor(op, g, dt, lh[q]))
    return k


def qt_step_shifted(state, jumps, dt, u, gate_fn, chi_max, cutoff):
    k = qt_jump_shifted(state, jumps, dt, u)
    if k < 0:
        trotter_step(state, gate_fn, 1, dt, chi_max, cutoff)
    return k


def qsd_noise_shifted(state, jumps, dt, rnd_row, noise_kind="gauss"):
    _, _, lh = _shift_means(state, jumps)
    dWs = qsd_increments(jumps, dt, rnd_row, noise_kind)
    for q, (site, op, g) in enumerate(jumps):
        one = np.eye(op.shape[0], dtype=np.complex128)
        noise = one + dWs[q] * np.sqrt(g) * (op - lh[q] * one)
        apply_site_op(state, site, noise @ drift_factor(op, g, dt, lh[q]))


def qsd_step_shifted(state, jumps, dt, rnd_row, gate_fn, chi_max, cutoff, noise_kind="gauss"):
    trotter_step(state, gate_fn, 1, dt, chi_max, cutoff)
    qsd_noise_shifted(state, jumps, dt, rnd_row, noise_kind)


def qsd_estimators(states):
    """Batch estimators of the linear unravelling (Sec. 4.2): the histories are never
    renormalized, so <psi|psi> fluctuates around 1.  Returns (mean, ratio, mean_norm):
      mean  = (1/B) sum_b <psi_b|O|psi_b>, the estimator of the paper;
      ratio = sum_b <psi_b|O|psi_b> / sum_b <psi_b|psi_b>, which divides out the norm
              fluctuation of the sample;
      mean_norm = (1/B) sum_b <psi_b|psi_b>, whose expectation is 1.
    O runs over the c_i^+ c_j of the correlation matrix."""
    pairs = [corr_mps(st, normalize=False) for st in states]
    C_sum = sum(C for C, _ in pairs)
    n_sum = sum(n for _, n in pairs)
    B = len(states)
    return C_sum / B, C_sum / n_sum, n_sum / B
