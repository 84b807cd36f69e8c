"""Complex band structure of a periodic electrode cell and its folding from the
transverse primitive cell to a supercell (App. B: generalized Bloch conditions,
Eq. cmp, and the band-folding relations that close the appendix).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Built from the same
steps as ``transport`` (slice eigenpairs, interface S-matrices, star products);
no blocking or reordering beyond the appendix's equations.

Model: local potential only, so no non-local sphere crosses a cell boundary
(N_crosl = N_crosr = 0) and the unknowns of Eq. cmp are 2N plane-wave-slice
amplitudes.  The cell holds slices 1..M (the periodic electrode's unit cell
along z, a3 along z so a3_perp = 0); slice M+1 is the next cell's slice 1.
Reference planes as in ``transport``: z_p is the right end of slice p, so
z_{M+1} = z_1 + d with d the cell length.

The Bloch conditions (Eqs. bc1, bc2) on the wave and its z-derivative say
that the amplitudes in slice M+1 are lam = e^{i k d} times those in slice 1:
A^{M+1} = lam A^1, B^{M+1} = lam B^1.  The cell's S-matrix S = S(1, M+1)
gives [A^{M+1}; B^1] = S [A^1; B^{M+1}] (Eq. smm3_0 without the C terms).
Taking the cell's incoming amplitudes X = [A^1; B^{M+1}] as the unknowns
(the choice of App. B), the two block rows read

    lam A^1 = S11 A^1 + S12 B^{M+1}
    B^{M+1} = lam (S21 A^1 + S22 B^{M+1})

i.e.  P X = lam Q X  with  P = [[S11, S12], [0, I]],  Q = [[I, 0], [S21, S22]],
the generalized eigenproblem of Eq. cmp.  |lam| = 1: propagating Bloch
states; |lam| < 1: evanescent states decaying towards +z; |lam| > 1: decaying
towards -z.

Readings (listed in the design notes): the cell's first slice is repeated as
slice M+1 so that both Bloch planes are reference planes of the same slice
basis; k = -i log(lam) / d on the principal branch (Re k in (-pi/d, pi/d]).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .transport import (LEAD_THRESHOLD, ThresholdError, cascade, interface_smatrix, overlap,
                        wavevectors)

__all__ = ["cell_smatrix", "bloch_pencil", "complex_bands", "mode_flux", "flux_matrix", "electrode_modes",
           "transmission_bands", "fold_indices", "fold_mode", "PROPAGATING_TOL", "LAM_RANGE"]

# |lam| within this of 1: a propagating Bloch state
PROPAGATING_TOL = 1e-8
# Bloch factors outside [1/LAM_RANGE, LAM_RANGE] (evanescent states that change by more than
# this over one cell) are not resolved as numbers in FP64: S22 of the cell is then singular to
# working precision and Eq. cmp has numerically infinite eigenvalues, so ``complex_bands``
# refuses to list their k.  The states themselves stay well defined when each is read at the
# plane where it is largest (``electrode_modes``), so the matching does not need the range.
LAM_RANGE = 1e13


def _cell_slices(prep: dict):
    """Slices 1..M of a prepared cell (``transport.prepare``; its lead entries are unused)."""
    m = prep["n_slices"]
    if m < 1:
        raise ValueError("the cell needs at least one slice")
    return [prep["eps"][p] for p in range(1, m + 1)], [prep["u"][p] for p in range(1, m + 1)], \
        [float(prep["dz"][p]) for p in range(1, m + 1)]


def cell_smatrix(prep: dict, energy: float) -> dict:
    """S(1, M+1) of one electrode cell: the interfaces 1|2, ..., M-1|M and M|1' (slice 1
    of the next cell, thickness dz_1), joined by star products (Eq. recurrence1)."""
    eps, us, dz = _cell_slices(prep)
    for e in eps:
        if np.min(np.abs(energy - np.asarray(e))) < LEAD_THRESHOLD:
            raise ThresholdError("energy on a slice channel threshold (k = 0)")
    ks = [wavevectors(energy, e) for e in eps]
    m = len(eps)
    smats = []
    for p in range(m):
        q = (p + 1) % m                       # the next slice; after slice M, slice 1 again
        smats.append(interface_smatrix(overlap(us[p], us[q]), ks[p], ks[q], dz[q]))
    return cascade(smats)


def bloch_pencil(s: dict):
    """P, Q of Eq. cmp from the cell's S-matrix blocks (S11, S12, S21, S22) = (t, rp, r, tp)."""
    n = s["t"].shape[0]
    eye = np.eye(n, dtype=np.complex128)
    zero = np.zeros((n, n), dtype=np.complex128)
    p = np.block([[s["t"], s["rp"]], [zero, eye]])
    q = np.block([[eye, zero], [s["r"], s["tp"]]])
    return p, q


def complex_bands(prep: dict, energy: float, check_range: bool = True) -> dict:
    """Eq. cmp at one energy: lam [2N], X [2N][2N] (columns [A^1; B^{M+1}], unit 2-norm),
    k = -i log(lam) / d, the cell length d, and the pencil (P, Q).  With check_range, Bloch
    factors beyond LAM_RANGE raise."""
    s = cell_smatrix(prep, energy)
    p, q = bloch_pencil(s)
    lam, x = sla.eig(p, q)
    mag = np.abs(lam)
    if check_range and (not np.all(np.isfinite(lam)) or mag.min() < 1.0 / LAM_RANGE or mag.max() > LAM_RANGE):
        raise ValueError(f"Bloch factors span [{mag.min():.1e}, {mag.max():.1e}], beyond what FP64 resolves "
                         f"([{1.0 / LAM_RANGE:.0e}, {LAM_RANGE:.0e}]): a thinner cell or a smaller basis")
    x = x / np.linalg.norm(x, axis=0)[None, :]
    d = float(np.sum(_cell_slices(prep)[2]))
    with np.errstate(divide="ignore", invalid="ignore"):   # lam of 0 or inf without check_range
        k = -1j * np.log(lam) / d
    return dict(lam=lam, x=x, k=k, d=d, p=p, q=q)


def mode_flux(prep: dict, energy: float, lam: complex, x: np.ndarray) -> float:
    """Probability current of one mode (H = -nabla^2, per cell area) at the reference plane of
    slice 1: sum over its channels of 2 k (|A|^2 - |B|^2) (real k) or 4 kappa Im(conj(A) B)
    (k = i kappa), with B^1 = B^{M+1} / lam; the slice eigenstates are orthonormal, so the
    channels do not mix."""
    eps = _cell_slices(prep)[0][0]
    k = wavevectors(energy, eps)
    n = k.size
    a, b = x[:n], x[n:] / lam
    real = np.abs(k.imag) <= np.abs(k.real)
    j = np.sum(2.0 * k.real[real] * (np.abs(a[real]) ** 2 - np.abs(b[real]) ** 2))
    j += np.sum(4.0 * k.imag[~real] * np.imag(np.conj(a[~real]) * b[~real]))
    return float(j)


def flux_matrix(k, a_u, b_u, a_v, b_v) -> np.ndarray:
    """Cross flux J(u_i, v_j) = -i (conj(u) v' - conj(u') v) of two sets of modes given by
    their channel amplitudes (columns) at a reference plane, where u = a + b and
    u' = i k (a - b) per channel:  J = (A_u + B_u)^H K (A_v - B_v) + (A_u - B_u)^H K^* (A_v + B_v),
    K = diag(k).  J(u, u) is ``mode_flux``; Bloch states of different lam on the unit circle
    carry no cross flux."""
    k = np.asarray(k)
    su, du = a_u + b_u, a_u - b_u
    sv, dv = a_v + b_v, a_v - b_v
    return su.conj().T @ (k[:, None] * dv) + du.conj().T @ (np.conj(k)[:, None] * sv)


def electrode_modes(prep: dict, energy: float) -> dict:
    """The Bloch states of an electrode cell at one energy, with their amplitudes (a, b) in the
    slice-1 eigenbasis at a slice-1 reference plane (plane 1 for |lam| <= 1, plane M+1 for the
    others: each where it is largest, so that states decaying by more than FP64 spans over one
    cell stay well defined), sorted into
    right-going (propagating with positive flux, or decaying towards +z: |lam| < 1) and
    left-going ones (negative flux, or |lam| > 1).  Each set must hold N states."""
    bands = complex_bands(prep, energy, check_range=False)
    lam, x, p, q = bands["lam"], bands["x"], bands["p"], bands["q"]
    n = x.shape[0] // 2
    xt, xb = x[:n], x[n:]
    # each state where it is largest, through the cell's S-matrix (no division by lam): states
    # with |lam| <= 1 at plane 1, (A^1, B^1 = S21 A^1 + S22 B^{M+1}); the others at plane M+1,
    # (A^{M+1} = S11 A^1 + S12 B^{M+1}, B^{M+1}).  Both are slice-1 planes of the electrode.
    grow = np.abs(lam) > 1.0
    a = np.where(grow[None, :], p[:n, :n] @ xt + p[:n, n:] @ xb, xt)
    b = np.where(grow[None, :], xb, q[n:, :n] @ xt + q[n:, n:] @ xb)
    k = wavevectors(energy, _cell_slices(prep)[0][0])
    prop = np.abs(np.abs(lam) - 1.0) < PROPAGATING_TOL
    flux = np.real(np.diag(flux_matrix(k, a, b, a, b)))
    right = np.where((prop & (flux > 0)) | (~prop & (np.abs(lam) < 1.0)))[0]
    left = np.where((prop & (flux < 0)) | (~prop & (np.abs(lam) > 1.0)))[0]
    if right.size != n or left.size != n:
        raise ValueError(f"{right.size} right- and {left.size} left-going states, expected {n} each "
                         "(an energy at a band edge?)")
    return dict(lam=lam, a=a, b=b, k=k, prop=prop, flux=flux, right=right, left=left, u1=_cell_slices(prep)[1][0])


def transmission_bands(left_cell: dict, scatter: dict, right_cell: dict, energy: float) -> dict:
    """T and R between two periodic electrodes through a scattering region (App. C in the
    S-matrix form of Sec. II.A).  The left electrode ends with a copy of its cell's slice 1
    (reference plane: its right end), the scattering region's slices 1..N follow, and the right
    electrode starts with its cell's slice 1 (reference plane: its right end); the region's
    S-matrix S = S(L1, R1) joins those two planes.  Left of it the wave is an incident
    right-going propagating state plus the left-going states (amplitudes rho), right of it the
    right-going states (amplitudes tau): per incident state,

        T_a tau              = S11 (a_in + R_a rho) + S12 T_b tau
        b_in + R_b rho       = S21 (a_in + R_a rho) + S22 T_b tau

    (T_a, T_b: the right electrode's right-going states, R_a, R_b: the left electrode's
    left-going ones).  With incident states j and flux matrices J,
    T = Tr[(tau_p^H J_out tau_p) J_in^-1] over the propagating transmitted states, R likewise
    with -J over the propagating reflected ones; T + R = number of incident states."""
    for cell in (left_cell, right_cell):
        if not np.allclose(cell["kin"], scatter["kin"], rtol=0, atol=1e-12):
            raise ValueError("the electrodes and the scattering region need the same transverse basis")
    lm = electrode_modes(left_cell, energy)
    rm = electrode_modes(right_cell, energy)
    eps_s, us, dz = ([scatter["eps"][p] for p in range(1, scatter["n_slices"] + 1)],
                     [scatter["u"][p] for p in range(1, scatter["n_slices"] + 1)],
                     [float(scatter["dz"][p]) for p in range(1, scatter["n_slices"] + 1)])
    le, lu, _ = _cell_slices(left_cell)
    re_, ru, rdz = _cell_slices(right_cell)
    eps = [le[0]] + eps_s + [re_[0]]
    uu = [lu[0]] + us + [ru[0]]
    ws = [0.0] + dz + [rdz[0]]
    for e in eps:
        if np.min(np.abs(energy - np.asarray(e))) < LEAD_THRESHOLD:
            raise ThresholdError("energy on a slice channel threshold (k = 0)")
    ks = [wavevectors(energy, e) for e in eps]
    s = cascade([interface_smatrix(overlap(uu[p], uu[p + 1]), ks[p], ks[p + 1], ws[p + 1])
                 for p in range(len(eps) - 1)])
    inc = lm["right"][lm["prop"][lm["right"]]]
    ta, tb = rm["a"][:, rm["right"]], rm["b"][:, rm["right"]]
    ra, rb = lm["a"][:, lm["left"]], lm["b"][:, lm["left"]]
    ia, ib = lm["a"][:, inc], lm["b"][:, inc]
    m = np.block([[ta - s["rp"] @ tb, -s["t"] @ ra], [-s["tp"] @ tb, rb - s["r"] @ ra]])
    d = np.vstack([s["t"] @ ia, s["r"] @ ia - ib])
    y = np.linalg.solve(m, d)
    n = ta.shape[0]
    tau, rho = y[:n], y[n:]
    tp = rm["prop"][rm["right"]]
    rp = lm["prop"][lm["left"]]
    j_in = flux_matrix(lm["k"], ia, ib, ia, ib)
    j_out = flux_matrix(rm["k"], ta[:, tp], tb[:, tp], ta[:, tp], tb[:, tp])
    j_ref = -flux_matrix(lm["k"], ra[:, rp], rb[:, rp], ra[:, rp], rb[:, rp])
    jinv = np.linalg.inv(j_in)
    tt = float(np.real(np.trace(tau[tp].conj().T @ j_out @ tau[tp] @ jinv)))
    rr = float(np.real(np.trace(rho[rp].conj().T @ j_ref @ rho[rp] @ jinv)))
    return dict(T=tt, R=rr, n_in=int(inc.size), S=s, tau=tau, rho=rho)


def fold_indices(miller_prim, c, mk, miller_super) -> np.ndarray:
    """Position in the supercell basis of each primitive plane wave k_perp + m b1 + n b2 with
    k_perp = K_perp + m^k B1 + n^k B2, b1 = c11 B1 + c12 B2, b2 = c21 B1 + c22 B2: the wave
    is K_perp + (m^k + m c11 + n c21) B1 + (n^k + m c12 + n c22) B2 (App. B).  Raises if a
    folded wave is not in the supercell basis."""
    mp = np.asarray(miller_prim, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64).reshape(2, 2)
    big = np.stack([mk[0] + mp[:, 0] * c[0, 0] + mp[:, 1] * c[1, 0],
                    mk[1] + mp[:, 0] * c[0, 1] + mp[:, 1] * c[1, 1]], axis=1)
    where = {tuple(v): i for i, v in enumerate(np.asarray(miller_super, dtype=np.int64))}
    try:
        return np.array([where[tuple(v)] for v in big], dtype=np.int64)
    except KeyError as e:
        raise ValueError(f"folded plane wave {e} is not in the supercell basis")


def fold_mode(x_prim: np.ndarray, u1_prim, u1_super, idx: np.ndarray, n_super: int) -> np.ndarray:
    """A primitive-cell mode [A^1; B^{M+1}] (slice-1 eigenbasis of the primitive cell) as the
    supercell's unknowns: both halves to plane-wave coefficients (U^1 a), re-indexed by
    ``fold_indices``, then to the supercell's slice-1 eigenbasis (U^1_super^dagger)."""
    n = x_prim.shape[0] // 2
    out = np.zeros(2 * n_super, dtype=np.complex128)
    for h in range(2):
        pw = np.zeros(n_super, dtype=np.complex128)
        pw[idx] = u1_prim @ x_prim[h * n:(h + 1) * n]
        out[h * n_super:(h + 1) * n_super] = u1_super.conj().T @ pw
    return out
