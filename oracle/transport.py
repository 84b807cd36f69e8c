"""Plain FP64 reference of the transport method (Li, Chu, Zhang, Cheng,
"Electron transport in graphene/graphene side-contact junction by plane-wave
multiple scattering method", arXiv:1504.01462).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Slow and direct on
purpose: NumPy/SciPy in complex128, library routines (eigh, LU solve) as the
only building blocks, no blocking, fusion or reordering beyond the paper's
equations.

Model (local potential only; the non-local projector terms C, H^a, H^b,
h^a, h^b of the paper are zero here):  -nabla^2 psi + V psi = E psi in Ry/bohr
units, V periodic in the transverse plane, z-independent inside each slice,
V = const (default 0) in the two leads.

Notation follows the paper: slices p = 1..N between the left lead (p = 0) and
the right lead (p = N+1); the reference plane z_p of slice p is its right
end; in slice p the wave is sum_n phi_n^p [A_n e^{i k_n (z-z_p)} +
B_n e^{-i k_n (z-z_p)}].  S(p,p+1) maps [A^p; B^{p+1}] to [A^{p+1}; B^p]
(Sec. II.A, Eq. smm2); its blocks (S11, S12, S21, S22) are stored as
(t, rp, r, tp).

Readings where the paper is silent or garbled (each listed in the design
notes):
* k_n^p = sqrt(E - E_n^p) (the printed /hbar means /hbar^2; hbar^2/2m = 1),
  branch Im k >= 0, Re k > 0 on the real axis (forward = propagating or
  decaying towards +z).
* S(p,p+1) uses the thickness of slice p+1; the right lead has thickness 0.
* The overlap sum_s (M^{p+1}_{js})^* M^p_{ns} is (U^{p dagger} U^{p+1})_{nj}
  with unit-norm eigenvectors as the columns of U^p.
* T = sum_{i,j open} (k_i / k_j) |t_ij|^2 (flux-normalised), R likewise.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = [
    "recurrence2_step", "cond1", "mixed_doubling",
    "ThresholdError", "SingularError", "kinetic", "slice_hamiltonians", "slice_eigen",
    "prepare", "wavevectors", "overlap", "interface_xy", "interface_smatrix",
    "transfer_matrix", "smatrix_from_transfer", "identity_smatrix", "star", "cascade",
    "recurrence2_cascade", "interface_smatrices", "iter_interface_smatrices", "transmission_from_smatrix",
    "transmission", "global_system", "transfer_product", "born_reflection",
    "LEAD_THRESHOLD", "kpar_average", "slice_amplitudes", "dT_dV", "dT_dV_real",
]

LEAD_THRESHOLD = 1e-10


class ThresholdError(ValueError):
    """The energy sits on a lead channel threshold E = |k_par + G|^2 (+V_lead)."""


class SingularError(ValueError):
    """A matrix that must be inverted (X or I - S12 S21) is singular."""


# --------------------------------------------------------------------------------------
# E-independent part: Hamiltonians and slice eigenproblems (Sec. II.A, Eq. loc; App. A, Eq. A8)
# --------------------------------------------------------------------------------------

def kinetic(miller, bvec, kpar) -> np.ndarray:
    """|k_par + G|^2 for every basis vector (the kinetic term of Eq. loc)."""
    g = np.asarray(miller, dtype=np.float64) @ np.asarray(bvec, dtype=np.float64)
    return np.sum((np.asarray(kpar, dtype=np.float64) + g) ** 2, axis=1)


def slice_hamiltonians(kin, vq, q_of_ij) -> np.ndarray:
    """H^p_{ij} = |k_par+G_i|^2 delta_ij + V^p(G_i - G_j)  (Eq. loc), shape (N_s, N, N)."""
    h = np.ascontiguousarray(np.asarray(vq)[:, np.asarray(q_of_ij)])
    idx = np.arange(len(kin))
    h[:, idx, idx] += kin
    return h


def slice_eigen(h):
    """Eigenpairs of each slice Hamiltonian: E^p_n ascending, U^p columns = phi^p_n(G)."""
    eps = np.empty(h.shape[:2])
    u = np.empty(h.shape, dtype=np.complex128)
    for p in range(h.shape[0]):
        eps[p], u[p] = sla.eigh(h[p])
    return eps, u


def prepare(inp: dict, vlead_left=0.0, vlead_right=0.0) -> dict:
    """Slice data for one k_par: lists over p = 0..N+1 of E^p (N,), U^p (None = identity), dz_p."""
    kin = kinetic(inp["miller"], inp["bvec"], inp["kpar"])
    h = slice_hamiltonians(kin, inp["vq"], inp["q_of_ij"])
    eps_s, u_s = slice_eigen(h)
    ns = h.shape[0]
    eps = [kin + vlead_left] + [eps_s[p] for p in range(ns)] + [kin + vlead_right]
    us = [None] + [u_s[p] for p in range(ns)] + [None]
    dz = np.concatenate([[0.0], np.asarray(inp["dz"], dtype=np.float64), [0.0]])
    return dict(kin=kin, eps=eps, u=us, dz=dz, n=len(kin), n_slices=ns)


# --------------------------------------------------------------------------------------
# Per-energy part
# --------------------------------------------------------------------------------------

def wavevectors(energy: float, eps) -> np.ndarray:
    """k_n = sqrt(E - E_n) with Im k >= 0 (propagating: k > 0; evanescent: k = i kappa)."""
    k = np.sqrt(energy - np.asarray(eps, dtype=np.float64) + 0j)
    return np.where(k.imag < 0, -k, k)


def overlap(up, uq) -> np.ndarray:
    """O_nj = sum_s (M^{q}_{js})^* M^{p}_{ns} = (U^{p dagger} U^{q})_{nj}  (App. A, Eq. app)."""
    if up is None and uq is None:
        raise ValueError("two lead blocks cannot be adjacent")
    if up is None:
        return np.array(uq, copy=True)
    if uq is None:
        return up.conj().T.copy()
    return np.ascontiguousarray(up.conj().T) @ uq


def interface_xy(o, kp, kq):
    """X_nj = O_nj (k^p_n + k^{p+1}_j)/(2 k^p_n), Y_nj = O_nj (k^p_n - k^{p+1}_j)/(2 k^p_n)
    -- the bracketed coefficients of App. A, Eqs. (app) and (bpp)."""
    x = o * (kp[:, None] + kq[None, :]) / (2.0 * kp[:, None])
    y = o * (kp[:, None] - kq[None, :]) / (2.0 * kp[:, None])
    return x, y


def transfer_matrix(o, kp, kq, dzq):
    """The transfer matrix I(p,p+1) of App. A, Eq. (transfer), as the four blocks
    (I11, I12, I21, I22) = (X P^-1, Y P, Y P^-1, X P) with P = diag e^{i k^{p+1} dz}."""
    x, y = interface_xy(o, kp, kq)
    ph = np.exp(1j * kq * dzq)
    return x / ph[None, :], y * ph[None, :], y / ph[None, :], x * ph[None, :]


def smatrix_from_transfer(i11, i12, i21, i22) -> dict:
    """App. A, Eq. (scatter) taken literally: S11 = I11^-1, S12 = -I11^-1 I12,
    S21 = I21 S11, S22 = I22 + I21 S12."""
    s11 = np.linalg.inv(i11)
    s12 = -s11 @ i12
    return dict(t=s11, rp=s12, r=i21 @ s11, tp=i22 + i21 @ s12)


def interface_smatrix(o, kp, kq, dzq) -> dict:
    """S(p,p+1) from Eq. (scatter) with the transfer blocks of Eq. (transfer) inserted
    and the growing factor P^-1 = e^{-i k dz} cancelled analytically:

        S11 = P X^-1,  S12 = -P X^-1 Y P,  S21 = Y X^-1,  S22 = (X - Y X^-1 Y) P.
    """
    x, y = interface_xy(o, kp, kq)
    ph = np.exp(1j * kq * dzq)
    try:
        lu = sla.lu_factor(x, check_finite=True)
    except (sla.LinAlgError, ValueError) as e:  # pragma: no cover
        raise SingularError(str(e))
    if np.any(np.abs(np.diag(lu[0])) == 0):
        raise SingularError("X is singular")
    n = x.shape[0]
    xinv = np.ascontiguousarray(sla.lu_solve(lu, np.eye(n, dtype=np.complex128)))
    xinv_y = xinv @ y
    return dict(t=ph[:, None] * xinv,
                rp=-(ph[:, None] * xinv_y) * ph[None, :],
                r=y @ xinv,
                tp=(x - y @ xinv_y) * ph[None, :])


def identity_smatrix(n: int) -> dict:
    """S(p,p) = I (Sec. II.A, below Eq. smm2)."""
    e = np.eye(n, dtype=np.complex128)
    z = np.zeros((n, n), dtype=np.complex128)
    return dict(t=e, rp=z, r=z.copy(), tp=e.copy())


def star(a: dict, b: dict) -> dict:
    """Layer doubling, Eq. (recurrence1) / App. A Eq. (recurrence) without the h terms:
    a = S(m,n), b = S(n,k)  ->  S(m,k)."""
    n = a["t"].shape[0]
    f = np.eye(n, dtype=np.complex128) - a["rp"] @ b["r"]
    lu = sla.lu_factor(f)
    if np.any(np.abs(np.diag(lu[0])) == 0):
        raise SingularError("I - S12(m,n) S21(n,k) is singular")
    finv_t = np.ascontiguousarray(sla.lu_solve(lu, a["t"]))      # [I - S12 S21]^-1 S11(m,n)
    finv_rp = np.ascontiguousarray(sla.lu_solve(lu, a["rp"]))    # [I - S12 S21]^-1 S12(m,n)
    return dict(t=b["t"] @ finv_t,
                rp=b["rp"] + b["t"] @ finv_rp @ b["tp"],
                r=a["r"] + a["tp"] @ b["r"] @ finv_t,
                tp=a["tp"] @ b["tp"] + a["tp"] @ b["r"] @ finv_rp @ b["tp"])


def cascade(smats, order: str = "left") -> dict:
    """S(first, last) = s[0] * s[1] * ... (star products; the grouping is free because
    doubling combines any split m < n < k)."""
    smats = list(smats)
    if order == "left":
        acc = smats[0]
        for s in smats[1:]:
            acc = star(acc, s)
        return acc
    if order == "right":
        acc = smats[-1]
        for s in reversed(smats[:-1]):
            acc = star(s, acc)
        return acc
    if order == "tree":
        level = smats
        while len(level) > 1:
            nxt = [star(level[i], level[i + 1]) for i in range(0, len(level) - 1, 2)]
            if len(level) % 2:
                nxt.append(level[-1])
            level = nxt
        return level[0]
    raise ValueError(order)


def recurrence2_cascade(transfers_and_smats) -> dict:
    """Left fold with the mixed recurrence of App. A, Eq. (recurrence2): carry
    (I11, I12, S21, S22); convert to S at the end through Eq. (scatter)."""
    it = iter(transfers_and_smats)
    a = dict(next(it))
    for b in it:
        m = a["i11"] + a["i12"] @ b["r"]
        minv = np.linalg.inv(m)
        a = dict(i11=m @ b["i11"],
                 i12=m @ b["i12"] + a["i12"] @ b["tp"],
                 r=a["r"] + a["tp"] @ b["r"] @ minv,
                 tp=a["tp"] @ b["tp"] - a["tp"] @ b["r"] @ minv @ a["i12"] @ b["tp"])
    s11 = np.linalg.inv(a["i11"])
    return dict(t=s11, rp=-s11 @ a["i12"], r=a["r"], tp=a["tp"])


def recurrence2_step(a: dict, b: dict) -> dict:
    """One step of the mixed recurrence of App. A, Eq. (recurrence2), without the h
    terms: a = (I11, I12, S21, S22)(m,n), b = (I11, I12, S21, S22)(n,k)  ->  (m,k)."""
    m = a["i11"] + a["i12"] @ b["r"]
    minv = np.linalg.inv(m)
    return dict(i11=m @ b["i11"],
                i12=m @ b["i12"] + a["i12"] @ b["tp"],
                r=a["r"] + a["tp"] @ b["r"] @ minv,
                tp=a["tp"] @ b["tp"] - a["tp"] @ b["r"] @ minv @ a["i12"] @ b["tp"])


def cond1(a) -> float:
    """1-norm condition number ||A||_1 ||A^-1||_1 (dense inverse)."""
    return float(np.linalg.norm(a, 1) * np.linalg.norm(np.linalg.inv(a), 1))


def mixed_doubling(prep: dict, energy: float, max_cond: float) -> dict:
    """Whole S by doubling, as App. A describes after Eq. (recurrence2): the interface
    blocks (I11, I12, S21, S22) are combined pairwise, level after level, with the mixed
    recurrence while cond_1(I11) of every block stays at or below max_cond; then every
    block is turned into S through Eq. (scatter) (S11 = I11^-1, S12 = -I11^-1 I12) and
    the remaining levels use the star product of Eq. (recurrence).  Pairs are formed
    left to right; an odd last block moves up a level unchanged.  Returns the whole S
    and the number of levels done in the mixed form."""
    _lead_check(energy, prep["eps"][0])
    _lead_check(energy, prep["eps"][-1])
    ks = [wavevectors(energy, e) for e in prep["eps"]]
    blocks = []
    for p in range(prep["n_slices"] + 1):
        o = overlap(prep["u"][p], prep["u"][p + 1])
        i11, i12, _, _ = transfer_matrix(o, ks[p], ks[p + 1], prep["dz"][p + 1])
        sm = interface_smatrix(o, ks[p], ks[p + 1], prep["dz"][p + 1])
        blocks.append(dict(i11=i11, i12=i12, r=sm["r"], tp=sm["tp"]))

    def to_s(blk):
        s11 = np.linalg.inv(blk["i11"])
        return dict(t=s11, rp=-s11 @ blk["i12"], r=blk["r"], tp=blk["tp"])

    levels = 0
    mixed = max(cond1(b["i11"]) for b in blocks) <= max_cond
    if not mixed:
        blocks = [to_s(b) for b in blocks]
    while len(blocks) > 1:
        pair = recurrence2_step if mixed else star
        nxt = [pair(blocks[i], blocks[i + 1]) for i in range(0, len(blocks) - 1, 2)]
        if len(blocks) % 2:
            nxt.append(blocks[-1])
        blocks = nxt
        if mixed:
            levels += 1
            if max(cond1(b["i11"]) for b in blocks) > max_cond:
                mixed = False
                blocks = [to_s(b) for b in blocks]
    whole = to_s(blocks[0]) if mixed else blocks[0]
    return dict(S=whole, mixed_levels=levels)


def _lead_check(energy, eps_lead):
    if np.min(np.abs(energy - np.asarray(eps_lead))) < LEAD_THRESHOLD:
        raise ThresholdError(f"E = {energy} is within {LEAD_THRESHOLD} of a lead channel threshold")


def iter_interface_smatrices(prep: dict, energy: float, reverse: bool = False):
    """S(p,p+1) for p = 0..N (or N..0), produced one at a time."""
    _lead_check(energy, prep["eps"][0])
    _lead_check(energy, prep["eps"][-1])
    ks = [wavevectors(energy, e) for e in prep["eps"]]
    order = range(prep["n_slices"] + 1)
    for p in (reversed(order) if reverse else order):
        o = overlap(prep["u"][p], prep["u"][p + 1])
        yield interface_smatrix(o, ks[p], ks[p + 1], prep["dz"][p + 1])


def interface_smatrices(prep: dict, energy: float):
    """[S(p,p+1) for p = 0..N] at one energy."""
    return list(iter_interface_smatrices(prep, energy))


def transmission_from_smatrix(s: dict, energy: float, eps_left, eps_right):
    """T and R of the whole junction for waves incident from the left:
    A^0 = I, B^{N+1} = 0 gives t = A^{N+1} = S11, r = B^0 = S21 (App. C)."""
    _lead_check(energy, eps_left)
    _lead_check(energy, eps_right)
    kl = wavevectors(energy, eps_left)
    kr = wavevectors(energy, eps_right)
    ol = np.where(np.asarray(eps_left) < energy)[0]
    orr = np.where(np.asarray(eps_right) < energy)[0]
    t = s["t"][np.ix_(orr, ol)]
    r = s["r"][np.ix_(ol, ol)]
    tt = float(np.sum((kr[orr].real[:, None] / kl[ol].real[None, :]) * np.abs(t) ** 2))
    rr = float(np.sum((kl[ol].real[:, None] / kl[ol].real[None, :]) * np.abs(r) ** 2))
    return tt, rr, int(ol.size)


def transmission(prep: dict, energy: float, order: str = "left") -> dict:
    """Full path at one (E, k_par): slice S-matrices, star cascade, T and R."""
    if order == "left":            # streamed: S(0,1) * S(1,2) * ...
        it = iter_interface_smatrices(prep, energy)
        s = next(it)
        for b in it:
            s = star(s, b)
    elif order == "right":         # streamed: ... * (S(N-1,N) * S(N,N+1))
        it = iter_interface_smatrices(prep, energy, reverse=True)
        s = next(it)
        for a in it:
            s = star(a, s)
    else:
        s = cascade(interface_smatrices(prep, energy), order)
    tt, rr, n_open = transmission_from_smatrix(s, energy, prep["eps"][0], prep["eps"][-1])
    return dict(T=tt, R=rr, n_open=n_open, S=s)


# --------------------------------------------------------------------------------------
# Second exact route and cross-checks (tiny inputs)
# --------------------------------------------------------------------------------------

def global_system(prep: dict, energy: float):
    """t and r from one dense linear system: continuity of psi and psi' at every
    interface in the G basis, no S-matrices.  Inside slice p the wave is written
    as U^p [a^p e^{ik(z - z_{p-1})} + B^p e^{-ik(z - z_p)}] so every coefficient
    is bounded.  Unknowns r = B^0, (a^p, B^p)_{p=1..N}, t = A^{N+1}; incidence
    A^0 = e_j, B^{N+1} = 0 for every j.  Returns (t, r), each (N, N)."""
    n, ns = prep["n"], prep["n_slices"]
    ks = [wavevectors(energy, e) for e in prep["eps"]]
    dz = prep["dz"]
    nunk = 2 * n * (ns + 1)
    m = np.zeros((nunk, nunk), dtype=np.complex128)
    rhs = np.zeros((nunk, n), dtype=np.complex128)
    eye = np.eye(n)

    def col(p, which):          # column offset of an unknown block
        if p == 0:
            return 0                                   # r
        if p == ns + 1:
            return n + 2 * n * ns                      # t
        return n + 2 * n * (p - 1) + (0 if which == "a" else n)

    for p in range(ns + 1):     # interface at z_p between block p and p+1
        r0 = 2 * n * p
        # left side (block p) at its right end z_p
        up = eye if prep["u"][p] is None else prep["u"][p]
        kp = ks[p]
        if p == 0:
            # lead: psi = e_j + r ;  -i psi' = K (e_j - r)
            m[r0:r0 + n, col(0, "b"):col(0, "b") + n] += eye
            m[r0 + n:r0 + 2 * n, col(0, "b"):col(0, "b") + n] += -np.diag(kp)
            rhs[r0:r0 + n] -= eye
            rhs[r0 + n:r0 + 2 * n] -= np.diag(kp)
        else:
            php = np.exp(1j * kp * dz[p])
            ca, cb = col(p, "a"), col(p, "b")
            m[r0:r0 + n, ca:ca + n] += up * php[None, :]
            m[r0:r0 + n, cb:cb + n] += up
            m[r0 + n:r0 + 2 * n, ca:ca + n] += (up * kp[None, :]) * php[None, :]
            m[r0 + n:r0 + 2 * n, cb:cb + n] += -(up * kp[None, :])
        # right side (block p+1) at its left end z_p, subtracted
        q = p + 1
        uq = eye if prep["u"][q] is None else prep["u"][q]
        kq = ks[q]
        if q == ns + 1:
            ct = col(q, "a")
            m[r0:r0 + n, ct:ct + n] -= eye
            m[r0 + n:r0 + 2 * n, ct:ct + n] -= np.diag(kq)
        else:
            phq = np.exp(1j * kq * dz[q])
            ca, cb = col(q, "a"), col(q, "b")
            m[r0:r0 + n, ca:ca + n] -= uq
            m[r0:r0 + n, cb:cb + n] -= uq * phq[None, :]
            m[r0 + n:r0 + 2 * n, ca:ca + n] -= uq * kq[None, :]
            m[r0 + n:r0 + 2 * n, cb:cb + n] -= -(uq * kq[None, :]) * phq[None, :]
    sol = np.linalg.solve(m, rhs)
    return sol[col(ns + 1, "a"):col(ns + 1, "a") + n], sol[0:n]


def transfer_product(prep: dict, energy: float):
    """t and r from the literal product of the transfer matrices I(p,p+1) of
    App. A, Eq. (smm1)/(transfer): [A^0; B^0] = I(0,1) ... I(N,N+1) [A^{N+1}; B^{N+1}].
    Numerically unstable for evanescent modes (the reason the paper moves to
    S-matrices); only for thin, shallow inputs."""
    n = prep["n"]
    ks = [wavevectors(energy, e) for e in prep["eps"]]
    tot = np.eye(2 * n, dtype=np.complex128)
    for p in range(prep["n_slices"] + 1):
        o = overlap(prep["u"][p], prep["u"][p + 1])
        i11, i12, i21, i22 = transfer_matrix(o, ks[p], ks[p + 1], prep["dz"][p + 1])
        tot = tot @ np.block([[i11, i12], [i21, i22]])
    m11, m21 = tot[:n, :n], tot[n:, :n]
    t = np.linalg.inv(m11)
    return t, m21 @ t


def born_reflection(kin, vq, q_of_ij, dz, energy: float) -> np.ndarray:
    """First-order (Born) reflection amplitude between free-lead channels:
    r_ij = -(i / 2k_i) sum_p V^p(G_i - G_j) (e^{i kappa z_p} - e^{i kappa z_{p-1}})/(i kappa),
    kappa = k_i + k_j, from the 1D Green's function e^{ik|z|}/(2ik) of App. A
    (below Eq. A10) applied to the sliced potential."""
    k = wavevectors(energy, kin)
    z = np.concatenate([[0.0], np.cumsum(dz)])
    kap = k[:, None] + k[None, :]
    v = np.asarray(vq)[:, np.asarray(q_of_ij)]                  # (N_s, N, N)
    ph = (np.exp(1j * kap[None] * z[1:, None, None]) - np.exp(1j * kap[None] * z[:-1, None, None])) / (1j * kap[None])
    return -(1j / (2.0 * k[:, None])) * np.sum(v * ph, axis=0)


def kpar_average(t_k, n_open_k):
    """Per-energy average over the k_par mesh, Sec. II.B Eq. (T1_d):
    T_bar(E) = (1 / N^x N^y) sum_k T(E, k); also sum_k T / sum_k N_open.
    Arrays are [n_k][n_e]."""
    t_k = np.asarray(t_k, dtype=np.float64)
    n = np.asarray(n_open_k, dtype=np.float64)
    tbar = t_k.sum(axis=0) / t_k.shape[0]
    tot = n.sum(axis=0)
    per = np.where(tot > 0, t_k.sum(axis=0) / np.where(tot > 0, tot, 1.0), 0.0)
    return tbar, per


# --------------------------------------------------------------------------------------
# First variation of T with respect to the slice potentials
# --------------------------------------------------------------------------------------

def slice_amplitudes(prep: dict, energy: float, a0, bn1):
    """(A^p, B^p) for p = 0..N+1 of the solution with incoming amplitudes A^0 = a0 (left
    lead) and B^{N+1} = bn1 (right lead), columns = several solutions.  From the left
    cascade L = S(0,p) and the right cascade R = S(p,N+1) (Sec. II.A, Eq. smm2):
    A^p = L11 A^0 + L12 B^p and B^p = R21 A^p + R22 B^{N+1}, i.e.
    (I - L12 R21) A^p = L11 A^0 + L12 R22 B^{N+1}."""
    smats = interface_smatrices(prep, energy)
    n, ns = prep["n"], prep["n_slices"]
    left = [identity_smatrix(n)]
    for s_ in smats:
        left.append(star(left[-1], s_))                 # left[p] = S(0,p)
    right = [identity_smatrix(n)]
    for s_ in reversed(smats):
        right.append(star(s_, right[-1]))              # right[k] = S(N+1-k, N+1)
    right = right[::-1]                                 # right[p] = S(p, N+1)
    out = []
    for p in range(ns + 2):
        lp, rp_ = left[p], right[p]
        f = np.eye(n, dtype=np.complex128) - lp["rp"] @ rp_["r"]
        a = np.linalg.solve(f, lp["t"] @ a0 + lp["rp"] @ (rp_["tp"] @ bn1))
        b = rp_["r"] @ a + rp_["tp"] @ bn1
        out.append((a, b))
    return out, left[-1]


def _exp_integral(kappa, width):
    """int_{-w}^{0} e^{i kappa s} ds, elementwise (w >= 0)."""
    x = 1j * kappa * width
    small = np.abs(x) < 1e-8
    safe = np.where(small, 1.0, kappa)
    val = (1.0 - np.exp(-x)) / (1j * safe)
    return np.where(small, width * (1.0 - 0.5 * x), val)


def dT_dV(prep: dict, energy: float, q_of_ij, n_q: int) -> np.ndarray:
    """g[p][Q] (slices p = 1..N as rows 0..N-1) with dT = 2 Re sum_{p,Q} g[p][Q] dV^p(Q) to
    first order, for any perturbation dV of the slice potentials' Fourier coefficients
    (H^p_ab = |k+G_a|^2 delta_ab + V^p(G_a - G_b)).

    Derivation (not in the paper; the sliced model as in Sec. II): with the Wronskian
    W[f, g] = f^dagger g' - f'^dagger g, dW/dz = f^dagger dH g when f solves the unperturbed
    equation and g the perturbed one.  Taking g = psi_j (incident from the left in open
    channel j: A^0 = e_j, B^{N+1} = 0) and f = phi_i (outgoing only into the right lead's open
    channel i: the open rows of B^0 vanish, those of A^{N+1} equal e_i, the incoming
    amplitudes only on open channels) gives dt_ij = (1/(2 i k_i)) int phi_i^dagger dH psi_j dz,
    and dT = sum_ij (k_i/k_j) 2 Re(conj(t_ij) dt_ij).  Inside slice p both are
    U^p [A e^{ik(z-z_p)} + B e^{-ik(z-z_p)}], so the z integral is a sum of exponential
    integrals over the slice."""
    n, ns = prep["n"], prep["n_slices"]
    _lead_check(energy, prep["eps"][0])
    _lead_check(energy, prep["eps"][-1])
    kl = wavevectors(energy, prep["eps"][0])
    kr = wavevectors(energy, prep["eps"][-1])
    ol = np.where(np.asarray(prep["eps"][0]) < energy)[0]
    orr = np.where(np.asarray(prep["eps"][-1]) < energy)[0]
    g = np.zeros((ns, n_q), dtype=np.complex128)
    if ol.size == 0 or orr.size == 0:
        return g
    # in-states psi_j
    a0 = np.zeros((n, ol.size), dtype=np.complex128)
    a0[ol, np.arange(ol.size)] = 1.0
    amp_in, whole = slice_amplitudes(prep, energy, a0, np.zeros_like(a0))
    t = whole["t"][np.ix_(orr, ol)]
    # out-states phi_i: solve [r_OO t'_OR; t_RO r'_RR] [x; y] = [0; e_i] on the open channels
    sys_ = np.block([[whole["r"][np.ix_(ol, ol)], whole["tp"][np.ix_(ol, orr)]],
                     [whole["t"][np.ix_(orr, ol)], whole["rp"][np.ix_(orr, orr)]]])
    rhs = np.zeros((ol.size + orr.size, orr.size), dtype=np.complex128)
    rhs[ol.size + np.arange(orr.size), np.arange(orr.size)] = 1.0
    xy = np.linalg.solve(sys_, rhs)
    fa0 = np.zeros((n, orr.size), dtype=np.complex128)
    fa0[ol, :] = xy[:ol.size]
    fb = np.zeros((n, orr.size), dtype=np.complex128)
    fb[orr, :] = xy[ol.size:]
    amp_out, _ = slice_amplitudes(prep, energy, fa0, fb)
    # weights w_ij = (k_i / k_j) conj(t_ij) / (2 i k_i) = conj(t_ij) / (2 i k_j)
    w = np.conj(t) / (2j * kl[ol][None, :])                    # (i in orr, j in ol)
    q = np.asarray(q_of_ij)
    for p in range(1, ns + 1):
        k = wavevectors(energy, prep["eps"][p])
        width = prep["dz"][p]
        a_j, b_j = amp_in[p]
        c_i, d_i = amp_out[p]
        kc = np.conj(k)[:, None]
        km = k[None, :]
        m = (_exp_integral(km - kc, width) * (c_i.conj() @ w @ a_j.T)
             + _exp_integral(-km - kc, width) * (c_i.conj() @ w @ b_j.T)
             + _exp_integral(km + kc, width) * (d_i.conj() @ w @ a_j.T)
             + _exp_integral(-km + kc, width) * (d_i.conj() @ w @ b_j.T))
        u = prep["u"][p]
        kmat = u.conj() @ m @ u.T                                # K_ab = sum_nm conj(U_an) M_nm U_bm
        g[p - 1] = np.bincount(q.ravel(), weights=kmat.real.ravel(), minlength=n_q) + \
            1j * np.bincount(q.ravel(), weights=kmat.imag.ravel(), minlength=n_q)
    return g


def dT_dV_real(g: np.ndarray, q_miller) -> tuple:
    """The gradient with respect to real parameters on a half-set of Q (V(-Q) = conj V(Q)
    keeps H Hermitian): for each Q with its partner -Q, dT/dRe V(Q) = 2 Re(g(Q) + g(-Q)) and
    dT/dIm V(Q) = 2 Im(g(-Q) - g(Q)); for Q = -Q only the real part, 2 Re g(Q).  Returns
    (index of Q, index of -Q, d/dRe, d/dIm) arrays over the half-set."""
    qm = np.asarray(q_miller)
    index = {tuple(v): i for i, v in enumerate(qm.tolist())}
    partner = np.array([index[tuple((-v).tolist())] for v in qm])
    keep = np.arange(len(qm)) <= partner
    qi = np.where(keep)[0]
    qj = partner[qi]
    self_ = qi == qj
    d_re = 2.0 * np.real(g[:, qi] + np.where(self_[None, :], 0.0, g[:, qj]))
    d_im = np.where(self_[None, :], 0.0, 2.0 * np.imag(g[:, qj] - g[:, qi]))
    return qi, qj, d_re, d_im
