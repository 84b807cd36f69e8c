"""Pins of the complex-band oracle (App. B, Eq. cmp, and the band folding) against
results fixed independently of it: the closed form of a constant potential, the
1D transfer-matrix (Kronig-Penney) dispersion of potentials that depend on z only,
the symmetry lam -> 1/conj(lam) and zero flux of evanescent states, and the
primitive-cell -> supercell folding checked on the supercell's own eigenproblem."""
import numpy as np
import pytest

import msgen
import oracle as orc
from msgen.lattice import Cell, difference_set, plane_wave_basis
from msgen.potential import vq_gaussian_wells

KPAR = (0.07, -0.11)


def _cell_inputs(n_g, dz, vz=None, kpar=KPAR):
    """config1's transverse cell and wells over slices of thickness dz; with vz, a potential
    that depends on z only (V^p(Q) = vz[p] at Q = 0, zero elsewhere)."""
    j = msgen.config1()
    j.dz = np.asarray(dz, dtype=np.float64)
    inp = msgen.junction_inputs(j, kpar, n_g)
    if vz is not None:
        q0 = int(np.where((inp["q_miller"] == 0).all(axis=1))[0][0])
        vq = np.zeros_like(inp["vq"])
        vq[:, q0] = vz
        inp["vq"] = vq
    return inp


def _match(got, want, tol):
    """Every wanted eigenvalue has its own computed one within tol (relative)."""
    got = list(got)
    assert len(got) == len(want)
    for w in want:
        d = [abs(g - w) / abs(w) for g in got]
        i = int(np.argmin(d))
        assert d[i] < tol, (w, got[i], d[i])
        got.pop(i)


def _kp_lambdas(e, vz, dz):
    """Bloch factors of a 1D piecewise-constant potential at energy e: the roots of
    lam^2 - tr(T) lam + 1 = 0, T the product of the layers' (psi, psi') transfer matrices
    [[cos qw, sin(qw)/q], [-q sin qw, cos qw]], q = sqrt(e - v) (textbook Kronig-Penney)."""
    t = np.eye(2, dtype=np.complex128)
    for v, w in zip(vz, dz):
        q = np.sqrt(complex(e - v))
        layer = np.array([[np.cos(q * w), np.sin(q * w) / q], [-q * np.sin(q * w), np.cos(q * w)]])
        t = layer @ t
    tr = np.trace(t)
    r = np.sqrt(tr * tr - 4.0)
    return [(tr + r) / 2.0, (tr - r) / 2.0]


@pytest.mark.parametrize("n_slices", [1, 3])
def test_constant_potential_closed_form(n_slices):
    """V = v0 everywhere: lam = e^{+- i k_n d} with k_n = sqrt(E - |k+G_n|^2 - v0)."""
    dz = np.full(n_slices, 1.5 / n_slices)
    v0, e = 0.3, 2.1
    inp = _cell_inputs(9, dz, vz=np.full(n_slices, v0))
    prep = orc.prepare(inp)
    b = orc.complex_bands(prep, e)
    k = np.sqrt(e - prep["kin"] - v0 + 0j)
    want = list(np.exp(1j * k * 1.5)) + list(np.exp(-1j * k * 1.5))
    _match(b["lam"], want, 1e-11)
    assert abs(b["d"] - 1.5) < 1e-15


@pytest.mark.parametrize("e", [0.45, 1.3, 2.9])
def test_z_only_potential_matches_kronig_penney(e):
    """V(z) piecewise constant over four slices, uniform across the plane: every transverse
    channel n is the 1D problem at energy E - |k+G_n|^2, whose Bloch factors the layers'
    transfer matrices fix (propagating and evanescent alike)."""
    dz = np.array([0.3, 0.5, 0.2, 0.4])
    vz = np.array([0.0, 0.8, -0.5, 0.25])
    inp = _cell_inputs(9, dz, vz=vz)
    prep = orc.prepare(inp)
    b = orc.complex_bands(prep, e)
    want = []
    for kin in prep["kin"]:
        want += _kp_lambdas(e - kin, vz, dz)
    _match(b["lam"], want, 1e-9)


def test_wells_symmetry_and_flux():
    """A potential varying across the plane (config1's wells over three slices): the
    spectrum is closed under lam -> 1/conj(lam) (real energy, Hermitian H); evanescent
    states carry no flux; propagating states come in equal numbers of each direction."""
    dz = np.array([0.5, 0.6, 0.4])
    inp = _cell_inputs(13, dz)
    prep = orc.prepare(inp)
    e = 1.1
    b = orc.complex_bands(prep, e)
    lam = b["lam"]
    _match(lam, list(1.0 / np.conj(lam)), 1e-9)
    prop = np.abs(np.abs(lam) - 1.0) < 1e-8
    assert prop.sum() >= 2
    fluxes = [orc.mode_flux(prep, e, lam[i], b["x"][:, i]) for i in range(lam.size)]
    scale = max(abs(f) for f in fluxes)
    for i in np.where(~prop)[0]:
        assert abs(fluxes[i]) < 1e-10 * scale, (lam[i], fluxes[i])
    right = sum(1 for i in np.where(prop)[0] if fluxes[i] > 0)
    left = sum(1 for i in np.where(prop)[0] if fluxes[i] < 0)
    assert right == left == prop.sum() // 2
    for i in np.where(prop)[0]:
        assert abs(fluxes[i]) > 1e-6 * scale


def test_threshold_raises():
    inp = _cell_inputs(9, [0.5, 0.5], vz=np.array([0.0, 0.0]))
    prep = orc.prepare(inp)
    with pytest.raises(orc.ThresholdError):
        orc.complex_bands(prep, float(prep["kin"][0]))


@pytest.mark.parametrize("nmat", [((2, 0), (0, 1)), ((1, 1), (-1, 1))])
def test_folding_primitive_to_supercell(nmat):
    """Transverse supercells A_i = sum_k N_ik a_k of a potential with the primitive period
    (N = [[2, 0], [0, 1]], and the rotated [[1, 1], [-1, 1]]): then b_i = sum_j c_ij B_j with
    c = N^T, and the primitive waves at k and k + B1 fold onto the supercell's at K = k.  With
    the supercell basis made of both primitive bases folded by the appendix's index map, the
    supercell's complex bands are those of the primitive cell at k and at k + B1, and every
    folded primitive mode solves the supercell's Eq. cmp."""
    j = msgen.config1()
    dz = np.array([0.5, 0.7, 0.3])
    prim = j.cell
    nm = np.asarray(nmat, dtype=np.int64)
    a = np.asarray(prim.avec)
    sup = Cell(a1=tuple(nm[0] @ a), a2=tuple(nm[1] @ a))
    c = nm.T
    b1s = sup.bvec[0]
    assert np.allclose(c @ sup.bvec, prim.bvec)
    kpar = np.asarray(KPAR)
    n_p = 8
    sets = []
    for mk, kp in (((0, 0), kpar), ((1, 0), kpar + b1s)):
        miller = plane_wave_basis(prim, kp, n_p)
        qm, qij = difference_set(miller)
        inp = dict(miller=miller, q_miller=qm, q_of_ij=qij, vq=vq_gaussian_wells(prim, qm, j.wells, dz),
                   dz=dz, bvec=prim.bvec, kpar=kp)
        sets.append((mk, kp, miller, orc.prepare(inp)))
    m_sup = np.concatenate([np.asarray(mk) + m.astype(np.int64) @ c for mk, _, m, _ in sets])
    qm, qij = difference_set(m_sup)
    # the supercell potential: the primitive coefficient where Q = (m, n) c is a primitive
    # reciprocal vector, zero elsewhere
    mn = qm @ np.linalg.inv(c.astype(np.float64))
    prim_q = np.all(np.abs(mn - np.round(mn)) < 1e-9, axis=1)
    vq = np.zeros((dz.size, qm.shape[0]), dtype=np.complex128)
    vq[:, prim_q] = vq_gaussian_wells(prim, np.round(mn[prim_q]).astype(np.int64), j.wells, dz)
    psup = orc.prepare(dict(miller=m_sup, q_miller=qm, q_of_ij=qij, vq=vq, dz=dz, bvec=sup.bvec, kpar=kpar))
    # the folded primitive waves are exactly the supercell's basis vectors
    for mk, kp, m, prep in sets:
        idx = orc.fold_indices(m, c, mk, m_sup)
        assert np.allclose(orc.kinetic(m, prim.bvec, kp), psup["kin"][idx], rtol=0, atol=1e-12)
    e = 0.9
    bs = orc.complex_bands(psup, e)
    want = []
    for mk, kp, m, prep in sets:
        bp = orc.complex_bands(prep, e)
        want += list(bp["lam"])
        idx = orc.fold_indices(m, c, mk, m_sup)
        for i in range(bp["lam"].size):
            xf = orc.fold_mode(bp["x"][:, i], prep["u"][1], psup["u"][1], idx, m_sup.shape[0])
            res = bs["p"] @ xf - bp["lam"][i] * (bs["q"] @ xf)
            assert np.linalg.norm(res) < 1e-10 * max(1.0, abs(bp["lam"][i])), (i, np.linalg.norm(res))
    _match(bs["lam"], want, 1e-9)


# ---------------------------------------------------------------- transmission between
# periodic electrodes (App. C through the region's S-matrix)
def _with(inp, dz, vq):
    out = dict(inp)
    out["dz"] = np.asarray(dz, dtype=np.float64)
    out["vq"] = np.asarray(vq)
    return out


def test_free_electrodes_reproduce_free_lead_transmission():
    """Electrode cells of zero potential (one slice and two of other thicknesses): their Bloch
    states are the free plane waves, so T and R equal those of the free-lead path (itself
    pinned to closed forms and a second exact route)."""
    dz = np.array([0.5, 0.7, 0.3, 0.6])
    inp = _cell_inputs(11, dz)
    scatter = orc.prepare(inp)
    zero = np.zeros((1, inp["vq"].shape[1]), dtype=np.complex128)
    left = orc.prepare(_with(inp, [0.9], zero))
    right = orc.prepare(_with(inp, [0.4, 0.35], np.zeros((2, inp["vq"].shape[1]))))
    for e in (0.45, 1.3, 2.2):
        ref = orc.transmission(scatter, e)
        got = orc.transmission_bands(left, scatter, right, e)
        assert got["n_in"] == ref["n_open"]
        assert abs(got["T"] - ref["T"]) < 1e-10, (e, got["T"], ref["T"])
        assert abs(got["R"] - ref["R"]) < 1e-10


def test_crystal_continued_through_the_region_transmits_perfectly():
    """A scattering region that continues the electrodes' crystal (their cell's slices 2..M, 1
    repeated, ending with 2..M): every incident Bloch state is transmitted, T = the number of
    incident states, R = 0."""
    dz = np.array([0.5, 0.6, 0.4])
    inp = _cell_inputs(11, dz)
    cell = orc.prepare(inp)
    order = [1, 2, 0, 1, 2, 0, 1, 2]
    region = orc.prepare(_with(inp, dz[order], inp["vq"][order]))
    for e in (0.8, 1.7):
        got = orc.transmission_bands(cell, region, cell, e)
        assert got["n_in"] >= 1
        assert abs(got["T"] - got["n_in"]) < 1e-9, (e, got)
        assert abs(got["R"]) < 1e-9


def test_different_electrodes_conserve_flux():
    """A wells electrode on the left, a z-only crystal on the right, a random region between:
    T + R equals the number of incident Bloch states, and both lie in [0, n_in]."""
    dz = np.array([0.5, 0.6, 0.4])
    inp = _cell_inputs(11, dz)
    left = orc.prepare(inp)
    q0 = int(np.where((inp["q_miller"] == 0).all(axis=1))[0][0])
    vr = np.zeros((2, inp["vq"].shape[1]), dtype=np.complex128)
    vr[:, q0] = [0.3, -0.4]
    right = orc.prepare(_with(inp, [0.45, 0.55], vr))
    rng = np.random.default_rng(7)
    dzs = np.array([0.3, 0.5, 0.4, 0.2, 0.6])
    vq = inp["vq"][rng.integers(0, 3, dzs.size)] * 1.7
    region = orc.prepare(_with(inp, dzs, vq))
    for e in (0.9, 1.6, 2.4):
        got = orc.transmission_bands(left, region, right, e)
        assert abs(got["T"] + got["R"] - got["n_in"]) < 1e-9, (e, got["T"], got["R"], got["n_in"])
        assert -1e-12 < got["T"] < got["n_in"] + 1e-12 and got["R"] > -1e-12


def test_flux_matrix_diagonal_and_cross_flux():
    """The flux matrix's diagonal is each state's own flux, and two propagating Bloch states
    of different lam carry no cross flux (current conservation from cell to cell: J(u, v) is
    multiplied by conj(lam_u) lam_v per cell, which is not 1)."""
    dz = np.array([0.5, 0.6, 0.4])
    inp = _cell_inputs(13, dz)
    prep = orc.prepare(inp)
    e = 1.9
    m = orc.electrode_modes(prep, e)
    j = orc.flux_matrix(m["k"], m["a"], m["b"], m["a"], m["b"])
    lam = m["lam"]
    for i in range(lam.size):
        assert abs(j[i, i].real - orc.mode_flux(prep, e, lam[i], np.concatenate([m["a"][:, i],
                                                                                 m["b"][:, i] * lam[i]]))) \
            < 1e-12 * np.max(np.abs(j))
    prop = np.where(m["prop"])[0]
    assert prop.size >= 4
    scale = np.max(np.abs(np.diag(j)[prop]))
    for a in prop:
        for b in prop:
            if a != b and abs(lam[a] - lam[b]) > 1e-6:
                assert abs(j[a, b]) < 1e-10 * scale, (lam[a], lam[b], j[a, b])


def test_far_evanescent_states():
    """A cell whose evanescent states change by far more than FP64 spans per cell (N = 137, a
    5 bohr cell: S22 singular to working precision, some lam numerically infinite).  The list
    of k values is refused, but the states read at the plane where each is largest, through
    the cell's S-matrix, still match exactly: flux is conserved, free electrodes reproduce the
    free-lead path and a region that continues the crystal transmits perfectly."""
    j = msgen.config1()
    dz = np.full(3, 5.0 / 3)
    j.dz = dz
    inp = msgen.junction_inputs(j, KPAR, 137)
    cell = orc.prepare(inp)
    with pytest.raises(ValueError, match="beyond what FP64 resolves"):
        orc.complex_bands(cell, 1.3)
    rng = np.random.default_rng(3)
    region = orc.prepare(_with(inp, [0.3, 0.5, 0.4, 0.2], inp["vq"][rng.integers(0, 3, 4)] * 1.3))
    got = orc.transmission_bands(cell, region, cell, 1.3)
    assert abs(got["T"] + got["R"] - got["n_in"]) < 1e-11
    free = orc.prepare(_with(inp, [5.0], np.zeros((1, inp["vq"].shape[1]))))
    ref = orc.transmission(region, 1.3)
    assert abs(orc.transmission_bands(free, region, free, 1.3)["T"] - ref["T"]) < 1e-10
    order = [1, 2, 0, 1, 2, 0, 1, 2]
    crystal = orc.prepare(_with(inp, dz[order], inp["vq"][order]))
    got = orc.transmission_bands(cell, crystal, cell, 1.3)
    assert abs(got["T"] - got["n_in"]) < 1e-10 and abs(got["R"]) < 1e-10


def test_config3_electrode_cell_is_one_period():
    """The config-3 sheet electrode cell: its slices equal those of the sheet continued far along
    z (every well within 8 bohr of the cell included), in its first period and in the next one,
    and the top sheet's cell is the bottom one moved by +gap along y (a transverse phase per Q)."""
    from msgen.configs import _zigzag_sheet
    j = msgen.config3_electrode("bottom", n_g=61, n_slices=20)
    per = j.meta["period"]
    inp = msgen.junction_inputs(j, (0.0, 0.0))
    wide = msgen.Wells(_zigzag_sheet(20.0 - 6.3 / 2, -4 * per, 6 * per, zshift=-12 * per), 1.2, 0.6)
    two = msgen.Junction("two", j.cell, wide, np.full(40, per / 20), j.energies, j.kpars, j.n_g)
    inp2 = msgen.junction_inputs(two, (0.0, 0.0))
    scale = np.max(np.abs(inp["vq"]))
    assert np.max(np.abs(inp2["vq"][:20] - inp["vq"])) < 1e-13 * scale
    assert np.max(np.abs(inp2["vq"][20:] - inp["vq"])) < 1e-13 * scale
    top = msgen.junction_inputs(msgen.config3_electrode("top", n_g=61, n_slices=20), (0.0, 0.0))
    qv = np.asarray(inp["q_miller"], dtype=np.float64) @ np.asarray(inp["bvec"])
    phase = np.exp(-1j * qv[:, 1] * 6.3)        # every well moved by +gap along y
    assert np.max(np.abs(top["vq"] - inp["vq"] * phase[None, :])) < 1e-13 * scale
