"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test checks a closed form,
an invariant, a special case that reduces to a textbook result, or a second
exact algorithm (the global linear system, the literal transfer-matrix
product) written without S-matrices.
"""
import numpy as np
import pytest

import msgen
import oracle as orc


def _c1(kpar=(0.0, 0.0), n_g=None, n_slices=None, slab=6.0):
    j = msgen.config1()
    if n_slices is not None:
        j.dz = np.full(n_slices, slab / n_slices)
    return j, msgen.junction_inputs(j, kpar, n_g)


def _with_vq(inp, vq):
    d = dict(inp)
    d["vq"] = vq
    return d


def _const_vq(inp, vz):
    """V^p(Q) = vz[p] at Q = 0 only (a potential that depends on z alone)."""
    q0 = np.where((inp["q_miller"] == 0).all(axis=1))[0][0]
    vq = np.zeros((len(vz), inp["q_miller"].shape[0]), dtype=np.complex128)
    vq[:, q0] = vz
    return vq


# ---------------------------------------------------------------- inputs ---------------

def test_basis_closed_shell_and_negation():
    _, inp = _c1()
    m = inp["miller"]
    s = (m.astype(int) ** 2).sum(1)
    assert m.shape == (37, 2) and s.max() == 10
    assert sum(1 for a in range(-4, 5) for b in range(-4, 5) if a * a + b * b <= 10) == 37
    assert set(map(tuple, m)) == set(map(tuple, -m))


def test_vq_matches_brute_force_quadrature():
    """Closed-form V^p(Q) against a real-space grid (periodic images summed), Gauss-Legendre
    in z over each slice and a 2D FFT."""
    j, inp = _c1()
    a = 5.0
    n = 64
    x = np.arange(n) * a / n
    gl_x, gl_w = np.polynomial.legendre.leggauss(16)
    z = msgen.slice_edges(j.dz)
    for p in (0, 7, 23):
        zz = 0.5 * (z[p] + z[p + 1]) + 0.5 * (z[p + 1] - z[p]) * gl_x
        v = np.zeros((n, n))
        for c, d, s in zip(j.wells.centres, j.wells.depth, j.wells.sigma):
            for ix in range(-2, 3):
                for iy in range(-2, 3):
                    dx = x[:, None] - c[0] - ix * a
                    dy = x[None, :] - c[1] - iy * a
                    fz = np.sum(0.5 * gl_w * np.exp(-(zz - c[2]) ** 2 / (2 * s * s)))
                    v += -d * np.exp(-(dx ** 2 + dy ** 2) / (2 * s * s)) * fz
        f = np.fft.fft2(v) / n ** 2
        qm = inp["q_miller"]
        ref = f[qm[:, 0] % n, qm[:, 1] % n]
        assert np.max(np.abs(ref - inp["vq"][p])) < 1e-12


# ---------------------------------------------------------------- slices ----------------

def test_slice_eigen_residuals():
    _, inp = _c1()
    kin = orc.kinetic(inp["miller"], inp["bvec"], inp["kpar"])
    h = orc.slice_hamiltonians(kin, inp["vq"], inp["q_of_ij"])
    assert np.allclose(h, np.conj(np.transpose(h, (0, 2, 1))), atol=1e-15)
    eps, u = orc.slice_eigen(h)
    for p in range(h.shape[0]):
        assert np.linalg.norm(h[p] @ u[p] - u[p] * eps[p]) / np.linalg.norm(h[p]) < 1e-13
        assert np.linalg.norm(u[p].conj().T @ u[p] - np.eye(37)) < 5e-12


def test_fresnel_decoupled_interface():
    """V depending on z only and U = I: each channel is a 1D step, whose S-matrix is the
    Fresnel result, including evanescent channels."""
    e = 0.8
    eps_p = np.array([0.0, 0.3, 1.2, 5.0, -0.4])
    eps_q = np.array([0.5, 0.1, 0.7, 4.0, 0.2])
    kp, kq = orc.wavevectors(e, eps_p), orc.wavevectors(e, eps_q)
    dz = 0.37
    s = orc.interface_smatrix(np.eye(5, dtype=complex), kp, kq, dz)
    ph = np.exp(1j * kq * dz)
    assert np.allclose(np.diag(s["r"]), (kp - kq) / (kp + kq), atol=1e-14, rtol=0)
    assert np.allclose(np.diag(s["t"]), 2 * kp / (kp + kq) * ph, atol=1e-14, rtol=0)
    assert np.allclose(np.diag(s["rp"]), (kq - kp) / (kp + kq) * ph ** 2, atol=1e-14, rtol=0)
    assert np.allclose(np.diag(s["tp"]), 2 * kq / (kp + kq) * ph, atol=1e-14, rtol=0)
    for b in s.values():
        assert np.max(np.abs(b - np.diag(np.diag(b)))) < 1e-15


@pytest.mark.parametrize("vc", [0.0, 0.35])
def test_free_propagation(vc):
    """Constant potential in slab and leads: t = diag(e^{i k L}), r = 0, T = N_open."""
    j, inp = _c1()
    inp = _with_vq(inp, _const_vq(inp, np.full(j.n_slices, vc)))
    prep = orc.prepare(inp, vc, vc)
    for e in (0.5, 2.2, 4.1):
        out = orc.transmission(prep, e)
        k = orc.wavevectors(e, prep["kin"] + vc)
        assert np.max(np.abs(out["S"]["t"] - np.diag(np.exp(1j * k * j.length)))) < 1e-13
        assert np.max(np.abs(out["S"]["r"])) < 1e-13
        assert abs(out["T"] - out["n_open"]) < 1e-13 and out["n_open"] == int(np.sum(prep["kin"] + vc < e))


def _barrier_closed(eps, v0, b):
    if eps > v0:
        q = np.sqrt(eps - v0)
        return 1.0 / (1.0 + v0 ** 2 * np.sin(q * b) ** 2 / (4 * eps * (eps - v0)))
    kap = np.sqrt(v0 - eps)
    return 1.0 / (1.0 + v0 ** 2 * np.sinh(kap * b) ** 2 / (4 * eps * (v0 - eps)))


@pytest.mark.parametrize("v0", [0.5, -0.5])
def test_square_barrier(v0):
    """V(z) = V0 on [0.5, 2.5] bohr (edges on slice boundaries): every open channel is the
    textbook 1D barrier, T = sum_G [1 + V0^2 sin^2(q b) / (4 eps (eps - V0))]^-1."""
    j, inp = _c1(n_slices=12, slab=3.0)
    vz = np.zeros(12)
    vz[2:10] = v0
    inp = _with_vq(inp, _const_vq(inp, vz))
    prep = orc.prepare(inp)
    for e in (0.2, 0.45, 0.7, 1.0, 2.0, 3.5):
        out = orc.transmission(prep, e)
        ref = sum(_barrier_closed(e - kk, v0, 2.0) for kk in prep["kin"] if kk < e)
        assert abs(out["T"] - ref) < 1e-12
        assert abs(out["T"] + out["R"] - out["n_open"]) < 1e-12


def _flux_s(s, e, kin):
    o = np.where(kin < e)[0]
    k = orc.wavevectors(e, kin)[o].real
    sq, isq = np.sqrt(k), 1 / np.sqrt(k)
    blk = lambda m: (sq[:, None] * m[np.ix_(o, o)]) * isq[None, :]
    return np.block([[blk(s["t"]), blk(s["rp"])], [blk(s["r"]), blk(s["tp"])]])


def test_current_conservation_and_unitarity():
    _, inp = _c1()
    prep = orc.prepare(inp)
    for e in np.linspace(0.1, 1.0, 8).tolist() + [2.0, 3.7]:
        out = orc.transmission(prep, e)
        assert abs(out["T"] + out["R"] - out["n_open"]) < 1e-12
        st = _flux_s(out["S"], e, prep["kin"])
        assert np.max(np.abs(st.conj().T @ st - np.eye(st.shape[0]))) < 1e-12


def test_reciprocity():
    """Real V (time reversal): t~(k)_ij = t~'(-k)_ji and r~(k)_ij = r~(-k)_ji, with the basis
    at -k_par the negation of the basis at k_par."""
    j = msgen.config1()
    kpar = np.array([0.31, 0.17])
    inp = msgen.junction_inputs(j, kpar)
    neg = dict(inp)
    neg["kpar"] = -kpar
    neg["miller"] = -inp["miller"]
    neg["q_miller"], neg["q_of_ij"] = msgen.difference_set(neg["miller"])
    neg["vq"] = msgen.vq_gaussian_wells(j.cell, neg["q_miller"], j.wells, j.dz)
    pa, pb = orc.prepare(inp), orc.prepare(neg)
    assert np.allclose(pa["kin"], pb["kin"], atol=1e-14)
    for e in (0.4, 2.5):
        sa = _flux_s(orc.transmission(pa, e)["S"], e, pa["kin"])
        sb = _flux_s(orc.transmission(pb, e)["S"], e, pb["kin"])
        m = sa.shape[0] // 2
        assert np.max(np.abs(sa[:m, :m] - sb[m:, m:].T)) < 1e-12   # t(k) vs t'(-k)^T
        assert np.max(np.abs(sa[m:, :m] - sb[m:, :m].T)) < 1e-12   # r(k) vs r(-k)^T
        ta, tb = orc.transmission(pa, e)["T"], orc.transmission(pb, e)["T"]
        assert abs(ta - tb) < 1e-12


def test_associativity_of_the_cascade():
    _, inp = _c1()
    prep = orc.prepare(inp)
    sm = orc.interface_smatrices(prep, 0.63)
    a, b, c = (orc.cascade(sm, o) for o in ("left", "right", "tree"))
    for key in ("t", "rp", "r", "tp"):
        scale = max(1.0, np.max(np.abs(a[key])))
        assert np.max(np.abs(a[key] - b[key])) < 1e-12 * scale
        assert np.max(np.abs(a[key] - c[key])) < 1e-12 * scale


def test_identity_element():
    _, inp = _c1()
    prep = orc.prepare(inp)
    s = orc.interface_smatrices(prep, 0.5)[5]
    i = orc.identity_smatrix(37)
    for x in (orc.star(i, s), orc.star(s, i)):
        for key in s:
            assert np.max(np.abs(x[key] - s[key])) < 1e-15


@pytest.mark.parametrize("n_g,n_slices", [(13, 8), (37, 24)])
def test_global_linear_system(n_g, n_slices):
    """Second exact route: one dense system of psi / psi' continuity conditions."""
    _, inp = _c1(n_g=n_g, n_slices=n_slices)
    prep = orc.prepare(inp)
    for e in (0.3, 0.9, 2.6):
        s = orc.transmission(prep, e)["S"]
        t, r = orc.global_system(prep, e)
        assert np.max(np.abs(t - s["t"])) < 1e-12
        assert np.max(np.abs(r - s["r"])) < 1e-12


def test_transfer_product_and_literal_scatter():
    """Thin, shallow case: the literal transfer-matrix product (Eq. smm1/transfer) and the
    literal Eq. (scatter) agree with the cancelled-form S cascade."""
    _, inp = _c1(n_g=13, n_slices=8, slab=0.8)
    prep = orc.prepare(inp)
    e = 0.7
    s = orc.transmission(prep, e)["S"]
    t, r = orc.transfer_product(prep, e)
    assert np.max(np.abs(t - s["t"])) < 1e-11 and np.max(np.abs(r - s["r"])) < 1e-11
    ks = [orc.wavevectors(e, x) for x in prep["eps"]]
    for p in range(prep["n_slices"] + 1):
        o = orc.overlap(prep["u"][p], prep["u"][p + 1])
        lit = orc.smatrix_from_transfer(*orc.transfer_matrix(o, ks[p], ks[p + 1], prep["dz"][p + 1]))
        can = orc.interface_smatrix(o, ks[p], ks[p + 1], prep["dz"][p + 1])
        for key in can:
            assert np.max(np.abs(lit[key] - can[key])) < 1e-12


def test_recurrence2_matches_recurrence():
    """The mixed transfer/scattering doubling (App. A, Eq. recurrence2) reproduces the
    pure scattering-matrix doubling (Eq. recurrence) on a few slices."""
    _, inp = _c1(n_g=13, n_slices=8, slab=2.0)
    prep = orc.prepare(inp)
    e = 0.55
    ks = [orc.wavevectors(e, x) for x in prep["eps"]]
    items = []
    for p in range(prep["n_slices"] + 1):
        o = orc.overlap(prep["u"][p], prep["u"][p + 1])
        i11, i12, _, _ = orc.transfer_matrix(o, ks[p], ks[p + 1], prep["dz"][p + 1])
        s = orc.interface_smatrix(o, ks[p], ks[p + 1], prep["dz"][p + 1])
        items.append(dict(i11=i11, i12=i12, r=s["r"], tp=s["tp"]))
    a = orc.recurrence2_cascade(items)
    b = orc.transmission(prep, e)["S"]
    for key in ("t", "rp", "r", "tp"):
        assert np.max(np.abs(a[key] - b[key])) < 1e-10 * max(1.0, np.max(np.abs(b[key])))


def test_mixed_doubling_matches_star_cascade():
    """Doubling with the mixed recurrence until cond_1(I11) passes a threshold, then the
    star product (App. A after Eq. recurrence2), gives the whole S of the plain left fold
    of star products, whatever the threshold: 1 (pure S from the start), a moderate one
    (a switch part-way) and none (mixed to the end)."""
    _, inp = _c1(n_g=13, n_slices=8, slab=2.0)
    prep = orc.prepare(inp)
    e = 0.55
    ref = orc.transmission(prep, e)["S"]
    nb = prep["n_slices"] + 1
    full_levels = int(np.ceil(np.log2(nb)))
    seen = set()
    for max_cond, levels in ((1.0, 0), (None, None), (np.inf, full_levels)):
        if max_cond is None:    # a threshold between the conds of levels 1 and 2
            ks = [orc.wavevectors(e, x) for x in prep["eps"]]
            b = []
            for p in range(nb):
                o = orc.overlap(prep["u"][p], prep["u"][p + 1])
                i11, i12, _, _ = orc.transfer_matrix(o, ks[p], ks[p + 1], prep["dz"][p + 1])
                sm = orc.interface_smatrix(o, ks[p], ks[p + 1], prep["dz"][p + 1])
                b.append(dict(i11=i11, i12=i12, r=sm["r"], tp=sm["tp"]))
            c = []
            for _ in range(2):
                nxt = [orc.recurrence2_step(b[i], b[i + 1]) for i in range(0, len(b) - 1, 2)]
                if len(b) % 2:
                    nxt.append(b[-1])
                b = nxt
                c.append(max(orc.cond1(x["i11"]) for x in b))
            assert c[1] > c[0] * 1.5
            max_cond, levels = float(np.sqrt(c[0] * c[1])), 2
        out = orc.mixed_doubling(prep, e, max_cond)
        assert out["mixed_levels"] == levels, (max_cond, out["mixed_levels"])
        seen.add(out["mixed_levels"])
        for key in ("t", "rp", "r", "tp"):
            assert np.max(np.abs(out["S"][key] - ref[key])) < 1e-10 * max(1.0, np.max(np.abs(ref[key]))), key
    assert len(seen) == 3


def test_cond1_pins():
    """cond_1 of a diagonal matrix is max|d| / min|d|; of a unitary permutation, 1."""
    d = np.array([3.0, -0.5, 2j, 8.0])
    assert abs(orc.cond1(np.diag(d)) - 16.0) < 1e-12
    assert abs(orc.cond1(np.eye(5)[[3, 0, 4, 1, 2]]) - 1.0) < 1e-12


def test_slice_splitting():
    """One slice of thickness 2 dz is the same as two identical slices of dz."""
    j, inp = _c1(n_slices=12)
    thick = dict(inp)
    thin = dict(inp)
    thin["vq"] = np.repeat(inp["vq"], 2, axis=0)
    thin["dz"] = np.repeat(inp["dz"] / 2, 2)
    for e in (0.35, 1.7):
        a = orc.transmission(orc.prepare(thick), e)
        b = orc.transmission(orc.prepare(thin), e)
        assert np.max(np.abs(a["S"]["t"] - b["S"]["t"])) < 1e-12
        assert np.max(np.abs(a["S"]["r"] - b["S"]["r"])) < 1e-12


def test_first_born_limit():
    """r(lambda V)/lambda -> first-order Born amplitude (pins the channel coupling, index
    order of V(G_i - G_j) and the phase reference planes)."""
    _, inp = _c1()
    kin = orc.kinetic(inp["miller"], inp["bvec"], inp["kpar"])
    e = 0.6
    rb = orc.born_reflection(kin, inp["vq"], inp["q_of_ij"], inp["dz"], e)
    h = 5e-4
    f = []
    for lam in (h, 2 * h, 4 * h):
        prep = orc.prepare(_with_vq(inp, lam * inp["vq"]))
        f.append(orc.transmission(prep, e)["S"]["r"] / lam)
    extrap = (8 * f[0] - 6 * f[1] + f[2]) / 3.0
    assert np.max(np.abs(rb)) > 1e-2
    assert np.max(np.abs(extrap - rb)) < 1e-8 * max(1.0, np.max(np.abs(rb)))


def test_transverse_translation():
    j = msgen.config1()
    inp = msgen.junction_inputs(j, (0.0, 0.0))
    delta = np.array([0.7, -1.3])
    moved = msgen.Wells(j.wells.centres + np.r_[delta, 0.0], j.wells.depth, j.wells.sigma)
    inp2 = _with_vq(inp, msgen.vq_gaussian_wells(j.cell, inp["q_miller"], moved, j.dz))
    e = 2.4
    a = orc.transmission(orc.prepare(inp), e)
    b = orc.transmission(orc.prepare(inp2), e)
    g = inp["miller"] @ inp["bvec"]
    ph = np.exp(-1j * ((g[:, None, :] - g[None, :, :]) @ delta))
    assert abs(a["T"] - b["T"]) < 1e-12
    assert np.max(np.abs(b["S"]["r"] - ph * a["S"]["r"])) < 1e-12


def test_z_mirror():
    """V(z) -> V(L - z): r(mirror) = r'(original), t(mirror) = t'(original)."""
    _, inp = _c1()
    mir = _with_vq(inp, inp["vq"][::-1].copy())
    mir["dz"] = inp["dz"][::-1].copy()
    e = 1.9
    a = orc.transmission(orc.prepare(inp), e)
    b = orc.transmission(orc.prepare(mir), e)
    assert np.max(np.abs(b["S"]["r"] - a["S"]["rp"])) < 1e-12
    assert np.max(np.abs(b["S"]["t"] - a["S"]["tp"])) < 1e-12
    assert abs(a["T"] - b["T"]) < 1e-12


def test_dz_convergence_order_two():
    """Slice-averaged smooth wells: the error of T falls as dz^2."""
    ts = []
    for ns in (30, 60, 120, 240):
        _, inp = _c1(n_slices=ns)
        ts.append(orc.transmission(orc.prepare(inp), 0.55)["T"])
    d = np.abs(np.diff(ts))
    orders = np.log2(d[:-1] / d[1:])
    assert np.all(np.abs(orders - 2.0) < 0.2), orders


def test_lead_threshold_raises():
    _, inp = _c1()
    prep = orc.prepare(inp)
    with pytest.raises(orc.ThresholdError):
        orc.transmission(prep, float(prep["kin"][5]))


def test_singular_star_raises():
    n = 4
    e, z = np.eye(n, dtype=complex), np.zeros((n, n), dtype=complex)
    a = dict(t=e, rp=e.copy(), r=z, tp=e.copy())
    b = dict(t=e.copy(), rp=z.copy(), r=e.copy(), tp=e.copy())
    with pytest.raises(orc.SingularError):
        orc.star(a, b)


def test_kpar_average():
    """Eq. (T1_d): the mesh average; when T does not depend on k_y it reduces to the
    k_x average of Eq. (T2_d); per-channel transmission is sum T / sum N_open."""
    rng = np.random.default_rng(5)
    tx = rng.uniform(0, 3, size=(6, 4))              # T(m_x, E)
    nx = rng.integers(1, 5, size=(6, 4))
    t2 = np.repeat(tx, 3, axis=0)                    # the same for 3 values of k_y
    n2 = np.repeat(nx, 3, axis=0)
    tbar2, per2 = orc.kpar_average(t2, n2)
    tbar1, per1 = orc.kpar_average(tx, nx)
    assert np.allclose(tbar2, tx.mean(axis=0), rtol=1e-15) and np.allclose(tbar1, tbar2, rtol=1e-15)
    assert np.allclose(per1, tx.sum(0) / nx.sum(0), rtol=1e-15) and np.allclose(per1, per2, rtol=1e-15)
    tb, pc = orc.kpar_average(np.zeros((2, 3)), np.zeros((2, 3), dtype=int))
    assert np.all(tb == 0) and np.all(pc == 0)


# ---------------------------------------------------------------- dT/dV (first variation) --
def test_dT_dV_square_barrier_closed_form():
    """z-only barrier: d/dV0 of the textbook T(E; V0) (the closed form differentiated by
    central differences) equals the first-variation gradient summed over the barrier's
    slices at Q = 0."""
    j, inp = _c1(n_slices=12, slab=3.0)
    v0 = 0.5
    vz = np.zeros(12)
    vz[2:10] = v0
    inp = _with_vq(inp, _const_vq(inp, vz))
    prep = orc.prepare(inp)
    q0 = int(np.where((inp["q_miller"] == 0).all(axis=1))[0][0])
    for e in (0.45, 1.0, 3.5):
        g = orc.dT_dV(prep, e, inp["q_of_ij"], inp["vq"].shape[1])
        grad = float(2.0 * np.real(np.sum(g[2:10, q0])))
        h = 1e-6
        closed = lambda v: sum(_barrier_closed(e - kk, v, 2.0) for kk in prep["kin"] if kk < e)
        ref = (closed(v0 + h) - closed(v0 - h)) / (2 * h)
        assert abs(grad - ref) < 1e-8 * max(1.0, abs(ref)), (e, grad, ref)
        # a z-only potential keeps the channels decoupled (t diagonal), so a first-order
        # change of T comes only from the diagonal of dH, which is carried by Q = 0
        others = np.delete(g, q0, axis=1)
        assert np.max(np.abs(others)) < 1e-12 * max(1.0, np.max(np.abs(g[:, q0])))


def test_dT_dV_matches_central_differences():
    """Coupled channels (config1 wells, 13 plane waves, k_par off symmetry, 5 open
    channels): dT/dRe V^p(Q) and dT/dIm V^p(Q) with V(-Q) = conj V(Q) kept, against
    central differences of T (h = 1e-6) on 8 seeded coefficients."""
    j, inp = _c1(kpar=(0.07, -0.11), n_g=13, n_slices=6)
    prep = orc.prepare(inp)
    e = 2.3
    g = orc.dT_dV(prep, e, inp["q_of_ij"], inp["vq"].shape[1])
    qi, qj, dre, dim = orc.dT_dV_real(g, inp["q_miller"])
    rng = np.random.default_rng(20)
    h = 1e-6
    checked = 0
    for _ in range(8):
        p, c = int(rng.integers(0, 6)), int(rng.integers(0, len(qi)))
        for part in ("re", "im"):
            if part == "im" and qi[c] == qj[c]:
                continue
            vals = []
            for sgn in (1, -1):
                vq = inp["vq"].copy()
                d = h * (1 if part == "re" else 1j) * sgn
                vq[p, qi[c]] += d
                if qj[c] != qi[c]:
                    vq[p, qj[c]] += np.conj(d)
                vals.append(orc.transmission(orc.prepare(_with_vq(inp, vq)), e)["T"])
            fd = (vals[0] - vals[1]) / (2 * h)
            an = dre[p, c] if part == "re" else dim[p, c]
            assert abs(fd - an) < 2e-8 + 1e-5 * abs(an), (p, c, part, fd, an)
            checked += 1
    assert checked >= 12


def test_dT_dV_born_limit():
    """Weak potential (lambda V, lambda -> 0): t = diag(e^{ikL}) + O(lambda), so to first
    order dT is the diagonal Born transmission change, whose real part vanishes (current
    conservation); the gradient must be O(lambda) while T - N_open = O(lambda^2)."""
    j, inp = _c1(n_slices=8)
    e = 1.7
    grads = []
    for lam in (1e-3, 2e-3):
        ii = _with_vq(inp, inp["vq"] * lam)
        prep = orc.prepare(ii)
        g = orc.dT_dV(prep, e, ii["q_of_ij"], ii["vq"].shape[1])
        grads.append(np.max(np.abs(np.real(g))))
    assert grads[1] / grads[0] == pytest.approx(2.0, rel=1e-2)
