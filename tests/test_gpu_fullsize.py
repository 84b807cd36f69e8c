"""Full-size checks at N_G = 1200, 400 slices (the benchmark workload), in the launch
configuration bench.py times: one (gap, k_par) with its 32 energies per batch.

The oracle takes about 13 minutes per point here, so its values at sample points
(gaps 5.0, 6.3 and 7.5 bohr, k_par off the symmetric centre) are stored
(tests/golden/make_golden.py, which calls only the oracle); every other point is
checked through properties that hold at any size: current conservation
R + T = N_open and the agreement of the FP32-MFMA form with the FP64 form."""
import numpy as np
import pytest

import msgen
from gpu_common import golden_points

pytestmark = pytest.mark.gpu

_CACHE = {}


@pytest.fixture(scope="module")
def ms():
    import paper_1504_01462_amd as m
    return m


@pytest.fixture(scope="module")
def full(ms):
    pts = golden_points("config3")
    assert pts, "tests/golden/oracle_points.json has no config3 points"
    p0 = pts[0]
    j = msgen.config3(p0["meta"]["gap"], p0["meta"]["registry"])
    inp = msgen.junction_inputs(j, j.kpars[p0["k_index"]])
    ctx = ms.Context(0)
    s = ms.prepare_from_inputs(ctx, inp)
    T, R, no, st = (x.cpu().numpy() for x in ms.ms_transmission_batch(ctx, s, j.energies, "fp64"))
    ctx.sync()
    yield dict(ctx=ctx, s=s, j=j, pts=pts, T=T, R=R, no=no, st=st)
    ctx.close()


def test_config3_fp64_against_oracle(full):
    T, R, no, st, j = full["T"], full["R"], full["no"], full["st"], full["j"]
    assert np.all(st == 0)
    assert np.max(np.abs(T + R - no)) < 1e-9
    p0 = full["pts"][0]
    same = [p for p in full["pts"] if p["junction"] == p0["junction"] and p["k_index"] == p0["k_index"]]
    for p in same:
        i = p["e_index"]
        assert abs(j.energies[i] - p["energy"]) < 1e-15
        assert int(no[i]) == p["n_open"]
        assert abs(T[i] - p["T"]) < 1e-10, (p["energy"], T[i], p["T"])


def test_config3_other_gaps_and_kpar_against_oracle(ms, full):
    """The stored oracle points of the other (gap, k_par) groups of the benchmark workload:
    each group's slices prepared at its own k_par, folded at the stored energies."""
    ctx = full["ctx"]
    p0 = full["pts"][0]
    groups = {}
    for p in full["pts"]:
        if (p["junction"], p["k_index"]) != (p0["junction"], p0["k_index"]):
            groups.setdefault((p["junction"], p["k_index"]), []).append(p)
    assert len(groups) >= 3, "stored points cover gaps 5.0 and 7.5 and a second k_par at 6.3"
    for (name, ik), pts in groups.items():
        j = msgen.config3(pts[0]["meta"]["gap"], pts[0]["meta"]["registry"])
        assert j.name == name
        s = ms.prepare_from_inputs(ctx, msgen.junction_inputs(j, j.kpars[ik]))
        T, R, no, st = (x.cpu().numpy() for x in ms.ms_transmission_batch(ctx, s, [p["energy"] for p in pts]))
        ctx.sync()
        assert np.all(st == 0)
        for i, p in enumerate(pts):
            assert int(no[i]) == p["n_open"], (name, ik, p["energy"])
            assert abs(T[i] - p["T"]) < 1e-10, (name, ik, p["energy"], T[i], p["T"])
            assert abs(R[i] - p["R"]) < 1e-10, (name, ik, p["energy"], R[i], p["R"])
        del s


FP32_TARGET = 1e-6


def _config3_fp32(ms, full):
    ctx, s, j = full["ctx"], full["s"], full["j"]
    if "T32" not in full:
        T32, R32, no32, st32 = (x.cpu().numpy() for x in ms.ms_transmission_batch(ctx, s, j.energies, "fp32"))
        ctx.sync()
        full.update(T32=T32, R32=R32, no32=no32, st32=st32)
    return full["T32"], full["R32"], full["no32"], full["st32"]


def test_config3_fp32_form_meets_target(ms, full):
    """The FP32-MFMA form on the 32 points of a config3 k_par: every point valid, |dT| <= 1e-6
    against FP64 (the form's target), current conserved to the same order."""
    T32, R32, no32, st32 = _config3_fp32(ms, full)
    assert np.all(st32 == 0)
    dT = np.max(np.abs(T32 - full["T"]))
    print(f"\nconfig3 FP32-MFMA form: max |dT| vs FP64 over {T32.size} points = {dT:.3e}")
    assert dT <= FP32_TARGET
    assert np.max(np.abs(T32 + R32 - no32)) < 1e-6


def test_config3_slices_sampled_against_oracle(ms, full):
    """a1-a3 at full size on sampled slices: eigenvalues against the oracle's dense
    eigensolver, eigen-residuals, and the stored overlaps against U^p^dagger U^(p+1)
    formed from the returned eigenvectors."""
    import oracle as orc
    import torch
    j, ctx = full["j"], full["ctx"]
    p0 = full["pts"][0]
    inp = msgen.junction_inputs(j, j.kpars[p0["k_index"]])
    s = ms.prepare_from_inputs(ctx, inp, with_evec=True)
    ctx.sync()
    kin = orc.kinetic(inp["miller"], inp["bvec"], inp["kpar"])
    eps = s.eps.cpu().numpy()
    for p in (0, 137, 398):   # slice index p is the paper's slice p+1
        h = orc.slice_hamiltonians(kin, inp["vq"][p:p + 1], inp["q_of_ij"])[0]
        lam_ref, _ = orc.slice_eigen(h[None])
        lam_ref = lam_ref[0]
        scale = np.max(np.abs(lam_ref))
        assert np.max(np.abs(eps[p + 1] - lam_ref)) < 1e-11 * scale, p
        u = s.evec[p].cpu().numpy()
        res = np.linalg.norm(h @ u - u * eps[p + 1][None, :]) / np.linalg.norm(h)
        assert res < 1e-12, (p, res)
        assert np.linalg.norm(u.conj().T @ u - np.eye(u.shape[0])) < 1e-11
        un = s.evec[p + 1].cpu().numpy()
        o = s.ovl[p + 1].cpu().numpy()
        assert np.max(np.abs(o - u.conj().T @ un)) < 1e-12, p
    del s
    torch.cuda.empty_cache()


def test_uneven_instances_config4_sample(ms, full):
    """Instances of the uneven workload at their real sizes (N_G 200 / 450 / 800 with 150-390
    slices, one energy each), folded in one captured graph: every instance equals its own
    ms_transmission_batch, conserves current, the FP32 form stays near it, and the cheapest
    instance matches the oracle."""
    import oracle as orc
    ctx = full["ctx"]
    inst = msgen.config4_instances()
    pick = [3, 7, 10, 6, 12, 13]                    # n_g 200, 450, 200, 800, 200, 450
    inps, sets, es = [], [], []
    for i in pick:
        j = inst[i]["junction"]
        inp = msgen.junction_inputs(j, j.kpars[inst[i]["k_index"]])
        inps.append(inp)
        sets.append(ms.prepare_from_inputs(ctx, inp))
        es.append([inst[i]["energy"]])
    T, R, no, st = (x.cpu().numpy() for x in ms.ms_transmission_uneven(ctx, sets, es, "fp64", graph=True))
    T32 = ms.ms_transmission_uneven(ctx, sets, es, "fp32", graph=True)[0].cpu().numpy()
    ctx.sync()
    assert np.all(st == 0)
    assert np.max(np.abs(T + R - no)) < 1e-8
    for k, s in enumerate(sets):
        t1 = ms.ms_transmission_batch(ctx, s, es[k], "fp64")[0].cpu().numpy()
        ctx.sync()
        assert abs(T[k] - t1[0]) < 1e-11, k
    assert np.max(np.abs(T32 - T)) <= FP32_TARGET
    k = pick.index(12)                              # n_g = 200, 248 slices
    ref = orc.transmission(orc.prepare(inps[k]), es[k][0])
    assert abs(T[k] - ref["T"]) < 1e-10 and int(no[k]) == ref["n_open"]


EPS_T = 1e-13   # bound on the change of T when one slice's eigenproblem is solved again (measured: 3.4e-14)


def test_dT_dV_full_size_central_differences(ms, full):
    """The adjoint workload at full size (config3 gap 6.3, k_par = 0, N_G = 1200, 400 slices,
    checkpoints every 20 planes): 20 seeded real parameters (Re and Im parts of V^p(Q) with
    V(-Q) = conj V(Q) kept; 19 with Q != 0) against central differences of the GPU's own T.

    Each difference re-solves only the perturbed slice (a one-slice ms_slices_prepare with its
    eigenvectors) and replaces its eigenvalues and the two overlaps it enters, formed with the
    library's GEMM from the neighbours' eigenvectors.  A re-solved slice changes T by up to
    EPS_T (the eigensolver's convergence tolerance, about 3e-14 relative, carried through 401
    interfaces), so a central difference at step h carries a rounding floor of EPS_T / h:
    1e-7 absolute at the specified h = 1e-6, which is above 1e-6 of the smaller derivatives.
    Each coefficient is therefore checked twice: (a) at h = 1e-6 within 1e-6 relative plus
    that floor; (b) by Richardson extrapolation of the differences at h = 1e-4 and 2e-4
    (truncation O(h^4), floor 1.5 EPS_T / 1e-4 = 1.5e-9) within 1e-6 relative plus its floor.
    The six perturbed sets of a coefficient are folded in one ms_transmission_multi call."""
    import torch
    import oracle as orc
    ctx = full["ctx"]
    j = msgen.config5()
    inp = msgen.junction_inputs(j, j.kpars[0])
    s = ms.prepare_from_inputs(ctx, inp, with_evec=True)
    n, ns = s.n_g, s.n_slices
    q = torch.as_tensor(np.ascontiguousarray(inp["q_of_ij"], dtype=np.int32), device="cuda")
    e = float(j.energies[8])
    g, tr, no = ms.ms_dT_dV(ctx, s, e, q, inp["vq"].shape[1], 20)
    ctx.sync()
    g = g.cpu().numpy()
    qi, qj, dre, dim = orc.dT_dV_real(g, inp["q_miller"])
    eye = torch.eye(n, dtype=torch.complex128, device="cuda")
    dz = inp["dz"]
    steps = [1e-6, 1e-4, 2e-4]
    # one slice set per (step, sign): the base set itself and five copies of its slice data
    sets = [s] + [ms.Slices(n, ns, s.dz, s.eps.clone(), s.ovl.clone()) for _ in range(2 * len(steps) - 1)]

    def set_slice(dst, p, vrow):
        """dst's slice p (vq row p) re-solved from the potential row vrow."""
        one = ms.prepare_from_inputs(ctx, dict(inp, vq=vrow[None, :].copy(), dz=dz[p:p + 1].copy()), with_evec=True)
        u = one.evec[0]
        left = s.evec[p - 1] if p > 0 else eye
        right = s.evec[p + 1] if p < ns - 1 else eye
        dst.eps[p + 1].copy_(one.eps[1])
        ms.ms_debug_gemm(ctx, left.contiguous(), u.contiguous(), dst.ovl[p], op_a=2, op_b=0)
        ms.ms_debug_gemm(ctx, u.contiguous(), right.contiguous(), dst.ovl[p + 1], op_a=2, op_b=0)

    saved = {}

    def restore(dst, p):
        e0, o0, o1 = saved[p]
        dst.eps[p + 1].copy_(e0)
        dst.ovl[p].copy_(o0)
        dst.ovl[p + 1].copy_(o1)

    T0 = ms.ms_transmission_batch(ctx, s, [e])[0].cpu().numpy()[0]
    ctx.sync()
    assert abs(tr.cpu().numpy()[0] - T0) < 1e-9
    rng = np.random.default_rng(5)
    qm = inp["q_miller"][qi]
    low = np.where((np.abs(qm).sum(axis=1) > 0) & (np.abs(qm[:, 0]) <= 2) & (np.abs(qm[:, 1]) <= 8))[0]
    c0 = int(np.where(np.abs(qm).sum(axis=1) == 0)[0][0])
    picks = [(int(rng.integers(0, ns)), c0, "re")]
    picks += [(int(rng.integers(0, ns)), int(rng.choice(low)), "re" if k % 2 else "im") for k in range(19)]
    print(f"\nfull-size dT/dV: T = {T0:.12f}, EPS_T = {EPS_T:.0e}")
    noise = []
    for p, c, part in picks:
        saved[p] = (s.eps[p + 1].clone(), s.ovl[p].clone(), s.ovl[p + 1].clone())
        k = 0
        for h in steps:
            for sgn in (1, -1):
                d = sgn * h * (1.0 if part == "re" else 1j)
                v = inp["vq"][p].copy()
                v[qi[c]] += d
                if qj[c] != qi[c]:
                    v[qj[c]] += np.conj(d)
                set_slice(sets[k], p, v)
                k += 1
        Tv = ms.ms_transmission_multi(ctx, sets, np.full((len(sets), 1), e))[0].cpu().numpy()[:, 0]
        ctx.sync()
        for dst in sets:
            restore(dst, p)
        fd = [(Tv[2 * i] - Tv[2 * i + 1]) / (2 * h) for i, h in enumerate(steps)]
        rich = (4.0 * fd[1] - fd[2]) / 3.0
        an = dre[p, c] if part == "re" else dim[p, c]
        noise.append(steps[0] * abs(fd[0] - rich))
        print(f"  p={p:3d} Q={tuple(int(x) for x in inp['q_miller'][qi[c]])} {part}: adjoint={an:+.10e} "
              f"fd(1e-6)={fd[0]:+.10e} richardson(1e-4,2e-4)={rich:+.10e} rel={abs(rich - an) / abs(an):.1e}")
        assert abs(rich - an) <= 1e-6 * abs(an) + 1.5 * EPS_T / steps[1], (p, c, part, rich, an)
        assert abs(fd[0] - an) <= 1e-6 * abs(an) + EPS_T / steps[0], (p, c, part, fd[0], an)
    print(f"  T noise implied by the h = 1e-6 differences: up to {max(noise):.1e} (EPS_T = {EPS_T:.0e})")
