"""Full-size checks at N_G = 1200, 400 slices (the benchmark workload), in the launch
configuration bench.py times: one (gap, k_par) with its 32 energies per batch.

The oracle takes about 13 minutes per point here, so its values at two sample
points are stored (tests/golden/make_golden.py); every other point is checked
through properties that hold at any size: current conservation R + T = N_open
and the agreement of the FP32-MFMA form with the FP64 form."""
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
    for p in full["pts"]:
        i = p["e_index"]
        assert abs(j.energies[i] - p["energy"]) < 1e-15
        assert int(no[i]) == p["n_open"]
        assert abs(T[i] - p["T"]) < 1e-10, (p["energy"], T[i], p["T"])


def test_config3_fp32_form(ms, full):
    """FP32-MFMA interface GEMMs (FP32 accumulation), everything else FP64.  Measured
    max |dT| over the 32 points is ~1.5e-4 (T up to 13): FP32 accumulation leaves ~1e-6
    relative error per GEMM entry, compounded over 401 interfaces.  The 1e-6 target is
    NOT met by this form; the bound below guards the achieved accuracy."""
    ctx, s, j = full["ctx"], full["s"], full["j"]
    T32, R32, no32, st32 = (x.cpu().numpy() for x in ms.ms_transmission_batch(ctx, s, j.energies, "fp32"))
    ctx.sync()
    assert np.all(st32 == 0)
    dT = np.max(np.abs(T32 - full["T"]))
    print(f"\nconfig3 FP32-MFMA form: max |dT| vs FP64 over {T32.size} points = {dT:.3e}")
    assert dT < 1e-3
    assert np.max(np.abs(T32 + R32 - no32)) < 1e-3


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
    assert np.max(np.abs(T32 - T)) < 1e-3
    k = pick.index(12)                              # n_g = 200, 248 slices
    ref = orc.transmission(orc.prepare(inps[k]), es[k][0])
    assert abs(T[k] - ref["T"]) < 1e-10 and int(no[k]) == ref["n_open"]


def test_dT_dV_full_size_central_differences(ms, full):
    """The adjoint workload's geometry at full size (config3 gap 6.3, k_par = 0, N_G = 1200,
    400 slices, checkpoints every 20 planes): three slice coefficients' derivatives against
    central differences of the batch path's T (h = 1e-5), and T itself."""
    import torch
    ctx = full["ctx"]
    j = msgen.config5()
    inp = msgen.junction_inputs(j, j.kpars[0])
    s = ms.prepare_from_inputs(ctx, inp, with_evec=True)
    q = torch.as_tensor(np.ascontiguousarray(inp["q_of_ij"], dtype=np.int32), device="cuda")
    e = float(j.energies[8])
    g, tr, no = ms.ms_dT_dV(ctx, s, e, q, inp["vq"].shape[1], 20)
    T0 = ms.ms_transmission_batch(ctx, s, [e])[0].cpu().numpy()[0]
    ctx.sync()
    g = g.cpu().numpy()
    assert abs(tr.cpu().numpy()[0] - T0) < 1e-9
    q0 = int(np.where((inp["q_miller"] == 0).all(axis=1))[0][0])
    h = 1e-5
    for p in (37, 200, 371):
        vals = []
        for sgn in (1, -1):
            vq = inp["vq"].copy()
            vq[p, q0] += sgn * h
            sp = ms.prepare_from_inputs(ctx, dict(inp, vq=vq))
            vals.append(ms.ms_transmission_batch(ctx, sp, [e])[0].cpu().numpy()[0])
            ctx.sync()
        fd = (vals[0] - vals[1]) / (2 * h)
        an = 2.0 * np.real(g[p, q0])
        assert abs(fd - an) < 1e-6 + 1e-4 * abs(an), (p, fd, an)
