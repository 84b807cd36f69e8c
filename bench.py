#!/usr/bin/env python3
"""Throughput benchmark of the plane-wave multiple-scattering transport path on one MI355X.

Workload (default): the side-contact overlap junction -- rectangular 4.65 x 40
bohr cell, two graphene-like Gaussian-well sheets overlapping 15 bohr along
the transport direction, N_G = 1200 plane waves, 400 slices of 0.05 bohr,
free-electron leads, 32 energies at each of 8 k_par for 3 vacuum gaps (768
points).  One step = the eight k_par of one gap (256 points): slice Hamiltonians,
eigenpairs and overlaps (E-independent) of each, the fused slice-S /
star-product fold of all 256 points in one batch, T and R per point, and the
k_par average.  Successive steps walk through the 3 gaps (`--kpar-per-step 4`:
the 6 (gap, k_par quartet) groups of 128 points).
Inputs are seeded and synthetic, generated once per distinct (gap, k_par) in
worker processes before the GPU is touched, and resident in HBM before timing.

Timing: min(W, 1) untimed warmup steps, then the FP64 form over K steps, or
over as many as the wall budget `--time-budget` holds (at least one; the line
reports the steps actually timed in `steps`).  Then the FP32-MFMA form over the
first timed steps (`--fp32-steps`), with its largest |dT| against the FP64
results of the same points; its number is the headline only when that stays
below 1e-6.  Optional legs (each skipped when the process's wall budget
`--wall-budget` would not hold it): the paper's mixed transfer/scattering
doubling (`--mixed`), the gradient dT/dV (`--adjoint N`), uneven instances
(`--uneven N`).  `--all-points` runs every group once in both forms (the
|dT| chain over the whole workload) with no time budget.

    python bench.py [--steps K] [--warmup W] [--config config3|config2|config1]
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "(E,k∥) transmission points/s at N_G=1200; FP32-MFMA vs FP64 at |ΔT|<1e-6"
PEAK = {"fp64": 78.6, "fp32": 157.3}      # dense MFMA TFLOP/s
HBM_PEAK = 8000.0                          # GB/s
T_START = time.perf_counter()


def elapsed():
    return time.perf_counter() - T_START


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="config3", choices=["config1", "config2", "config3"])
    ap.add_argument("--time-budget", type=float, default=150.0,
                    help="seconds of the timed FP64 leg: fewer than --steps are timed when they would not fit")
    ap.add_argument("--wall-budget", type=float, default=450.0,
                    help="seconds from start after which optional legs are skipped")
    ap.add_argument("--fp32-steps", type=int, default=1,
                    help="timed steps of the FP32-MFMA form (the first timed FP64 steps' points); 0 skips it")
    ap.add_argument("--all-points", action="store_true",
                    help="every (gap, k_par pair) group once, in both forms, without time budget")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kpar-per-step", type=int, default=8,
                    help="k_par values of one junction folded together in one batch per step")
    ap.add_argument("--mixed", action="store_true",
                    help="also time the paper's mixed-recurrence doubling (ms_mixed_doubling) at one point")
    ap.add_argument("--roofline-kernel", default="iface_gemm",
                    help="profiler category reported in 'roofline'")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default GEMM tile rule instead of timing both edges first")
    ap.add_argument("--uneven", type=int, default=0,
                    help="instances of the uneven workload (N_G 200-1200, 100-400 slices) to fold; 0 skips it")
    ap.add_argument("--adjoint", type=int, default=0,
                    help="energies of the adjoint workload (dT/dV at N_G = 1200) to time; 0 skips it")
    ap.add_argument("--overlap", action="store_true",
                    help="prepare the next step's slices on a second stream while the current step folds")
    ap.add_argument("--uneven-only", action="store_true",
                    help="measure only the uneven workload (--uneven instances) and print its JSON line")
    ap.add_argument("--no-event-profile", action="store_true",
                    help="record no HIP events around launches (no roofline figure; for external profilers)")
    ap.add_argument("--workers", type=int, default=16, help="processes generating the seeded inputs")
    ap.add_argument("--probe", choices=["iface64", "iface32", "lu", "eigh", "copy"],
                    help="run one kernel at the benchmark's launch shape (for profiler counters) and exit: "
                         "the interface product with the fold's fused epilogue (FP64 or FP32 MFMA, n_g 1200, 32 "
                         "energies), the LU solve of "
                         "32 augmented systems, 8 slice eigenproblems, or a 1 GiB device copy (calibration)")
    ap.add_argument("--probe-launches", type=int, default=5)
    ap.add_argument("--electrode-only", type=int, default=0, metavar="N_G",
                    help="time the periodic-electrode path at this basis size and exit: the complex bands of "
                         "one config-3 sheet cell (one z-period, 40 slices) and the transmission from the bottom "
                         "sheet's electrode through the config-3 junction (400 slices) into the top sheet's")
    ap.add_argument("--electrode-bands-only", action="store_true",
                    help="with --electrode-only: time the complex bands only")
    ap.add_argument("--electrode-energies", type=int, default=1,
                    help="energies (spread over the config-3 window) for --electrode-only")
    return ap.parse_args()


def probe(kind, launches):
    """One kernel kind at the benchmark's launch shape, timed with stream events; one JSON line."""
    import torch
    import paper_1504_01462_amd as ms
    ctx = ms.Context(0)
    dev = ctx.device
    g = torch.Generator(device=dev).manual_seed(1)
    n, batch = 1200, 32

    def crand(*shape, dtype=torch.complex128):
        return torch.randn(*shape, generator=g, device=dev, dtype=dtype)

    if kind.startswith("iface"):   # as the fold launches it: the fused epilogue reads Y and P
        dt = torch.complex128 if kind == "iface64" else torch.complex64
        a, o = crand(batch, n, n, dtype=dt), crand(n, n) / n ** 0.5
        kp, kq = crand(batch, n), crand(batch, n) + 1.5
        y, pq = crand(batch, n, n), crand(batch, n)
        run = lambda: ms.ms_debug_iface_fused(ctx, a, o, kp, kq, y, pq, "fp64" if kind == "iface64" else "fp32")
        work = {"flop": 8.0 * n * 2 * n * n * batch,
                "bytes": batch * n * n * a.element_size() + 16.0 * n * n + 2 * 16.0 * batch * n + 16.0 * batch * 2 * n * n
                         + 16.0 * batch * n * n}
    elif kind == "lu":
        nrhs = n + 13
        src = crand(batch, n, n + nrhs)
        src[:, :, :n] += 4.0 * n ** 0.5 * torch.eye(n, device=dev, dtype=torch.complex128)
        aug = src.clone()
        run = lambda: (aug.copy_(src), ms.ms_debug_lu_solve(ctx, aug, n))
        work = {"flop": 8.0 * batch * (n ** 3 / 3.0 + n * n * nrhs), "bytes": 16.0 * batch * n * (n + nrhs)}
    elif kind == "eigh":
        nb = 8
        h = crand(nb, n, n)
        h = (h + h.conj().transpose(1, 2)).contiguous()
        shift = torch.full((nb,), 6.0 * n ** 0.5, dtype=torch.float64, device=dev)   # > the spectral radius
        run = lambda: ms.ms_debug_eigh(ctx, h, shift)
        work = {"flop": 8.0 * nb * 3.0 * n ** 3, "bytes": 16.0 * nb * 2 * n * n}
    else:
        x = torch.empty(1 << 26, dtype=torch.complex128, device=dev)
        y = torch.empty_like(x)
        run = lambda: y.copy_(x)
        work = {"flop": 0.0, "bytes": 2.0 * x.numel() * 16}
    run()
    ctx.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(launches):
        run()
    e1.record()
    ctx.sync()
    torch.cuda.synchronize()
    ms_per = e0.elapsed_time(e1) / launches
    print(json.dumps({"probe": kind, "launches": launches, "ms_per_launch": ms_per,
                      "tflops": work["flop"] / ms_per / 1e9 if work["flop"] else None,
                      "gbps": work["bytes"] / ms_per / 1e6, **work}), flush=True)
    ctx.close()


def electrode_measure(n_g, n_e, bands_only=False):
    """Periodic electrodes (NEXT-4) at config-3 shape: per energy, the complex bands of the bottom
    sheet's cell (one QZ of the 2 N_G pencil) and the electrode transmission bottom sheet ->
    junction -> top sheet (two cells' bands, the region's S, the matching); one JSON line."""
    import msgen
    import torch
    import paper_1504_01462_amd as ms
    ctx = ms.Context(0)
    jl = msgen.config3_electrode("bottom", n_g=n_g, n_slices=40)
    jr = msgen.config3_electrode("top", n_g=n_g, n_slices=40)
    jg = msgen.config3(6.3, "AA", n_g=n_g)
    kp = jg.kpars[3]
    sl, sr, sg = (ms.prepare_from_inputs(ctx, msgen.junction_inputs(j, kp), with_evec=True) for j in (jl, jr, jg))
    ctx.sync()
    energies = np.linspace(0.3, 0.9, n_e) if n_e > 1 else np.array([0.5])
    rows = []
    # one energy at a time: all of them for the bands alone, else the first (compared with the batch)
    for e in (energies if bands_only else energies[:1]):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        al, be, _ = ms.ms_complex_bands(ctx, sl, float(e))
        ctx.sync()
        t1 = time.perf_counter()
        lam = (al / be).cpu().numpy()
        rows.append(dict(energy=float(e), bands_s=round(t1 - t0, 3),
                         propagating=int(np.sum(np.abs(np.abs(lam) - 1.0) < 1e-8))))
        if not bands_only:
            T, R, no = ms.ms_electrode_transmission(ctx, sl, sg, sr, float(e))
            ctx.sync()
            rows[-1].update(transmission_s=round(time.perf_counter() - t1, 3), T=float(T[0]), R=float(R[0]),
                            n_in=int(no[0]))
        print(f"[bench] electrode E={e:.3f}: {rows[-1]}", file=sys.stderr, flush=True)
    batch = None
    if n_e > 1 and not bands_only:   # all energies in one call: both cells' pencils in one QZ launch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T, R, no = ms.ms_electrode_transmission_batch(ctx, sl, sg, sr, energies)
        ctx.sync()
        tb = time.perf_counter() - t0
        Th = T.cpu().numpy()
        batch = dict(energies=int(n_e), seconds=round(tb, 3), seconds_per_energy=round(tb / n_e, 3),
                     single_call_seconds=rows[0]["transmission_s"], T=[float(x) for x in Th],
                     n_in=[int(x) for x in no.cpu().numpy()],
                     abs_T_minus_single_call_first_energy=float(abs(Th[0] - rows[0]["T"])))
        print(f"[bench] electrode batch of {n_e}: {tb:.2f} s", file=sys.stderr, flush=True)
    ctx.close()
    return dict(n_g=n_g, pencil=2 * n_g, cell_slices=40, region_slices=int(jg.dz.size), k_par=[float(x) for x in kp],
                points=rows, batch=batch,
                note="one workgroup per pencil (complex QZ); transmission = both cells' bands + the region's "
                     "S-matrix + the matching solve; batch = all energies in one call")


def workload(name):
    """(groups of (key, [k_par indices]) in step order, junction factory, description)."""
    import msgen
    if name == "config3":
        combos = [(gap, ik) for gap in (6.3, 5.0, 7.5) for ik in range(8)]
        make = lambda gap: msgen.config3(gap, "AA")
        desc = ("side-contact overlap junction: 4.65x40 bohr cell, two Gaussian-well sheets overlapping 15 bohr, "
                "N_G=1200, 400 slices x 0.05 bohr, 32 energies per k_par, 8 k_par x 3 gaps")
    elif name == "config2":
        combos = [(reg, ik) for reg in ("AA", "AB") for ik in range(16)]
        make = lambda reg: msgen.config2(reg)
        desc = "bilayer-gap junction: 2x2 hexagonal supercell, N_G=300, 160 slices x 0.1 bohr, 64 energies per k_par"
    else:
        combos = [(None, 0)]
        make = lambda _: msgen.config1()
        desc = "square cell, 4 wells, N_G=37, 24 slices x 0.25 bohr, 8 energies at k_par=0"
    return combos, make, desc


def step_groups(combos, kps):
    groups = []
    for key, ik in combos:
        if groups and groups[-1][0] == key and len(groups[-1][1]) < kps:
            groups[-1][1].append(ik)
        else:
            groups.append((key, [ik]))
    return groups


def host_inputs_of(task):
    """Seeded inputs of one (config, key, k_par index) as host arrays (no GPU)."""
    name, key, ik = task
    _, make, _ = workload(name)
    import msgen
    j = make(key)
    inp = msgen.junction_inputs(j, j.kpars[ik])
    return dict(miller=np.ascontiguousarray(inp["miller"], dtype=np.int32),
                q=np.ascontiguousarray(inp["q_of_ij"], dtype=np.int32), vq=np.ascontiguousarray(inp["vq"]),
                dz=np.ascontiguousarray(inp["dz"]), bvec=np.asarray(inp["bvec"]).reshape(4),
                kpar=np.asarray(inp["kpar"]))


def adjoint_energy_indices(n_total, n_e):
    """n_e distinct energy indices spread evenly over [0, n_total) (all of them when n_e >= n_total)."""
    n_e = max(1, min(n_e, n_total))
    if n_e == 1:
        return np.array([n_total // 2])
    return np.round(np.linspace(0, n_total - 1, n_e)).astype(int)


def cpu_baseline(name, budget_s):
    """The oracle, untuned, on a bounded sample of one point of the workload: consecutive slice
    eigenproblems (about a third of the budget) and the interface S-matrices + star products of
    the chain they form (the rest), scaled to one point."""
    import msgen
    import oracle as orc
    blas_threads = None
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        pass
    combos, make, _ = workload(name)
    j = make(combos[0][0])
    inp = msgen.junction_inputs(j, j.kpars[combos[0][1]])
    kin = orc.kinetic(inp["miller"], inp["bvec"], inp["kpar"])
    e = float(j.energies[len(j.energies) // 2])
    ns = j.n_slices
    t0 = time.perf_counter()
    n_eig = 0
    us = []
    while n_eig < ns and (n_eig < 2 or time.perf_counter() - t0 < 0.33 * budget_s):
        h = orc.slice_hamiltonians(kin, inp["vq"][n_eig:n_eig + 1], inp["q_of_ij"])
        eps, u = orc.slice_eigen(h)
        us.append((eps[0], u[0]))
        n_eig += 1
    t_eig = (time.perf_counter() - t0) / n_eig
    t1 = time.perf_counter()
    acc = orc.identity_smatrix(len(kin))
    n_if = 0
    while n_if < len(us) - 1 and (n_if == 0 or time.perf_counter() - t1 < 0.67 * budget_s):
        o = orc.overlap(us[n_if][1], us[n_if + 1][1])
        s = orc.interface_smatrix(o, orc.wavevectors(e, us[n_if][0]), orc.wavevectors(e, us[n_if + 1][0]),
                                  float(inp["dz"][n_if]))
        acc = orc.star(acc, s)
        n_if += 1
    t_if = (time.perf_counter() - t1) / max(1, n_if)
    # one point = its share of the E-independent eigenproblems + (n_slices + 1) interfaces
    t_point = t_eig * ns / len(j.energies) + t_if * (ns + 1)
    try:
        affinity = len(os.sched_getaffinity(0))
    except Exception:
        affinity = None
    return {"value": 1.0 / t_point, "unit": "points/s", "cores": int(blas_threads or affinity or os.cpu_count() or 1),
            "kind": "oracle", "blas_threads": blas_threads, "host_cpus": os.cpu_count(), "affinity_cpus": affinity,
            "sample": (f"{name} first (gap/registry, k_par), E={e:.4f} Ry: {n_eig} consecutive slice eigenproblems "
                       f"({t_eig:.2f} s each) and the {n_if} interface S-matrices + star products between them "
                       f"({t_if:.2f} s each), scaled to one point = eigen share over {len(j.energies)} energies + "
                       f"{ns + 1} interfaces (extrapolated from the sample, not a full point)")}


def measured_traffic(cat, flops_per_launch, form, tile):
    """HBM bytes per launch of the roofline kernel from the committed rocprofv3 counter
    summary of that form, or None when it covers another kernel, tile shape or launch shape,
    or when the kernel source has changed since the counters were taken."""
    name = {"fp64": f"{cat}_config3_counters.txt", "fp32": f"{cat}32_config3_counters.txt"}.get(form)
    path = os.path.join(ROOT, "profiles", name) if name else ""
    if not path or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        src = open(os.path.join(ROOT, kv["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != kv["source_sha256"]:
            return None
        n = 1200
        if abs(flops_per_launch - 8.0 * 2 * n * n * n * int(kv["batch"])) > 1.0:
            return None
        if int(kv.get("tile", "128")) != tile or kv.get("form", "fp64") != form:
            return None
        return float(kv["traffic_bytes"])
    except (KeyError, ValueError, OSError):
        return None


def mixed_doubling_measure(ms, ctx, st, buf, results, log):
    """The paper's doubling with the mixed recurrence (App. A, Eq. recurrence2) and the switch
    to star products, at one (E, k_par) point of the same workload: time per point, the
    number of mixed levels, and its T against the fused fold's T for the same point."""
    import torch
    j = st["j"]
    kk = st["ks"][0]
    ie = len(j.energies) // 2
    e = float(j.energies[ie])
    ms.ms_slices_prepare(ctx, kk["miller"], kk["bvec"], kk["kpar"], kk["q"], kk["vq"], kk["dz"], out=buf)
    eps_l, eps_r = buf.eps[0].contiguous(), buf.eps[-1].contiguous()
    ms.ms_mixed_doubling(ctx, buf, e, 1e6)            # warmup (workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    whole, levels = ms.ms_mixed_doubling(ctx, buf, e, 1e6)
    T, R, no = ms.ms_transmission(ctx, whole, e, eps_l, eps_r)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.sync()
    t_fold = float(results["fp64"]["T"][ie]) if "fp64" in results else None
    n, ns = j.n_g, j.n_slices
    log(f"mixed doubling: {dt:.2f} s per point, {levels} mixed levels")
    return {"config": f"first timed (gap, k_par) of the workload, E = {e:.6f} Ry, max_cond = 1e6",
            "seconds_per_point": dt, "mixed_levels": levels, "T": float(T.cpu()[0]),
            "T_fused_fold": t_fold, "abs_dT": abs(float(T.cpu()[0]) - t_fold) if t_fold is not None else None,
            "n_open": int(no.cpu()[0]),
            "note": (f"whole S of {ns + 1} interfaces by a doubling tree: about 9 1/3 N^3 complex MACs per mixed "
                     "pair, 10 1/3 per star pair and 4/3 N^3 per block for the condition numbers, against "
                     "3 1/3 N^3 per interface for the fused fold")}


def uneven_inputs(i):
    """Seeded inputs of uneven instance i (host arrays; no GPU)."""
    import msgen
    it = msgen.config4_instances()[i]
    j = it["junction"]
    inp = msgen.junction_inputs(j, j.kpars[it["k_index"]])
    return dict(n_g=j.n_g, ns=len(j.dz), e=float(it["energy"]),
                miller=np.ascontiguousarray(inp["miller"], dtype=np.int32),
                q=np.ascontiguousarray(inp["q_of_ij"], dtype=np.int32), vq=np.ascontiguousarray(inp["vq"]),
                dz=np.ascontiguousarray(inp["dz"]), bvec=np.asarray(inp["bvec"]).reshape(4),
                kpar=np.asarray(inp["kpar"]))


def uneven_measure(ms, ctx, count, log, replays=2, prep_streams=3, chunk_bytes=64e9, host_inputs=None):
    """The uneven workload: the first `count` seeded instances of the bilayer junction with
    N_G drawn from {200, 450, 800, 1200}, 100-400 slices and one (E, k_par) each, taken in
    chunks of consecutive instances whose overlaps fit `chunk_bytes` of HBM.  Per chunk the
    slice eigenproblems and overlaps are prepared on `prep_streams` contexts (timed), then
    all instances of the chunk are folded in one call, in the FP32-MFMA form and in FP64
    (timed; |dT| between the forms per instance), with GEMM tile edges chosen per basis size
    by ms_autotune.  The first chunk's instances with N_G <= 450 are also folded in one
    captured hipGraph, whose replays are timed and checked against the direct call (a graph
    holds at most 96000 kernels, which the first 16 instances together, about 213000, exceed)."""
    import torch
    import msgen
    dev = ctx.device
    inst = msgen.config4_instances()[:count]
    chunks, cur, acc = [], [], 0.0
    for i, it in enumerate(inst):
        nb = (len(it["junction"].dz) + 1) * it["junction"].n_g ** 2 * 16.0
        if cur and acc + nb > chunk_bytes:
            chunks.append(cur)
            cur, acc = [], 0.0
        cur.append(i)
        acc += nb
    chunks.append(cur)
    pctx = [ctx] + [ms.Context(0, stream=torch.cuda.Stream()) for _ in range(prep_streams - 1)]
    n_gs = sorted({it["junction"].n_g for it in inst})
    tuned, tune_s = {}, 0.0
    tot = dict(prep=0.0, fp32=0.0, fp64=0.0)
    res_T = {"fp32": np.zeros(count), "fp64": np.zeros(count)}
    res_R64, res_no64 = np.zeros(count), np.zeros(count, dtype=np.int64)
    bad = 0
    graph = None
    for ci, chunk in enumerate(chunks):
        staged = []
        for i in chunk:
            h = host_inputs[i] if host_inputs is not None else uneven_inputs(i)
            staged.append(dict(h, miller=torch.as_tensor(h["miller"], device=dev),
                               q=torch.as_tensor(h["q"], device=dev), vq=torch.as_tensor(h["vq"], device=dev),
                               dz=torch.as_tensor(h["dz"], device=dev)))
        bufs = [ms.Slices.empty(x["n_g"], x["ns"], x["dz"], dev) for x in staged]
        # the instances' slice eigenproblems are independent: spread them over contexts on
        # separate streams (heaviest first onto the least loaded), one host thread each
        load = [0.0] * len(pctx)
        place = [0] * len(staged)
        for i in sorted(range(len(staged)), key=lambda i: -staged[i]["ns"] * staged[i]["n_g"] ** 3):
            r = min(range(len(pctx)), key=lambda r: load[r])
            load[r] += staged[i]["ns"] * staged[i]["n_g"] ** 3
            place[i] = r
        torch.cuda.synchronize()
        t0 = time.perf_counter()

        def prepare_on(r):   # one host thread per context: each preparation waits for its stream
            for i, (b, x) in enumerate(zip(bufs, staged)):
                if place[i] == r:
                    c = pctx[r]
                    ms.ms_slices_prepare(c, x["miller"], x["bvec"], x["kpar"], x["q"], x["vq"], x["dz"], out=b)

        with ThreadPoolExecutor(max_workers=len(pctx)) as pool:
            list(pool.map(prepare_on, range(len(pctx))))
        torch.cuda.synchronize()
        prep_s = time.perf_counter() - t0
        tot["prep"] += prep_s
        if ci == 0:   # GEMM tile edges per basis size, timed on synthetic systems of a chunk's batch
            t0 = time.perf_counter()
            for n_g in n_gs:
                nb = max(1, max(sum(1 for i in ch if inst[i]["junction"].n_g == n_g) for ch in chunks))
                choice, times = ms.ms_autotune(ctx, n_g, 8, nb)
                tuned[str(n_g)] = dict(batch=nb, choice=choice, lu_ms=[round(v, 3) for v in times[:4]],
                                       iface_ms=[round(v, 3) for v in times[4:]])
            tune_s = time.perf_counter() - t0
            log(f"uneven: autotuned {len(tuned)} basis sizes in {tune_s:.2f} s: "
                + ", ".join(f"{k}: {v['choice']}" for k, v in tuned.items()))
        es = [[x["e"]] for x in staged]
        for prec in ("fp32", "fp64"):
            if len(chunks) == 1:
                ms.ms_transmission_uneven(ctx, bufs, es, prec)          # warm: workspace
                torch.cuda.synchronize()
            t0 = time.perf_counter()
            T, R, no, st = ms.ms_transmission_uneven(ctx, bufs, es, prec)
            torch.cuda.synchronize()
            tot[prec] += time.perf_counter() - t0
            res_T[prec][chunk] = T.cpu().numpy()
            bad += int(np.sum(st.cpu().numpy() != 0))
            if prec == "fp64":
                res_R64[chunk] = R.cpu().numpy()
                res_no64[chunk] = no.cpu().numpy()
        log(f"uneven chunk {ci + 1}/{len(chunks)}: {len(chunk)} instances, prepare {prep_s:.2f} s, "
            f"folds so far fp32 {tot['fp32']:.2f} s / fp64 {tot['fp64']:.2f} s")
        small = [i for i, x in enumerate(staged) if x["n_g"] <= 450]
        if ci == 0 and small:
            sb, se = [bufs[i] for i in small], [es[i] for i in small]
            t0 = time.perf_counter()
            Tg = ms.ms_transmission_uneven(ctx, sb, se, "fp32", graph=True)[0]
            torch.cuda.synchronize()
            first_s = time.perf_counter() - t0
            ts = []
            for _ in range(replays):
                Tg.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ms.ms_graph_replay(ctx)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            ms.ms_transmission_uneven(ctx, sb, se, "fp32")           # the same instances, no graph
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Te = ms.ms_transmission_uneven(ctx, sb, se, "fp32")[0]
            torch.cuda.synchronize()
            eager_s = time.perf_counter() - t0
            graph = {
                "instances": len(small), "which": [chunk[i] for i in small], "form": "fp32",
                "capture_and_first_launch_s": round(first_s, 4),
                "replay_s": round(min(ts), 4),
                "direct_call_s": round(eager_s, 4),
                "max_abs_T_replay_minus_direct": float(np.max(np.abs(Tg.cpu().numpy() - Te.cpu().numpy()))),
            }
            log(f"uneven graph ({len(small)} instances): capture+launch {first_s:.2f} s, replay {min(ts):.3f} s, "
                f"direct {eager_s:.3f} s")
        del bufs, staged
        torch.cuda.empty_cache()
    for c in pctx[1:]:
        c.close()
    dT = np.abs(res_T["fp32"] - res_T["fp64"])
    mix = {}
    for it in inst:
        mix[str(it["junction"].n_g)] = mix.get(str(it["junction"].n_g), 0) + 1
    res = {
        "workload": "uneven instances of the bilayer-gap junction (hexagonal 2x2 cell, 16 bohr): "
                    "N_G in {200, 450, 800, 1200}, 100-400 slices, one (E, k_par) each, seeded; "
                    f"the first {count} of 512",
        "instances": count,
        "chunks": len(chunks),
        "n_g_mix": mix,
        "slices_total": int(sum(len(it["junction"].dz) for it in inst)),
        "prepare_s": round(tot["prep"], 4),
        "prepare_streams": prep_streams,
        "autotune": {"seconds": round(tune_s, 3), "per_n_g": tuned},
        "fold_s": {"fp32": round(tot["fp32"], 4), "fp64": round(tot["fp64"], 4)},
        "instances_per_s_fold": {"fp32": round(count / tot["fp32"], 3), "fp64": round(count / tot["fp64"], 3)},
        "instances_per_s_end_to_end": {"fp32": round(count / (tot["prep"] + tot["fp32"]), 3),
                                       "fp64": round(count / (tot["prep"] + tot["fp64"]), 3)},
        "max_abs_dT_fp32_vs_fp64": float(dT.max()),
        "max_abs_R_plus_T_minus_Nopen_fp64": float(np.max(np.abs(res_T["fp64"] + res_R64 - res_no64))),
        "bad_points": bad,
    }
    res["worst_dT"] = [dict(instance=int(i), n_g=int(inst[i]["junction"].n_g), slices=len(inst[i]["junction"].dz),
                            energy=round(float(inst[i]["energy"]), 4), n_open=int(res_no64[i]),
                            T=round(float(res_T["fp64"][i]), 6), dT=float(f"{dT[i]:.3g}"))
                       for i in np.argsort(-dT)[:3]]
    if count <= 32:
        res["abs_dT_fp32_vs_fp64"] = [float(f"{v:.3g}") for v in dT]
    else:
        res["abs_dT_fp32_vs_fp64_quantiles"] = {q: float(f"{np.quantile(dT, float(q)):.3g}")
                                                for q in ("0.5", "0.9", "0.99", "1.0")}
    if graph:
        res["graph"] = graph
    return res


def adjoint_measure(ms, ctx, n_e, log, fd_slices=(37, 200, 371)):
    """The adjoint workload: dT/dV^p(Q) for every slice and Fourier coefficient of the
    side-contact junction at gap 6.3 bohr, k_par = 0 (N_G = 1200, 400 slices, the right
    cascade of every plane kept), at `n_e` of its 16 energies in one call (split over three
    streams, each stream's energies batched through every launch); seconds per energy, and the
    derivative with respect to Re V^p(0) on three slices against central differences of T
    (h = 1e-5)."""
    import torch
    import msgen
    j = msgen.config5()
    inp = msgen.junction_inputs(j, j.kpars[0])
    dev = ctx.device
    q = torch.as_tensor(np.ascontiguousarray(inp["q_of_ij"], dtype=np.int32), device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = ms.prepare_from_inputs(ctx, inp, with_evec=True)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    idx = adjoint_energy_indices(len(j.energies), n_e)
    es = [float(j.energies[i]) for i in idx]
    free_gb = torch.cuda.mem_get_info(dev)[0] / 1e9
    log(f"adjoint: {free_gb:.0f} GB of device memory free before the call")
    t0 = time.perf_counter()
    gall, trall, _ = ms.ms_dT_dV(ctx, s, es, q, inp["vq"].shape[1], 1)   # every plane kept
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    trall = trall.cpu().numpy()
    log(f"adjoint: {n_e} energies in {total:.2f} s ({total / n_e:.2f} s per energy), T = {trall[:, 0]}")
    times = [total / n_e] * n_e
    grads = [(es[0], gall[0].cpu().numpy(), trall[0], 0)]
    e, g, tr, _ = grads[0]
    q0 = int(np.where((inp["q_miller"] == 0).all(axis=1))[0][0])
    h, rel = 1e-5, []
    for p in fd_slices:
        vals = []
        for sgn in (1, -1):
            vq = inp["vq"].copy()
            vq[p, q0] += sgn * h
            sp = ms.prepare_from_inputs(ctx, dict(inp, vq=vq))
            vals.append(float(ms.ms_transmission_batch(ctx, sp, [e])[0].cpu().numpy()[0]))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(2.0 * np.real(g[p, q0]))
        rel.append(abs(fd - an) / max(abs(an), 1e-12))
    n, ns = j.n_g, len(j.dz)
    # per interface: three reduced star products (4 1/3 n^3 complex MACs each), two slice
    # S-matrices (4 n^3 each), and per slice I - L12 R21, its LU and conj(U) M U^T (3 1/3 n^3)
    flop = 8.0 * (2 * 13.0 / 3 + 8 + 10.0 / 3) * n ** 3 * (ns + 1)   # two star products per plane
    return {
        "workload": "dT/dV^p(Q) of the side-contact junction at gap 6.3 bohr, k_par = 0: N_G = 1200, "
                    f"400 slices, {inp['vq'].shape[1]} Fourier coefficients per slice, the right cascade of "
                    "every plane kept",
        "energies": es,
        "T": [float(x) for x in trall[:, 0]],
        "concurrent_streams": min(3, n_e),
        "energies_per_batch": -(-n_e // min(3, n_e)),
        "prepare_with_eigenvectors_s": round(prep_s, 3),
        "seconds_per_energy": [round(x, 3) for x in times],
        "gradient_entries_per_energy": int(ns * inp["vq"].shape[1]),
        "approx_flop_per_energy": flop,
        "approx_tflops": round(flop / np.mean(times) / 1e12, 2),
        "fd_check": {"coefficient": "Re V^p(Q=0)", "slices": list(fd_slices), "h": h,
                     "max_rel_diff": float(max(rel))},
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the path shards over (E, k_par) points with no "
              "communication between GPUs, so it has no multi-GPU step to time; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print(f"[bench {elapsed():6.1f}s] {msg}", file=sys.stderr, flush=True)

    if args.probe:
        probe(args.probe, max(1, args.probe_launches))
        return
    if args.electrode_only:
        out = electrode_measure(args.electrode_only, max(1, args.electrode_energies), args.electrode_bands_only)
        print(json.dumps({"electrode": out, "n_gpus": 1, "data": "synthetic"}), flush=True)
        return
    # ---- seeded inputs, generated in worker processes before this process loads the GPU
    # library or touches the GPU (the pool and its workers are gone before that)
    from concurrent.futures import ProcessPoolExecutor
    workers = max(1, min(args.workers, os.cpu_count() or 1))
    uneven_host = None
    if args.uneven_only:
        import msgen  # noqa: F401
        with ProcessPoolExecutor(max_workers=workers) as pool:
            uneven_host = list(pool.map(uneven_inputs, range(max(1, args.uneven)), chunksize=4))
        log(f"uneven inputs generated ({len(uneven_host)} instances)")
    combos, make, desc = workload(args.config)
    kps = max(1, args.kpar_per_step)
    groups = step_groups(combos, kps)
    warm = min(max(0, args.warmup), 1)
    if args.all_points:
        plan = groups[:]                              # every group once, all timed
        warm = 0
    else:
        nmax = max(1, args.steps)
        plan = [groups[i % len(groups)] for i in range(warm + nmax)]
    host = {}
    if not args.uneven_only:
        tasks = sorted({(args.config, key, ik) for key, iks in plan for ik in iks}, key=str)
        with ProcessPoolExecutor(max_workers=min(workers, len(tasks))) as pool:
            for t, h in zip(tasks, pool.map(host_inputs_of, tasks)):
                host[(t[1], t[2])] = h
        log(f"inputs generated: {len(tasks)} distinct (key, k_par) of {args.config} in {workers} processes")

    import torch
    import paper_1504_01462_amd as ms

    if args.uneven_only:
        n_u = max(1, args.uneven)
        ctx = ms.Context(0)
        u = uneven_measure(ms, ctx, n_u, log, host_inputs=uneven_host)
        ctx.close()
        print(json.dumps({"uneven_batch": u, "n_gpus": 1, "data": "synthetic"}), flush=True)
        return

    ctx = ms.Context(0)
    dev = ctx.device
    juncs = {}
    dev_in = {}
    for (key, ik), h in host.items():      # resident in HBM before any timing
        if key not in juncs:
            juncs[key] = make(key)
        dev_in[(key, ik)] = dict(h, miller=torch.as_tensor(h["miller"], device=dev),
                                 q=torch.as_tensor(h["q"], device=dev), vq=torch.as_tensor(h["vq"], device=dev),
                                 dz=torch.as_tensor(h["dz"], device=dev))
    staged = [dict(j=juncs[key], key=key, iks=list(iks), ks=[dev_in[(key, ik)] for ik in iks]) for key, iks in plan]
    j0 = staged[0]["j"]
    n_e, n_k = len(j0.energies), len(j0.kpars)
    bufsets = [[ms.Slices.empty(j0.n_g, j0.n_slices, staged[0]["ks"][0]["dz"], dev) for _ in range(kps)]
               for _ in range(2 if args.overlap else 1)]
    bufs = bufsets[0]
    sp = torch.cuda.Stream(dev) if args.overlap else None   # default priority
    ctx_p = ms.Context(0, stream=sp) if args.overlap else None
    t_store = torch.zeros((n_k, n_e), dtype=torch.float64, device=dev)
    no_store = torch.zeros((n_k, n_e), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    log(f"inputs resident: {len(staged)} planned steps of {args.config}, {kps} k_par per step")

    tuned_main = None
    if args.autotune:   # GEMM tile edges for this basis size and batch (never changes a result)
        t0 = time.perf_counter()
        choice, times = ms.ms_autotune(ctx, j0.n_g, min(j0.n_g, 13), kps * n_e)
        tuned_main = dict(seconds=round(time.perf_counter() - t0, 3), choice=choice,
                          lu_ms=[round(v, 3) for v in times[:4]], iface_ms=[round(v, 3) for v in times[4:]])
        log(f"autotune n_g={j0.n_g}, batch {kps * n_e}: {choice}")

    main_stream = torch.cuda.current_stream(dev)

    def fold(st, prec, bset, outs, evs):
        m = len(st["ks"])
        es = np.tile(np.asarray(st["j"].energies, dtype=np.float64), (m, 1))
        T, R, no, status = ms.ms_transmission_multi(ctx, bset[:m], es, prec)
        for r, ik in enumerate(st["iks"]):
            t_store[ik].copy_(T[r])
            no_store[ik].copy_(no[r])
        ms.ms_kpar_average(ctx, t_store, no_store)
        if evs is not None:
            evs.append(torch.cuda.Event(enable_timing=True))
            evs[-1].record(main_stream)
        outs.append((T.reshape(-1), R.reshape(-1), no.reshape(-1), status.reshape(-1)))

    def run(steps, prec, label):
        """One step: the slice eigenproblems and overlaps of each of its k_par, the fused fold
        over all their energies in one batch, T and R, the k_par average.  Without --overlap all
        on the current stream, one after the other, with stream events between preparation and
        fold (the E-independent share of each step); with it, step i+1's slices are prepared on a
        second context and stream while step i folds, ordered by events."""
        outs, evs = [], []
        if not args.overlap:
            evs.append(torch.cuda.Event(enable_timing=True))
            evs[-1].record(main_stream)
            for i, st in enumerate(steps):
                for b, kk in zip(bufs, st["ks"]):
                    ms.ms_slices_prepare(ctx, kk["miller"], kk["bvec"], kk["kpar"], kk["q"], kk["vq"], kk["dz"],
                                         out=b)
                evs.append(torch.cuda.Event(enable_timing=True))
                evs[-1].record(main_stream)
                fold(st, prec, bufs, outs, evs)
                log(f"{label} step {i + 1}/{len(steps)} enqueued")
            return outs, evs
        ev_prep = [torch.cuda.Event() for _ in steps]
        ev_fold = [torch.cuda.Event() for _ in steps]
        start = torch.cuda.Event()
        start.record(main_stream)

        def prep(i):
            with torch.cuda.stream(sp):
                sp.wait_event(ev_fold[i - 2] if i >= 2 else start)
                for b, kk in zip(bufsets[i % 2], steps[i]["ks"]):
                    ms.ms_slices_prepare(ctx_p, kk["miller"], kk["bvec"], kk["kpar"], kk["q"], kk["vq"], kk["dz"],
                                         out=b)
                ev_prep[i].record(sp)

        with ThreadPoolExecutor(1) as pool:
            fut = pool.submit(prep, 0)
            for i, st in enumerate(steps):
                fut.result()
                if i + 1 < len(steps):
                    fut = pool.submit(prep, i + 1)
                main_stream.wait_event(ev_prep[i])
                fold(st, prec, bufsets[i % 2], outs, None)
                ev_fold[i].record(main_stream)
                log(f"{label} step {i + 1}/{len(steps)} enqueued")
            fut.result()
        return outs, None

    def collect(outs):
        return tuple(np.concatenate([o[i].cpu().numpy() for o in outs]) for i in range(4))

    evp = not args.no_event_profile
    cat = args.roofline_kernel
    results = {}
    # ---- FP64: warmup, then the timed steps (as many as the time budget holds)
    tw = time.perf_counter()
    if warm:
        run(staged[:warm], "fp64", "fp64 warmup")
        ctx.sync()
    t_warm = time.perf_counter() - tw
    pool_steps = staged[warm:]
    if args.all_points or not warm:
        n_timed = len(pool_steps)
    else:
        n_timed = max(1, min(len(pool_steps), int(args.time_budget // max(t_warm, 1e-3))))
    timed_steps = pool_steps[:n_timed]
    log(f"fp64 warmup: {warm} step(s) in {t_warm:.2f} s; timing {n_timed} of {args.steps} requested steps")
    forms = ["fp64"]
    if args.fp32_steps > 0:
        forms.append("fp32")
    for prec in forms:
        steps = timed_steps if prec == "fp64" or args.all_points else timed_steps[:max(1, args.fp32_steps)]
        if prec == "fp32" and not args.all_points:
            est = t_warm * len(steps)
            if elapsed() + est > args.wall_budget:
                log(f"fp32 leg skipped: {est:.0f} s would pass the wall budget")
                continue
        ms.ms_debug_profile(ctx, [cat] if evp else False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs, evs = run(steps, prec, prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.sync()
        log(f"{prec}: {len(steps)} timed steps in {dt:.2f} s")
        prof = ms.ms_debug_profile_read(ctx, cat)
        ms.ms_debug_profile(ctx, False)
        T, R, NO, ST = collect(outs)
        prep_s = fold_s = None
        if evs is not None:       # stream events: [start, after prep 1, after fold 1, after prep 2, ...]
            ms_t = [evs[i].elapsed_time(evs[i + 1]) / 1e3 for i in range(len(evs) - 1)]
            prep_s, fold_s = float(sum(ms_t[0::2])), float(sum(ms_t[1::2]))
        results[prec] = dict(seconds=dt, steps=len(steps), points=int(T.size), T=T, R=R, NO=NO, ST=ST, prof=prof,
                             prep_s=prep_s, fold_s=fold_s)

    base = results["fp64"]
    out_forms = {}
    for prec, r in results.items():
        d = dict(points_per_s=r["points"] / r["seconds"], steps=r["steps"], points=r["points"],
                 ms_per_step=1e3 * r["seconds"] / r["steps"],
                 max_abs_R_plus_T_minus_Nopen=float(np.max(np.abs(r["T"] + r["R"] - r["NO"]))),
                 bad_points=int(np.sum(r["ST"] != 0)),
                 T_sha1=hashlib.sha1(np.ascontiguousarray(r["T"]).tobytes()).hexdigest()[:16])
        if r["fold_s"]:
            d["per_point_work"] = {
                "points_per_s": r["points"] / r["fold_s"],
                "fold_s": round(r["fold_s"], 3), "prepare_s": round(r["prep_s"], 3),
                "note": "(i) the fold alone (a4-a6, k_par average) from stream events between each step's "
                        "slice preparation (a1-a3) and its fold; `points_per_s` of the form is (ii), end to end"}
        if prec != "fp64":
            m = r["points"]
            dT = np.abs(r["T"] - base["T"][:m])
            d["max_abs_dT_vs_fp64"] = float(np.max(dT))
            d["abs_dT_vs_fp64_quantiles"] = {q: float(f"{np.quantile(dT, float(q)):.3g}")
                                             for q in ("0.5", "0.9", "0.99", "1.0")}
            d["points_compared"] = m
        out_forms[prec] = d

    head = "fp64"
    f32 = out_forms.get("fp32")
    if f32 and f32["max_abs_dT_vs_fp64"] < 1e-6 and f32["bad_points"] == 0:
        head = "fp32"
    hr = results[head]
    tot_ms, launches, flops, nbytes = hr["prof"]
    avg_s = tot_ms / 1e3 / max(1, launches) or float("inf")
    fl_per = flops / max(1, launches)
    by_per = nbytes / max(1, launches)
    gemm_like = cat in ("iface_gemm", "lu_update", "lu_inner", "prep_gemm", "trsm", "jacobi")
    peak = PEAK["fp32" if (head == "fp32" and cat == "iface_gemm") else "fp64"]
    if gemm_like and fl_per / max(1.0, by_per) > peak * 1e12 / (HBM_PEAK * 1e9):
        roof = {"bound": "mfma", "achieved": fl_per / avg_s / 1e12, "peak": peak, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": by_per / avg_s / 1e9, "peak": HBM_PEAK, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"] if launches else None
    # the FP32 products always use 64 x 64 tiles; FP64 the tuned (or default 64) edge
    iface_tile = 64 if head == "fp32" else ((tuned_main["choice"]["iface"] if tuned_main else 0) or 64)
    roof["traffic"] = measured_traffic(cat, fl_per, head, iface_tile if cat == "iface_gemm" else 128)
    roof["kernel"] = cat
    if cat == "iface_gemm":
        roof["tile"] = "64x64" if iface_tile == 64 else "128x64"
        roof["algorithmic_flop_per_launch"] = fl_per
        roof["algorithmic_bytes_per_launch"] = by_per
    roof["avg_launch_ms"] = avg_s * 1e3
    roof["launches"] = launches
    roof["note"] = ("per-launch durations from HIP events that bracket the kernel's own execution "
                    "(hipExtLaunchKernel) on the stream it is launched on, over the timed region of the "
                    "headline form; the interface GEMM runs alone on the GPU; algorithmic flops are "
                    "8 M N K per complex product (the kernel issues three real MFMA products per "
                    "complex one, 6 M N K)")

    line = {
        "metric": METRIC,
        "value": out_forms[head]["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": results[head]["steps"],
        "warmup": warm,
        "ms_per_step": out_forms[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64-mfma+f64" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {desc}", "n_g": j0.n_g, "n_slices": j0.n_slices,
                   "energies_per_kpar": n_e, "kpar_per_step": kps, "points_per_step": kps * n_e,
                   "prepare_overlapped": bool(args.overlap),
                   "steps_requested": args.steps, "warmup_requested": args.warmup,
                   "time_budget_s": None if args.all_points else args.time_budget,
                   "steps_over": [[str(st["key"]), st["iks"]] for st in timed_steps],
                   "headline_form": head},
        "forms": out_forms,
        "roofline": roof,
        "autotune": tuned_main,
    }
    if ctx_p is not None:
        ctx_p.close()                       # the preparation context's workspace
    if args.mixed and args.config == "config3":
        if elapsed() + 60 < args.wall_budget:
            line["mixed_doubling"] = mixed_doubling_measure(ms, ctx, timed_steps[0], bufs[0], results, log)
        else:
            log("mixed doubling skipped (wall budget)")
    if args.adjoint > 0 and args.config == "config3":
        if elapsed() + 30 + 8 * args.adjoint < args.wall_budget:
            for bs in bufsets:
                bs.clear()
            torch.cuda.empty_cache()
            actx = ms.Context(0)            # its own context: the gradient's workspace is freed after
            line["adjoint"] = adjoint_measure(ms, actx, args.adjoint, log)
            actx.close()
            torch.cuda.empty_cache()
        else:
            log("adjoint leg skipped (wall budget)")
    if args.uneven > 0:
        if elapsed() + 2.5 * args.uneven < args.wall_budget:
            for bs in bufsets:
                bs.clear()
            torch.cuda.empty_cache()
            line["uneven_batch"] = uneven_measure(ms, ctx, args.uneven, log)
        else:
            log("uneven leg skipped (wall budget)")
    ctx.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        line["cpu_baseline"] = cpu_baseline(args.config, args.cpu_seconds)
    line["wall_s"] = round(elapsed(), 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
