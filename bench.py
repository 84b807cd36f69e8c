#!/usr/bin/env python3
"""Throughput benchmark of the plane-wave multiple-scattering transport path on one MI355X.

Workload (default): the side-contact overlap junction -- rectangular 4.65 x 40
bohr cell, two graphene-like Gaussian-well sheets overlapping 15 bohr along
the transport direction, N_G = 1200 plane waves, 400 slices of 0.05 bohr,
free-electron leads, 32 energies at each of 8 k_par for 3 vacuum gaps.  One
step = two k_par of one gap (64 points): slice Hamiltonians, eigenpairs and
overlaps (E-independent) of each, the fused slice-S / star-product fold of
all 64 points in one batch, T and R per point, and the k_par average.
Inputs are seeded and synthetic, uploaded to HBM before the timed region.

The steps run twice, in FP64 and in the FP32-MFMA form, over the same
(gap, k_par) pairs; the FP32 number is the headline only when its largest
|dT| against the FP64 run stays below 1e-6.  One point of the workload is
also solved with the paper's mixed transfer/scattering doubling, and the first
instances of the uneven workload (N_G from 200 to 1200, 100-400 slices, one point
each) are folded in one call, the small ones also in a captured hipGraph
(`uneven_batch`), and the gradient dT/dV of every slice coefficient is timed at three
energies of the adjoint workload (`adjoint`).

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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="config3", choices=["config1", "config2", "config3"])
    ap.add_argument("--forms", default="fp64,fp32")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kpar-per-step", type=int, default=2,
                    help="k_par values of one junction folded together in one batch per step")
    ap.add_argument("--no-next3", dest="next3", action="store_false",
                    help="skip the timing of the mixed-recurrence doubling (ms_mixed_doubling)")
    ap.add_argument("--roofline-kernel", default="iface_gemm",
                    help="profiler category reported in 'roofline' ('auto': the largest summed time in the warmup)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the default GEMM tile rule instead of timing both edges first")
    ap.add_argument("--uneven", type=int, default=16,
                    help="instances of the uneven workload (N_G 200-1200, 100-400 slices) folded in one "
                         "captured graph after the main measurement; 0 skips it")
    ap.add_argument("--adjoint", type=int, default=8,
                    help="energies of the adjoint workload (dT/dV at N_G = 1200) to time; 0 skips it")
    ap.add_argument("--overlap", action="store_true",
                    help="prepare the next step's slices on a second stream while the current step folds")
    ap.add_argument("--uneven-only", action="store_true",
                    help="measure only the uneven workload (--uneven instances) and print its JSON line")
    ap.add_argument("--no-event-profile", action="store_true",
                    help="record no HIP events around launches (no roofline figure; for external profilers)")
    return ap.parse_args()


def workload(name):
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


def cpu_baseline(name, budget_s):
    """The oracle, untuned, on a bounded sample of one point of the workload."""
    import msgen
    import oracle as orc
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    combos, make, _ = workload(name)
    j = make(combos[0][0])
    inp = msgen.junction_inputs(j, j.kpars[combos[0][1]])
    kin = orc.kinetic(inp["miller"], inp["bvec"], inp["kpar"])
    e = float(j.energies[len(j.energies) // 2])
    ns = j.n_slices
    t0 = time.perf_counter()
    n_eig = 0
    us = []
    while n_eig < 3 and (n_eig == 0 or time.perf_counter() - t0 < 0.35 * budget_s):
        h = orc.slice_hamiltonians(kin, inp["vq"][n_eig:n_eig + 1], inp["q_of_ij"])
        eps, u = orc.slice_eigen(h)
        us.append((eps[0], u[0]))
        n_eig += 1
    t_eig = (time.perf_counter() - t0) / n_eig
    t1 = time.perf_counter()
    acc = orc.identity_smatrix(len(kin))
    n_if = 0
    while n_if < len(us) - 1 and (n_if == 0 or time.perf_counter() - t1 < 0.6 * budget_s):
        o = orc.overlap(us[n_if][1], us[n_if + 1][1])
        s = orc.interface_smatrix(o, orc.wavevectors(e, us[n_if][0]), orc.wavevectors(e, us[n_if + 1][0]),
                                  float(inp["dz"][n_if]))
        acc = orc.star(acc, s)
        n_if += 1
    t_if = (time.perf_counter() - t1) / max(1, n_if)
    # one point = its share of the E-independent eigenproblems + (n_slices + 1) interfaces
    t_point = t_eig * ns / len(j.energies) + t_if * (ns + 1)
    return {"value": 1.0 / t_point, "unit": "points/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"{name} first (gap/registry, k_par), E={e:.4f} Ry: {n_eig} slice eigenproblems "
                       f"({t_eig:.2f} s each) and {n_if} interface S-matrix + star products ({t_if:.2f} s each), "
                       f"scaled to one point = eigen share over {len(j.energies)} energies + {ns + 1} interfaces; "
                       "extrapolated, not a full point")}


def measured_traffic(cat, flops_per_launch, form, tile=128):
    """HBM bytes per launch of the roofline kernel from the committed rocprofv3 counter
    summary, or None when it covers another kernel, tile shape, launch shape or form, or
    when the kernel source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{cat}_config3_counters.txt")
    if form != "fp64" or not os.path.exists(path):
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
        if int(kv.get("tile", "128")) != tile:
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
    idx = np.linspace(0, len(j.energies) - 1, n_e + 2)[1:-1].round().astype(int)
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
    host_inputs = None
    if args.uneven_only:
        # generate the seeded inputs in worker processes, before this process loads the GPU
        # library or touches the GPU; the pool and its workers are gone before that
        from concurrent.futures import ProcessPoolExecutor
        t0 = time.perf_counter()
        with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as pool:
            host_inputs = list(pool.map(uneven_inputs, range(max(1, args.uneven)), chunksize=4))
        print(f"[bench] uneven inputs generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    import torch
    import msgen
    import paper_1504_01462_amd as ms

    if args.uneven_only:
        n_u = max(1, args.uneven)
        ctx = ms.Context(0)
        u = uneven_measure(ms, ctx, n_u, lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True),
                           host_inputs=host_inputs)
        ctx.close()
        print(json.dumps({"uneven_batch": u, "n_gpus": 1, "data": "synthetic"}), flush=True)
        return
    combos, make, desc = workload(args.config)
    # a step takes kps consecutive k_par of one junction (one batch of kps x n_e points)
    kps = max(1, args.kpar_per_step)
    groups = []
    for key, ik in combos:
        if groups and groups[-1][0] == key and len(groups[-1][1]) < kps:
            groups[-1][1].append(ik)
        else:
            groups.append((key, [ik]))
    nsteps = args.warmup + args.steps
    sel = [groups[i % len(groups)] for i in range(nsteps)]
    ctx = ms.Context(0)
    dev = ctx.device
    # seeded inputs, uploaded to HBM before timing
    cache = {}
    staged = []
    for key, iks in sel:
        if key not in cache:
            cache[key] = make(key)
        j = cache[key]
        ks = []
        for ik in iks:
            inp = msgen.junction_inputs(j, j.kpars[ik])
            ks.append(dict(
                ik=ik,
                miller=torch.as_tensor(np.ascontiguousarray(inp["miller"], dtype=np.int32), device=dev),
                q=torch.as_tensor(np.ascontiguousarray(inp["q_of_ij"], dtype=np.int32), device=dev),
                vq=torch.as_tensor(np.ascontiguousarray(inp["vq"]), device=dev),
                dz=torch.as_tensor(np.ascontiguousarray(inp["dz"]), device=dev),
                bvec=np.asarray(inp["bvec"]).reshape(4), kpar=np.asarray(inp["kpar"])))
        staged.append(dict(j=j, key=key, iks=list(iks), ks=ks))
    j0 = staged[0]["j"]
    n_e, n_k = len(j0.energies), len(j0.kpars)
    # two sets of slice buffers: with --overlap the next step's slices are prepared into one set
    # (on a second context and stream) while the current step folds the other
    bufsets = [[ms.Slices.empty(j0.n_g, j0.n_slices, staged[0]["ks"][0]["dz"], dev) for _ in range(kps)]
               for _ in range(2 if args.overlap else 1)]
    bufs = bufsets[0]
    sp = torch.cuda.Stream(dev) if args.overlap else None   # default priority
    ctx_p = ms.Context(0, stream=sp) if args.overlap else None
    t_store = torch.zeros((n_k, n_e), dtype=torch.float64, device=dev)
    no_store = torch.zeros((n_k, n_e), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"inputs staged: {len(staged)} steps of {args.config}, {kps} k_par per step")
    tuned_main = None
    if args.autotune:   # GEMM tile edges for this basis size and batch (never changes a result)
        t0 = time.perf_counter()
        choice, times = ms.ms_autotune(ctx, j0.n_g, min(j0.n_g, 13), kps * n_e)
        tuned_main = dict(seconds=round(time.perf_counter() - t0, 3), choice=choice,
                          lu_ms=[round(v, 3) for v in times[:4]], iface_ms=[round(v, 3) for v in times[4:]])
        log(f"autotune n_g={j0.n_g}, batch {kps * n_e}: {choice} (LU ms {tuned_main['lu_ms']}, "
            f"interface ms {tuned_main['iface_ms']})")

    def fold(i, st, prec, bset, outs):
        m = len(st["ks"])
        es = np.tile(np.asarray(st["j"].energies, dtype=np.float64), (m, 1))
        T, R, no, status = ms.ms_transmission_multi(ctx, bset[:m], es, prec)
        for r, ik in enumerate(st["iks"]):
            t_store[ik].copy_(T[r])
            no_store[ik].copy_(no[r])
        ms.ms_kpar_average(ctx, t_store, no_store)
        outs.append((T.reshape(-1), R.reshape(-1), no.reshape(-1), status.reshape(-1)))

    def run(steps, prec):
        """One step: the slice eigenproblems and overlaps of each of its k_par, the fused fold
        over all their energies in one batch, T and R, the k_par average.  Without --overlap all
        on the current stream, one after the other; with it, step i+1's slices are prepared on a
        second context and stream (enqueued by a worker thread, since the preparation's host
        steps wait for its stream) while step i folds, ordered by events: a fold waits for its
        slices, a preparation for the fold that last read its buffer set."""
        outs = []
        if not args.overlap:
            for i, st in enumerate(steps):
                for b, kk in zip(bufs, st["ks"]):
                    ms.ms_slices_prepare(ctx, kk["miller"], kk["bvec"], kk["kpar"], kk["q"], kk["vq"], kk["dz"],
                                         out=b)
                fold(i, st, prec, bufs, outs)
                log(f"{prec} step {i + 1}/{len(steps)} enqueued")
            return outs
        main = torch.cuda.current_stream(dev)
        ev_prep = [torch.cuda.Event() for _ in steps]
        ev_fold = [torch.cuda.Event() for _ in steps]
        start = torch.cuda.Event()
        start.record(main)

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
                main.wait_event(ev_prep[i])
                fold(i, st, prec, bufsets[i % 2], outs)
                ev_fold[i].record(main)
                log(f"{prec} step {i + 1}/{len(steps)} enqueued")
            fut.result()
        return outs

    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    results = {}
    prof_pick = None
    evp = not args.no_event_profile
    for prec in forms:
        # warmup (the first form's warmup also picks the dominant kernel)
        ms.ms_debug_profile(ctx, evp)
        tw = time.perf_counter()
        run(staged[:args.warmup], prec)
        ctx.sync()
        log(f"{prec} warmup ({args.warmup} steps): {time.perf_counter() - tw:.2f} s")
        prof = {c: ms.ms_debug_profile_read(ctx, c) for c in ms.PROFILE_CATEGORIES}
        if prof_pick is None:
            prof_pick = args.roofline_kernel
            if prof_pick == "auto":
                prof_pick = max(prof, key=lambda c: prof[c][0]) if evp and args.warmup > 0 else "iface_gemm"
        ms.ms_debug_profile(ctx, [prof_pick] if evp else False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = run(staged[args.warmup:], prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.sync()
        log(f"{prec}: {args.steps} timed steps in {dt:.2f} s")
        timed = {c: ms.ms_debug_profile_read(ctx, c) for c in ms.PROFILE_CATEGORIES}
        ms.ms_debug_profile(ctx, False)
        T = np.concatenate([o[0].cpu().numpy() for o in outs])
        R = np.concatenate([o[1].cpu().numpy() for o in outs])
        NO = np.concatenate([o[2].cpu().numpy() for o in outs])
        ST = np.concatenate([o[3].cpu().numpy() for o in outs])
        results[prec] = dict(seconds=dt, points=int(T.size), T=T, R=R, NO=NO, ST=ST, prof=timed,
                             warm_prof=prof)

    base = results[forms[0]]
    out_forms = {}
    for prec, r in results.items():
        d = dict(points_per_s=r["points"] / r["seconds"], ms_per_step=1e3 * r["seconds"] / args.steps,
                 max_abs_R_plus_T_minus_Nopen=float(np.max(np.abs(r["T"] + r["R"] - r["NO"]))),
                 bad_points=int(np.sum(r["ST"] != 0)),
                 T_sha1=hashlib.sha1(np.ascontiguousarray(r["T"]).tobytes()).hexdigest()[:16])
        if prec != forms[0]:
            d["max_abs_dT_vs_" + forms[0]] = float(np.max(np.abs(r["T"] - base["T"])))
        d["warmup_kernel_ms_per_step"] = {c: round(v[0] / max(1, args.warmup), 3)
                                          for c, v in r["warm_prof"].items() if v[1]}
        d["warmup_kernel_launches_per_step"] = {c: int(v[1] / max(1, args.warmup))
                                                for c, v in r["warm_prof"].items() if v[1]}
        out_forms[prec] = d

    head = forms[0]
    if "fp32" in results and "fp64" in results and \
            out_forms["fp32"].get("max_abs_dT_vs_fp64", 1.0) < 1e-6 and out_forms["fp32"]["bad_points"] == 0:
        head = "fp32"
    hr = results[head]
    cat = prof_pick
    tot_ms, launches, flops, nbytes = hr["prof"][cat]
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
    iface_tile = (tuned_main["choice"]["iface"] if tuned_main else 0) or 128
    roof["traffic"] = measured_traffic(cat, fl_per, head, iface_tile if cat == "iface_gemm" else 128)
    roof["kernel"] = cat
    if cat == "iface_gemm":
        roof["tile"] = f"{iface_tile}x{iface_tile}"
    roof["avg_launch_ms"] = avg_s * 1e3
    roof["launches"] = launches
    roof["note"] = ("per-launch durations from HIP events that bracket the kernel's own execution "
                    "(hipExtLaunchKernel) on the stream it is launched on; the interface GEMM runs alone on the GPU")

    line = {
        "metric": METRIC,
        "value": out_forms[head]["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": out_forms[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64-mfma+f64" if head == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {desc}", "n_g": j0.n_g, "n_slices": j0.n_slices,
                   "energies_per_kpar": n_e, "kpar_per_step": kps, "prepare_overlapped": bool(args.overlap),
                   "steps_over": [[str(st["key"]), st["iks"]] for st in staged],
                   "headline_form": head},
        "forms": out_forms,
        "roofline": roof,
        "autotune": tuned_main,
    }
    if args.next3 and args.config == "config3":
        line["mixed_doubling"] = mixed_doubling_measure(ms, ctx, staged[args.warmup], bufs[0], results, log)
    if ctx_p is not None:
        ctx_p.close()                       # the preparation context's workspace
    if args.adjoint > 0 and args.config == "config3":
        for bs in bufsets:
            bs.clear()
        torch.cuda.empty_cache()
        actx = ms.Context(0)                # its own context: the gradient's workspace is freed after
        line["adjoint"] = adjoint_measure(ms, actx, args.adjoint, log)
        actx.close()
        torch.cuda.empty_cache()
    if args.uneven > 0:
        for bs in bufsets:                  # the main workload's slice buffers
            bs.clear()
        torch.cuda.empty_cache()
        line["uneven_batch"] = uneven_measure(ms, ctx, args.uneven, log)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        line["cpu_baseline"] = cpu_baseline(args.config, args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
