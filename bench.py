#!/usr/bin/env python3
"""Throughput of the Monte Carlo / rigorous-Mie photon walk on one MI355X.

One step is one pass of the whole hot path on the headline workload: the Mie
table build on the device (series, phase function, CDF, inverse table) and
the photon walk of 1e8 photons through a 10 mm water cube holding 5 um
polystyrene spheres at optical depth 4 (Philox seed 1234, 16384-entry inverse
CDF, 512 x 512 side and transmitted images).  `value` is scatter events per
second over the timed steps, inputs resident on the device.  Image exits go
through the exit log (MC_EXIT_LOG) unless --atomic-tally is given.

The JSON line also carries
  roofline      the walk kernel's achieved issue rate from an operation census
                of the method (counts of steps, interactions, boundary steps
                and exits, each priced in full-rate FP32 VALU issue slots by
                instruction class) over its measured average duration (HIP
                events the library attaches to that kernel's dispatch on the
                launch stream), against the chip's FP32 VALU peak (the
                published 157.3 TFLOP/s as fused multiply-adds); the same
                census over the whole mc_simulate (with the log binning and
                finalize kernels) is reported beside it;
  cpu_baseline  the FP64 oracle timed on this host: one thread on a leading
                sample of the workload and every thread of the CPU share on
                the whole workload (or a bounded leading part), with the CPU
                model and core counts;
  tally_error   per workload, the GPU path against the FP64 oracle at matched
                seeds: largest |difference| per image bin in units of the bin's
                Monte Carlo sigma, relative L2 norm of the image difference,
                bins beyond 3 sigma, the energy-balance residual of each side,
                and for the differentiation workload the path-moment images and
                a gradient (--no-tally-error skips it; both come from the
                oracle leg, which --no-cpu-baseline skips);
  sweep         the paper-scale workload at optical depths 1, 2 and 8 and the
                HG run at 4: scatter events/s over mc_simulate and the census
                fraction of each walk kernel (--no-sweep skips it);
  adjoint       after the timed steps, the same walk run forward only
                (mc_simulate, then a stream wait) and forward + adjoint
                (mc_simulate with the path-moment tallies, then mc_grad for
                an L2 loss, which waits), each over --steps launches on the
                same seed: the wall-clock ratio t(fwd + adjoint) / t(fwd);
  batch         the 256-medium batched launch (particle diameters, depths,
                albedos and photon counts from the seeded batch sampler,
                5.75e8 photons): launch shape from mc_autotune_batch on a
                1/16 photon sample, then scatter events/s of the batched
                launch against the best rate any of its media reaches when
                run alone with mc_simulate (--no-batch skips it);
  heavy         polydisperse heavy scattering: lognormal sizes (median 5 um,
                sigma_ln 0.05, 64 bins), tau = 16, 1e9 photons, 1024 x 1024
                int64 fixed-point images; table build time, forward scatter
                events/s, and forward + adjoint against forward time
                (--no-heavy skips it);
  analysis      the paper's image comparison on simulated side images: at
                each optical depth of Tables 3 and 4, a Mie and an HG run
                with the 1.25 mm-radius parallel beam (1e8 photons, 512 x 512)
                and an independent Mie run (other seed) as the reference;
                RMSE and r of both against it, the three radial zone errors,
                the radial correlation and the share of annuli where Mie is
                closer, and the time of mc_image_metrics (--no-analysis skips it).

    python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mie MC scatter events/s (τ=4, 1e8 photons); fwd+adjoint vs fwd-only time"

# Operation census: the fewest gfx950 VALU instructions that perform the
# walk's arithmetic per unit of work, by issue class.  gfx950 issues a wave64
# full-rate instruction (FP32 add/mul/fma, 32-bit integer add, and/or/xor,
# move, all operands in vector registers) in 2 SIMD cycles, half-rate ones
# (compares, selects, min/max/med3, shifts and funnel shifts, conversions,
# 32x32-bit products including v_mad_u64_u32, three-input bit operations) in
# 4, transcendentals (rcp, sqrt, log, sin, cos) in 8; measured by
# bench/issue_cost_probe.hip at 2.3-2.6, 3.7-4.4 and 8.0-8.2 cycles.  A slot
# is one full-rate lane-instruction, so a unit costs full + 2 half + 4 trans
# slots.  A uniform is one funnel shift (23 random bits under the exponent of
# 1.0) and one subtraction: 1 full, 1 half.
#   step         Philox4x32-10 (20 products, 20 three-input XORs: 40 half);
#                the free-path uniform (1 full, 1 half), its log and the
#                product by -1/mu (1 full, 1 trans); three wall distances
#                (per axis a reciprocal, a difference, two products and a
#                three-way maximum: 9 full, 3 half, 3 trans); nearest wall
#                (min3), hit test and step length (3 half); move (3 full);
#                step count (1 full)  = 15 full, 47 half, 4 trans.  (The path
#                length is summed only by the kernels that tally path
#                moments or records.)
#   interaction  event count, absorption and weight (3 full); roulette test
#                (1 half); two uniforms (2 full, 2 half); inverse-CDF
#                product, two conversions, fraction, difference and lerp
#                (4 full, 2 half); cos and sin of the polar angle from
#                v = 1 - cos (3 full, 1 trans); cos and sin of the azimuth
#                (2 trans); the orthonormal basis of Duff et al. (copysign,
#                sum and reciprocal, 9 products and fmas: 9 full, 1 half,
#                1 trans); new direction (12 full); Newton renormalisation
#                (7 full)  = 40 full, 6 half, 4 trans.  With Henyey-Greenstein
#                (Eq. 11) the table's 4 full, 2 half give way to the closed-
#                form inverse and a clamp of v (4 full, 1 half, 1 trans:
#                fma, reciprocal, product, fma, product, maximum)
#                = 40 full, 5 half, 5 trans
#   boundary     the reflection uniform (1 full, 1 half); wall axis and its
#                direction component (2 compares, 4 selects); clamp onto the
#                box (3 med3); unpolarised Fresnel with TIR (cos of
#                refraction: 3 full, 1 trans; the two amplitude ratios over
#                one reciprocal of the product of their denominators: 9 full,
#                1 trans; R: 3 full; TIR compare and select: 2 half);
#                reflect-or-leave (1 compare, 3 selects); exit face (1
#                compare, 1 shift-or, 1 select)  = 16 full, 19 half, 2 trans.
#                (Reflections are not counted per step: steps - events - exits.)
#   exit         imaged faces: pixel row and column (scale, floor, clamp), key,
#                weight added (3 full, 5 half); other faces: face total (2 full)
CENSUS = {"step": {"full": 15, "half": 47, "trans": 4},
          "interaction": {"full": 40, "half": 6, "trans": 4},
          "interaction_hg": {"full": 40, "half": 5, "trans": 5},
          "boundary": {"full": 16, "half": 19, "trans": 2},
          "imaged_exit": {"full": 3, "half": 5, "trans": 0},
          "other_exit": {"full": 2, "half": 0, "trans": 0}}
SLOTS_PER_CLASS = {"full": 1, "half": 2, "trans": 4}


def unit_slots(unit: str) -> int:
    return sum(SLOTS_PER_CLASS[k] * n for k, n in CENSUS[unit].items())


# MI355X: 256 CUs x 4 SIMDs x 32 full-rate FP32 lanes per clock at the
# 2.4 GHz peak engine clock: the published 157.3 TFLOP/s FP32 vector rate
# counted as fused multiply-adds.
PEAK_SLOTS_PER_S = 256 * 4 * 32 * 2.4e9

# HBM traffic of one walk_kernel launch on this workload with the exit log,
# from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by
# what the same counters read for a 256 MiB device copy (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0); valid only for the tally path and kernel code it was
# measured on (profiles/walk_tau4_counters.md): the digest covers the walk
# sources without comments and whitespace, so a comment edit keeps it.
TRAFFIC = {"tally": "log", "sources_sha256": "38c308aadf57ff13455a2aed5542f66d0dec4c300fd06419b7cc5937b107dc34",
           "fetch_kib": 374.3, "write_kib": 558765.0, "fetch_factor": 2.0, "write_factor": 1.0}
WALK_SOURCES = ("paper_2507_23189_amd/csrc/walk.hip", "paper_2507_23189_amd/csrc/philox.hpp")


def code_digest(text: str) -> str:
    """SHA-256 of C++ source text with its comments and all whitespace removed."""
    import hashlib
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return hashlib.sha256(re.sub(r"\s+", "", text).encode()).hexdigest()


def walk_sources_digest() -> str:
    return code_digest("".join(open(os.path.join(ROOT, f)).read() for f in WALK_SOURCES))


def measured_traffic(args):
    """Bytes per launch if the walk kernel is the one the counters were taken on, else None."""
    if args.atomic_tally != (TRAFFIC["tally"] == "atomic"):
        return None
    if walk_sources_digest() != TRAFFIC["sources_sha256"]:
        return None
    return 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_factor"] + TRAFFIC["write_kib"] * TRAFFIC["write_factor"])


def tally_flags(mc, args):
    """Image exits go through the exit log unless --atomic-tally."""
    return 0 if args.atomic_tally else mc.MC_EXIT_LOG


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def census_slots(scal, hg=False):
    """Algorithmic issue slots of one launch from its scalar tallies.  The
    imaged share of exits is taken from the exit weights (every exit weight
    is w0 * albedo^k, equal to 1e-3 at albedo 0.9999)."""
    steps, events, photons = scal[14], scal[9], scal[10]
    exits = photons - scal[11] - scal[12]
    faces = scal[0:6]
    imaged = exits * (faces[1] + faces[5]) / max(faces.sum(), 1e-300)
    return (unit_slots("step") * steps + unit_slots("interaction_hg" if hg else "interaction") * events
            + unit_slots("boundary") * (steps - events)
            + unit_slots("imaged_exit") * imaged + unit_slots("other_exit") * (exits - imaged))


def host_cpu():
    """CPU model, logical CPUs, CPUs this process may run on, and the share of
    them the benchmark uses: OMP_NUM_THREADS when set (a shared host may allot each
    GPU a fixed share of its cores), else every CPU in the affinity set."""
    try:
        model = open("/proc/cpuinfo").read().split("model name")[1].split("\n")[0].strip(" :\t")
    except Exception:
        model = "unknown"
    total = os.cpu_count() or 1
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else total
    share = int(os.environ.get("OMP_NUM_THREADS") or affinity)
    return model, total, affinity, max(1, min(affinity, share))


def cpu_baseline(w, target_s: float, gpu_value: float):
    """FP64 oracle on the host: one thread on a leading sample of the workload,
    then every thread of the CPU share on the whole workload (or on as much
    of it as fits in about target_s), both on the same seed and draws."""
    from oracle import walk as owalk
    model, total, affinity, threads = host_cpu()
    wk = owalk.Walk(w)
    n1 = 250_000
    r1 = wk.run(n_photons=n1, threads=1, chunks=1)
    if r1.seconds < 0.15 * target_s:
        n1 = int(min(w.n_photons, n1 * 0.15 * target_s / max(r1.seconds, 1e-3)))
        r1 = wk.run(n_photons=n1, threads=1, chunks=1)
    one = r1.scalars[9] / r1.seconds
    n = int(min(w.n_photons, one * threads * target_s / max(r1.scalars[9] / n1, 1e-9)))
    res = wk.run(n_photons=n, threads=threads)
    ev = res.scalars[9]
    allc = ev / res.seconds
    return {"value": allc, "unit": "scatter events/s", "cores": threads, "kind": "oracle",
            "sample": f"photons 0..{n - 1} of the same workload (same seed and draws), FP64 C oracle on "
                      f"{threads} host threads, {res.seconds:.1f} s, {ev:.3e} events; one thread on photons "
                      f"0..{n1 - 1}, {r1.seconds:.1f} s",
            "cpu_model": model, "cores_total": total, "cores_affinity": affinity,
            "one_core": {"value": one, "photons": n1, "seconds": r1.seconds},
            "all_cores": {"value": allc, "threads": threads, "photons": n, "seconds": res.seconds},
            "gpu_over_all_cores": gpu_value / allc, "gpu_over_one_core": gpu_value / one}


def _image_error(g, o, o_w2, n, max_w=1.0):
    """GPU image g against the oracle's o at matched seeds: largest |g - o| in
    units of the bin's Monte Carlo sigma (sigma^2 = sum w^2 - (sum w)^2 / N,
    from the oracle), the relative L2 norm of g - o, bins beyond 3 sigma, and
    bins the oracle leaves empty where the GPU holds more than 3 photon weights."""
    import numpy as np
    sig = np.sqrt(np.maximum(o_w2 - o * o / n, 0.0))
    d = np.abs(g - o)
    m = sig > 0
    return {"max_dev_over_sigma": float((d[m] / sig[m]).max()) if m.any() else 0.0,
            "rel_l2": float(np.linalg.norm(g - o) / max(float(np.linalg.norm(o)), 1e-300)),
            "bins_beyond_3sigma": int(np.sum(m & (d > 3.0 * sig))),
            "empty_oracle_bins_over_3w": int(np.sum(~m & (d > 3.0 * max_w)))}


def _energy_residual(s, n, w0):
    """Energy bookkeeping (Eq. 16): the weight that left, was absorbed or was
    capped, less roulette's net change, over the weight that entered, minus 1."""
    return float((float(s[0:6].sum()) + s[6] + s[8] - s[7]) / (n * w0) - 1.0)


def tally_error(mc, W, dev, args):
    """Tally error of the benchmarked GPU path against the FP64 oracle at
    matched seeds (same photon ids, Philox draws and tables' definitions), per
    workload: the parity workload in full, the paper-scale optical depths and
    the HG run, the differentiation workload (images, path-moment images and a
    gradient), three batched media and the heavy polydisperse workload, each
    on its leading photons."""
    import numpy as np
    import torch
    from oracle import mie as omie
    from oracle import walk as owalk
    from oracle import poly as opoly
    lg = tally_flags(mc, args)
    sub = 1_000_000
    rows = []

    def compare(label, w, g, o, fix=False):
        scale = 2.0 ** -32 if fix else 1.0
        gs = np.asarray(g["scalars"], dtype=np.float64)
        w0 = 1.0 - owalk.fresnel(w.src_dir[2], w.n_outside, w.particle.n_medium)
        maxw = max(1.0, w.roulette_w / w.roulette_p)
        row = {"config": label, "workload": w.name, "photons": w.n_photons,
               "side": _image_error(g["side"] * scale, o.side, o.side_w2, w.n_photons, maxw),
               "trans": _image_error(g["trans"] * scale, o.trans, o.trans_w2, w.n_photons, maxw),
               "energy_residual": {"gpu": _energy_residual(gs, w.n_photons, w0),
                                   "oracle": _energy_residual(o.scalars, w.n_photons, w0)},
               "events_rel_diff": float(abs(gs[9] - o.scalars[9]) / max(o.scalars[9], 1.0)),
               "absorbed_rel_diff": float(abs(gs[6] - o.scalars[6]) / max(abs(o.scalars[6]), 1e-300))}
        rows.append(row)
        return row

    def gpu(w, table, flags, g=None, moments=False, fix=False):
        _, med, src, geo, det, run = mc.args_from_workload(w, table, g=g, flags=flags)
        t = mc.Tally.alloc(det, dev, moments=moments, fix64=fix, log_photons=w.n_photons)
        mc.mc_simulate(med, src, geo, det, run, t)
        torch.cuda.synchronize()
        return dict(side=t.side.cpu().numpy().astype(np.float64), trans=t.trans.cpu().numpy().astype(np.float64),
                    scalars=t.scalars.cpu().numpy(), tally=t, med=med, geo=geo, det=det)

    # The parity workload in full.
    w = W.TINY
    tab = mc.mie_table_build(mc.args_from_workload(w)[0], dev)
    compare("parity tau=1 1e5", w, gpu(w, tab, lg), owalk.Walk(w).run())
    # Paper scale: each optical depth and the HG run, leading 1e6 photons.
    for tau in W.PAPER_TAUS:
        w = W.paper_scale(tau).replace(n_photons=sub)
        tab = mc.mie_table_build(mc.args_from_workload(w)[0], dev)
        compare(f"paper tau={tau:g} mie", w, gpu(w, tab, lg), owalk.Walk(w).run())
    w = W.paper_scale(4.0, phase=W.PHASE_HG).replace(n_photons=sub)
    tab = mc.mie_table_build(mc.args_from_workload(w)[0], dev)
    compare("paper tau=4 hg", w, gpu(w, tab, lg, g=tab.g),
            owalk.Walk(w, g=omie.table_from_workload(w).g).run())
    # Differentiation workload: images, path moments and the gradient of a
    # fixed random linear loss against the oracle's per-photon records.
    w = W.DIFF.replace(n_photons=sub)
    tab = mc.mie_table_build(mc.args_from_workload(w)[0], dev)
    g = gpu(w, tab, lg | mc.MC_MOMENTS, moments=True)
    o = owalk.Walk(w).run(records=True)
    row = compare("differentiation tau=4", w, g, o)
    n = w.side_px
    sel = (o.rec("face") == 1) & (o.rec("cause") == 0)
    r_ = np.clip(np.floor(o.rec("py")[sel] / w.size_mm[1] * n).astype(int), 0, n - 1)
    c_ = np.clip(np.floor(o.rec("pz")[sel] / w.size_mm[2] * n).astype(int), 0, n - 1)
    wk = np.zeros((n, n)); wl = np.zeros((n, n))
    np.add.at(wk, (r_, c_), o.rec("w")[sel] * o.rec("k")[sel])
    np.add.at(wl, (r_, c_), o.rec("w")[sel] * o.rec("L")[sel])
    gk, gl = g["tally"].side_wk.cpu().numpy(), g["tally"].side_wl.cpu().numpy()
    row["moments_rel_l2"] = {"sum_wk": float(np.linalg.norm(gk - wk) / np.linalg.norm(wk)),
                             "sum_wl": float(np.linalg.norm(gl - wl) / np.linalg.norm(wl))}
    gimg = np.random.default_rng(5).normal(size=(n, n))
    d_ms, d_ma, _ = mc.mc_grad(g["med"], g["geo"], g["det"], g["tally"], torch.tensor(gimg, device=dev))
    mu_s = w.albedo * w.tau / w.size_mm[2]
    term_s = gimg[r_, c_] * o.rec("w")[sel] * (o.rec("k")[sel] / mu_s - o.rec("L")[sel])
    term_a = -gimg[r_, c_] * o.rec("w")[sel] * o.rec("L")[sel]
    row["gradient_rel_diff"] = {"mu_sca": float(abs(d_ms - term_s.sum()) / np.abs(term_s).sum()),
                                "mu_abs": float(abs(d_ma - term_a.sum()) / np.abs(term_a).sum()),
                                "what": "|GPU - oracle| / sum of |per-photon terms| for a fixed random "
                                        "dLoss/dI (numpy seed 5)"}
    # Three batched media: the smallest, middle and largest particles.
    ws = W.batch_workloads(256)
    order = sorted(range(len(ws)), key=lambda i: ws[i].particle.diameter_um)
    pick = [ws[order[0]], ws[order[len(ws) // 2]], ws[order[-1]]]
    pick = [x.replace(n_photons=min(x.n_photons, sub)) for x in pick]
    tabs = [mc.mie_table_build(mc.args_from_workload(x)[0], dev) for x in pick]
    _, _, src, geo, det, run = mc.args_from_workload(pick[0])
    tb = mc.Tally.alloc_batch(det, len(pick), dev)
    mc.mc_simulate_batch([mc.batch_item(x, t) for x, t in zip(pick, tabs)], pick[0].n_cdf, src, geo, det, run, tb)
    torch.cuda.synchronize()
    for i, x in enumerate(pick):
        gi = dict(side=tb.side[i].cpu().numpy(), trans=tb.trans[i].cpu().numpy(), scalars=tb.scalars[i].cpu().numpy())
        compare(f"batch medium {x.instance} d={x.particle.diameter_um:.2f}um tau={x.tau:.2f} "
                f"albedo={x.albedo:.4f}", x, gi, owalk.Walk(x).run())
    # Heavy polydisperse workload, leading 1e6 photons, int64 images.
    w = W.HEAVY.replace(n_photons=sub)
    tab = mc.table_for_workload(w, dev)
    compare("heavy polydisperse tau=16", w, gpu(w, tab, lg | mc.MC_FIX64, fix=True),
            owalk.Walk(w, opoly.poly_table_from_workload(w)).run(), fix=True)
    return rows


def oracle_leg(mc, W, w, dev, args, gpu_value):
    """The part of the benchmark that runs the oracle: its timing on the host
    and the tally error of the GPU path against it."""
    log("bench: timing the oracle on the host")
    base = cpu_baseline(w, args.cpu_seconds, gpu_value)
    err = None
    if not args.no_tally_error:
        log("bench: tally error against the oracle")
        t0 = time.perf_counter()
        err = tally_error(mc, W, dev, args)
        log(f"bench: tally error done in {time.perf_counter() - t0:.1f} s")
    return base, err


def sweep_timing(mc, W, dev, args):
    """The paper-scale workload at its other optical depths and the HG run on
    the headline's seeds: scatter events/s and the census fraction of each,
    mc_simulate timed with HIP events on the launch stream."""
    import torch
    out = []
    for tau, phase in [(t, W.PHASE_MIE) for t in W.PAPER_TAUS if t != 4.0] + [(4.0, W.PHASE_HG)]:
        w = W.paper_scale(tau, phase=phase)
        table = mc.mie_table_build(mc.args_from_workload(w)[0], dev)
        g = table.g if phase == W.PHASE_HG else None
        _, med, src, geo, det, run = mc.args_from_workload(w, table, g=g, flags=tally_flags(mc, args))
        t = mc.Tally.alloc(det, dev, log_photons=w.n_photons)
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        wev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        run.time_walk(*wev)
        run.time_sim(*ev)
        for _ in range(3):
            mc.mc_simulate(med, src, geo, det, run, t)
        ms, wms = [], []
        for _ in range(max(3, args.steps // 2)):
            mc.mc_simulate(med, src, geo, det, run, t)
            torch.cuda.synchronize()
            ms.append(ev[0].elapsed_time(ev[1]))
            wms.append(wev[0].elapsed_time(wev[1]))
        s = t.scalars.cpu().numpy()
        sim_s = sum(ms) / len(ms) * 1e-3
        walk_s = sum(wms) / len(wms) * 1e-3
        slots = census_slots(s, phase == W.PHASE_HG)
        out.append({"workload": w.name, "tau": tau, "phase": "mie" if phase == W.PHASE_MIE else "hg",
                    "photons": w.n_photons, "events_per_photon": float(s[9] / s[10]),
                    "steps_per_photon": float(s[14] / s[10]), "mc_simulate_ms": sim_s * 1e3,
                    "walk_kernel_ms": walk_s * 1e3, "events_per_s": float(s[9]) / sim_s,
                    "frac": slots / walk_s / PEAK_SLOTS_PER_S,
                    "frac_mc_simulate": slots / sim_s / PEAK_SLOTS_PER_S})
    return out


def adjoint_timing(mc, w, dev, args):
    """Wall-clock of forward-only and forward + adjoint walks of `w` (table
    built once), each launch followed by a wait, as an optimiser step would."""
    import torch
    spec = mc.args_from_workload(w)[0]
    table = mc.mie_table_build(spec, dev)
    g_hg = table.g if w.phase == mc.MC_PHASE_HG else None
    kw = dict(g=g_hg, block_size=args.block_size, grid_blocks=args.grid_blocks)
    lg = tally_flags(mc, args)
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=lg, **kw)
    _, med_a, _, _, det_a, _ = mc.args_from_workload(w, table, flags=lg | mc.MC_MOMENTS, **kw)
    _, med_p, _, _, det_p, _ = mc.args_from_workload(w, table, flags=lg | mc.MC_MOMENTS | mc.MC_MOMENTS_PIXEL2,
                                                     **kw)
    t_fwd = mc.Tally.alloc(det, dev, log_photons=w.n_photons)
    t_adj = mc.Tally.alloc(det_a, dev, moments=True, log_photons=w.n_photons, workspace=t_fwd.workspace)
    t_pix = mc.Tally.alloc(det_p, dev, moments=True, pixel2=True, log_photons=w.n_photons,
                           workspace=t_fwd.workspace)
    gen = torch.Generator(device="cpu").manual_seed(7)
    dloss = torch.randn(w.side_px, w.side_px, generator=gen, dtype=torch.float64).to(dev)
    d2loss = torch.full_like(dloss, 2.0)

    def fwd():
        mc.mc_simulate(med, src, geo, det, run, t_fwd)
        torch.cuda.synchronize()

    def adj():
        mc.mc_simulate(med_a, src, geo, det_a, run, t_adj)
        return mc.mc_grad(med_a, geo, det_a, t_adj, dloss, d2loss_uniform=2.0)

    def adj_pixel():
        mc.mc_simulate(med_p, src, geo, det_p, run, t_pix)
        return mc.mc_grad(med_p, geo, det_p, t_pix, dloss, d2loss)

    def clock(fn):
        fn()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = fn()
        return (time.perf_counter() - t0) / args.steps * 1e3, out

    fwd_ms, _ = clock(fwd)
    adj_ms, grad = clock(adj)
    pix_ms, _ = clock(adj_pixel)
    return {"ratio": adj_ms / fwd_ms, "fwd_ms": fwd_ms, "fwd_adjoint_ms": adj_ms,
            "ratio_pixel_hessian": pix_ms / fwd_ms, "fwd_adjoint_pixel_hessian_ms": pix_ms,
            "grad_mu_sca_mu_abs_c": list(grad),
            "what": "fwd = mc_simulate (images, scalars); fwd+adjoint = mc_simulate with MC_MOMENTS "
                    "(side images of sum w k and sum w L, image-wide sums of w^2, w^2 k, w^2 L), then "
                    "mc_grad with dLoss/dI and a uniform d2Loss/dI2 = 2 (L2 loss); the pixel-Hessian "
                    "variant adds the per-pixel w^2 k and w^2 L images (MC_MOMENTS_PIXEL2)"}


def batch_timing(mc, W, dev, args):
    """Batched launch of the 256 sampled media against each medium run alone."""
    import torch
    ws = W.batch_workloads(256)
    tables = [mc.mie_table_build(mc.args_from_workload(w)[0], dev) for w in ws]
    _, _, src, geo, det, run = mc.args_from_workload(ws[0], flags=tally_flags(mc, args))
    items = [mc.batch_item(w, t) for w, t in zip(ws, tables)]
    tal = mc.Tally.alloc_batch(det, len(ws), dev, log_photons=sum(w.n_photons for w in ws))
    t0 = time.perf_counter()
    blk, chk, best, table = mc.mc_autotune_batch(items, ws[0].n_cdf, src, geo, det, run, tal, 1.0 / 16)
    tune_s = time.perf_counter() - t0
    run.block_size, run.chunk = blk, chk
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    mc.mc_simulate_batch(items, ws[0].n_cdf, src, geo, det, run, tal)
    ms = []
    for _ in range(max(1, args.steps)):
        ev[0].record()
        mc.mc_simulate_batch(items, ws[0].n_cdf, src, geo, det, run, tal)
        ev[1].record()
        torch.cuda.synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    scal = tal.scalars.cpu().numpy()
    events = float(scal[:, 9].sum())
    batch_ms = sorted(ms)[len(ms) // 2]
    # Every medium alone (default launch shape, the same tally path), timed
    # the same way.
    single = []
    for w, t in zip(ws, tables):
        _, med, s1, g1, d1, r1 = mc.args_from_workload(w, t, flags=tally_flags(mc, args))
        one = mc.Tally.alloc(d1, dev, log_photons=w.n_photons)
        mc.mc_simulate(med, s1, g1, d1, r1, one)
        ev[0].record()
        mc.mc_simulate(med, s1, g1, d1, r1, one)
        ev[1].record()
        torch.cuda.synchronize()
        t_ms = ev[0].elapsed_time(ev[1])
        single.append((float(one.scalars[9]) / (t_ms * 1e-3), t_ms))
    best_single = max(r for r, _ in single)
    return {"media": len(ws), "photons": int(sum(w.n_photons for w in ws)), "events": events,
            "tally": "atomic" if args.atomic_tally else "exit log",
            "batch_ms": batch_ms, "events_per_s": events / (batch_ms * 1e-3),
            "best_single_events_per_s": best_single,
            "ratio_to_best_single": events / (batch_ms * 1e-3) / best_single,
            "sum_of_single_ms": float(sum(m for _, m in single)),
            "autotune": {"block_size": blk, "chunk": chk, "sample_ms": best, "seconds": tune_s,
                         "candidates_ms": {f"{b}x{c}": v for (b, c), v in table.items()}}}


def heavy_timing(mc, W, dev, args):
    """The polydisperse tau = 16 workload: table, forward, forward + adjoint."""
    import torch
    w = W.HEAVY
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    table = mc.table_for_workload(w, dev)
    table_ms = (time.perf_counter() - t0) * 1e3
    lg = tally_flags(mc, args)
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=mc.MC_FIX64 | lg)
    _, med_a, _, _, det_a, _ = mc.args_from_workload(w, table, flags=mc.MC_FIX64 | mc.MC_MOMENTS | lg)
    t_f = mc.Tally.alloc(det, dev, fix64=True, log_photons=w.n_photons)
    t_a = mc.Tally.alloc(det_a, dev, fix64=True, moments=True, log_photons=w.n_photons, workspace=t_f.workspace)
    dloss = torch.ones((w.side_px, w.side_px), dtype=torch.float64, device=dev)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def clock(fn, reps=2):
        fn()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            out.append((time.perf_counter() - t) * 1e3)
        return min(out)

    def fwd():
        ev[0].record()
        mc.mc_simulate(med, src, geo, det, run, t_f)
        ev[1].record()

    def adj():
        mc.mc_simulate(med_a, src, geo, det_a, run, t_a)
        mc.mc_grad(med_a, geo, det_a, t_a, dloss, d2loss_uniform=2.0)

    fwd_ms = clock(fwd)
    kernel_ms = ev[0].elapsed_time(ev[1])
    adj_ms = clock(adj)
    s = t_f.scalars.cpu().numpy()
    return {"workload": w.name, "photons": w.n_photons, "tau": w.tau, "bins": w.particle.n_bins,
            "images": [w.side_px, w.trans_px], "events": float(s[9]),
            "events_per_photon": float(s[9] / s[10]), "table_ms": table_ms, "fwd_ms": fwd_ms,
            "mc_simulate_ms": kernel_ms, "events_per_s": float(s[9]) / (kernel_ms * 1e-3),
            "fwd_adjoint_ms": adj_ms, "adjoint_ratio": adj_ms / fwd_ms}


def analysis_timing(mc, W, dev, args):
    """Tables 3 and 4's measures between simulated images, per optical depth."""
    import torch
    rows = []
    metric_ms = []
    for od in W.ANALYSIS_ODS:
        wm = W.analysis_workload(od)
        table = mc.mie_table_build(mc.args_from_workload(wm)[0], dev)
        imgs = {}
        ws = None
        for name, w, g in (("mie", wm, None), ("ref", wm.replace(seed=W.ANALYSIS_REF_SEED), None),
                           ("mie2", wm.replace(seed=W.ANALYSIS_REF_SEED + 1), None),
                           ("hg", wm.replace(phase=W.PHASE_HG), table.g)):
            _, med, src, geo, det, run = mc.args_from_workload(w, table, g=g, flags=tally_flags(mc, args))
            t = mc.Tally.alloc(det, dev, log_photons=w.n_photons, workspace=ws)
            ws = t.workspace
            mc.mc_simulate(med, src, geo, det, run, t)
            imgs[name] = t.side
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m_mie = mc.image_metrics(imgs["mie"], imgs["ref"], imgs["hg"])
        metric_ms.append((time.perf_counter() - t0) * 1e3)
        m_hg = mc.image_metrics(imgs["hg"], imgs["ref"])
        # Noise level of the zone errors: two independent Mie runs differ from
        # the Mie reference by noise alone (shot noise, and the rescaling by a
        # noisy brightest pixel), so their zone errors are what noise gives at
        # this photon count.  HG's difference from Mie counts as resolved in a
        # zone only where its error is over twice the larger of the two.
        m_mie2 = mc.image_metrics(imgs["mie2"], imgs["ref"])
        noise = [max(a, b) for a, b in zip(m_mie["zone_rmse"], m_mie2["zone_rmse"])]
        resolved = [h > 2.0 * n for h, n in zip(m_hg["zone_rmse"], noise)]
        rows.append({"od": od,
                     "rmse": {"hg": m_hg["rmse"], "mie": m_mie["rmse"], "mie2": m_mie2["rmse"]},
                     "r": {"hg": m_hg["r"], "mie": m_mie["r"], "mie2": m_mie2["r"]},
                     "zone_rmse": {"hg": m_hg["zone_rmse"], "mie": m_mie["zone_rmse"],
                                   "mie2": m_mie2["zone_rmse"]},
                     "zone_noise": noise, "zone_resolved": resolved,
                     "radial_r": {"hg": m_hg["radial_r"], "mie": m_mie["radial_r"]},
                     "mie_better": m_mie["better"]})
    return {"images": "side, 512 x 512, 1e8 photons, beam radius 1.25 mm; reference: Mie, seed "
                      f"{W.ANALYSIS_REF_SEED}; mie2: a second Mie run, seed {W.ANALYSIS_REF_SEED + 1}, "
                      "against the same reference; zone_noise: the larger Mie zone error (noise alone); "
                      "zone_resolved: HG's zone error over twice that (mie_better, the paper's share of "
                      "annuli, reports noise where the zones are not resolved)",
            "per_od": rows, "metrics_ms": sorted(metric_ms)[len(metric_ms) // 2]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tau", type=float, default=4.0)
    ap.add_argument("--photons", type=int, default=100_000_000)
    ap.add_argument("--phase", choices=("mie", "hg"), default="mie")
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-heavy", action="store_true")
    ap.add_argument("--no-analysis", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the other optical depths and the HG run")
    ap.add_argument("--no-tally-error", action="store_true", help="skip the tally error against the oracle")
    ap.add_argument("--atomic-tally", action="store_true",
                    help="tally image exits with global atomics instead of the exit log")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the walk would shard by photon range across GPUs, but this library runs on a single device.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2507_23189_amd as mc
    import workloads as W

    phase = W.PHASE_MIE if args.phase == "mie" else W.PHASE_HG
    w = W.paper_scale(args.tau, phase=phase, n_photons=args.photons)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    spec, *_ = mc.args_from_workload(w)
    stream = torch.cuda.current_stream()

    flags = tally_flags(mc, args)
    det_probe = mc.args_from_workload(w, flags=flags)[4]
    tallies = [mc.Tally.alloc(det_probe, dev, log_photons=w.n_photons)]
    tallies += [mc.Tally.alloc(det_probe, dev, log_photons=w.n_photons, workspace=tallies[0].workspace)
                for _ in range(args.warmup + args.steps - 1)]
    # Per step: HIP events that the library sets to the start and end of the
    # walk kernel and, on every fourth timed step, to the start of
    # mc_simulate's first kernel and the end of its last (init, walk, log
    # binning, finalize).  They ride on the kernels' dispatches; each pair
    # still costs the device a few microseconds per step (about 3 us for the
    # walk's, 8 us for the whole call's), hence the sampling of the second.
    # Each event is created (recorded once) here, outside the timed steps.
    sim_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.warmup + args.steps)]
    sim_timed = set(range(args.warmup, args.warmup + args.steps, 4))
    walk_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.warmup + args.steps)]
    for pair in sim_ev + walk_ev:
        for e in pair:
            e.record(stream)
    torch.cuda.synchronize()

    # One step = the table build (device) followed by the walk on the same
    # stream.  With the Mie phase the table is enqueued without a host wait, so
    # steps pipeline; the HG step needs g on the host and waits for the table.
    inv_cdf = torch.empty(w.n_cdf, dtype=torch.float32, device=dev)
    result = torch.empty(4, dtype=torch.float64, device=dev)
    table_work = torch.empty(w.n_angles, dtype=torch.float64, device=dev)
    g_hg = mc.mie_table_build(spec, dev).g if phase == W.PHASE_HG else None

    def step(i):
        if phase == W.PHASE_MIE:
            table = mc.mie_table_enqueue(spec, dev, inv_cdf=inv_cdf, result=result, work=table_work)
        else:
            table = mc.mie_table_build(spec, dev)
        _, med, src, geo, det, run = mc.args_from_workload(w, table, g=g_hg, flags=flags,
                                                           block_size=args.block_size, grid_blocks=args.grid_blocks)
        run.time_walk(*walk_ev[i])
        run.time_sim(*(sim_ev[i] if i in sim_timed else (None, None)))
        mc.mc_simulate(med, src, geo, det, run, tallies[i])
        return table

    log(f"bench: workload {w.name}, warmup {args.warmup}, steps {args.steps}")
    keep = []
    for i in range(args.warmup):
        keep.append(step(i))
    torch.cuda.synchronize()
    log("bench: warmup done")
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        keep.append(step(i))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("bench: timed steps done")
    sweep = None if args.no_sweep else sweep_timing(mc, W, dev, args)
    log("bench: optical-depth sweep done")
    adjoint = adjoint_timing(mc, w, dev, args)
    log("bench: adjoint timing done")
    batch = None if args.no_batch else batch_timing(mc, W, dev, args)
    log("bench: batch timing done")
    heavy = None if args.no_heavy else heavy_timing(mc, W, dev, args)
    log("bench: heavy timing done")
    analysis = None if args.no_analysis else analysis_timing(mc, W, dev, args)
    log("bench: analysis done")

    scal = [t.scalars.cpu().numpy() for t in tallies[args.warmup:]]
    events = float(sum(s[9] for s in scal))
    photons = float(sum(s[10] for s in scal))
    elapsed = t1 - t0
    timed = range(args.warmup, args.warmup + args.steps)
    walk_avg_s = sum(walk_ev[i][0].elapsed_time(walk_ev[i][1]) for i in timed) / args.steps * 1e-3
    sim_avg_s = sum(sim_ev[i][0].elapsed_time(sim_ev[i][1]) for i in sim_timed) / len(sim_timed) * 1e-3
    slots = census_slots(scal[-1])
    achieved = slots / walk_avg_s
    s_last = scal[-1]

    out = {
        "metric": METRIC,
        "value": events / elapsed,
        "unit": "scatter events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "tau": w.tau, "photons": w.n_photons, "phase": args.phase,
                   "particle": "polystyrene d=5um n=1.59 in water n=1.33, lambda 532 nm",
                   "cuboid_mm": list(w.size_mm), "n_cdf": w.n_cdf, "images": [w.side_px, w.trans_px],
                   "seed": w.seed, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_SLOTS_PER_S / 1e12,
                     "unit": "Tslot/s", "frac": achieved / PEAK_SLOTS_PER_S,
                     "traffic": measured_traffic(args) if (args.tau == 4.0 and args.photons == 100_000_000
                                                           and phase == W.PHASE_MIE) else None,
                     "kernel": "walk_kernel (the photon walk; HIP events the library attaches to its dispatch)",
                     "tally": "atomic" if args.atomic_tally else "exit log",
                     "kernel_ms": walk_avg_s * 1e3, "slots_per_launch": slots,
                     "mc_simulate_ms": sim_avg_s * 1e3,
                     "frac_mc_simulate": slots / sim_avg_s / PEAK_SLOTS_PER_S,
                     "mc_simulate": ("init, walk_kernel, finalize" if args.atomic_tally else
                                     "init, walk_kernel, log_bin, finalize") +
                                    f" (every fourth timed step, {len(sim_timed)} of {args.steps})"},
        "photons_per_s": photons / elapsed,
        "events_per_photon": s_last[9] / s_last[10],
        "steps_per_photon": s_last[14] / s_last[10],
        "adjoint_ratio": adjoint["ratio"],
        "adjoint": adjoint,
        "batch": batch,
        "heavy": heavy,
        "analysis": analysis,
        "sweep": sweep,
    }
    if batch is not None:
        batch["ratio_to_headline"] = batch["events_per_s"] / out["value"]
    if not args.no_cpu_baseline:
        base, err = oracle_leg(mc, W, w, dev, args, out["value"])
        out["cpu_baseline"] = base
        if not args.no_tally_error:
            out["tally_error"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
