"""Shared test helpers: run the HIP path and the oracle on the same workload
and compare them.  Imported by the test modules only."""
from __future__ import annotations

import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

IREC = ("face", "cause", "k", "steps")
FREC = ("px", "py", "pz", "dx", "dy", "dz", "w", "L", "A")


def gpu_run(w, *, table=None, records=False, record_stride=1, sigma=True, g=None, block_size=0,
            grid_blocks=0, n_photons=None, photon_offset=0, flags_extra=0, tally=None, table_kw=None,
            fix64=False):
    """Build the table (unless given) and run mc_simulate; return numpy results."""
    import torch
    import paper_2507_23189_amd as mc
    dev = torch.device("cuda:0")
    spec, *_ = mc.args_from_workload(w)
    if table is None:
        table = mc.mie_table_build(spec, dev, **(table_kw or {}))
    flags = (mc.MC_SIGMA if sigma else 0) | (mc.MC_RECORD if records else 0) | (mc.MC_FIX64 if fix64 else 0) \
        | flags_extra
    _, med, src, geo, det, run = mc.args_from_workload(w, table, g=g, flags=flags, record_stride=record_stride,
                                                       block_size=block_size, grid_blocks=grid_blocks,
                                                       n_photons=n_photons, photon_offset=photon_offset)
    n = run.n_photons
    rows = (n + record_stride - 1) // record_stride if records else 0
    if tally is None:
        tally = mc.Tally.alloc(det, dev, sigma=sigma, record_rows=rows, fix64=fix64)
    mc.mc_simulate(med, src, geo, det, run, tally)
    torch.cuda.synchronize()
    out = dict(side=tally.side.cpu().numpy(), trans=tally.trans.cpu().numpy(),
               scalars=tally.scalars.cpu().numpy(), table=table, tally=tally)
    if sigma:
        out["side_w2"] = tally.side_w2.cpu().numpy()
        out["trans_w2"] = tally.trans_w2.cpu().numpy()
    if records and tally.rec_i is not None:
        ri = tally.rec_i.cpu().numpy()
        rf = tally.rec_f.cpu().numpy().astype(np.float64)
        out["rec"] = {k: ri[i] for i, k in enumerate(IREC)}
        out["rec"].update({k: rf[i] for i, k in enumerate(FREC)})
    return out


def oracle_rec(res):
    return {k: res.rec(k) for k in IREC + FREC}


def trajectory_match(g, o, box):
    """Per-photon agreement: same face, cause and scatter count; position,
    direction, weight and path length within 1e-4 relative (floors: 1e-4 of
    the box for positions and path length, 1e-4 for directions)."""
    ok = (g["face"] == o["face"]) & (g["cause"] == o["cause"]) & (g["k"] == o["k"])
    for c in ("px", "py", "pz"):
        ok &= np.abs(g[c] - o[c]) <= 1e-4 * np.maximum(np.abs(o[c]), box)
    for c in ("dx", "dy", "dz"):
        ok &= np.abs(g[c] - o[c]) <= 1e-4
    ok &= np.abs(g["w"] - o["w"]) <= 1e-4 * np.abs(o["w"]) + 1e-12
    ok &= np.abs(g["L"] - o["L"]) <= 1e-4 * np.maximum(o["L"], box)
    return ok


def image_within_3sigma(img_g, img_o, w2_o, n_photons, max_w=1.0):
    """Every bin within 3 sigma of the oracle, sigma^2 = sum w^2 - (sum w)^2 / N;
    a bin the oracle leaves empty may hold at most 3 photon weights."""
    var = np.maximum(w2_o - img_o ** 2 / n_photons, 0.0)
    tol = 3.0 * np.sqrt(var)
    tol = np.where(img_o == 0.0, 3.0 * max_w, tol)
    return np.abs(img_g - img_o) <= tol + 1e-9 * np.abs(img_o)


def unmatched_totals(rec, bad):
    """Per-face exit weight, absorbed weight, scatter events, roulette kills,
    capped photons, wall reflections and steps of the photons flagged in
    `bad`, from one side's per-photon records (a photon's reflections are its
    steps less its interactions and its exit): subtracted from that side's
    scalar tallies, they leave the sums over the photons both sides walked
    alike."""
    out = np.zeros(15)
    exited = bad & (rec["cause"] == 0)
    for f in range(6):
        out[f] = np.sum(rec["w"][exited & (rec["face"] == f)], dtype=np.float64)
    out[6] = np.sum(rec["A"][bad], dtype=np.float64)
    out[9] = np.sum(rec["k"][bad].astype(np.float64))
    out[11] = np.sum(bad & (rec["cause"] == 1))
    out[12] = np.sum(bad & (rec["cause"] == 2))
    steps = rec["steps"][bad].astype(np.float64)
    out[13] = np.sum(steps - rec["k"][bad].astype(np.float64)) - np.sum(exited)
    out[14] = np.sum(steps)
    return out


def assert_matched_scalars(g_scal, g_rec, o_scal, o_rec, ok, rtol=1e-4):
    """Scalar tallies restricted to trajectory-matched photons: face totals
    and absorbed weight agree to rtol (FP32 transport against FP64); scatter
    events, roulette kills, capped photons, reflections and steps exactly
    (matched photons take the same path)."""
    gs = np.asarray(g_scal[:15], dtype=np.float64) - unmatched_totals(g_rec, ~ok)
    os_ = np.asarray(o_scal[:15], dtype=np.float64) - unmatched_totals(o_rec, ~ok)
    for i in list(range(7)):
        assert abs(gs[i] - os_[i]) <= rtol * abs(os_[i]) + 1e-9, (i, gs[i], os_[i])
    for i in (9, 11, 12, 13, 14):
        assert gs[i] == os_[i], (i, gs[i], os_[i])
