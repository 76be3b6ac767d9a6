"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Bars: Philox words bit-exact; Mie coefficients, efficiencies and phase table
to FP64 rounding, inverse table to one FP32 ulp; per-photon trajectories
(face, cause, scatter count, end position, direction, weight, path length)
within 1e-4 for at least 99.9 % of photons; every image bin within 3 sigma of
Monte Carlo noise at matched seeds; launch-shape and photon-range invariance
bit-exact on records."""
import math

import numpy as np
import pytest

import workloads as W
from _helpers import assert_matched_scalars, gpu_run, image_within_3sigma, oracle_rec, trajectory_match
from oracle import mie, philox
from oracle import walk as owalk

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def mc():
    import paper_2507_23189_amd as m
    m.lib()
    return m


# ---------------------------------------------------------------- Philox

def test_philox_words_bit_exact(mc, cuda_device):
    torch = _torch()
    rng = np.random.default_rng(11)
    ids = np.concatenate([np.arange(5, dtype=np.uint64), rng.integers(0, 2**40, 27, dtype=np.uint64),
                          np.array([2**32 - 1, 2**32, 2**63 + 7], dtype=np.uint64)])
    for seed, inst, step0, nst in [(1234, 0, 0, 9), (2**40 + 99, 3, 1 << 20, 4), (0, 0, 2**32 - 3, 3)]:
        ids_t = torch.tensor(ids.view(np.int64), device=cuda_device)
        out = torch.empty(len(ids) * nst * 4, dtype=torch.int32, device=cuda_device)
        mc.mc_philox_blocks(seed, inst, ids_t, step0, nst, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32).reshape(len(ids), nst, 4)
        for i, pid in enumerate(ids):
            for s in range(nst):
                ref = philox.step_block(seed, int(pid), step0 + s, instance=inst)
                assert tuple(int(v) for v in got[i, s]) == ref, (seed, pid, step0 + s)


# ------------------------------------------------------------- Mie table

TABLE_CASES = [
    dict(d=5.0, m_re=1.59, m_im=0.0, n_med=1.33, lam=532.0, na=1801, nc=4096),      # tiny workload
    dict(d=5.0, m_re=1.59, m_im=0.0, n_med=1.33, lam=532.0, na=1801, nc=16384),     # paper scale
    dict(d=5.0, m_re=1.594, m_im=0.00033, n_med=1.333, lam=532.0, na=3001, nc=4096),  # printed indices, 3000-point grid
    dict(d=0.5, m_re=1.59, m_im=0.0, n_med=1.33, lam=532.0, na=1801, nc=4096),      # x ~ 3.9
    dict(d=10.0, m_re=1.59, m_im=0.0, n_med=1.33, lam=532.0, na=1801, nc=2),        # x ~ 78.5, smallest table
    dict(d=0.02, m_re=1.5, m_im=0.1, n_med=1.0, lam=532.0, na=3, nc=5),             # Rayleigh, smallest grid
    dict(d=120.0, m_re=1.59, m_im=0.0, n_med=1.33, lam=532.0, na=3001, nc=16384),   # x ~ 942: 984 of the 1024 terms
    # |m| x ~ 1.6e-5: the downward D_n steps have |k| = n / |mx| up to 1.3e6, so the
    # homogeneous recurrence's power-of-two rescaling is what keeps P_n, Q_n finite.
    dict(d=0.02, m_re=1.33e-4, m_im=0.0, n_med=1.33, lam=532.0, na=181, nc=64),
    dict(d=0.05, m_re=2e-3, m_im=1e-3, n_med=1.0, lam=532.0, na=181, nc=64),     # absorbing, |m| x ~ 6.6e-4
    dict(d=2.0, m_re=0.05, m_im=0.0, n_med=1.0, lam=532.0, na=1801, nc=4096),    # m < 1 at x ~ 11.8
]


@pytest.mark.parametrize("case", TABLE_CASES)
def test_mie_table_parity(mc, cuda_device, case):
    c = case
    spec = mc.MieSpec(n_medium=c["n_med"], m_re=c["m_re"], m_im=c["m_im"], diameter_um=c["d"],
                      wavelength_nm=c["lam"], n_angles=c["na"], n_cdf=c["nc"])
    t = mc.mie_table_build(spec, cuda_device, phase=True, cdf=True, coef=True)
    o = mie.build_table(c["d"], c["m_re"], c["m_im"], c["n_med"], c["lam"], c["na"], c["nc"])
    assert t.x == pytest.approx(o.x, rel=1e-15)
    assert t.n_terms == len(o.a)
    coef = t.coef.cpu().numpy()
    ga = coef[:, 0] + 1j * coef[:, 1]
    gb = coef[:, 2] + 1j * coef[:, 3]
    # Two FP64 evaluations of the same recurrence agree to ~1e-14 of the largest
    # coefficient, except on a sharp resonance (a term whose |b_n| swings by ~1
    # over dx ~ 1e-3), where rounding is amplified by the term's conditioning;
    # 1e-11 covers that without hiding a wrong term (those are O(1) off).
    big = max(np.abs(o.a).max(), np.abs(o.b).max())
    assert np.abs(ga - o.a).max() <= 1e-11 * big
    assert np.abs(gb - o.b).max() <= 1e-11 * big
    for name in ("q_ext", "q_sca", "g", "sigma_ext_mm2"):
        assert getattr(t, name) == pytest.approx(getattr(o, name), rel=1e-11, abs=1e-300)
    assert t.q_abs == pytest.approx(o.q_abs, abs=1e-11 * o.q_ext)
    gP = t.phase.cpu().numpy()
    np.testing.assert_allclose(gP, o.P, rtol=1e-10, atol=1e-14 * o.P.max())
    # The CDF is a normalised sum of P with positive weights, so a relative
    # error eps in every P moves it by at most 2 eps, plus the sums' own
    # rounding (below 1e-13).  P agrees to ~1e-15 at small x and to ~1e-13
    # near the 1024-term limit (the series' conditioning), so a fixed 1e-12
    # holds for every case.
    np.testing.assert_allclose(t.cdf.cpu().numpy(), o.F, rtol=0, atol=1e-12)
    inv = t.inv_cdf.cpu().numpy()
    ref32 = o.v.astype(np.float32)
    ulp = np.spacing(np.abs(ref32)).astype(np.float64)
    assert np.all(np.abs(inv.astype(np.float64) - ref32.astype(np.float64)) <= ulp + 1e-30)


def test_mie_table_enqueue_matches_build(mc, cuda_device):
    torch = _torch()
    w = W.HEADLINE
    spec, *_ = mc.args_from_workload(w)
    t = mc.mie_table_build(spec, cuda_device)
    e = mc.mie_table_enqueue(spec, cuda_device)
    torch.cuda.synchronize()
    assert math.isnan(e.q_ext) and e.n_terms == t.n_terms and e.x == t.x
    torch.testing.assert_close(e.inv_cdf, t.inv_cdf, rtol=0, atol=0)
    r = e.result.cpu().numpy()
    assert (r[0], r[1], r[2], r[3]) == (t.q_ext, t.q_sca, t.g, t.n_terms)


# ------------------------------------------------------- trajectories, images

def _oracle(w, records=True, ids=None, g=None):
    return owalk.Walk(w, g=g).run(records=records, ids=ids)


@pytest.mark.parametrize("phase", [W.PHASE_MIE, W.PHASE_HG])
def test_tiny_workload_trajectories_and_images(mc, cuda_device, phase):
    w = W.TINY.replace(phase=phase)
    g = gpu_run(w, records=True)
    o = _oracle(w, g=None if phase == W.PHASE_MIE else mie.table_from_workload(w).g)
    ok = trajectory_match(g["rec"], oracle_rec(o), box=10.0)
    assert ok.mean() >= 0.999, (ok.mean(), np.flatnonzero(~ok)[:10])
    assert image_within_3sigma(g["side"], o.side, o.side_w2, w.n_photons).all()
    assert image_within_3sigma(g["trans"], o.trans, o.trans_w2, w.n_photons).all()
    gs, os_ = g["scalars"], o.scalars
    assert gs[10] == w.n_photons
    # Over the photons both sides walked alike the totals agree to FP32 rounding.
    assert_matched_scalars(gs, g["rec"], os_, oracle_rec(o), ok)
    # Squared-weight images against the oracle too.
    assert image_within_3sigma(g["side_w2"], o.side_w2, o.side_w2, w.n_photons).all()


@pytest.mark.parametrize("g", [-0.5, 0.0, 0.99])
def test_hg_trajectories_across_asymmetry(mc, cuda_device, g):
    """Eq. 11 sampling at back-scattering, isotropic and strongly forward g."""
    w = W.TINY.replace(phase=W.PHASE_HG, tau=3.0, n_photons=20000)
    gr = gpu_run(w, records=True, g=g)
    o = _oracle(w, g=g)
    ok = trajectory_match(gr["rec"], oracle_rec(o), box=10.0)
    assert ok.mean() >= 0.999, (g, ok.mean())
    assert image_within_3sigma(gr["trans"], o.trans, o.trans_w2, w.n_photons).all()


@pytest.mark.parametrize("kw", [
    dict(tau=4.0, n_cdf=16384, side_px=512, trans_px=512, n_photons=20000),
    dict(tau=8.0, n_photons=20000, albedo=0.9),
    dict(tau=6.0, albedo=0.5, roulette_w=0.01, n_photons=20000),          # roulette fires often
    dict(tau=2.0, n_outside=1.33, n_photons=20000),                       # index-matched walls
    dict(tau=3.0, n_photons=12345, side_px=3, trans_px=5, size_mm=(4.0, 7.0, 10.0),
         src_pos_mm=(1.0, 2.0, 0.0), src_dir=(0.3, -0.2, 0.9)),            # ragged, oblique beam
    dict(tau=8.0, max_steps=4, n_photons=5000),                            # step cap
    dict(tau=2.0, n_photons=5000, src_pos_mm=(0.0, 0.0, 0.0), src_dir=(-0.0, 0.0, 1.0)),  # along an edge
    dict(tau=0.0, n_photons=5000, src_dir=(0.2, 0.1, 0.97)),              # no medium: walls only
    dict(tau=3.0, albedo=1.0, n_photons=10000),                           # no absorption
])
def test_trajectory_parity_variants(mc, cuda_device, kw):
    w = W.TINY.replace(**kw)
    g = gpu_run(w, records=True)
    o = _oracle(w)
    ok = trajectory_match(g["rec"], oracle_rec(o), box=max(w.size_mm))
    assert ok.mean() >= 0.999, (kw, ok.mean())
    assert_matched_scalars(g["scalars"], g["rec"], o.scalars, oracle_rec(o), ok)
    assert image_within_3sigma(g["side"], o.side, o.side_w2, w.n_photons, max_w=10.0).all()
    assert image_within_3sigma(g["trans"], o.trans, o.trans_w2, w.n_photons, max_w=10.0).all()


PAPER_SCALE = [(1.0, W.PHASE_MIE), (2.0, W.PHASE_MIE), (4.0, W.PHASE_MIE), (8.0, W.PHASE_MIE), (4.0, W.PHASE_HG)]


@pytest.mark.parametrize("tau,phase", PAPER_SCALE, ids=lambda v: str(v))
def test_full_size_sampled_trajectories(mc, cuda_device, tau, phase):
    """Every paper-scale workload (tau 1, 2, 4, 8 with the Mie table and the
    HG run with g = g_Mie; 1e8 photons, 16384-entry table, 512 x 512 images)
    at full size in the default launch shape: every 50 000th photon is
    recorded and replayed one by one in the oracle."""
    w = W.paper_scale(tau, phase=phase)
    stride = 50_000
    g = gpu_run(w, records=True, record_stride=stride, sigma=False)
    ids = np.arange(0, w.n_photons, stride, dtype=np.uint64)
    o = _oracle(w, ids=ids, g=None if phase == W.PHASE_MIE else mie.table_from_workload(w).g)
    ok = trajectory_match(g["rec"], oracle_rec(o), box=10.0)
    assert ok.mean() >= 0.999, ok.mean()
    s = g["scalars"]
    assert s[10] == w.n_photons
    # Energy bookkeeping at full size: start weight + roulette = exits + absorbed + capped.
    w0 = 1.0 - ((1.0 - 1.33) / 2.33) ** 2
    assert s[0:6].sum() + s[6] + s[8] == pytest.approx(w.n_photons * w0 + s[7], rel=1e-5)
    # Events per photon agree with the oracle's sample within 4 sigma.
    k = o.rec("k").astype(float)
    assert abs(s[9] / s[10] - k.mean()) <= 4 * k.std() / math.sqrt(len(k))


# ------------------------------------------------------------ invariances

def test_launch_shape_and_photon_ranges_are_invariant(mc, cuda_device):
    """Fixed-point tallies make every result independent of how photons are
    scheduled: other launch shapes give bit-identical records, images and
    scalars, and photon ranges accumulated into one MC_FIX64 tally equal the
    single run exactly."""
    torch = _torch()
    w = W.TINY.replace(tau=3.0, n_photons=30000)
    a = gpu_run(w, records=True)
    b = gpu_run(w, records=True, block_size=64, grid_blocks=7, table=a["table"])
    c = gpu_run(w, records=True, block_size=320, grid_blocks=3, table=a["table"])
    for other in (b, c):
        for k in a["rec"]:
            np.testing.assert_array_equal(a["rec"][k], other["rec"][k])
        for k in ("side", "trans", "side_w2", "trans_w2", "scalars"):
            np.testing.assert_array_equal(a[k], other[k])
    # Photon ranges accumulated into one fixed-point tally equal the single run.
    f = gpu_run(w, fix64=True, table=a["table"])
    p1 = gpu_run(w, fix64=True, n_photons=11111, table=a["table"])
    tal = p1["tally"]
    gpu_run(w, fix64=True, n_photons=w.n_photons - 11111, photon_offset=11111, table=a["table"], tally=tal,
            flags_extra=mc.MC_ACCUMULATE)
    torch.cuda.synchronize()
    for k in ("side", "trans", "side_w2", "trans_w2"):
        np.testing.assert_array_equal(getattr(tal, k).cpu().numpy(), f[k])
    np.testing.assert_allclose(tal.scalars.cpu().numpy()[:15], f["scalars"][:15], rtol=1e-15, atol=0)
    # Fixed-point images are the double images scaled by 2^32; the +x and +z
    # face totals are exactly the image sums.
    np.testing.assert_array_equal(f["side"].astype(np.float64) * 2.0**-32, a["side"])
    assert f["side"].sum() * 2.0**-32 == f["scalars"][1]
    assert f["trans"].sum() * 2.0**-32 == f["scalars"][5]


def test_full_chip_launches_are_bit_identical(mc, cuda_device):
    """Full-chip launches of the tau = 4 workload (16384-entry table in LDS,
    every CU busy): repeated runs and another block size give identical
    fixed-point images and scalars.  Each photon's walk depends only on its
    id, so any difference means a wave read shared state (the table, the
    scalar words, the cache) before the block had finished setting it up."""
    w = W.paper_scale(4.0)
    a = gpu_run(w, fix64=True, n_photons=4_000_000)
    runs = [gpu_run(w, fix64=True, n_photons=4_000_000, table=a["table"]) for _ in range(2)]
    runs.append(gpu_run(w, fix64=True, n_photons=4_000_000, table=a["table"], block_size=256))
    for other in runs:
        for k in ("side", "trans", "side_w2", "trans_w2", "scalars"):
            np.testing.assert_array_equal(a[k], other[k], err_msg=k)


@pytest.mark.parametrize("kw", [dict(), dict(albedo=0.8, roulette_w=0.5, roulette_p=0.2)],
                         ids=["default", "weights_above_one"])
def test_fixed_point_tallies_are_exact_sums_of_record_weights(mc, cuda_device, kw):
    """MC_FIX64 tallies hold, per pixel and per face, the sum of each exit
    weight rounded to nearest (ties to even) at 2^32 per unit, bit for bit:
    recomputed here from the per-photon records, with the pixel of each exit
    from its recorded position by the same FP32 floor(coord * (n / size)),
    n / size rounded once to FP32 as the library does.  The second case sets
    roulette to raise weights to up to 2.5, past the walk's shortcut for
    weights below 1."""
    w = W.TINY.replace(tau=3.0, n_photons=30000, side_px=97, trans_px=131, **kw)
    f = gpu_run(w, records=True, fix64=True)
    r = f["rec"]
    f32 = np.float32

    def q(x):
        return np.rint(np.asarray(x, dtype=np.float64) * 2.0**32).astype(np.int64)

    wf = r["w"].astype(f32)
    out = r["cause"] == 0
    for face, img, row_c, col_c, col_size, n in ((1, "side", "py", "pz", w.size_mm[2], w.side_px),
                                                 (5, "trans", "py", "px", w.size_mm[0], w.trans_px)):
        sel = out & (r["face"] == face)
        row = np.floor(r[row_c][sel].astype(f32) * f32(n / w.size_mm[1])).astype(np.int64).clip(0, n - 1)
        col = np.floor(r[col_c][sel].astype(f32) * f32(n / col_size)).astype(np.int64).clip(0, n - 1)
        for name, vals in ((img, q(wf[sel])), (img + "_w2", q(wf[sel] * wf[sel]))):
            expect = np.zeros(n * n, dtype=np.int64)
            np.add.at(expect, row * n + col, vals)
            np.testing.assert_array_equal(f[name].reshape(-1), expect, err_msg=name)
    s = f["scalars"]
    for face in range(6):
        assert s[face] == q(wf[out & (r["face"] == face)]).sum() * 2.0**-32, face
    assert s[6] == q(r["A"].astype(f32)).sum() * 2.0**-32


def test_zero_and_single_photon(mc, cuda_device):
    w = W.TINY
    z = gpu_run(w, n_photons=0, records=True)
    assert np.all(z["side"] == 0) and np.all(z["trans"] == 0) and np.all(z["scalars"][:15] == 0)
    one = gpu_run(w, n_photons=1, records=True)
    o = _oracle(w.replace(n_photons=1))
    assert trajectory_match(one["rec"], oracle_rec(o), box=10.0).all()
    assert one["scalars"][10] == 1


def test_gpu_physics_pins(mc, cuda_device):
    # Beer-Lambert ballistic fraction and the pure absorber on the HIP path.
    tau = 1.0
    w = W.TINY.replace(tau=tau, n_outside=1.33, n_photons=200000)
    g = gpu_run(w, records=True)
    ball = (g["rec"]["k"] == 0) & (g["rec"]["face"] == 5)
    p = math.exp(-tau)
    assert abs(ball.sum() - w.n_photons * p) <= 4 * math.sqrt(w.n_photons * p * (1 - p))
    wa = W.TINY.replace(tau=1.5, n_outside=1.33, albedo=0.0, roulette_w=0.0, n_photons=200000)
    ga = gpu_run(wa)
    assert ga["side"].sum() == 0.0
    p = math.exp(-1.5)
    assert abs(ga["trans"].sum() - wa.n_photons * p) <= 4 * math.sqrt(wa.n_photons * p * (1 - p))
    # HG sampling: mean cosine of the first scatter is g (single-scatter setup).
    big = 1e6
    wh = W.TINY.replace(size_mm=(big, big, big), src_pos_mm=(big / 2, big / 2, 0.0), tau=big, max_steps=1,
                        phase=W.PHASE_HG, n_photons=200000, roulette_w=0.0)
    gh = gpu_run(wh, records=True, g=0.8668)
    mu = gh["rec"]["dz"]
    assert abs(mu.mean() - 0.8668) <= 4 * mu.std() / math.sqrt(len(mu))


def test_medium_forms_give_the_same_walk(mc, cuda_device):
    """The optical-depth, coefficient and concentration forms of one medium
    (Eq. 1, Eq. 16, Eq. 17) give the same FP32 walk constants and hence the
    same tallies, bit for bit."""
    torch = _torch()
    w = W.TINY.replace(n_photons=20000, tau=2.0, albedo=0.75)
    spec, *_ = mc.args_from_workload(w)
    table = mc.mie_table_build(spec, cuda_device)
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=mc.MC_FIX64)
    lz = geo.size_mm[2]
    mu_ext = w.tau / lz
    forms = [med]
    m_mu = mc.Medium.from_buffer_copy(med)
    m_mu.input, m_mu.mu_sca, m_mu.mu_abs = mc.MC_MEDIUM_MU, 0.75 * mu_ext, 0.25 * mu_ext
    forms.append(m_mu)
    m_c = mc.Medium.from_buffer_copy(med)
    m_c.input, m_c.concentration_per_mm3 = mc.MC_MEDIUM_CONCENTRATION, 1.0e4
    m_c.sigma_sca_mm2, m_c.sigma_abs_mm2, m_c.mu_abs_host = 0.75 * mu_ext / 1.0e4, 0.0, 0.25 * mu_ext
    forms.append(m_c)
    consts = set()
    for m in forms:
        c = mc.mc_medium_coefficients(m, geo)
        consts.add((np.float32(-math.log(2.0) / c["mu_ext"]), np.float32(c["albedo"]), np.float32(1.0 - c["albedo"])))
    assert len(consts) == 1, consts
    outs = []
    for m in forms:
        t = mc.Tally.alloc(det, cuda_device, fix64=True)
        mc.mc_simulate(m, src, geo, det, run, t)
        torch.cuda.synchronize()
        outs.append(t)
    for t in outs[1:]:
        assert torch.equal(t.side, outs[0].side) and torch.equal(t.trans, outs[0].trans)
        assert torch.equal(t.scalars, outs[0].scalars)


def test_walk_kernel_timing_events(mc, cuda_device):
    """Events passed in the run are set to the walk kernel's start and end,
    and to the start and end of the call's kernels: the walk times less than
    the call's kernels, which time less than the host-recorded bracket, and
    the results do not change."""
    torch = _torch()
    w = W.TINY.replace(n_photons=200_000, tau=3.0)
    spec, *_ = mc.args_from_workload(w)
    table = mc.mie_table_build(spec, cuda_device)
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=mc.MC_FIX64)
    a = mc.Tally.alloc(det, cuda_device, fix64=True)
    mc.mc_simulate(med, src, geo, det, run, a)
    walk = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    whole = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    sim = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    run.time_walk(*walk)
    run.time_sim(*sim)
    b = mc.Tally.alloc(det, cuda_device, fix64=True)
    whole[0].record()
    mc.mc_simulate(med, src, geo, det, run, b)
    whole[1].record()
    torch.cuda.synchronize()
    t_walk, t_whole = walk[0].elapsed_time(walk[1]), whole[0].elapsed_time(whole[1])
    t_sim = sim[0].elapsed_time(sim[1])
    assert 0.0 < t_walk <= t_sim <= t_whole
    assert torch.equal(a.side, b.side) and torch.equal(a.scalars, b.scalars)
