"""GPU checks of the perturbation Monte Carlo adjoint (mc_grad over the moment
tallies of mc_simulate with MC_MOMENTS): moments and gradients against the
oracle's per-photon records at matched seeds, against central finite
differences with common random numbers, and a small fit of the optical depth
to a lateral image through torch.autograd."""
import math

import numpy as np
import pytest

import workloads as W
from _helpers import FREC, IREC, gpu_run, oracle_rec, trajectory_match
from oracle import walk as owalk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import paper_2507_23189_amd as m
    m.lib()
    return m


def _oracle_moments(w, r):
    """Side-image moments sum w k, sum w L and sum (w k)^2 from the oracle's records."""
    ny = nx = w.side_px
    wk = np.zeros((ny, nx)); wl = np.zeros((ny, nx)); wk2 = np.zeros((ny, nx)); wl2 = np.zeros((ny, nx))
    sel = (r.rec("face") == 1) & (r.rec("cause") == 0)
    rows = np.clip(np.floor(r.rec("py")[sel] / w.size_mm[1] * ny).astype(int), 0, ny - 1)
    cols = np.clip(np.floor(r.rec("pz")[sel] / w.size_mm[2] * nx).astype(int), 0, nx - 1)
    a = r.rec("w")[sel] * r.rec("k")[sel]
    b = r.rec("w")[sel] * r.rec("L")[sel]
    np.add.at(wk, (rows, cols), a); np.add.at(wl, (rows, cols), b)
    np.add.at(wk2, (rows, cols), a * a); np.add.at(wl2, (rows, cols), b * b)
    return wk, wl, wk2, wl2, sel


def test_moments_and_gradient_match_oracle(mc, cuda_device):
    import torch
    w = W.TINY.replace(tau=4.0, n_photons=60000)
    # Moments need their buffers: allocate the tally with moments=True.
    spec, *_ = mc.args_from_workload(w)
    table = mc.mie_table_build(spec, cuda_device)
    _, med, src, geo, det, run = mc.args_from_workload(
        w, table, flags=mc.MC_MOMENTS | mc.MC_MOMENTS_PIXEL2 | mc.MC_RECORD)
    tal = mc.Tally.alloc(det, cuda_device, moments=True, pixel2=True, record_rows=w.n_photons)
    mc.mc_simulate(med, src, geo, det, run, tal)
    torch.cuda.synchronize()
    r = owalk.Walk(w).run(records=True)
    wk, wl, wk2, wl2, sel = _oracle_moments(w, r)
    gk, gl = tal.side_wk.cpu().numpy(), tal.side_wl.cpu().numpy()
    # Matched seeds: per pixel within 3 sigma of the moment's own MC noise.
    assert np.all(np.abs(gk - wk) <= 3 * np.sqrt(wk2) + 1e-9 + 3 * max(1.0, np.abs(wk).max() * 1e-6))
    assert np.all(np.abs(gl - wl) <= 3 * np.sqrt(wl2) + 1e-9 + 3 * max(1.0, np.abs(wl).max() * 1e-6))
    assert gk.sum() == pytest.approx(wk.sum(), rel=2e-3)
    assert gl.sum() == pytest.approx(wl.sum(), rel=2e-3)
    # Gradient of a random linear loss: library vs the oracle's records.
    rng = np.random.default_rng(5)
    gimg = rng.normal(size=(w.side_px, w.side_px))
    d_ms, d_ma, d_c = mc.mc_grad(med, geo, det, tal, torch.tensor(gimg, device=cuda_device))
    mu_t = w.tau / w.size_mm[2]
    mu_s = w.albedo * mu_t
    rows = np.clip(np.floor(r.rec("py")[sel] / w.size_mm[1] * w.side_px).astype(int), 0, w.side_px - 1)
    cols = np.clip(np.floor(r.rec("pz")[sel] / w.size_mm[2] * w.side_px).astype(int), 0, w.side_px - 1)
    gp = gimg[rows, cols]
    o_ms = np.sum(gp * r.rec("w")[sel] * (r.rec("k")[sel] / mu_s - r.rec("L")[sel]))
    o_ma = -np.sum(gp * r.rec("w")[sel] * r.rec("L")[sel])
    scale_s = np.sqrt(np.sum((gp * r.rec("w")[sel] * (r.rec("k")[sel] / mu_s - r.rec("L")[sel])) ** 2))
    scale_a = np.sqrt(np.sum((gp * r.rec("w")[sel] * r.rec("L")[sel]) ** 2))
    assert abs(d_ms - o_ms) <= 0.05 * scale_s
    assert abs(d_ma - o_ma) <= 0.05 * scale_a
    # Over the photons both sides walked alike (same trajectory to 1e-4 and
    # the same side pixel), the gradient agrees to 1e-4 of the sum of its
    # terms' sizes: the library's value less the GPU records' terms of the
    # other photons against the oracle's terms of the matched ones.
    ri, rf = tal.rec_i.cpu().numpy(), tal.rec_f.cpu().numpy().astype(np.float64)
    grec = {k: ri[i] for i, k in enumerate(IREC)}
    grec.update({k: rf[i] for i, k in enumerate(FREC)})
    orec = oracle_rec(r)
    n = w.side_px
    f32 = np.float32
    g_side = (grec["face"] == 1) & (grec["cause"] == 0)
    o_side = (orec["face"] == 1) & (orec["cause"] == 0)
    g_pix = (np.floor(grec["py"].astype(f32) * f32(n / w.size_mm[1])).astype(np.int64).clip(0, n - 1) * n
             + np.floor(grec["pz"].astype(f32) * f32(n / w.size_mm[2])).astype(np.int64).clip(0, n - 1))
    o_pix = (np.floor(orec["py"] / w.size_mm[1] * n).astype(np.int64).clip(0, n - 1) * n
             + np.floor(orec["pz"] / w.size_mm[2] * n).astype(np.int64).clip(0, n - 1))
    ok = trajectory_match(grec, orec, box=10.0) & (g_side == o_side) & (~g_side | (g_pix == o_pix))
    assert ok.mean() >= 0.999
    gflat = gimg.reshape(-1)

    def terms(rec, side, pix, sel):
        m = side & sel
        gp, wv = gflat[pix[m]], rec["w"][m]
        return gp * wv * (rec["k"][m] / mu_s - rec["L"][m]), -gp * wv * rec["L"][m]

    gs_bad, ga_bad = terms(grec, g_side, g_pix, ~ok)
    os_ok, oa_ok = terms(orec, o_side, o_pix, ok)
    assert abs((d_ms - gs_bad.sum()) - os_ok.sum()) <= 1e-4 * np.abs(os_ok).sum()
    assert abs((d_ma - ga_bad.sum()) - oa_ok.sum()) <= 1e-4 * np.abs(oa_ok).sum()
    assert d_c == pytest.approx(table.sigma_sca_mm2 * d_ms + table.sigma_abs_mm2 * d_ma, rel=1e-12)
    # Second-order moments, per pixel (MC_MOMENTS_PIXEL2) and summed over the
    # image (scalars), and the self-correlation correction (h = 2).
    w_s, k_s, l_s = r.rec("w")[sel], r.rec("k")[sel], r.rec("L")[sel]
    w2k = np.zeros_like(wk); w2l = np.zeros_like(wl)
    np.add.at(w2k, (rows, cols), w_s ** 2 * k_s)
    np.add.at(w2l, (rows, cols), w_s ** 2 * l_s)
    g2k, g2l = tal.side_w2k.cpu().numpy(), tal.side_w2l.cpu().numpy()
    assert g2k.sum() == pytest.approx(w2k.sum(), rel=2e-3)
    assert g2l.sum() == pytest.approx(w2l.sum(), rel=2e-3)
    sc = tal.scalars.cpu().numpy()
    assert sc[mc.MC_S_SIDE_W2] == pytest.approx(np.sum(w_s ** 2), rel=2e-3)
    assert sc[mc.MC_S_SIDE_W2K] == pytest.approx(g2k.sum(), rel=1e-12)
    assert sc[mc.MC_S_SIDE_W2L] == pytest.approx(g2l.sum(), rel=1e-12)
    gdev = torch.tensor(gimg, device=cuda_device)
    h2 = torch.full((w.side_px, w.side_px), 2.0, dtype=torch.float64, device=cuda_device)
    c_ms, c_ma, _ = mc.mc_grad(med, geo, det, tal, gdev, h2)
    q_s = 2 * np.sum(w_s ** 2 * (k_s / mu_s - l_s))
    q_a = -2 * np.sum(w_s ** 2 * l_s)
    assert c_ms == pytest.approx(d_ms - q_s, abs=0.05 * scale_s + 1e-3 * abs(q_s))
    assert c_ma == pytest.approx(d_ma - q_a, abs=0.05 * scale_a + 1e-3 * abs(q_a))
    # A uniform second derivative through the image-wide sums gives the same.
    u_ms, u_ma, _ = mc.mc_grad(med, geo, det, tal, gdev, d2loss_uniform=2.0)
    assert u_ms == pytest.approx(c_ms, rel=1e-9, abs=1e-9 * abs(q_s))
    assert u_ma == pytest.approx(c_ma, rel=1e-9, abs=1e-9 * abs(q_a))


def _walk(mc, dev, w, table, mu_s, mu_a, moments, tau_albedo=None):
    """One walk at (mu_s, mu_a); `tau_albedo` sets the medium's tau and albedo
    directly (so that mu_ext is bit-identical between two runs)."""
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=(mc.MC_MOMENTS if moments else 0) | mc.MC_SIGMA)
    mu_t = mu_s + mu_a
    med.tau, med.albedo = tau_albedo if tau_albedo is not None else (mu_t * w.size_mm[2], mu_s / mu_t)
    tal = mc.Tally.alloc(det, dev, sigma=True, moments=moments)
    mc.mc_simulate(med, src, geo, det, run, tal)
    return med, geo, det, tal


def _coefficients(w):
    mu_t = w.tau / w.size_mm[2]
    return w.albedo * mu_t, (1 - w.albedo) * mu_t


def test_gradient_of_a_linear_functional_matches_crn_differences(mc, cuda_device):
    """A smooth linear functional of the 512 x 512 lateral image at tau = 4:
    the pMC derivative against central differences with relative step 1e-3
    and common random numbers (same seed and draws on both sides), to 2 %.
    1e9 photons per evaluation keep the differences' own noise (decisions that
    flip between the two runs) near 0.5 %; at 1e7 it is ~3 %."""
    import torch
    w = W.DIFF.replace(n_photons=1_000_000_000)
    spec, *_ = mc.args_from_workload(w)
    table = mc.mie_table_build(spec, cuda_device)
    mu_s, mu_a = _coefficients(w)
    n = w.side_px
    yy, zz = torch.meshgrid(torch.linspace(-1, 1, n, dtype=torch.float64, device=cuda_device),
                            torch.linspace(-1, 1, n, dtype=torch.float64, device=cuda_device), indexing="ij")
    g = (torch.exp(-(yy ** 2 + zz ** 2)) * (1 + zz)).contiguous()
    med, geo, det, tal = _walk(mc, cuda_device, w, table, mu_s, mu_a, True)
    d_ms, d_ma, _ = mc.mc_grad(med, geo, det, tal, g)
    h = 1e-3
    fp = float((_walk(mc, cuda_device, w, table, mu_s * (1 + h), mu_a, False)[3].side * g).sum())
    fm = float((_walk(mc, cuda_device, w, table, mu_s * (1 - h), mu_a, False)[3].side * g).sum())
    fd = (fp - fm) / (2 * h * mu_s)
    print(f"linear functional dF/dmu_s: pMC {d_ms:.6e}  CRN-FD {fd:.6e}")
    assert d_ms == pytest.approx(fd, rel=0.02)


def test_corrected_l2_gradient_matches_crn_differences(mc, cuda_device):
    """L2 loss of the 512 x 512 lateral image against the tau = 4.5 target
    (seed 99).  At these pixel counts the plain loss is dominated by Monte
    Carlo variance, so the comparison uses the variance-corrected loss
    sum[(I - T)^2 - sum w^2] and the self-correlation-corrected pMC gradient
    (mc_grad with a uniform second derivative 2); both estimate the gradient
    of |E[I] - T|^2.
    Relative step 1e-2 and 4e8 photons per evaluation keep the differences'
    noise below 1 % (at step 1e-3 the pixel crossings of a 512^2 image need
    ~1e10 photons)."""
    w = W.DIFF.replace(n_photons=400_000_000)
    spec, *_ = mc.args_from_workload(w)
    table = mc.mie_table_build(spec, cuda_device)
    tw = W.DIFF_TARGET.replace(n_photons=400_000_000)
    T = _walk(mc, cuda_device, tw, table, *_coefficients(tw), False)[3].side.clone()
    mu_s, mu_a = _coefficients(w)
    med, geo, det, tal = _walk(mc, cuda_device, w, table, mu_s, mu_a, True)
    diff = tal.side - T
    d_ms, d_ma, _ = mc.mc_grad(med, geo, det, tal, (2 * diff).contiguous(), d2loss_uniform=2.0)
    # The image-wide sum of w^2 in the scalars is the squared-weight image's sum.
    assert float(tal.scalars[mc.MC_S_SIDE_W2]) == pytest.approx(float(tal.side_w2.sum()), rel=1e-6)

    def clean(tt):
        return float(((tt.side - T) ** 2).sum() - tt.side_w2.sum())

    h = 1e-2
    fd = (clean(_walk(mc, cuda_device, w, table, mu_s * (1 + h), mu_a, False)[3]) -
          clean(_walk(mc, cuda_device, w, table, mu_s * (1 - h), mu_a, False)[3])) / (2 * h * mu_s)
    print(f"corrected L2 dL/dmu_s: pMC {d_ms:.6e}  CRN-FD {fd:.6e}")
    assert d_ms == pytest.approx(fd, rel=0.02)
    # The absorption derivative, checked along the albedo at fixed mu_ext: with
    # common random numbers every trajectory is then the same on both sides and
    # only the weights a^k change, so the difference has no pixel-crossing
    # noise (a step in mu_abs alone rescales mu_ext by ~1e-5, whose crossings
    # swamp the absorption signal).  d/da at fixed mu_ext = mu_ext (d/dmu_s - d/dmu_a).
    mu_t = mu_s + mu_a
    da = 5e-5
    fd_a = (clean(_walk(mc, cuda_device, w, table, (w.albedo + da) * mu_t, (1 - w.albedo - da) * mu_t, False,
                        tau_albedo=(w.tau, w.albedo + da))[3]) -
            clean(_walk(mc, cuda_device, w, table, (w.albedo - da) * mu_t, (1 - w.albedo + da) * mu_t, False,
                        tau_albedo=(w.tau, w.albedo - da))[3])) / (2 * da)
    pmc_a = mu_t * (d_ms - d_ma)
    print(f"corrected L2 dL/da at fixed mu_ext: pMC {pmc_a:.6e}  CRN-FD {fd_a:.6e}  (dL/dmu_a pMC {d_ma:.6e})")
    assert pmc_a == pytest.approx(fd_a, rel=0.02)


@pytest.mark.parametrize("exit_log", [False, True])
def test_autograd_fits_optical_depth_to_a_lateral_image(mc, cuda_device, exit_log):
    """20 Adam steps on tau through torch.autograd (side_l2_loss), 1e7 photons
    per evaluation, 512 x 512 lateral image, from tau = 4 towards the target
    made at tau = 4.5 with seed 99, with image exits tallied by atomics or
    through the exit log (one workspace shared by all walks).  Adam's step is
    nearly independent of the gradient's scale; betas (0.5, 0.9) and rate 0.1
    settle within 1e-3 of the optimum of a quadratic 0.5 away in 20 steps."""
    import torch
    w = W.DIFF
    spec, *_ = mc.args_from_workload(w)
    table = mc.mie_table_build(spec, cuda_device)
    target = gpu_run(W.DIFF_TARGET, table=table, sigma=False)["tally"].side
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=mc.MC_EXIT_LOG if exit_log else 0)
    sim = mc.SideImage(med, src, geo, det, run, cuda_device)
    L = w.size_mm[2]
    tau = torch.tensor(4.0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tau], lr=0.1, betas=(0.5, 0.9))
    for it in range(20):
        opt.zero_grad()
        mu_t = tau / L
        loss = mc.side_l2_loss(mu_t * w.albedo, mu_t * (1 - w.albedo), target, sim)
        loss.backward()
        opt.step()
    print(f"fitted tau {tau.item():.4f} (target 4.5)")
    assert abs(tau.item() - 4.5) < 0.05
