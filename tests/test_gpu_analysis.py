"""GPU checks of the paper's image comparison on simulated images: the finite
parallel beam of the walk, and the comparison measures of Tables 3 and 4
(mc_image_metrics) against the oracle's measures on the same images."""
import math

import numpy as np
import pytest

import workloads as W
from _helpers import gpu_run, image_within_3sigma, oracle_rec, trajectory_match
from oracle import metrics as M
from oracle import walk as owalk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import paper_2507_23189_amd as m
    m.lib()
    return m


def test_finite_beam_trajectories_and_images(mc, cuda_device):
    w = W.TINY.replace(tau=2.0, beam_radius_mm=2.0, n_photons=30000)
    g = gpu_run(w, records=True)
    o = owalk.Walk(w).run(records=True)
    ok = trajectory_match(g["rec"], oracle_rec(o), box=10.0)
    assert ok.mean() >= 0.999, ok.mean()
    assert image_within_3sigma(g["side"], o.side, o.side_w2, w.n_photons).all()
    assert image_within_3sigma(g["trans"], o.trans, o.trans_w2, w.n_photons).all()


def test_finite_beam_enters_uniformly_on_its_disk(mc, cuda_device):
    R = 2.0
    w = W.TINY.replace(tau=1e-9, n_outside=1.33, beam_radius_mm=R, n_photons=200000)
    g = gpu_run(w, records=True)
    r = g["rec"]
    assert np.all(r["face"] == 5)
    dx, dy = r["px"] - 5.0, r["py"] - 5.0
    rho2 = dx * dx + dy * dy
    n = w.n_photons
    assert rho2.max() <= R * R * (1 + 1e-6)
    assert abs(np.mean(rho2 < (R / 2) ** 2) - 0.25) <= 4 * math.sqrt(0.25 * 0.75 / n)
    assert abs(rho2.mean() / (R * R) - 0.5) <= 4 / math.sqrt(12 * n)


def test_finite_beam_batch_equals_separate_runs(mc, cuda_device):
    import torch
    ws = [w.replace(beam_radius_mm=1.25) for w in W.batch_workloads(6, photon_scale=1e-3)]
    tables = [mc.mie_table_build(mc.args_from_workload(w)[0], cuda_device) for w in ws]
    _, _, src, geo, det, run = mc.args_from_workload(ws[0], flags=mc.MC_FIX64)
    items = [mc.batch_item(w, t) for w, t in zip(ws, tables)]
    tal = mc.Tally.alloc_batch(det, len(ws), cuda_device, fix64=True)
    mc.mc_simulate_batch(items, ws[0].n_cdf, src, geo, det, run, tal)
    torch.cuda.synchronize()
    for i, (w, t) in enumerate(zip(ws, tables)):
        one = gpu_run(w, table=t, fix64=True, sigma=False)
        np.testing.assert_array_equal(tal.trans[i].cpu().numpy(), one["trans"])
        np.testing.assert_array_equal(tal.side[i].cpu().numpy(), one["side"])


def _check_against_oracle(mc, a, b, c, cx, cy, r_max):
    import torch
    ta, tb = torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")
    tc = torch.tensor(c, device="cuda") if c is not None else None
    g = mc.image_metrics(ta, tb, tc, cx=cx, cy=cy, r_max=r_max, profiles=True)
    o = M.image_metrics(a, b, cx, cy, r_max, c=c)
    for k in ("rmse", "r", "radial_r"):
        if math.isnan(o[k]):
            assert math.isnan(g[k]), k
        else:
            assert g[k] == pytest.approx(o[k], rel=1e-9, abs=1e-12), k
    np.testing.assert_allclose(g["zone_rmse"], o["zone_rmse"], rtol=1e-8, atol=1e-11)
    assert g["n_annuli"] == o["n_annuli"]
    np.testing.assert_array_equal(g["count"].cpu().numpy(), o["count"])
    np.testing.assert_allclose(g["profile_a"].cpu().numpy(), o["profile_a"], rtol=0, atol=1e-11)
    np.testing.assert_allclose(g["profile_b"].cpu().numpy(), o["profile_b"], rtol=0, atol=1e-11)
    if c is not None:
        assert g["better"] == pytest.approx(o["better"], abs=1.5 / o["n_annuli"])
    return g, o


def test_metrics_on_synthetic_images(mc, cuda_device):
    n = 96
    yy, xx = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    a = np.exp(-((xx - 48) ** 2 + (yy - 40) ** 2) / 300.0) + 0.05 * np.sin(xx / 5.0) ** 2
    b = np.exp(-((xx - 50) ** 2 + (yy - 48) ** 2) / 500.0)
    c = b + 0.2 * np.cos(yy / 9.0) ** 2
    g, _ = _check_against_oracle(mc, a, b, c, 48.0, 48.0, 48.0)
    same, _ = _check_against_oracle(mc, a, 3.0 * a, None, 48.0, 48.0, 40.0)
    assert same["rmse"] == pytest.approx(0.0, abs=1e-15) and same["r"] == pytest.approx(1.0, abs=1e-12)
    comp = (a - a.min()) / (a.max() - a.min())
    anti, _ = _check_against_oracle(mc, comp, 1.0 - comp, None, 30.0, 60.0, 25.5)
    assert anti["r"] == pytest.approx(-1.0, abs=1e-12)
    flat, _ = _check_against_oracle(mc, np.ones((n, n)), b, None, 48.0, 48.0, 48.0)
    assert math.isnan(flat["r"])


def test_metrics_on_simulated_mie_and_hg_images(mc, cuda_device):
    """The side images of a Mie and an HG run (finite beam, OD 5) against an
    independent Mie run: the measures of Tables 3 and 4, on the device and
    in the oracle, on the same images."""
    n = 2_000_000
    wm = W.analysis_workload(5.0, n_photons=n).replace(n_cdf=4096, side_px=256, trans_px=256)
    table = mc.mie_table_build(mc.args_from_workload(wm)[0], cuda_device)
    mie_img = gpu_run(wm, table=table, sigma=False)["side"]
    ref_img = gpu_run(wm.replace(seed=W.ANALYSIS_REF_SEED), table=table, sigma=False)["side"]
    hg_img = gpu_run(wm.replace(phase=W.PHASE_HG), table=table, sigma=False, g=table.g)["side"]
    _check_against_oracle(mc, mie_img, ref_img, hg_img, 128.0, 128.0, 128.0)
    _check_against_oracle(mc, hg_img, ref_img, None, 128.0, 128.0, 128.0)
    _check_against_oracle(mc, mie_img, hg_img, None, 100.0, 140.0, 90.0)
