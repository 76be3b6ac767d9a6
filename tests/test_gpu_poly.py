"""GPU checks of the polydisperse table (mie_table_build_poly) and of the
heavy-scattering walk built on it (lognormal sizes, tau = 16, 1024 x 1024
fixed-point images), against the oracle's polydisperse table and walk."""
import math

import numpy as np
import pytest

import workloads as W
from _helpers import gpu_run, image_within_3sigma, oracle_rec, trajectory_match
from oracle import mie, poly
from oracle import walk as owalk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import paper_2507_23189_amd as m
    m.lib()
    return m


POLY_CASES = [
    dict(d=5.0, sigma=0.05, bins=64, na=1801, nc=16384),     # heavy-scattering workload
    dict(d=1.0, sigma=0.3, bins=64, na=1801, nc=4096),       # wide distribution of small spheres
    dict(d=3.0, sigma=0.1, bins=5, na=3001, nc=2),           # few bins, smallest table
]


@pytest.mark.parametrize("case", POLY_CASES)
def test_poly_table_parity(mc, cuda_device, case):
    c = case
    spec = mc.MieSpec(n_medium=1.33, m_re=1.59, m_im=0.0, diameter_um=c["d"], wavelength_nm=532.0,
                      n_angles=c["na"], n_cdf=c["nc"])
    t = mc.mie_table_build_poly(spec, c["sigma"], c["bins"], cuda_device, phase=True, cdf=True)
    o = poly.build_poly_table(c["d"], c["sigma"], c["bins"], 1.59, 0.0, 1.33, 532.0, c["na"], c["nc"])
    assert t.x == pytest.approx(o.x, rel=1e-15)
    assert t.n_terms == max(mie.n_terms(mie.size_parameter(dk, 532.0, 1.33)) for dk in o.diameters_um)
    for name in ("g", "sigma_ext_mm2", "sigma_sca_mm2"):
        assert getattr(t, name) == pytest.approx(getattr(o, name), rel=1e-11)
    assert t.q_ext == pytest.approx(o.q_ext, rel=1e-11)
    np.testing.assert_allclose(t.phase.cpu().numpy(), o.P, rtol=1e-10, atol=1e-14 * o.P.max())
    np.testing.assert_allclose(t.cdf.cpu().numpy(), o.F, rtol=0, atol=1e-13)
    inv = t.inv_cdf.cpu().numpy().astype(np.float64)
    ref32 = o.v.astype(np.float32)
    ulp = np.spacing(np.abs(ref32)).astype(np.float64)
    assert np.all(np.abs(inv - ref32.astype(np.float64)) <= ulp + 1e-30)


def test_zero_width_equals_single_size(mc, cuda_device):
    spec = mc.MieSpec(n_medium=1.33, m_re=1.59, m_im=0.0, diameter_um=5.0, wavelength_nm=532.0,
                      n_angles=1801, n_cdf=4096)
    single = mc.mie_table_build(spec, cuda_device)
    mixed = mc.mie_table_build_poly(spec, 0.0, 8, cuda_device)
    a, b = single.inv_cdf.cpu().numpy(), mixed.inv_cdf.cpu().numpy()
    assert np.all(np.abs(a.astype(np.float64) - b) <= np.spacing(np.abs(a)).astype(np.float64) + 1e-30)
    assert mixed.g == pytest.approx(single.g, rel=1e-13)
    assert mixed.sigma_ext_mm2 == pytest.approx(single.sigma_ext_mm2, rel=1e-13)


@pytest.fixture(scope="module")
def heavy(mc, cuda_device):
    w = W.HEAVY
    return w, mc.table_for_workload(w, cuda_device), poly.poly_table_from_workload(w)


def test_heavy_subsample_trajectories_and_images(mc, cuda_device, heavy):
    """The first 1e6 photons of the heavy workload (their trajectories are
    those of the full 1e9-photon run): per-photon records and the 1024 x 1024
    images against the oracle's FP64 walk on the oracle's own table."""
    w, table, otab = heavy
    ws = w.replace(n_photons=1_000_000)
    g = gpu_run(ws, table=table, records=True)
    o = owalk.Walk(ws, table=otab).run(records=True)
    ok = trajectory_match(g["rec"], oracle_rec(o), box=10.0)
    print(f"heavy subsample: {ok.mean():.5f} of trajectories match; events/photon "
          f"{g['scalars'][9] / g['scalars'][10]:.3f}")
    assert ok.mean() >= 0.999, ok.mean()
    assert image_within_3sigma(g["side"], o.side, o.side_w2, ws.n_photons).all()
    assert image_within_3sigma(g["trans"], o.trans, o.trans_w2, ws.n_photons).all()
    np.testing.assert_allclose(g["scalars"][:7], o.scalars[:7], rtol=2e-3, atol=2.0)
    assert abs(g["scalars"][9] - o.scalars[9]) <= 1e-3 * o.scalars[9]


def test_heavy_full_size_sampled_with_moments(mc, cuda_device, heavy):
    """The full heavy launch (1e9 photons, int64 fixed-point images, path
    moments for the adjoint) as the benchmark runs it: every 1e6-th photon
    recorded and replayed one by one in the oracle; fixed-point face totals
    equal the image sums; energy bookkeeping closes."""
    w, table, otab = heavy
    stride = 1_000_000
    _, med, src, geo, det, run = mc.args_from_workload(
        w, table, flags=mc.MC_FIX64 | mc.MC_MOMENTS | mc.MC_RECORD, record_stride=stride)
    rows = w.n_photons // stride
    tal = mc.Tally.alloc(det, cuda_device, fix64=True, moments=True, record_rows=rows)
    mc.mc_simulate(med, src, geo, det, run, tal)
    import torch
    torch.cuda.synchronize()
    s = tal.scalars.cpu().numpy()
    assert s[10] == w.n_photons
    side, trans = tal.side.cpu().numpy(), tal.trans.cpu().numpy()
    assert side.sum() * 2.0**-32 == s[1] and trans.sum() * 2.0**-32 == s[5]
    w0 = 1.0 - ((1.0 - 1.33) / 2.33) ** 2
    assert s[0:6].sum() + s[6] + s[8] == pytest.approx(w.n_photons * w0 + s[7], rel=1e-5)
    ri, rf = tal.rec_i.cpu().numpy(), tal.rec_f.cpu().numpy().astype(np.float64)
    from _helpers import FREC, IREC
    rec = {k: ri[i] for i, k in enumerate(IREC)}
    rec.update({k: rf[i] for i, k in enumerate(FREC)})
    ids = np.arange(0, w.n_photons, stride, dtype=np.uint64)
    o = owalk.Walk(w, table=otab).run(ids=ids, records=True)
    assert trajectory_match(rec, oracle_rec(o), box=10.0).mean() >= 0.999
    # The adjoint on the full launch: finite, and the concentration derivative
    # is the cross-section combination of the other two.
    g = (torch.ones_like(tal.side_wk)).contiguous()
    d_ms, d_ma, d_c = mc.mc_grad(med, geo, det, tal, g)
    assert math.isfinite(d_ms) and math.isfinite(d_ma)
    assert d_c == pytest.approx(table.sigma_sca_mm2 * d_ms + table.sigma_abs_mm2 * d_ma, rel=1e-12)
