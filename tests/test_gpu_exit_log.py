"""GPU checks of the exit-log tally path (MC_EXIT_LOG).  It computes the same
integer sums as the atomic path, so its images and scalars must equal that
path's bit for bit on the same photons.  The atomic path is itself checked
against the oracle elsewhere; one case here also compares the log path with
the oracle directly.  Covered: both phase functions, with and without squared
weights, float64 and int64 outputs, ragged image shapes (keys that do not
fill the last 512-key group), a log too small for the walk (exits fall back
to atomics), no log at all, accumulation into earlier results, a workspace
shared by walks in a row, and the full 1e8-photon tau = 4 launch."""
import numpy as np
import pytest

import workloads as W
from _helpers import image_within_3sigma
from oracle import walk as owalk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import paper_2507_23189_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def table(mc, cuda_device):
    w = W.paper_scale(4.0)
    spec, *_ = mc.args_from_workload(w)
    return mc.mie_table_build(spec, cuda_device)


def _run(mc, dev, w, table, flags, *, n_photons, det_shape=None, log_photons=None, workspace=None,
         tally=None, phase=None, grid_blocks=0):
    import torch
    w = w if phase is None else w.replace(phase=phase)
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=flags, n_photons=n_photons,
                                                       grid_blocks=grid_blocks)
    if det_shape is not None:
        det.side_nx, det.side_ny, det.trans_nx, det.trans_ny = det_shape
    if tally is None:
        tally = mc.Tally.alloc(det, dev, sigma=bool(flags & mc.MC_SIGMA), fix64=bool(flags & mc.MC_FIX64),
                               log_photons=log_photons if log_photons is not None else n_photons,
                               workspace=workspace)
    mc.mc_simulate(med, src, geo, det, run, tally)
    torch.cuda.synchronize()
    out = {k: getattr(tally, k).cpu().numpy() for k in ("side", "trans", "scalars")}
    if flags & mc.MC_SIGMA:
        out["side_w2"] = tally.side_w2.cpu().numpy()
        out["trans_w2"] = tally.trans_w2.cpu().numpy()
    out["tally"] = tally
    out["fallback"] = int(tally.workspace[21].item())   # exits added directly: the log was full
    return out


def _same(a, b):
    for k in ("side", "trans", "scalars", "side_w2", "trans_w2"):
        if k in a or k in b:
            assert a[k].dtype == b[k].dtype
            assert np.array_equal(a[k], b[k]), k


CASES = [
    dict(phase="mie", fix64=True, sigma=False),
    dict(phase="mie", fix64=True, sigma=True),
    dict(phase="mie", fix64=False, sigma=False),
    dict(phase="hg", fix64=True, sigma=True),
    dict(phase="hg", fix64=False, sigma=False),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['phase']}-{'fix64' if c['fix64'] else 'f64'}"
                         f"{'-sigma' if c['sigma'] else ''}")
def test_log_equals_atomic_path(mc, cuda_device, table, case):
    w = W.paper_scale(4.0)
    phase = W.PHASE_MIE if case["phase"] == "mie" else W.PHASE_HG
    flags = (mc.MC_FIX64 if case["fix64"] else 0) | (mc.MC_SIGMA if case["sigma"] else 0)
    n = 2_000_000
    a = _run(mc, cuda_device, w, table, flags, n_photons=n, phase=phase)
    b = _run(mc, cuda_device, w, table, flags | mc.MC_EXIT_LOG, n_photons=n, phase=phase)
    assert a["scalars"][10] == n
    assert a["side"].sum() > 0 and a["trans"].sum() > 0
    _same(a, b)


def test_log_with_finite_beam_and_heavy_weights(mc, cuda_device, table):
    """The analysis workload's 1.25 mm beam (no first-step counting, so the
    beam's unscattered exits go through the log too) and roulette settings
    that raise weights above 1: the log still equals the atomic path."""
    w = W.analysis_workload(8.0).replace(roulette_w=0.5, roulette_p=0.2, albedo=0.98)
    flags = mc.MC_FIX64 | mc.MC_SIGMA
    n = 1_000_000
    a = _run(mc, cuda_device, w, table, flags, n_photons=n)
    b = _run(mc, cuda_device, w, table, flags | mc.MC_EXIT_LOG, n_photons=n)
    assert a["scalars"][10] == n and a["trans"].sum() > 0
    _same(a, b)


@pytest.mark.parametrize("shape", [(37, 23, 61, 19), (1, 1, 1, 1), (5, 300, 700, 3), (512, 512, 1024, 1024)])
def test_log_ragged_shapes(mc, cuda_device, table, shape):
    """Image sizes whose key count is not a multiple of 512, a single pixel
    per image, and keys beyond one histogram part of a range."""
    w = W.paper_scale(4.0)
    flags = mc.MC_FIX64 | mc.MC_SIGMA
    n = 500_000
    a = _run(mc, cuda_device, w, table, flags, n_photons=n, det_shape=shape)
    b = _run(mc, cuda_device, w, table, flags | mc.MC_EXIT_LOG, n_photons=n, det_shape=shape)
    _same(a, b)


@pytest.mark.parametrize("cap", [-1, 0, 64, 1000, 12000])
def test_log_capacity_fallback(mc, cuda_device, table, cap):
    """A launch of two 1024-lane blocks whose log holds 0, 64, 1000 or 12000
    entries per block and range: each block adds about 5400 exits to every
    range, so with small regions most of them find the log full and are
    added directly.  With no room even for the region counts (-1) the walk
    takes the atomic path.  The results do not change."""
    import torch
    w = W.paper_scale(4.0)
    flags = mc.MC_FIX64 | mc.MC_SIGMA
    n = 1_000_000
    _, _, _, _, det, _ = mc.args_from_workload(w, flags=flags | mc.MC_EXIT_LOG)
    regions = 64 * 2
    ws_bytes = mc.mc_workspace_bytes(det) + (regions * 4 + regions * cap * 8 if cap >= 0 else 0)
    small = mc.Tally.alloc(det, cuda_device, sigma=True, fix64=True, log_photons=0)
    small.workspace = torch.empty((ws_bytes + 7) // 8, dtype=torch.int64, device=cuda_device)
    a = _run(mc, cuda_device, w, table, flags, n_photons=n, grid_blocks=2)
    b = _run(mc, cuda_device, w, table, flags | mc.MC_EXIT_LOG, n_photons=n, tally=small, grid_blocks=2)
    _same(a, b)
    print(f"cap {cap}: {b['fallback']} exits added directly")
    if 0 <= cap <= 1000:
        assert b["fallback"] > 0
    else:
        assert b["fallback"] == 0


def test_log_accumulate_and_shared_workspace(mc, cuda_device, table):
    """Two walks in a row on one workspace: the second, with MC_ACCUMULATE,
    adds its photons (ids after the first's) to the first's results."""
    import torch
    w = W.paper_scale(4.0)
    flags = mc.MC_FIX64 | mc.MC_SIGMA
    n = 1_000_000
    full = _run(mc, cuda_device, w, table, flags, n_photons=2 * n)
    t = _run(mc, cuda_device, w, table, flags | mc.MC_EXIT_LOG, n_photons=n)["tally"]
    other = _run(mc, cuda_device, w, table, flags | mc.MC_EXIT_LOG, n_photons=n, workspace=t.workspace)
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=flags | mc.MC_EXIT_LOG | mc.MC_ACCUMULATE,
                                                       n_photons=n, photon_offset=n)
    mc.mc_simulate(med, src, geo, det, run, t)
    torch.cuda.synchronize()
    got = {k: getattr(t, k).cpu().numpy() for k in ("side", "trans", "side_w2", "trans_w2")}
    for k in ("side", "trans", "side_w2", "trans_w2"):
        assert np.array_equal(got[k], full[k]), k
    s = t.scalars.cpu().numpy()
    assert s[10] == 2 * n and s[9] == full["scalars"][9]
    # The walk that shared the workspace before still holds its own result.
    first = _run(mc, cuda_device, w, table, flags, n_photons=n)
    _same(first, {k: v for k, v in other.items() if k != "tally"})


def test_log_against_oracle(mc, cuda_device):
    """The log path on the tiny workload against the oracle's FP64 walk."""
    w = W.TINY
    spec, *_ = mc.args_from_workload(w)
    tab = mc.mie_table_build(spec, cuda_device)
    g = _run(mc, cuda_device, w, tab, mc.MC_SIGMA | mc.MC_EXIT_LOG, n_photons=w.n_photons)
    o = owalk.Walk(w).run()
    assert image_within_3sigma(g["side"], o.side, o.side_w2, w.n_photons).all()
    assert image_within_3sigma(g["trans"], o.trans, o.trans_w2, w.n_photons).all()
    np.testing.assert_allclose(g["scalars"][:7], o.scalars[:7], rtol=2e-3, atol=2.0)


def test_log_full_size_launch(mc, cuda_device, table):
    """The full tau = 4 launch of 1e8 photons (512 x 512 images) in the
    launch configuration the benchmark times: the log path equals the atomic
    path, and the record-writing kernel whose sampled trajectories the parity
    tests replay in the oracle, bit for bit; nearly every exit went through
    the log."""
    import torch
    w = W.paper_scale(4.0)
    a = _run(mc, cuda_device, w, table, mc.MC_FIX64, n_photons=w.n_photons)
    b = _run(mc, cuda_device, w, table, mc.MC_FIX64 | mc.MC_EXIT_LOG, n_photons=w.n_photons)
    _same(a, b)
    stride = 50_000
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=mc.MC_FIX64 | mc.MC_RECORD,
                                                       record_stride=stride)
    t = mc.Tally.alloc(det, cuda_device, fix64=True, record_rows=w.n_photons // stride)
    mc.mc_simulate(med, src, geo, det, run, t)
    torch.cuda.synchronize()
    _same(b, {k: getattr(t, k).cpu().numpy() for k in ("side", "trans", "scalars")})
    assert int(t.rec_i[0].ge(0).sum()) > 0
    assert a["scalars"][10] == w.n_photons
    # Waves that take more than their share of photons can run out of chunks
    # in a range; those few exits are added directly.
    print(f"exits added directly: {b['fallback']}")
    assert b["fallback"] <= 1e-3 * w.n_photons


@pytest.mark.parametrize("fix64", [True, False])
def test_log_with_path_moments_and_adjoint(mc, cuda_device, table, fix64):
    """MC_EXIT_LOG with MC_MOMENTS: the images equal the atomic path's bit
    for bit; the FP64 path moments and second-moment scalars (sums whose order
    differs from run to run) and the adjoint agree to rounding."""
    import torch
    w = W.paper_scale(4.0)
    n = 2_000_000
    base = mc.MC_MOMENTS | (mc.MC_FIX64 if fix64 else 0)
    out = []
    for flags in (base, base | mc.MC_EXIT_LOG):
        _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=flags, n_photons=n)
        t = mc.Tally.alloc(det, cuda_device, fix64=fix64, moments=True, log_photons=n)
        mc.mc_simulate(med, src, geo, det, run, t)
        g = (torch.arange(w.side_px * w.side_px, dtype=torch.float64, device=cuda_device) % 7 - 3.0).reshape(
            w.side_px, w.side_px).contiguous()
        grad = mc.mc_grad(med, geo, det, t, g, d2loss_uniform=2.0)
        torch.cuda.synchronize()
        out.append(dict(side=t.side.cpu().numpy(), trans=t.trans.cpu().numpy(), s=t.scalars.cpu().numpy(),
                        wk=t.side_wk.cpu().numpy(), wl=t.side_wl.cpu().numpy(), grad=np.array(grad)))
    a, b = out
    assert np.array_equal(a["side"], b["side"]) and np.array_equal(a["trans"], b["trans"])
    assert np.array_equal(a["s"][:16], b["s"][:16])
    np.testing.assert_allclose(b["s"][16:19], a["s"][16:19], rtol=1e-12)
    np.testing.assert_allclose(b["wk"], a["wk"], rtol=1e-12, atol=1e-12 * np.abs(a["wk"]).max())
    np.testing.assert_allclose(b["wl"], a["wl"], rtol=1e-12, atol=1e-12 * np.abs(a["wl"]).max())
    np.testing.assert_allclose(b["grad"], a["grad"], rtol=1e-9)
