"""The allocation-free walk (mc_simulate_noalloc): through the C ABI, its
tallies equal mc_simulate's with a caller workspace, bit for bit with int64
fixed-point images, on two calls in a row on the library's one scratch array,
the second with fewer photons and smaller images (so it must not see what the
first left behind)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _run(mc, dev, w, table, flags, noalloc, n_photons, shape):
    import torch
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=flags, n_photons=n_photons)
    det.side_nx, det.side_ny, det.trans_nx, det.trans_ny = shape
    sigma = bool(flags & mc.MC_SIGMA)
    moments = bool(flags & mc.MC_MOMENTS)
    t = mc.Tally.alloc(det, dev, sigma=sigma, fix64=bool(flags & mc.MC_FIX64), moments=moments,
                       record_rows=n_photons if flags & mc.MC_RECORD else 0)
    if noalloc:
        t.workspace = None
        mc.mc_simulate_noalloc(med, src, geo, det, run, t)
    else:
        mc.mc_simulate(med, src, geo, det, run, t)
    torch.cuda.synchronize()
    names = ["side", "trans", "scalars"] + (["side_w2", "trans_w2"] if sigma else []) \
        + (["side_wk", "side_wl"] if moments else []) + (["rec_i", "rec_f"] if flags & mc.MC_RECORD else [])
    return {k: getattr(t, k).cpu().numpy() for k in names}


@pytest.mark.parametrize("phase", [W.PHASE_MIE, W.PHASE_HG])
def test_noalloc_equals_mc_simulate_on_two_calls(phase, cuda_device):
    import paper_2507_23189_amd as mc
    w = W.paper_scale(2.0).replace(phase=phase)
    spec, *_ = mc.args_from_workload(w)
    table = mc.mie_table_build(spec, cuda_device)
    flags = mc.MC_FIX64 | mc.MC_SIGMA
    calls = [(3_000_000, (512, 512, 512, 512)), (200_000, (97, 61, 33, 129))]
    for n, shape in calls:
        ref = _run(mc, cuda_device, w, table, flags, False, n, shape)
        got = _run(mc, cuda_device, w, table, flags, True, n, shape)
        print(f"noalloc: phase {phase}, {n} photons, images {shape}", flush=True)
        for k in ref:
            assert np.array_equal(ref[k], got[k]), k
        assert got["scalars"][10] == n


def test_noalloc_records_moments_and_double_images(cuda_device):
    """The other tally options through the one scratch copy: float64 images
    (sums of the same fixed-point integers, so equal), per-photon records and
    path moments (FP64 sums in another order: equal to rounding)."""
    import paper_2507_23189_amd as mc
    w = W.TINY.replace(tau=3.0, n_photons=40000)
    spec, *_ = mc.args_from_workload(w)
    table = mc.mie_table_build(spec, cuda_device)
    shape = (w.side_px, w.side_px, w.trans_px, w.trans_px)
    ref = _run(mc, cuda_device, w, table, mc.MC_RECORD, False, w.n_photons, shape)
    got = _run(mc, cuda_device, w, table, mc.MC_RECORD, True, w.n_photons, shape)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k
    ref = _run(mc, cuda_device, w, table, mc.MC_MOMENTS, False, w.n_photons, shape)
    got = _run(mc, cuda_device, w, table, mc.MC_MOMENTS, True, w.n_photons, shape)
    for k in ("side", "trans"):
        assert np.array_equal(ref[k], got[k]), k
    np.testing.assert_array_equal(ref["scalars"][:16], got["scalars"][:16])
    for k in ("side_wk", "side_wl"):
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-12, atol=1e-12 * np.abs(ref[k]).max())


def test_noalloc_refuses_what_does_not_fit(cuda_device):
    import paper_2507_23189_amd as mc
    w = W.TINY
    spec, *_ = mc.args_from_workload(w)
    table = mc.mie_table_build(spec, cuda_device)
    _, med, src, geo, det, run = mc.args_from_workload(w, table, flags=mc.MC_SIGMA)
    det.side_nx = det.side_ny = det.trans_nx = det.trans_ny = 1024      # 2^21 pixels, 2^22 words with sigma
    t = mc.Tally.alloc(det, cuda_device, sigma=True)
    with pytest.raises(mc.McError) as e:
        mc.mc_simulate_noalloc(med, src, geo, det, run, t)
    assert e.value.code == mc.MC_EINVAL and "scratch" in str(e.value)
    det.flags = mc.MC_EXIT_LOG
    t = mc.Tally.alloc(det, cuda_device, log_photons=w.n_photons)
    with pytest.raises(mc.McError) as e:
        mc.mc_simulate_noalloc(med, src, geo, det, run, t)
    assert e.value.code == mc.MC_EINVAL
