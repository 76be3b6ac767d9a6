"""GPU checks of the batched launch (mc_simulate_batch) and its autotuner.

A photon of a batched medium follows exactly the walk mc_simulate gives it for
that medium alone (same table, coefficients, Philox counter word and id), so
with fixed-point tallies every medium's images and scalars must equal a
separate mc_simulate of it bit for bit, whatever the launch shape or schedule.
The separate runs are themselves checked against the oracle by
test_gpu_parity; one batched medium is also compared with the oracle here."""
import numpy as np
import pytest

import workloads as W
from _helpers import gpu_run, image_within_3sigma
from oracle import walk as owalk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import paper_2507_23189_amd as m
    m.lib()
    return m


def _tables(mc, ws, dev):
    return [mc.mie_table_build(mc.args_from_workload(w)[0], dev) for w in ws]


def _batch(mc, ws, tables, dev, *, fix64=True, sigma=True, block_size=0, chunk=0, grid_blocks=0, log=False,
           log_photons=None, workspace_bytes=None):
    import torch
    flags = (mc.MC_FIX64 if fix64 else 0) | (mc.MC_SIGMA if sigma else 0) | (mc.MC_EXIT_LOG if log else 0)
    _, _, src, geo, det, run = mc.args_from_workload(ws[0], flags=flags, block_size=block_size,
                                                     grid_blocks=grid_blocks)
    run.chunk = chunk
    items = [mc.batch_item(w, t) for w, t in zip(ws, tables)]
    n_all = sum(w.n_photons for w in ws)
    tal = mc.Tally.alloc_batch(det, len(ws), dev, sigma=sigma, fix64=fix64,
                               log_photons=n_all if log_photons is None else log_photons)
    if workspace_bytes is not None:
        tal.workspace = torch.empty((workspace_bytes + 7) // 8, dtype=torch.int64, device=dev)
    mc.mc_simulate_batch(items, ws[0].n_cdf, src, geo, det, run, tal)
    torch.cuda.synchronize()
    return tal


def test_batch_equals_separate_runs(mc, cuda_device):
    """16 media (sizes, depths, albedos and photon counts from the batch
    sampler, photons scaled by 1e-2): every image, squared-weight image and
    scalar of the batch equals that medium's own mc_simulate, bit for bit."""
    ws = W.batch_workloads(16, photon_scale=1e-2)
    tables = _tables(mc, ws, cuda_device)
    tal = _batch(mc, ws, tables, cuda_device)
    side, trans = tal.side.cpu().numpy(), tal.trans.cpu().numpy()
    side2, trans2 = tal.side_w2.cpu().numpy(), tal.trans_w2.cpu().numpy()
    scal = tal.scalars.cpu().numpy()
    for i, (w, t) in enumerate(zip(ws, tables)):
        one = gpu_run(w, table=t, fix64=True)
        np.testing.assert_array_equal(side[i], one["side"], err_msg=f"medium {i}")
        np.testing.assert_array_equal(trans[i], one["trans"], err_msg=f"medium {i}")
        np.testing.assert_array_equal(side2[i], one["side_w2"], err_msg=f"medium {i}")
        np.testing.assert_array_equal(trans2[i], one["trans_w2"], err_msg=f"medium {i}")
        np.testing.assert_array_equal(scal[i][:15], one["scalars"][:15], err_msg=f"medium {i}")
        assert scal[i][mc.MC_S_PHOTONS] == w.n_photons
    # Double images are the same fixed-point sums converted.
    tal_d = _batch(mc, ws, tables, cuda_device, fix64=False)
    np.testing.assert_array_equal(tal_d.side.cpu().numpy(), side.astype(np.float64) * 2.0**-32)
    np.testing.assert_array_equal(tal_d.scalars.cpu().numpy()[:, :15], scal[:, :15])


def test_batch_launch_shape_and_chunk_invariance(mc, cuda_device):
    ws = W.batch_workloads(24, photon_scale=3e-3)
    tables = _tables(mc, ws, cuda_device)
    ref = _batch(mc, ws, tables, cuda_device)
    for kw in (dict(block_size=256, chunk=64), dict(block_size=1024, chunk=1024),
               dict(block_size=512, chunk=200, grid_blocks=5)):
        other = _batch(mc, ws, tables, cuda_device, **kw)
        for k in ("side", "trans", "side_w2", "trans_w2", "scalars"):
            np.testing.assert_array_equal(getattr(ref, k).cpu().numpy(), getattr(other, k).cpu().numpy(),
                                          err_msg=f"{k} {kw}")


def test_batch_medium_against_oracle(mc, cuda_device):
    """Three batched media against the oracle's images within 3 sigma and
    its scalar totals."""
    ws = [w.replace(n_photons=20000) for w in W.batch_workloads(3)]
    tables = _tables(mc, ws, cuda_device)
    tal = _batch(mc, ws, tables, cuda_device, fix64=False)
    side, trans, scal = tal.side.cpu().numpy(), tal.trans.cpu().numpy(), tal.scalars.cpu().numpy()
    for i, w in enumerate(ws):
        o = owalk.Walk(w).run()
        assert image_within_3sigma(side[i], o.side, o.side_w2, w.n_photons).all(), i
        assert image_within_3sigma(trans[i], o.trans, o.trans_w2, w.n_photons).all(), i
        np.testing.assert_allclose(scal[i][:7], o.scalars[:7], rtol=2e-3, atol=2.0)
        assert abs(scal[i][9] - o.scalars[9]) <= 1e-3 * o.scalars[9]


def test_batch_with_empty_and_single_photon_media(mc, cuda_device):
    ws = W.batch_workloads(5, photon_scale=1e-3)
    ws[1] = ws[1].replace(n_photons=0)
    ws[3] = ws[3].replace(n_photons=1)
    tables = _tables(mc, ws, cuda_device)
    tal = _batch(mc, ws, tables, cuda_device)
    scal = tal.scalars.cpu().numpy()
    assert scal[1][mc.MC_S_PHOTONS] == 0 and np.all(tal.side[1].cpu().numpy() == 0)
    assert scal[3][mc.MC_S_PHOTONS] == 1
    for i in (0, 3, 4):
        one = gpu_run(ws[i], table=tables[i], fix64=True)
        np.testing.assert_array_equal(tal.trans[i].cpu().numpy(), one["trans"])


def test_autotuner_picks_a_timed_candidate(mc, cuda_device):
    import torch
    ws = W.batch_workloads(32, photon_scale=1e-2)
    tables = _tables(mc, ws, cuda_device)
    _, _, src, geo, det, run = mc.args_from_workload(ws[0], flags=mc.MC_FIX64)
    items = [mc.batch_item(w, t) for w, t in zip(ws, tables)]
    tal = mc.Tally.alloc_batch(det, len(ws), cuda_device, fix64=True)
    blk, chk, best, table = mc.mc_autotune_batch(items, ws[0].n_cdf, src, geo, det, run, tal, 0.25)
    assert blk in mc.AUTOTUNE_BLOCKS and chk in mc.AUTOTUNE_CHUNKS
    assert best == min(table.values()) == table[(blk, chk)] and best > 0
    # The tuned shape gives the same tallies as the default one.
    run.block_size, run.chunk = blk, chk
    mc.mc_simulate_batch(items, ws[0].n_cdf, src, geo, det, run, tal)
    torch.cuda.synchronize()
    ref = _batch(mc, ws, tables, cuda_device, sigma=False)
    np.testing.assert_array_equal(tal.side.cpu().numpy(), ref.side.cpu().numpy())
    np.testing.assert_array_equal(tal.scalars.cpu().numpy(), ref.scalars.cpu().numpy())


@pytest.mark.parametrize("case", ["full", "no_entries", "no_log", "shape"])
def test_batch_exit_log_equals_atomic_path(mc, cuda_device, case):
    """The batched launch with its image exits through the exit log (key
    ranges over all media's keys, 2^12 of them for 64 media of 256 x 256 +
    256 x 256 pixels) equals the atomic path bit for bit: with a log sized
    for the batch, with room for the region counts but no entries (every
    exit falls back to an atomic), with no room for the log at all (the
    atomic path) and in another launch shape."""
    import torch
    ws = W.batch_workloads(64, photon_scale=1e-2)
    tables = _tables(mc, ws, cuda_device)
    ref = _batch(mc, ws, tables, cuda_device)
    kw = dict(log=True)
    if case in ("no_entries", "no_log"):
        _, _, _, _, det, _ = mc.args_from_workload(ws[0], flags=mc.MC_FIX64 | mc.MC_SIGMA)
        det_s = mc.Detector(det.side_nx, det.side_ny, det.trans_nx, det.trans_ny, det.flags)
        base = mc.mc_workspace_bytes_batch(det_s, len(ws))
        grid = 2 * torch.cuda.get_device_properties(cuda_device).multi_processor_count
        nbytes = base + (((4096 * grid * 4) + 7) // 8 * 8 if case == "no_entries" else 0)
        kw["workspace_bytes"] = nbytes
    if case == "shape":
        kw.update(block_size=512, chunk=256)
    got = _batch(mc, ws, tables, cuda_device, **kw)
    for k in ("side", "trans", "side_w2", "trans_w2", "scalars"):
        np.testing.assert_array_equal(getattr(ref, k).cpu().numpy(), getattr(got, k).cpu().numpy(), err_msg=k)
    fallback = int(got.workspace[21].item())
    print(f"{case}: {fallback} exits added directly", flush=True)
    if case == "no_entries":
        assert fallback > 0
    else:
        assert fallback == 0
