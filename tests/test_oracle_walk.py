"""Pins of the oracle's photon walk (Sec. 3.1.3) against closed forms and
invariants: Beer-Lambert ballistic transmission (Eq. 1), exact per-photon
energy balance under Eq. 16, a pure absorber, Fresnel identities, the
orthonormal rotation basis, single-scatter statistics of the free path
(Eq. 15), polar angle (inverse CDF / Eq. 11) and azimuth (uniform on
[0, 2 pi)), the detector orientation, resumability by photon range, and the
adjoint's weight score against a common-random-number difference."""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import mie, philox
from oracle import walk as owalk

WATER = 1.33


def _matched(**kw):
    """Index-matched walls (no Fresnel term)."""
    return W.TINY.replace(n_outside=WATER, **kw)


def _binom_ok(count, n, p, k=4.0):
    return abs(count - n * p) <= k * math.sqrt(n * p * (1 - p)) + 1


@pytest.fixture(scope="module")
def c1_table():
    return mie.table_from_workload(W.TINY)


# ------------------------------------------------------------- Beer-Lambert

@pytest.mark.parametrize("tau", [0.5, 1.0, 2.0, 4.0])
def test_ballistic_fraction_is_beer_lambert(tau, c1_table):
    w = _matched(tau=tau, n_photons=40000)
    r = owalk.Walk(w, c1_table).run(records=True)
    k, face = r.rec("k"), r.rec("face")
    ball = (k == 0) & (face == 5)
    assert np.all(face[k == 0] == 5)                       # unscattered => straight through
    assert _binom_ok(ball.sum(), w.n_photons, math.exp(-tau))
    assert np.all(r.rec("px")[ball] == 5.0) and np.all(r.rec("py")[ball] == 5.0)
    assert np.all(r.rec("w")[ball] == 1.0)


def test_pure_absorber_transmits_exp_minus_tau(c1_table):
    # albedo 0: every interaction removes the whole weight (Eq. 16).
    tau = 1.5
    w = _matched(tau=tau, albedo=0.0, roulette_w=0.0, n_photons=40000)
    r = owalk.Walk(w, c1_table).run()
    assert r.side.sum() == 0.0
    assert _binom_ok(r.trans.sum(), w.n_photons, math.exp(-tau))
    assert r.scalars[6] == pytest.approx(w.n_photons - r.trans.sum(), rel=1e-12)


def test_no_extinction_every_photon_leaves_through_the_far_faces(c1_table):
    # tau = 0: each wall hit reflects with the normal-incidence R; the photon
    # leaves +z with probability 1/(1+R) and -z with R/(1+R).
    w = W.TINY.replace(tau=0.0, n_photons=100000)
    r = owalk.Walk(w, c1_table).run(records=True)
    R = ((1.0 - WATER) / (1.0 + WATER)) ** 2
    assert np.all(r.rec("k") == 0)
    faces = r.rec("face")
    assert set(np.unique(faces)) <= {4, 5}
    assert _binom_ok((faces == 4).sum(), w.n_photons, R / (1 + R))
    assert np.all(r.rec("w") == pytest.approx(1.0 - R, rel=1e-15))


# ----------------------------------------------------------- energy balance

def test_energy_balance_per_photon_without_roulette(c1_table):
    w = W.TINY.replace(tau=3.0, albedo=0.9, roulette_w=0.0, n_photons=5000)
    r = owalk.Walk(w, c1_table).run(records=True)
    w0 = 1.0 - ((1.0 - WATER) / (1.0 + WATER)) ** 2
    cause = r.rec("cause")
    out = np.where(cause == 0, r.rec("w"), 0.0) + np.where(cause == 2, r.rec("w"), 0.0)
    np.testing.assert_allclose(out + r.rec("A"), w0, rtol=0, atol=1e-12)


def test_energy_balance_with_roulette(c1_table):
    w = W.TINY.replace(tau=6.0, albedo=0.5, roulette_w=0.01, roulette_p=0.1, n_photons=40000)
    r = owalk.Walk(w, c1_table).run(records=True)
    s = r.scalars
    w0 = 1.0 - ((1.0 - WATER) / (1.0 + WATER)) ** 2
    assert s[11] > 1000                                         # roulette did fire
    # Exact bookkeeping: start weight + roulette gains/losses = exits + absorbed + capped.
    assert s[0:6].sum() + s[6] + s[8] == pytest.approx(w.n_photons * w0 + s[7], rel=1e-12)
    # Unbiasedness: mean (exit + absorbed) per photon is w0 within MC noise.
    per = np.where(r.rec("cause") == 0, r.rec("w"), 0.0) + r.rec("A")
    assert abs(per.mean() - w0) <= 4 * per.std() / math.sqrt(len(per))


def test_step_cap_is_counted(c1_table):
    w = W.TINY.replace(tau=8.0, max_steps=3, n_photons=5000)
    r = owalk.Walk(w, c1_table).run(records=True)
    s = r.scalars
    capped = r.rec("cause") == 2
    assert capped.sum() == s[12] > 0
    assert np.all(r.rec("steps")[capped] == 3)
    assert s[8] == pytest.approx(r.rec("w")[capped].sum(), rel=1e-12)


# ---------------------------------------------------------- Fresnel, basis

@pytest.mark.parametrize("n1,n2", [(1.33, 1.0), (1.0, 1.33), (1.5, 1.2)])
def test_fresnel_identities(n1, n2):
    f = owalk.fresnel
    assert f(1.0, n1, n2) == pytest.approx(((n1 - n2) / (n1 + n2)) ** 2, rel=1e-14)
    assert f(0.3, n1, n1) == 0.0
    for ci in (0.95, 0.8, 0.6):
        si = math.sqrt(1 - ci * ci)
        st = n1 / n2 * si
        if st >= 1:
            assert f(ci, n1, n2) == 1.0                         # total internal reflection
            continue
        ct = math.sqrt(1 - st * st)
        assert f(ci, n1, n2) == pytest.approx(f(ct, n2, n1), rel=1e-12)   # reciprocity
    # Brewster angle: R_p vanishes, so R = R_s / 2 = sin^2(i - t) / (2 sin^2(i + t)).
    ib = math.atan(n2 / n1)
    it = math.asin(n1 / n2 * math.sin(ib))
    assert f(math.cos(ib), n1, n2) == pytest.approx(
        0.5 * math.sin(ib - it) ** 2 / math.sin(ib + it) ** 2, rel=1e-12)
    if n1 < n2:
        assert f(1e-9, n1, n2) == pytest.approx(1.0, abs=1e-8)    # grazing


@pytest.mark.parametrize("d", [(0, 0, 1), (0, 0, -1), (1, 0, 0), (0.3, -0.4, 0.866),
                               (0.6, 0.0, -0.8), (1e-9, 0, -1)])
def test_rotation_basis_is_orthonormal_and_right_handed(d):
    d = np.array(d, float)
    d /= np.linalg.norm(d)
    e1 = owalk.rotate(d, 0.0, 1.0, 1.0, 0.0)
    e2 = owalk.rotate(d, 0.0, 1.0, 0.0, 1.0)
    np.testing.assert_allclose([e1 @ d, e2 @ d, e1 @ e2], 0.0, atol=1e-12)
    np.testing.assert_allclose(np.cross(e1, e2), d, atol=1e-12)
    rng = np.random.default_rng(1)
    for _ in range(20):
        th, ph = rng.uniform(0, math.pi), rng.uniform(0, 2 * math.pi)
        n = owalk.rotate(d, math.cos(th), math.sin(th), math.cos(ph), math.sin(ph))
        assert np.linalg.norm(n) == pytest.approx(1.0, abs=1e-14)
        assert n @ d == pytest.approx(math.cos(th), abs=1e-12)


# ------------------------------------------------ single-scatter statistics

def _single_scatter(phase, table=None, g=None, n=100000):
    """One interaction in an effectively infinite medium (mu_t = 1/mm):
    record the free path and the first scattered direction."""
    big = 1e6
    w = W.TINY.replace(size_mm=(big, big, big), src_pos_mm=(big / 2, big / 2, 0.0), tau=big,
                       max_steps=1, phase=phase, n_photons=n, roulette_w=0.0)
    return w, owalk.Walk(w, table, g=g).run(records=True)


def test_draw_use_matches_the_stated_mapping(c1_table):
    # Step 0 of photon i uses Philox words (u0, u1, u2) for free path, polar
    # angle and azimuth; checked against the independent Python Philox.
    w, r = _single_scatter(W.PHASE_MIE, c1_table, n=64)
    for i in range(64):
        r0, r1, r2, _ = philox.step_block(w.seed, i, 0)
        u0, u1, u2 = (philox.to_uniform(v) for v in (r0, r1, r2))
        assert r.rec("pz")[i] == pytest.approx(-math.log(u0), rel=1e-12)
        v = mie.sample_table(c1_table.v, u1)
        assert r.rec("dz")[i] == pytest.approx(1.0 - v, abs=1e-12)
        phi = math.atan2(r.rec("dy")[i], r.rec("dx")[i]) % (2 * math.pi)
        assert phi == pytest.approx(2 * math.pi * u2, abs=1e-9)


@pytest.mark.parametrize("g", [0.0, 0.8668, -0.3])
def test_single_scatter_hg_statistics(g):
    w, r = _single_scatter(W.PHASE_HG, g=g)
    mu = r.rec("dz")
    assert abs(mu.mean() - g) <= 4 * mu.std() / math.sqrt(len(mu))      # <cos> = g
    if g == 0.0:
        cdf = lambda m: (m + 1) / 2
    else:
        cdf = lambda m: (1 - g * g) / (2 * g) * ((1 + g * g - 2 * g * m) ** -0.5 - 1 / (1 + g))
    assert stats.kstest(mu, cdf).pvalue > 1e-3
    phi = np.arctan2(r.rec("dy"), r.rec("dx")) % (2 * math.pi)
    assert stats.kstest(phi / (2 * math.pi), "uniform").pvalue > 1e-3
    assert stats.kstest(r.rec("pz"), "expon").pvalue > 1e-3              # Eq. 15, mu_t = 1
    assert np.all(r.rec("k") == 1)


def test_single_scatter_mie_statistics(c1_table):
    w, r = _single_scatter(W.PHASE_MIE, c1_table)
    # Reference CDF of cos(theta) from Eqs. 5-9 on a fine grid, independent of
    # the 1801-angle table the walk samples.
    th = mie.angle_grid(36001)
    P = mie.phase_function(th, c1_table.x, c1_table.a, c1_table.b, c1_table.q_sca)
    F = mie.cdf_in_theta(th, P)
    mu_grid = np.cos(th)[::-1]
    G = (1.0 - F)[::-1]                      # P(cos <= mu)
    cdf = lambda m: np.interp(m, mu_grid, G)
    assert stats.kstest(r.rec("dz"), cdf).pvalue > 1e-3
    mu = r.rec("dz")
    assert abs(mu.mean() - c1_table.g) <= 4 * mu.std() / math.sqrt(len(mu))


# -------------------------------------------------------------- detector

def test_transmitted_image_orientation(c1_table):
    w = _matched(tau=0.0, src_pos_mm=(2.3, 7.9, 0.0), n_photons=100)
    r = owalk.Walk(w, c1_table).run()
    row, col = int(7.9 / 10 * 128), int(2.3 / 10 * 128)     # rows y, columns x
    assert r.trans[row, col] == 100.0 and r.trans.sum() == 100.0


def test_side_image_orientation(c1_table):
    a = math.radians(60.0)
    w = _matched(tau=0.0, src_pos_mm=(5.0, 3.3, 0.0), src_dir=(math.sin(a), 0.0, math.cos(a)),
                 n_photons=100)
    r = owalk.Walk(w, c1_table).run(records=True)
    z_exit = 5.0 / math.tan(a)
    assert np.all(r.rec("face") == 1)
    np.testing.assert_allclose(r.rec("pz"), z_exit, rtol=1e-12)
    row, col = int(3.3 / 10 * 128), int(z_exit / 10 * 128)  # rows y, columns z
    assert r.side[row, col] == 100.0 and r.side.sum() == 100.0


def test_lateral_faces_are_symmetric(c1_table):
    w = W.TINY.replace(tau=4.0, n_photons=60000)
    r = owalk.Walk(w, c1_table).run(records=True)
    face, wt = r.rec("face"), r.rec("w")
    tot = [wt[face == f].sum() for f in range(4)]
    sig = math.sqrt(max(tot) * 1.0)
    for f in range(1, 4):
        assert abs(tot[f] - tot[0]) <= 5 * sig
    # Images agree with the records they are tallied from.
    assert r.side.sum() == pytest.approx(tot[1], rel=1e-12)
    assert r.trans.sum() == pytest.approx(wt[face == 5].sum(), rel=1e-12)


def test_path_length_bounds_displacement(c1_table):
    w = W.TINY.replace(tau=4.0, n_photons=3000)
    r = owalk.Walk(w, c1_table).run(records=True)
    disp = np.sqrt((r.rec("px") - 5) ** 2 + (r.rec("py") - 5) ** 2 + r.rec("pz") ** 2)
    assert np.all(r.rec("L") >= disp - 1e-9)
    ex = r.rec("cause") == 0
    assert np.all(r.rec("steps")[ex] >= r.rec("k")[ex] + 1)


# ------------------------------------------------------- adjoint score

def test_albedo_score_equals_common_random_number_difference(c1_table):
    # The perturbation Monte Carlo score of the adjoint: at fixed mu_ext a
    # detected photon's weight is w0 a^k (Eq. 16 applied k times), so
    # d/da of any linear functional of the side image is sum g w k / a, and
    # d/da = mu_ext (d/dmu_sca - d/dmu_abs) with the scores k/mu_sca - L and
    # -L.  Walks at a +- delta with the same draws follow the same
    # trajectories (the albedo only scales weights), so their central
    # difference must equal that score sum to O(delta^2 k^2).
    w = W.TINY.replace(tau=4.0, n_photons=6000)
    base = owalk.Walk(w, c1_table).run(records=True)
    delta = 5e-5                                   # albedo 0.9999 +- delta stays at or below 1
    up = owalk.Walk(w.replace(albedo=w.albedo + delta), c1_table).run(records=True)
    dn = owalk.Walk(w.replace(albedo=w.albedo - delta), c1_table).run(records=True)
    for r in (up, dn):
        np.testing.assert_array_equal(r.irec, base.irec)
    g = np.random.default_rng(3).normal(size=base.side.shape)
    fd = (np.sum(g * up.side) - np.sum(g * dn.side)) / (2 * delta)
    sel = (base.rec("face") == 1) & (base.rec("cause") == 0)
    n = w.side_px
    rows = np.clip(np.floor(base.rec("py")[sel] / w.size_mm[1] * n).astype(int), 0, n - 1)
    cols = np.clip(np.floor(base.rec("pz")[sel] / w.size_mm[2] * n).astype(int), 0, n - 1)
    score = np.sum(g[rows, cols] * base.rec("w")[sel] * base.rec("k")[sel]) / w.albedo
    mu_t = w.tau / w.size_mm[2]
    mu_s, L = w.albedo * mu_t, base.rec("L")[sel]
    by_coefficients = mu_t * np.sum(g[rows, cols] * base.rec("w")[sel] * ((base.rec("k")[sel] / mu_s - L) + L))
    assert sel.sum() > 200
    assert fd == pytest.approx(score, rel=1e-4)
    assert by_coefficients == pytest.approx(score, rel=1e-12)


# -------------------------------------------------------------- resume

def test_photon_ranges_compose(c1_table):
    w = W.TINY.replace(tau=2.0, n_photons=4000)
    wk = owalk.Walk(w, c1_table)
    full = wk.run(records=True, chunks=1)
    a = wk.run(n_photons=1500, records=True, chunks=1)
    b = wk.run(n_photons=2500, photon_offset=1500, records=True, chunks=1)
    np.testing.assert_array_equal(np.concatenate([a.irec, b.irec], 1), full.irec)
    np.testing.assert_array_equal(np.concatenate([a.frec, b.frec], 1), full.frec)
    np.testing.assert_allclose(a.side + b.side, full.side, rtol=1e-12, atol=1e-15)
    ids = np.array([17, 3999, 0, 2048], dtype=np.uint64)
    c = wk.run(ids=ids, records=True)
    np.testing.assert_array_equal(c.frec, full.frec[:, ids.astype(int)])


def test_exit_refraction_restores_the_incident_direction(c1_table):
    # tau = 0: the beam refracts in at z = 0 and out at the parallel face
    # z = L (Snell twice), so photons leaving +z on their first wall hit carry
    # the incident direction again; those reflected first leave -z mirrored.
    d = np.array([0.3, -0.2, 0.9])
    d /= np.linalg.norm(d)
    w = W.TINY.replace(tau=0.0, src_pos_mm=(2.0, 8.0, 0.0), src_dir=tuple(d), size_mm=(50.0, 50.0, 10.0),
                       n_photons=2000)
    r = owalk.Walk(w, c1_table).run(records=True)
    out = np.stack([r.rec("dx"), r.rec("dy"), r.rec("dz")], 1)
    first = (r.rec("face") == 5) & (r.rec("steps") == 1)
    assert first.sum() > 1500
    np.testing.assert_allclose(out[first], np.broadcast_to(d, out[first].shape), atol=1e-14)
    back = r.rec("face") == 4
    np.testing.assert_allclose(out[back], np.broadcast_to(d * [1, 1, -1], out[back].shape), atol=1e-14)
