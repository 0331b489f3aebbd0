"""Pins of the CPU oracle against values fixed by the paper and by mathematics.

Each test targets a plausible mistake in the oracle: a wrong Philox round, a
dropped Klein-Nishina term, a wrong sign in the free-flight or score, a
transposed index in the geometry, a parity slip in localization.
"""
import math
import os

import numpy as np
import pytest

from workloads import configs as C
from workloads import meshgen as mg
from workloads import xsgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MEC2 = 510.99895


def _sigma_ok(x, expect, sigma, k=3.0):
    return abs(x - expect) <= k * sigma


# --------------------------------------------------------------------------
# Philox

def test_philox_known_answers(orc):
    rows = 0
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            assert orc.philox(w[0:4], w[4:6]) == w[6:10]
            rows += 1
    assert rows == 3


def test_philox_bytes_uniform(orc):
    # chi^2 of byte frequencies over 40k outputs (160 kB)
    counts = np.zeros(256)
    for i in range(10000):
        for x in orc.philox([i, 7, 0, 3], [0x1234, 0x5678]):
            for s in (0, 8, 16, 24):
                counts[(x >> s) & 0xFF] += 1
    e = counts.sum() / 256
    chi2 = ((counts - e) ** 2 / e).sum()
    # 255 dof: mean 255, sd ~22.6; p < 1e-4 beyond ~350
    assert 170 < chi2 < 350


# --------------------------------------------------------------------------
# Klein-Nishina / Thomson

@pytest.mark.parametrize("E", [1.0, 40.0, 100.0, 661.7, 1332.49, 3000.0])
def test_kn_total_matches_textbook(orc, E):
    k = E / MEC2
    assert orc.kn_sigma(k) == pytest.approx(float(xsgen.sigma_kn(E)), rel=1e-9)


def test_kn_value_at_cs137(orc):
    # sigma_KN(661.7 keV) = 0.25619 b per electron
    assert orc.kn_sigma(661.7 / MEC2) / 1e-24 == pytest.approx(0.25619, abs=5e-6)


def _kn_density(eps, k):
    # d sigma/d eps up to a constant: (1/eps + eps)(1 - eps sin^2/(1 + eps^2))
    ct = 1.0 - (1.0 / eps - 1.0) / k
    s2 = 1.0 - ct * ct
    return (1.0 / eps + eps) * (1.0 - eps * s2 / (1.0 + eps * eps))


@pytest.mark.parametrize("E", [40.0, 661.7, 2000.0])
def test_kn_sampler_histogram(orc, E):
    from scipy import integrate
    k = E / MEC2
    e0 = 1.0 / (1.0 + 2.0 * k)
    n = 40000
    rng = np.random.default_rng(5)
    eps = np.array([orc.kn_sample(k, u) for u in rng.random(n)])
    assert eps.min() >= e0 - 1e-12 and eps.max() <= 1.0 + 1e-12
    edges = np.linspace(e0, 1.0, 31)
    obs, _ = np.histogram(eps, edges)
    w = np.array([integrate.quad(_kn_density, a, b, args=(k,))[0] for a, b in zip(edges[:-1], edges[1:])])
    exp = n * w / w.sum()
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < 70  # 29 dof, p ~ 5e-5


def test_compton_edge(orc):
    # T_max = E 2k/(1+2k) = 477.374 keV at 661.7 keV
    E = 661.7
    k = E / MEC2
    eps_min = orc.kn_sample(k, 1e-15)
    assert E * (1 - eps_min) == pytest.approx(477.374, abs=2e-3)
    assert E * 2 * k / (1 + 2 * k) == pytest.approx(477.374, abs=1e-3)


def test_thomson_sampler(orc):
    n = 40000
    rng = np.random.default_rng(6)
    mu = np.array([orc.thomson_sample(u) for u in rng.random(n)])
    edges = np.linspace(-1, 1, 21)
    obs, _ = np.histogram(mu, edges)
    cdf = lambda x: (x ** 3 + 3 * x + 4) / 8
    exp = n * (cdf(edges[1:]) - cdf(edges[:-1]))
    assert ((obs - exp) ** 2 / exp).sum() < 55  # 19 dof
    assert orc.thomson_sample(0.5) == pytest.approx(0.0, abs=1e-12)


# --------------------------------------------------------------------------
# synthetic cross-section recipe

def test_xs_table_magnitudes():
    pe, c, coh = xsgen.mass_attenuation({"Ge": 1.0}, np.array([100.0, 661.7]))
    assert pe[0] == pytest.approx(0.3999, abs=2e-4)
    assert c[0] == pytest.approx(0.1307, abs=2e-4)
    assert c[1] == pytest.approx(0.06798, abs=2e-5)
    # K edge of Ge: photo drops by 7.5 just below 11.103 keV
    lo, hi = xsgen.mass_attenuation({"Ge": 1.0}, np.array([11.102, 11.103]))[0]
    assert hi / lo == pytest.approx(7.5 * (11.102 / 11.103) ** 3, rel=1e-9)


def test_oracle_interpolation_at_grid_points(orc):
    w = C.c1_bare()
    s = orc.scene_from_workload(w)
    lnE0, dlnE, n = w.grid
    pe, c, _ = w.tables[1]
    rho = float(np.float32(5.32))  # region densities travel as float32
    for k in (0, 100, 511, 1022):
        E = math.exp(lnE0 + k * dlnE)
        mu = s.mu(1, E)
        assert mu[0] == pytest.approx(0.1 * rho * pe[k], rel=1e-12)
        assert mu[1] == pytest.approx(0.1 * rho * c[k], rel=1e-12)
    # between grid points: log-log (geometric) interpolation
    E = math.exp(lnE0 + 100.5 * dlnE)
    assert s.mu(1, E)[1] == pytest.approx(0.1 * rho * math.sqrt(c[100] * c[101]), rel=1e-12)


# --------------------------------------------------------------------------
# geometry

def test_bvh_matches_brute_force(orc):
    w = C.c2_hpge(n_seg=32, n_phi=4)
    sc = w.scene
    a = orc.Scene(sc.xyz, sc.tri, sc.tri_region, sc.n_regions, use_bvh=True)
    b = orc.Scene(sc.xyz, sc.tri, sc.tri_region, sc.n_regions, use_bvh=False)
    rng = np.random.default_rng(11)
    for _ in range(300):
        o = rng.uniform([-45, -45, -110], [45, 45, 20])
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ta, fa = a.closest_hit(o, d)
        tb, fb = b.closest_hit(o, d)
        assert fa == fb and ta == tb
        assert a.locate(o) == b.locate(o)


def test_closest_hit_plane_distance(orc):
    scene, mats, tabs, grid = C.slab(5.0, 1.0)
    s = orc.Scene(scene.xyz, scene.tri, scene.tri_region, scene.n_regions)
    o = np.array([0.1234, 0.4321, 10.0])
    d = np.array([0.3, -0.2, -1.0])
    d /= np.linalg.norm(d)
    t, f = s.closest_hit(o, d)
    assert t == pytest.approx(10.0 / abs(d[2]), rel=1e-14)
    t2, f2 = s.closest_hit(o + t * d, d, exclude=f)
    assert t2 == pytest.approx(5.0 / abs(d[2]), rel=1e-12)


def test_locate_nested_spheres(orc):
    radii = (10.0, 20.0, 30.0)
    sc = C.nested_spheres(radii)
    s = orc.Scene(sc.xyz, sc.tri, sc.tri_region, sc.n_regions)
    rng = np.random.default_rng(12)
    checked = 0
    for _ in range(400):
        p = rng.uniform(-35, 35, size=3)
        r = np.linalg.norm(p)
        if min(abs(r - R) for R in radii) < 0.05 * 30:
            continue
        expect = 0
        # region ids: outermost sphere added first => region 1 = radius 30
        for rid, R in enumerate(sorted(radii, reverse=True), start=1):
            if r < R:
                expect = rid
        assert s.locate(p) == expect
        checked += 1
    assert checked > 200


def test_locate_hpge_regions(orc):
    w = C.c2_hpge(n_seg=64, n_phi=8)
    s = orc.scene_from_workload(w)
    sc = w.scene
    probes = {
        "world": (0, 0, 600), "air": (0, 0, 100), "endcap": (37.5, 0, -50),
        "window": (0, 0, 5.25), "interior": (0, 0, 2.0), "cup": (33.0, 0, -30),
        "dead": (0, 0, -0.3), "active": (20, 0, -30), "bore": (3.0, 0, -40),
        "pin": (0, 0, -40), "coldfinger": (0, 0, -80),
    }
    for name, p in probes.items():
        assert s.locate(np.array(p, float)) == sc.region_id(name), name


# --------------------------------------------------------------------------
# mesh generator (Eq. 1-6)

def test_generator_vertices_follow_eq1_to_eq4():
    N, R = 64, 30.0
    shell = mg.cylinder(R, -60, 0, N)
    th = np.arctan2(shell.V[:, 1], shell.V[:, 0])
    ring = shell.V[np.abs(np.hypot(shell.V[:, 0], shell.V[:, 1]) - R) < 1e-9]
    assert len(ring) == 2 * N
    i = np.round(np.mod(np.arctan2(ring[:, 1], ring[:, 0]), 2 * np.pi) / (2 * np.pi / N)).astype(int) % N
    assert np.allclose(ring[:, 0], R * np.cos(2 * np.pi * i / N), atol=1e-12)
    assert np.allclose(ring[:, 1], R * np.sin(2 * np.pi * i / N), atol=1e-12)
    # rounded edge: every arc vertex sits on the torus (rho - (R-Rc))^2 + (z - (z1-Rc))^2 = Rc^2
    Rr, Rc, z1 = 32.0, 3.0, 0.0
    sh = mg.rounded_cylinder(Rr, -60, z1, Rc, 128, 20)
    rho = np.hypot(sh.V[:, 0], sh.V[:, 1])
    arc = (sh.V[:, 2] >= z1 - Rc - 1e-12) & (rho > Rr - Rc - 1e-9)
    d = np.hypot(rho[arc] - (Rr - Rc), sh.V[arc, 2] - (z1 - Rc))
    assert np.allclose(d, Rc, atol=1e-12)
    zs = np.unique(np.round(sh.V[arc, 2], 12))
    phis = np.sort(np.arcsin(np.clip((zs - (z1 - Rc)) / Rc, -1, 1)))
    assert np.allclose(phis, 0.5 * np.pi * np.arange(21) / 20, atol=1e-9)


def test_generator_signed_volume_and_euler():
    N, r, h = 64, 30.0, 60.0
    sh = mg.cylinder(r, -60, 0, N)
    exact = 0.5 * N * r * r * math.sin(2 * math.pi / N) * h
    assert mg.signed_volume(sh.V, sh.F) == pytest.approx(exact, rel=1e-12)
    assert exact == pytest.approx(169373.6185, abs=1e-4)
    for s in (mg.rounded_cylinder(32, -60, 0, 3, 128, 20), mg.capsule_top(5, -60, -15, 64, 10),
              mg.cup(33.5, 32.5, -62, -1, 1, 64), mg.inverted_cup(70, 40, -60, 27.5, 20, 64),
              mg.box((-1, -1, -1), (1, 1, 1)), mg.uv_sphere(10, 24, 12)):
        assert mg.euler_characteristic(s.F) == 2
        assert mg.signed_volume(s.V, s.F) > 0
    # cup volume = outer prism - cavity prism (both inscribed N-gons)
    a = lambda rr: 0.5 * 64 * rr * rr * math.sin(2 * math.pi / 64)
    cupv = mg.signed_volume(*astuple(mg.cup(33.5, 32.5, -62, -1, 1, 64)))
    assert cupv == pytest.approx(a(33.5) * 61 - a(32.5) * 60, rel=1e-12)


def astuple(s):
    return s.V, s.F


def test_c1_has_256_facets_and_c2_about_20k():
    assert len(C.c1_bare().scene.tri) == 256
    n = len(C.c2_hpge(n_histories=1).scene.tri)
    assert 19000 < n < 21500


# --------------------------------------------------------------------------
# transport closed forms

def _slab_scene(orc, T, photo, compton=0.0, coherent=0.0, active=True):
    scene, mats, tabs, grid = C.slab(T, photo, compton, coherent, active=active)
    s = orc.Scene(scene.xyz, scene.tri, scene.tri_region, scene.n_regions)
    s.set_region(0, 0, 0.0)
    s.set_region(1, 1, 1.0, 0, active)
    for m, t in tabs.items():
        s.set_xs(m, grid, *t)
    return s


BEAM = C.Source(C.KIND_BEAM, pos=(0.1234, 0.4321, 10.0), direction=(0.0, 0.0, -1.0))


# --------------------------------------------------------------------------
# pair production (Sec. 2.4.1): closed forms

MEC2 = 510.99895


def _pair_slab(orc, T, pair, photo_below=None):
    """ACTIVE slab with a constant pair partial; photo_below (optional): a
    photoelectric partial that is large below 1000 keV and negligible above."""
    scene, mats, tabs, grid = C.slab(T, 0.0, mu_pair=pair)
    if photo_below is not None:
        E = xsgen.grid_energies(*grid)
        t = list(tabs[1])
        t[0] = np.where(E < 1000.0, photo_below, 1e-30)
        tabs[1] = tuple(t)
    s = orc.Scene(scene.xyz, scene.tri, scene.tri_region, scene.n_regions)
    s.set_region(0, 0, 0.0)
    s.set_region(1, 1, 1.0, 0, True)
    for m, t in tabs.items():
        s.set_xs(m, grid, *t)
    return s


def test_pair_partial_vanishes_at_threshold(orc):
    s = _pair_slab(orc, 5.0, 2.0)
    assert s.mu(1, 2000.0)[3] == pytest.approx(0.2, rel=1e-12)
    assert s.mu(1, 2 * MEC2)[3] == 0.0 and s.mu(1, MEC2)[3] == 0.0
    assert s.mu(1, 2 * MEC2 * (1 + 1e-9))[3] == pytest.approx(0.2, rel=1e-12)


def test_pair_double_escape_line(orc):
    # A slab that only makes pairs (mu t = 1 at 2 MeV) and is transparent to
    # the 511 keV annihilation photons: each interacting history deposits
    # exactly E0 - 2 m_e c^2 (the double-escape line), the two photons leave,
    # and the uncollided fraction is exp(-1).  Nothing is a full-energy event.
    s = _pair_slab(orc, 5.0, 2.0)
    n, E0 = 200_000, 2000.0
    r = s.run(BEAM, E0, n, 2301, n_channels=8192, channel_keV=0.25)
    t = r.tally
    ex = math.exp(-1.0)
    assert _sigma_ok(t.n_uncollided / n, ex, math.sqrt(ex * (1 - ex) / n))
    assert t.n_pair == n - t.n_uncollided
    assert t.n_fep == 0 and t.n_absorbed == 0 and t.n_escape == n
    assert t.n_balance_fail == 0 and t.n_lost == 0
    assert t.edep_active == pytest.approx(t.n_pair * (E0 - 2 * MEC2), rel=1e-12)
    assert t.e_escape == pytest.approx(t.n_uncollided * E0 + t.n_pair * 2 * MEC2, rel=1e-12)
    ch = int((E0 - 2 * MEC2) // 0.25)
    assert r.spectrum[ch] == t.n_pair and r.spectrum.sum() == t.n_pair


def test_pair_full_absorption(orc):
    # The same slab, but the 511 keV photons are photo-absorbed within about a
    # micrometre: every interacting history deposits all of E0, so the FEPE is
    # 1 - exp(-1) up to the rare pair event within a micrometre of a face.
    s = _pair_slab(orc, 5.0, 2.0, photo_below=1e4)
    n, E0 = 200_000, 2000.0
    r = s.run(BEAM, E0, n, 2302)
    t = r.tally
    ex = 1 - math.exp(-1.0)
    assert abs(r.fepe() - ex) <= 3 * r.fepe_sigma() + 2e-4
    assert t.n_fep == t.n_absorbed and t.n_pair >= t.n_fep
    # both annihilation photons are absorbed unless they leave the slab
    lost_511 = t.n_escape - t.n_uncollided
    assert 2 * (t.n_pair - lost_511) <= t.n_photo <= 2 * t.n_pair
    assert t.n_balance_fail == 0 and t.n_lost == 0


def test_slab_photo_only_fepe(orc):
    # pencil beam on a photo-only ACTIVE slab: FEPE = 1 - exp(-mu t)
    s = _slab_scene(orc, 5.0, 2.0)  # mu = 0.2 /mm, mu t = 1
    r = s.run(BEAM, 661.7, 400_000, 2101, scales=[1.0])
    assert _sigma_ok(r.fepe(), 1 - math.exp(-1.0), r.fepe_sigma())
    assert r.tally.n_fep + r.tally.n_escape == r.tally.n_histories
    assert r.tally.n_balance_fail == 0 and r.tally.n_lost == 0


def test_slab_uncollided_transmission(orc):
    # full physics: uncollided escape fraction = exp(-mu_tot t)
    s = _slab_scene(orc, 5.0, 0.5, 1.0, 0.3)  # mu_tot = 0.18 /mm
    n = 300_000
    r = s.run(BEAM, 300.0, n, 2102)
    p = r.tally.n_uncollided / n
    ex = math.exp(-0.18 * 5.0)
    assert _sigma_ok(p, ex, math.sqrt(ex * (1 - ex) / n))
    assert r.tally.n_balance_fail == 0


def test_slab_density_scale_enters_attenuation(orc):
    s = _slab_scene(orc, 5.0, 2.0)
    r = s.run(BEAM, 661.7, 300_000, 2103, scales=[1.7])
    assert _sigma_ok(r.fepe(), 1 - math.exp(-1.7), r.fepe_sigma())


@pytest.mark.parametrize("scale", [1.0, 1.3])
def test_slab_gradient_closed_form(orc, scale):
    # dFEPE/ds = mu t exp(-s mu t) for the photo-only slab
    s = _slab_scene(orc, 5.0, 2.0)
    r = s.run(BEAM, 661.7, 400_000, 2104, scales=[scale])
    g, gs = r.grad(1)[0], r.grad_sigma(1)[0]
    assert _sigma_ok(g, 1.0 * math.exp(-scale * 1.0), gs)
    # score has zero mean over all histories; |score| <= s mu t here
    assert abs(r.tally.sum_score[0] / r.n) < 3 * 1.3 / math.sqrt(r.n)


def test_slab_gradient_matches_crn_finite_difference(orc):
    s = _slab_scene(orc, 5.0, 1.0, 1.0)  # photo + Compton
    n, h = 300_000, 0.01
    up = s.run(BEAM, 200.0, n, 2105, scales=[1 + h])
    dn = s.run(BEAM, 200.0, n, 2105, scales=[1 - h])
    fd = (up.fepe() - dn.fepe()) / (2 * h)
    r = s.run(BEAM, 200.0, n, 2105, scales=[1.0])
    g, gs = r.grad(1)[0], r.grad_sigma(1)[0]
    assert abs(g - fd) <= max(0.02 * abs(fd), 3 * gs)


def test_black_absorber_solid_angle(orc):
    # photo-only, mu = 5320/mm cylinder; isotropic point on axis at d = 100:
    # FEPE = Omega/4pi of the faceted front face (Van Oosterom-Strackee).
    b = C.bare_crystal(64)
    scene = b.build()
    s = orc.Scene(scene.xyz, scene.tri, scene.tri_region, scene.n_regions)
    s.set_region(0, 0, 0.0)
    s.set_region(1, 1, 5.32, 0, True)
    n = xsgen.GRID_N
    lnE0, dlnE, _ = xsgen.grid()
    s.set_xs(0, (lnE0, dlnE, n), *xsgen.constant_table(n=n))
    s.set_xs(1, (lnE0, dlnE, n), *xsgen.constant_table(1e4, 0, 0, n=n))
    src = C.Source(C.KIND_POINT, pos=(0.0, 0.0, 100.0))
    # exact faceted solid angle from the top-cap fan
    V = scene.xyz.astype(np.float64)
    F = scene.tri
    top = [f for f in F if np.all(np.abs(V[f][:, 2]) < 1e-9)]
    P = np.array([0, 0, 100.0])
    om = 0.0
    for f in top:
        R1, R2, R3 = V[f[0]] - P, V[f[2]] - P, V[f[1]] - P  # as seen from the source
        num = np.dot(R1, np.cross(R2, R3))
        l1, l2, l3 = map(np.linalg.norm, (R1, R2, R3))
        den = l1 * l2 * l3 + np.dot(R1, R2) * l3 + np.dot(R1, R3) * l2 + np.dot(R2, R3) * l1
        om += 2 * math.atan2(num, den)
    frac = abs(om) / (4 * math.pi)
    assert frac == pytest.approx(0.0210551, abs=2e-7)
    disk = 0.5 * (1 - 100 / math.hypot(100, 30))
    assert disk == pytest.approx(0.021087, abs=1e-6)
    r = s.run(src, 661.7, 4_000_000, 2106)
    assert _sigma_ok(r.fepe(), frac, r.fepe_sigma())


def test_infinite_medium_absorbs_everything(orc):
    sh = mg.uv_sphere(1000.0, 48, 24)
    b = mg.SceneBuilder("vacuum", 0.0)
    b.add("ge", "Ge", 5.32, sh, group=0, active=True)
    scene = b.build()
    w = C.Workload("sphere", scene, ["vacuum", "Ge"], C._tables_for(["vacuum", "Ge"])[0],
                   xsgen.grid(), C.Source(C.KIND_POINT, pos=(0.0, 0.0, 0.0)), [661.7], 20000, 1)
    s = orc.scene_from_workload(w)
    r = s.run(w.source, 661.7, 20000, 2107)
    assert r.tally.n_fep == r.tally.n_histories
    assert r.tally.edep_total == pytest.approx(20000 * 661.7, rel=1e-12)
    assert r.tally.n_compton > 20000  # most histories scatter before absorption


def test_energy_conservation_full_detector(orc):
    w = C.c2_hpge(n_seg=64, n_phi=8, distance=20.0)
    s = orc.scene_from_workload(w)
    for E in (40.0, 661.7, 2000.0):
        r = s.run(w.source, E, 100_000, 2108, n_channels=8192, channel_keV=0.25)
        t = r.tally
        assert t.n_balance_fail == 0 and t.n_lost == 0 and t.n_killed == 0
        assert t.edep_total + t.e_escape == pytest.approx(t.n_histories * E, rel=1e-12)
        assert t.n_absorbed + t.n_escape == t.n_histories
        # FEP histories land in the channel holding E (or the one below when E
        # sits on a channel edge and the deposits sum to E minus rounding)
        c = int(E / 0.25)
        assert r.spectrum[c - 1:c + 1].sum() >= t.n_fep
        assert t.n_fep <= t.n_absorbed


def test_thin_photo_slab_spectrum_is_single_line(orc):
    s = _slab_scene(orc, 0.5, 2.0)
    r = s.run(BEAM, 100.0, 50_000, 2109, n_channels=1024, channel_keV=0.25)
    assert r.spectrum.sum() == r.tally.n_fep > 0
    assert r.spectrum[400] == r.tally.n_fep


def test_determinism_and_thread_invariance(orc):
    w = C.c1_bare()
    s = orc.scene_from_workload(w)
    a = s.run(w.source, 661.7, 50_000, 2110, n_channels=256, channel_keV=4.0, threads=1)
    b = s.run(w.source, 661.7, 50_000, 2110, n_channels=256, channel_keV=4.0, threads=7)
    for f in ("n_fep", "n_absorbed", "n_segments", "n_compton"):
        assert getattr(a.tally, f) == getattr(b.tally, f)
    assert np.array_equal(a.spectrum, b.spectrum)
    # disjoint history ranges add up
    c = s.run(w.source, 661.7, 20_000, 2110, first=0, threads=3)
    d = s.run(w.source, 661.7, 30_000, 2110, first=20_000, threads=2)
    assert c.tally.n_fep + d.tally.n_fep == a.tally.n_fep


def test_broadening_moments(orc):
    n, w = 8192, 0.25
    spec = np.zeros(n)
    spec[4000] = 1000.0
    out = orc.broaden(spec, w, 0.64, 0.0018)
    Ec = 4000.5 * w
    sigma = math.sqrt(0.64 + 0.0018 * Ec) / (2 * math.sqrt(2 * math.log(2)))
    centres = (np.arange(n) + 0.5) * w
    assert out.sum() == pytest.approx(1000.0, rel=1e-5)
    assert (out * centres).sum() / out.sum() == pytest.approx(Ec, abs=1e-9)
    var = (out * (centres - Ec) ** 2).sum() / out.sum()
    # channel-integrated Gaussian: variance sigma^2 + w^2/12 (Sheppard)
    assert var == pytest.approx(sigma * sigma + w * w / 12, rel=2e-3)


def test_scales_apply_only_to_listed_groups(orc):
    # a region whose group has no scale passed is transported at density 1
    w = C.c2_hpge(n_seg=32, n_phi=4)
    s = orc.scene_from_workload(w)
    cup = w.scene.region_id("cup")  # group 4
    base = s.mu(cup, 100.0)
    assert np.isfinite(base).all() and base.sum() > 0
    assert np.array_equal(s.mu(cup, 100.0, scales=[2.0]), base)
    scaled = s.mu(cup, 100.0, scales=[1.0, 1.0, 1.0, 1.0, 2.0])
    assert np.allclose(scaled, 2.0 * base, rtol=1e-15)
    dead = w.scene.region_id("dead")  # group 0
    assert np.allclose(s.mu(dead, 100.0, scales=[3.0]), 3.0 * s.mu(dead, 100.0), rtol=1e-15)


def test_grazing_crossings_keep_their_region(orc):
    # a pencil beam almost parallel to a face (d.n = 1e-5) crosses into nested
    # boxes; every crossing must still be localised (none lost) and the
    # transmitted fraction must follow the attenuation along the actual path
    b = mg.SceneBuilder("vacuum", 0.0)
    b.add("outer", "synthetic", 1.0, mg.box((-50, -50, -50), (50, 50, 50)), group=0, active=True)
    b.add("inner", "synthetic", 1.0, mg.box((-20, -20, -20), (20, 20, 20)), group=0, active=True)
    scene = b.build()
    s = orc.Scene(scene.xyz, scene.tri, scene.tri_region, scene.n_regions)
    s.set_region(0, 0, 0.0)
    s.set_region(1, 1, 1.0, 0, True)
    s.set_region(2, 1, 1.0, 0, True)
    lnE0, dlnE, n = xsgen.grid()
    s.set_xs(0, (lnE0, dlnE, n), *xsgen.constant_table(n=n))
    s.set_xs(1, (lnE0, dlnE, n), *xsgen.constant_table(0.01, 0, 0, n=n))  # mu = 1e-3 /mm
    d = np.array([1.0, 0.0, -1e-5])
    d /= np.linalg.norm(d)
    src = C.Source(C.KIND_BEAM, pos=(-60.0, 3.3, 20.0 + 6e-4), direction=tuple(d))
    r = s.run(src, 100.0, 100_000, 2111)
    t = r.tally
    assert t.n_lost == 0 and t.n_balance_fail == 0
    assert t.n_crossings >= 2 * t.n_escape


# --------------------------------------------------------------------------
# scattering rotation, volume emission, line draw, annihilation axis

def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


ROT_DIRS = [(0, 0, 1), (0, 0, -1), (1, 0, 0), (0, -1, 0),
            # |w| above and below the 0.99999 switch to the pole branch
            (math.sqrt(1 - 0.999995 ** 2), 0, 0.999995), (0, math.sqrt(1 - 0.99998 ** 2), -0.99998),
            (0.3, -0.5, 0.81), (-0.7, 0.1, -0.2)]


@pytest.mark.parametrize("d", ROT_DIRS)
def test_rotation_keeps_polar_angle_and_turns_rigidly(orc, d):
    # after a scattering of polar cosine ct the new direction is a unit vector
    # at angle arccos(ct) from the old one, and the azimuth is a rigid turn
    # about it: two azimuths phi1, phi2 give directions whose dot product is
    # ct^2 + st^2 cos(phi1 - phi2), whatever the basis the rotation uses
    d = _unit(d)
    for ct in (-1.0, -0.3, 0.0, 0.5, 0.99):
        st2 = 1.0 - ct * ct
        phis = np.linspace(0.0, 2 * math.pi, 13)[:-1] + 0.1
        outs = [orc.rotate(d, ct, ph) for ph in phis]
        for o in outs:
            assert np.linalg.norm(o) == pytest.approx(1.0, abs=1e-12)
            assert np.dot(o, d) == pytest.approx(ct, abs=1e-12)
        for i in range(len(phis)):
            for j in range(i):
                expect = ct * ct + st2 * math.cos(phis[i] - phis[j])
                assert np.dot(outs[i], outs[j]) == pytest.approx(expect, abs=1e-12)


@pytest.mark.parametrize("d", [ROT_DIRS[0], ROT_DIRS[4], ROT_DIRS[6]])
def test_rotation_azimuth_uniform(orc, d):
    # azimuth of the new direction in a basis of the test's own, for uniform
    # phi: chi-square against a flat histogram (pole branch included)
    from scipy import stats
    d = _unit(d)
    a = np.eye(3)[np.argmin(np.abs(d))]
    e1 = _unit(np.cross(d, a))
    e2 = np.cross(d, e1)
    rng = np.random.default_rng(21)
    n = 20000
    az = np.empty(n)
    for i, ph in enumerate(rng.uniform(0, 2 * math.pi, n)):
        o = orc.rotate(d, 0.2, ph)
        az[i] = math.atan2(np.dot(o, e2), np.dot(o, e1))
    obs, _ = np.histogram(az, np.linspace(-math.pi, math.pi, 37))
    assert stats.chisquare(obs).pvalue > 1e-3


def _box_scene(orc, boxes, vacuum_world=True):
    """Boxes (name, lo, hi, (photo, compton, coherent, pair) mass partials,
    active) in a vacuum world; material i+1 is box i's."""
    b = mg.SceneBuilder("vacuum", 0.0)
    for name, lo, hi, _, active in boxes:
        b.add(name, "synthetic", 1.0, mg.box(lo, hi), group=0, active=active)
    scene = b.build()
    s = orc.Scene(scene.xyz, scene.tri, scene.tri_region, scene.n_regions)
    lnE0, dlnE, n = xsgen.grid()
    s.set_region(0, 0, 0.0)
    s.set_xs(0, (lnE0, dlnE, n), *xsgen.constant_table(n=n))
    for i, (_, _, _, part, active) in enumerate(boxes):
        s.set_region(i + 1, i + 1, 1.0, 0, active)
        pe, cs, coh, pair = part
        s.set_xs(i + 1, (lnE0, dlnE, n), *xsgen.constant_table(pe, cs, coh, n=n, pair=pair))
    return s


def test_volume_emission_fills_the_annulus_uniformly(orc):
    # every try lies inside a box that contains the whole annulus, so each
    # history takes its first draw: r^2, the azimuth and z are each uniform
    from scipy import stats
    s = _box_scene(orc, [("big", (-200, -200, -200), (200, 200, 200), (1.0, 0, 0, None), False)])
    src = C.Source(C.KIND_CYL, pos=(1.0, -2.0, -5.0), r_in=10.0, r_out=40.0, h=30.0, region=1)
    n = 20000
    pts = np.empty((n, 3))
    for h in range(n):
        E, p, tries = s.emission(src, 77, h)
        assert tries == 1
        pts[h] = p
    x, y, z = pts[:, 0] - 1.0, pts[:, 1] + 2.0, pts[:, 2]
    r2 = x * x + y * y
    assert r2.min() >= 100.0 - 1e-9 and r2.max() <= 1600.0 + 1e-9
    for v, lo, hi in ((r2, 100.0, 1600.0), (np.arctan2(y, x), -math.pi, math.pi), (z, -5.0, 25.0)):
        obs, _ = np.histogram(v, np.linspace(lo, hi, 21))
        assert stats.chisquare(obs).pvalue > 1e-3


def test_volume_emission_acceptance_equals_volume_ratio(orc):
    # the sampling cylinder (r 40, h 60) encloses a 64-gon prism (r 20, z in
    # [0, 30]) that is the source region: the fraction of tries accepted is
    # the volume ratio, and the accepted points are uniform in the prism
    from scipy import stats
    b = mg.SceneBuilder("vacuum", 0.0)
    b.add("prism", "synthetic", 1.0, mg.cylinder(20.0, 0.0, 30.0, 64), group=0)
    scene = b.build()
    s = orc.Scene(scene.xyz, scene.tri, scene.tri_region, scene.n_regions)
    src = C.Source(C.KIND_CYL, pos=(0.0, 0.0, -15.0), r_in=0.0, r_out=40.0, h=60.0, region=1)
    n = 20000
    tries = np.empty(n)
    zs = np.empty(n)
    for h in range(n):
        E, p, t = s.emission(src, 78, h)
        assert t >= 1
        tries[h] = t
        zs[h] = p[2]
        assert 0.0 <= p[2] <= 30.0 and math.hypot(p[0], p[1]) <= 20.0
    v_prism = 0.5 * 64 * 20.0 ** 2 * math.sin(2 * math.pi / 64) * 30.0
    p_acc = v_prism / (math.pi * 40.0 ** 2 * 60.0)
    # tries per history are geometric: mean 1/p, variance (1 - p)/p^2
    m = tries.mean()
    assert abs(m - 1 / p_acc) <= 3 * math.sqrt((1 - p_acc) / p_acc ** 2 / n)
    obs, _ = np.histogram(zs, np.linspace(0, 30, 16))
    assert stats.chisquare(obs).pvalue > 1e-3


def test_line_draw_follows_the_weights(orc):
    # a point source inside a black absorber (photo only, mu = 1000 /mm,
    # ACTIVE): every history deposits its line energy, so the counts in the
    # lines' channels follow the weights and the mean deposit is sum(p E)/sum(p)
    from scipy import stats
    s = _box_scene(orc, [("black", (-10, -10, -10), (10, 10, 10), (1e4, 0, 0, None), True)])
    lines = [60.0, 300.0, 662.0, 1300.0]
    prob = [1.0, 2.0, 3.0, 4.0]
    src = C.Source(C.KIND_POINT, pos=(0.1, 0.2, 0.3), lines_keV=lines, lines_prob=prob)
    n = 200_000
    r = s.run(src, 0.0, n, 2201, n_channels=8192, channel_keV=0.25)
    t = r.tally
    assert t.n_fep == n and t.n_balance_fail == 0
    ch = [int(e / 0.25) for e in lines]
    obs = np.array([r.spectrum[c] for c in ch])
    assert obs.sum() == n
    p = np.array(prob) / sum(prob)
    assert stats.chisquare(obs, n * p).pvalue > 1e-3
    E, mean = np.array(lines), float(np.dot(p, lines))
    sd = math.sqrt(float(np.dot(p, (E - mean) ** 2)) / n)
    assert abs(t.edep_active / n - mean) <= 3 * sd


def test_annihilation_photons_fly_back_to_back(orc):
    # A 1 mm slab that only makes pairs (transparent at 511 keV, not ACTIVE)
    # lies just above a wide black ACTIVE absorber.  A 2 MeV pencil beam
    # starts in the slab and runs upward, away from the absorber.  Of the two
    # annihilation photons exactly one runs downward (back to back), so every
    # pair event puts 511 keV, never 1022 keV, into the absorber (but for the
    # rare downward photon so flat that it passes beside the absorber).
    s = _box_scene(orc, [
        ("slab", (-10, -10, -1.0), (10, 10, 0.0), (0, 0, 0, 2.0), False),
        ("black", (-500, -500, -500), (500, 500, -1.001), (1e4, 0, 0, None), True)])
    src = C.Source(C.KIND_BEAM, pos=(0.123, 0.432, -0.5), direction=(0.0, 0.0, 1.0))
    n = 200_000
    r = s.run(src, 2000.0, n, 2202, n_channels=8192, channel_keV=0.25)
    t = r.tally
    p_pair = 1 - math.exp(-0.2 * 0.5)
    assert abs(t.n_pair / n - p_pair) <= 3 * math.sqrt(p_pair * (1 - p_pair) / n)
    one, two = int(MEC2 / 0.25), int(2 * MEC2 / 0.25)
    assert r.spectrum[two] == 0 and r.spectrum.sum() == r.spectrum[one]
    assert r.spectrum[one] >= 0.99 * t.n_pair
    assert t.edep_active == pytest.approx(r.spectrum[one] * MEC2, rel=1e-12)
    assert t.n_fep == 0 and t.n_balance_fail == 0 and t.n_lost == 0


def test_thomson_sampler_moments(orc):
    # moments of 3/8 (1 + mu^2) on [-1, 1] by the inverse CDF on a midpoint
    # grid of u: E[mu] = 0, E[mu^2] = 2/5, E[mu^4] = 9/35 (independent of the
    # CDF the sampler inverts)
    n = 20000
    mu = np.array([orc.thomson_sample((i + 0.5) / n) for i in range(n)])
    assert mu.mean() == pytest.approx(0.0, abs=1e-9)
    assert (mu ** 2).mean() == pytest.approx(2 / 5, abs=1e-6)
    assert (mu ** 4).mean() == pytest.approx(9 / 35, abs=1e-6)


def _recoil_density(T, E):
    # Compton recoil-electron energy distribution, textbook form in s = T/E:
    # 2 + s^2/(k^2 (1-s)^2) + s/(1-s) (s - 2/k), k = E / m_e c^2
    k = E / MEC2
    s = T / E
    return 2 + s * s / (k * k * (1 - s) ** 2) + s / (1 - s) * (s - 2 / k)


def test_single_scatter_thin_slab_spectrum(orc):
    # pencil beam through a small Compton-only ACTIVE block (0.5 mm deep, 2 mm
    # wide, mu t = 0.01): almost every interacting history scatters once and
    # leaves, depositing the recoil energy T, so the deposit spectrum follows
    # d sigma / dT and the interacting fraction is 1 - exp(-mu t)
    from scipy import integrate, stats
    s = _box_scene(orc, [("thin", (-1, -1, -0.5), (1, 1, 0.0), (0, 0.2, 0, None), True)])
    src = C.Source(C.KIND_BEAM, pos=(0.0123, -0.0321, 10.0), direction=(0.0, 0.0, -1.0))
    E, n = 661.7, 3_000_000
    r = s.run(src, E, n, 2203, n_channels=8192, channel_keV=0.25)
    t = r.tally
    p_int = 1 - math.exp(-0.02 * 0.5)
    hit = int(r.spectrum.sum())
    assert abs(hit / n - p_int) <= 3 * math.sqrt(p_int * (1 - p_int) / n)
    k = E / MEC2
    tmax = E * 2 * k / (1 + 2 * k)
    # 24 bins of 80 channels (20 keV) up to 480 keV; the last holds the edge
    edges = np.arange(0, 25) * 80
    obs = np.array([r.spectrum[a:b].sum() for a, b in zip(edges[:-1], edges[1:])], float)
    w = np.array([integrate.quad(_recoil_density, a * 0.25, min(b * 0.25, tmax), args=(E,))[0]
                  for a, b in zip(edges[:-1], edges[1:])])
    # deposits above the Compton edge need a second scattering (about 0.3 %)
    assert hit - obs.sum() <= 0.01 * hit
    assert stats.chisquare(obs, obs.sum() * w / w.sum()).pvalue > 1e-3
    assert t.n_balance_fail == 0


# --------------------------------------------------------------------------
# secondary electrons: straight CSDA tracks (Katz-Penfold mass range)

def _electron_slab_fepe(mu, d, R):
    """FEPE of a normal pencil beam on a photo-only ACTIVE slab of thickness d
    whose photoelectrons leave isotropically from the absorption depth z and
    run a straight range R: one escapes through a face at distance h with
    probability (1 - h/R)/2 for h < R (the directions within arccos(h/R) of
    the face's normal), and then takes part of the energy out of the world."""
    from scipy import integrate

    def f(h):
        return max(0.0, 1.0 - h / R) / 2.0

    val, _ = integrate.quad(lambda z: mu * math.exp(-mu * z) * (1.0 - f(z) - f(d - z)), 0.0, d,
                            points=[R, d - R], limit=200)
    return val


@pytest.mark.parametrize("E", [400.0, 1000.0])
def test_photoelectron_escape_from_a_slab(orc, E):
    # density 5 g/cm3, photo partial 1 cm2/g: mu = 0.5 / mm; slab 2 mm
    rho, d = 5.0, 2.0
    scene, mats, tabs, grid = C.slab(d, 1.0, density=rho)
    s = orc.Scene(scene.xyz, scene.tri, scene.tri_region, scene.n_regions)
    s.set_region(0, 0, 0.0, -1, False)
    s.set_region(1, 1, rho, -1, True)
    for m, t in tabs.items():
        s.set_xs(m, grid, *t)
    s.set_electrons(True)
    R = 10.0 * orc.lib().orc_csda_range(E) / rho  # mm
    assert 0.1 < R < d / 2
    src = C.Source(C.KIND_BEAM, pos=(0.3, -0.2, 10.0), direction=(0.0, 0.0, -1.0))
    n = 600_000
    r = s.run(src, E, n, 77)
    expect = _electron_slab_fepe(0.5, d, R)
    p = r.fepe()
    sig = math.sqrt(expect * (1 - expect) / n)
    assert abs(p - expect) <= 3 * sig, (E, p, expect, sig)
    # without the electron tracks every absorbed photon is a full-energy event
    no_elec = 1.0 - math.exp(-0.5 * d)
    assert p < no_elec - 10 * sig
    t = r.tally
    assert t.n_balance_fail == 0 and t.n_lost == 0 and t.n_electrons == t.n_photo
    assert t.edep_total + t.e_escape == pytest.approx(n * E, rel=1e-9)


def test_csda_range_inverse_and_threshold(orc):
    L = orc.lib()
    for T in (12.0, 100.0, 661.7, 2499.0, 2501.0, 3000.0):
        assert L.orc_csda_energy(L.orc_csda_range(T)) == pytest.approx(T, rel=1e-9)
    rs = [L.orc_csda_range(T) for T in np.linspace(10.0, 3000.0, 400)]
    assert all(b > a for a, b in zip(rs, rs[1:]))
    # below 10 keV (the range relation's lower end) electrons deposit in place:
    # results equal those without electrons
    scene, mats, tabs, grid = C.slab(2.0, 1.0, density=5.0)
    out = []
    for on in (False, True):
        s = orc.Scene(scene.xyz, scene.tri, scene.tri_region, scene.n_regions)
        s.set_region(0, 0, 0.0, -1, False)
        s.set_region(1, 1, 5.0, -1, True)
        for m, t in tabs.items():
            s.set_xs(m, grid, *t)
        s.set_electrons(on)
        src = C.Source(C.KIND_BEAM, pos=(0.0, 0.0, 10.0), direction=(0.0, 0.0, -1.0))
        out.append(s.run(src, 8.0, 20_000, 5).tally)
    assert out[0].n_fep == out[1].n_fep and out[1].n_electrons == 0
