"""Pair production with annihilation on the GPU (Sec. 2.4.1 lists it among the
photon interactions), through the C interface: the double-escape line and the
full-absorption FEPE of a pair-only slab (closed forms), and the 20236-facet HPGe detector at
2 MeV with synthetic pair partials against the oracle.  Runs without a pair
partial are covered, unchanged, by the other GPU tests."""
import math

import numpy as np
import pytest

from workloads import configs as C
from workloads import xsgen

pytestmark = pytest.mark.gpu

MEC2 = 510.99895
BEAM = C.Source(C.KIND_BEAM, pos=(0.1234, 0.4321, 10.0), direction=(0.0, 0.0, -1.0))


@pytest.fixture(scope="module")
def G():
    from paper_2605_25963_amd import gadep
    gadep.lib()
    return gadep


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def _pair_slab(G, ctx, T, pair, photo_below=None):
    scene, mats, tabs, grid = C.slab(T, 0.0, mu_pair=pair)
    if photo_below is not None:
        E = xsgen.grid_energies(*grid)
        t = list(tabs[1])
        t[0] = np.where(E < 1000.0, photo_below, 1e-30)
        tabs[1] = tuple(t)
    for m, t in tabs.items():
        ctx.set_xs(m, grid, *t)
    ctx.load_scene(0, scene.xyz, scene.tri, scene.tri_region, [(0, 0.0, -1, 0), (1, 1.0, 0, G.ACTIVE)])


def test_pair_double_escape_line(G, ctx):
    # pair-only slab, mu t = 1 at 2 MeV, transparent at 511 keV: every
    # interacting history deposits exactly E0 - 2 m_e c^2 and both
    # annihilation photons leave
    _pair_slab(G, ctx, 5.0, 2.0)
    n, E0 = 4_000_000, 2000.0
    r = ctx.run(BEAM, [E0], n, 61, spectrum=(8192, 0.25))
    t = r.tallies[0]
    ex = math.exp(-1.0)
    assert abs(t.n_uncollided / n - ex) <= 3 * math.sqrt(ex * (1 - ex) / n)
    n_pair = n - t.n_uncollided
    assert t.n_fep == 0 and t.n_absorbed == 0 and t.n_escape == n
    assert t.n_lost == 0 and t.n_killed == 0
    # energies to the tally's 2^-16 keV resolution per history
    assert t.edep_active_keV == pytest.approx(n_pair * (E0 - 2 * MEC2), rel=1e-6)
    assert t.edep_total_keV + t.e_escape_keV == pytest.approx(t.e_source_keV, rel=1e-6)
    assert t.e_escape_keV == pytest.approx(t.n_uncollided * E0 + n_pair * 2 * MEC2, rel=1e-6)
    ch = int((E0 - 2 * MEC2) // 0.25)
    assert r.spectra[0][ch] == n_pair and r.spectra[0].sum() == n_pair


def test_pair_full_absorption(G, ctx):
    # the annihilation photons are photo-absorbed within about a micrometre:
    # FEPE = 1 - exp(-1) up to pair events within a micrometre of a face
    _pair_slab(G, ctx, 5.0, 2.0, photo_below=1e4)
    n = 4_000_000
    ctx.set_option(G.OPT_COUNTERS, 1)
    try:
        r = ctx.run(BEAM, [2000.0], n, 62)
        ev = ctx.get_counters()
    finally:
        ctx.set_option(G.OPT_COUNTERS, 0)
    t = r.tallies[0]
    ex = 1 - math.exp(-1.0)
    p = t.n_fep / n
    assert abs(p - ex) <= 3 * math.sqrt(ex * (1 - ex) / n) + 2e-4
    assert t.n_fep == t.n_absorbed and t.n_lost == 0 and t.n_killed == 0
    assert ev["pair"] == n - t.n_uncollided
    lost_511 = t.n_escape - t.n_uncollided
    assert 2 * (ev["pair"] - lost_511) <= ev["photo"] <= 2 * ev["pair"]
    assert t.edep_total_keV + t.e_escape_keV == pytest.approx(t.e_source_keV, rel=1e-6)


def test_c2_detector_with_pairs_matches_oracle(G, ctx, orc):
    # the 20236-facet HPGe detector at 2 MeV and 1.4 MeV with synthetic pair partials in
    # every material; 100 mm source for more detector events
    w = C.c2_hpge(n_histories=1, distance=100.0)
    w.tables, w.grid = C._tables_for(w.materials, coherent=False, pair=True)
    G.load_workload(ctx, w)
    s = orc.scene_from_workload(w)
    for E, seed in ((2000.0, 63), (1401.452, 64)):
        n = 20_000_000
        ctx.set_option(G.OPT_COUNTERS, 1)
        try:
            r = ctx.run(w.source, [E], n, seed)
            ev = ctx.get_counters()
        finally:
            ctx.set_option(G.OPT_COUNTERS, 0)
        t = r.tallies[0]
        assert t.n_lost == 0 and t.n_killed == 0
        assert t.edep_total_keV + t.e_escape_keV == pytest.approx(t.e_source_keV, rel=1e-6)
        o = s.run(w.source, E, 400_000, 1000 + seed).tally
        m = o.n_histories
        for gk, ok in ((t.n_fep, o.n_fep), (t.n_absorbed, o.n_absorbed)):
            pg, po = gk / n, ok / m
            sg = math.sqrt(max(pg * (1 - pg), 1 / n) / n)
            so = math.sqrt(max(po * (1 - po), 1 / m) / m)
            assert abs(pg - po) <= 3 * math.hypot(sg, so), (E, gk, ok)
        # pair events per history (several per history are impossible: 511 keV
        # photons cannot make pairs, so this is a probability)
        pg, po = ev["pair"] / n, o.n_pair / m
        sg = math.sqrt(max(pg * (1 - pg), 1 / n) / n)
        so = math.sqrt(max(po * (1 - po), 1 / m) / m)
        assert po > 0 and abs(pg - po) <= 3 * math.hypot(sg, so), (E, pg, po)
        assert o.n_balance_fail == 0
