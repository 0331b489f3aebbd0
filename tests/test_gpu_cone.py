"""Cone emission (GADEP_SRC_CONE, variance reduction for distant point
sources): histories start only in the cone that subtends the bounding sphere
of the detector's inner shells and stand for the weight Omega/4pi.  Its
weighted FEPE must equal the analog FEPE -- the GPU's own analog run and the
oracle, which has no cone code at all -- within 3 combined sigma; a source
inside that sphere falls back to 4 pi bit for bit; a region with a coherent
partial around the source is refused."""
import math

import numpy as np
import pytest

from workloads import configs as C

pytestmark = pytest.mark.gpu


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


def cone_of(src):
    return C.Source(C.KIND_CONE, pos=src.pos)


@pytest.mark.parametrize("cfg", ["c2_250mm", "c1_100mm"])
def test_cone_weighted_fepe_equals_analog(G, ctx, orc, cfg):
    if cfg == "c2_250mm":
        w = C.c2_hpge(n_histories=1)
        E = [40.0, 116.256, 2000.0]
        n_an, n_cone, n_orc = 1_000_000_000, 20_000_000, 10_000_000
    else:
        w = C.c1_bare()
        E = [100.0, 661.7]
        n_an, n_cone, n_orc = 200_000_000, 20_000_000, 4_000_000
    G.load_workload(ctx, w)
    cone = ctx.run(cone_of(w.source), E, n_cone, 1201)
    an = ctx.run(w.source, E, n_an, 1202)
    s = orc.scene_from_workload(w)
    wt = cone.weights()
    assert np.all(wt > 0) and np.all(wt < 0.1) and np.all(wt == wt[0])
    pc, sc = cone.fepe(), cone.fepe_sigma()
    pa, sa = an.fepe(), an.fepe_sigma()
    for k, e in enumerate(E):
        o = s.run(w.source, e, n_orc, 1300 + k)
        po, so = o.fepe(), o.fepe_sigma()
        print(f"cone {cfg} E {e:8.3f}: weight {wt[k]:.6f}  cone {pc[k]:.6e} +- {sc[k]:.1e}  "
              f"analog gpu {pa[k]:.6e} +- {sa[k]:.1e}  oracle {po:.6e} +- {so:.1e}", flush=True)
        assert abs(pc[k] - pa[k]) <= 3 * math.hypot(sc[k], sa[k]), (e, pc[k], pa[k])
        assert abs(pc[k] - po) <= 3 * math.hypot(sc[k], so), (e, pc[k], po)
        t = cone.tallies[k]
        # every cone history heads for the detector: about 1/weight analog
        # histories' worth of entering photons, so the rare FP32 boundary
        # misses the kernel counts as lost show up; they stay below 1e-6
        assert t.n_lost <= 1e-6 * n_cone and t.n_killed == 0 and t.n_histories == n_cone
        # the same relative error costs far fewer histories
        assert sc[k] / pc[k] < sa[k] / pa[k] * math.sqrt(n_an / n_cone) / 3


def test_cone_inside_the_sphere_is_the_point_source(G, ctx):
    w = C.c2_hpge(n_histories=1)
    G.load_workload(ctx, w)
    inside = C.Source(C.KIND_POINT, pos=(3.0, -2.0, -30.0))  # in the detector's vacuum
    a = ctx.run(inside, [661.7], 1_000_000, 1203)
    b = ctx.run(cone_of(inside), [661.7], 1_000_000, 1203)
    assert b.tallies[0].weight == 1.0
    for f in ("n_histories", "n_fep", "n_absorbed", "n_escape", "edep_active_keV", "e_escape_keV"):
        assert getattr(a.tallies[0], f) == getattr(b.tallies[0], f), f


def test_cone_refused_with_coherent_scattering_around_the_source(G, ctx):
    w = C.c5_stress(n_histories=1, n_seg=64, n_phi=8, z_slices=1)  # coherent partials on
    G.load_workload(ctx, w)
    with pytest.raises(G.GadepError) as e:
        ctx.run(C.Source(C.KIND_CONE, pos=(0.0, 0.0, 250.0)), [661.7], 1000, 1)
    assert e.value.name == "GADEP_E_ARG" and "coherent" in str(e.value)
