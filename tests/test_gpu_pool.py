"""The pooled transport kernel (GADEP_OPT_POOL = 1) against the per-lane
kernel (0, the default) on the same histories: every tally, spectrum channel,
gradient and event count that describes the histories (not the schedule) bit
for bit, over the paths the kernels have -- point and volume sources, line
spectra with coherent scattering, pair production, gradients, batches with
scenes and overrides -- and over the pooled kernel's own threshold."""
import numpy as np
import pytest

from workloads import configs as C

pytestmark = pytest.mark.gpu

FIELDS = ("n_histories", "n_absorbed", "n_fep", "n_escape", "n_uncollided", "n_lost", "n_killed",
          "n_glitch", "n_source_fail", "edep_active_keV", "edep_total_keV", "e_escape_keV",
          "e_source_keV", "spectrum_overflow")
# event counts that belong to the histories; loop iterations, passes and
# cycles depend on the schedule
HISTORY_EVENTS = ("segments", "crossings", "node_visits", "tri_tests", "photo", "compton",
                  "coherent", "rng_calls", "locates", "emissions", "plane_tests", "box_tests", "pair",
                  "cone_tests")


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


def same(a, b):
    assert len(a.tallies) == len(b.tallies)
    for k, (ta, tb) in enumerate(zip(a.tallies, b.tallies)):
        for f in FIELDS:
            assert getattr(ta, f) == getattr(tb, f), (k, f, getattr(ta, f), getattr(tb, f))
    if a.spectra is not None or b.spectra is not None:
        assert np.array_equal(a.spectra, b.spectra)
    if a.grad is not None or b.grad is not None:
        assert np.array_equal(a.grad, b.grad) and np.array_equal(a.grad_var, b.grad_var)


def both(G, ctx, fn, counters=True):
    """fn() with the pooled kernel and with the per-lane kernel; also their
    history event counts."""
    out = []
    default = ctx.get_option(G.OPT_POOL)
    for pool in (1, 0):
        ctx.set_option(G.OPT_POOL, pool)
        ctx.set_option(G.OPT_COUNTERS, 1 if counters else 0)
        try:
            r = fn()
            ev = ctx.get_counters() if counters else None
        finally:
            ctx.set_option(G.OPT_POOL, default)
            ctx.set_option(G.OPT_COUNTERS, 0)
        out.append((r, ev))
    (a, ea), (b, eb) = out
    same(a, b)
    if counters:
        for k in HISTORY_EVENTS:
            assert ea[k] == eb[k], (k, ea[k], eb[k])
    return a


def test_pool_equals_per_lane_point_sources(G, ctx):
    w = C.c2_hpge(n_histories=1, distance=20.0)
    G.load_workload(ctx, w)
    print("pool on/off: C2 at 20 mm, 4 energies x 2e6, spectra", flush=True)
    r = both(G, ctx, lambda: ctx.run(w.source, [40.0, 122.0, 661.7, 2000.0], 2_000_000, 7,
                                     spectrum=(8192, 0.25)))
    assert r.tallies[2].n_fep > 1000
    print("pool on/off: C2 at 250 mm (screening), 12 energies x 1e6", flush=True)
    w = C.c2_hpge(n_histories=1)
    G.load_workload(ctx, w)
    both(G, ctx, lambda: ctx.run(w.source, w.energies, 1_000_000, 8))


def test_pool_equals_per_lane_volume_source_with_gradients(G, ctx):
    w = C.c4_grad(n_histories=1)
    G.load_workload(ctx, w)
    print("pool on/off: C4 volume source with gradients, 3 energies x 1e6", flush=True)
    r = both(G, ctx, lambda: ctx.run_grad(w.source, [60.0, 400.0, 1500.0], 1_000_000, 9,
                                          [1.0, 1.1, 0.9, 1.0, 1.0, 1.2]))
    assert np.any(r.grad != 0)


def test_pool_equals_per_lane_lines_coherent_and_pairs(G, ctx):
    w = C.c5_stress(n_histories=1, n_seg=64, n_phi=8, z_slices=1)
    G.load_workload(ctx, w)
    print("pool on/off: Marinelli, 13 lines, coherent, spectra, 2e6", flush=True)
    both(G, ctx, lambda: ctx.run(w.source, None, 2_000_000, 10, spectrum=(8192, 0.25)))
    w = C.c2_hpge(n_histories=1, distance=100.0)
    w.tables, w.grid = C._tables_for(w.materials, coherent=False, pair=True)
    G.load_workload(ctx, w)
    print("pool on/off: C2 with pair production, 2000 keV x 2e6", flush=True)
    r = both(G, ctx, lambda: ctx.run(w.source, [2000.0], 2_000_000, 11))
    assert r.tallies[0].n_absorbed > 0


def test_pool_equals_per_lane_batch_with_scenes(G, ctx):
    jobs = C.c3_jobs(6)
    spec = []
    for k, j in enumerate(jobs):
        w = C.c3_job_workload(j)
        G.load_workload(ctx, w, scene=k)
        spec.append(dict(source=w.source, energies=w.energies[::5], n_histories=50_000 + 20_000 * k,
                         scene=k, stream=k))
    print("pool on/off: 6 bottle jobs x 4 energies, batched", flush=True)
    both(G, ctx, lambda: ctx.run_batch(spec, 12))


def test_pool_threshold_claims_and_autotune_do_not_change_tallies(G, ctx):
    w = C.c2_hpge(n_histories=1, distance=100.0)
    G.load_workload(ctx, w)
    ref = ctx.run(w.source, [59.5, 661.7], 1_000_000, 13)
    ctx.set_option(G.OPT_POOL, 1)
    try:
        for period, claim in ((8, 16), (48, 4), (63, 64)):
            ctx.set_option(G.OPT_PERIOD, period)
            ctx.set_option(G.OPT_CLAIM, claim)
            r = ctx.run(w.source, [59.5, 661.7], 1_000_000, 13)
            same(r, ref)
        job = [dict(source=w.source, energies=[59.5, 661.7], n_histories=1_000_000, stream=0)]
        block, period, claim = ctx.autotune(job, 200_000)
        assert block == 64 and period in (16, 24, 32, 40, 48) and claim in (16, 64)
        same(ctx.run(w.source, [59.5, 661.7], 1_000_000, 13), ref)
    finally:
        ctx.set_option(G.OPT_POOL, 0)
        ctx.set_option(G.OPT_PERIOD, 0)
        ctx.set_option(G.OPT_CLAIM, 16)
