"""Work claims (GADEP_OPT_GUIDE, GADEP_OPT_CLAIM): fixed-size and shrinking
claims hand the same histories to the kernel in different pieces, and each
history draws counter-keyed random numbers, so every tally, spectrum channel,
gradient and history event count is the same bit for bit whatever the claim
schedule -- on the per-lane and pooled kernels, for batches, and for the
no-allocation entry point."""
import numpy as np
import pytest

from workloads import configs as C
from test_gpu_pool import HISTORY_EVENTS, same

pytestmark = pytest.mark.gpu

# (guide, claim): fixed claims of 1024 histories, shrinking claims with the
# defaults, shrinking claims down to one wavefront of histories, coarse ones,
# fixed one-wavefront claims, many small batches
SCHEDULES = ((0, 16), (16, 16), (1, 1), (2, 4096), (0, 1), (8, 2))


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


def over_schedules(G, ctx, fn):
    g0, c0 = ctx.get_option(G.OPT_GUIDE), ctx.get_option(G.OPT_CLAIM)
    out = []
    try:
        for guide, claim in SCHEDULES:
            ctx.set_option(G.OPT_GUIDE, guide)
            ctx.set_option(G.OPT_CLAIM, claim)
            ctx.set_option(G.OPT_COUNTERS, 1)
            r = fn()
            out.append((r, ctx.get_counters()))
    finally:
        ctx.set_option(G.OPT_GUIDE, g0)
        ctx.set_option(G.OPT_CLAIM, c0)
        ctx.set_option(G.OPT_COUNTERS, 0)
    a, ea = out[0]
    for b, eb in out[1:]:
        same(a, b)
        for k in HISTORY_EVENTS:
            assert ea[k] == eb[k], (k, ea[k], eb[k])
    return a


def test_defaults(G, ctx):
    assert ctx.get_option(G.OPT_GUIDE) == 16 and ctx.get_option(G.OPT_CLAIM) == 16
    for bad in (-1, 17):
        with pytest.raises(G.GadepError):
            ctx.set_option(G.OPT_GUIDE, bad)


def test_claims_do_not_change_results_point_source(G, ctx):
    w = C.c2_hpge(n_histories=1)
    G.load_workload(ctx, w)
    print("claims: C2 at 250 mm, 12 energies x 4e6 (+ one ragged energy)", flush=True)
    E = list(w.energies)
    r = over_schedules(G, ctx, lambda: ctx.run(w.source, E, 4_000_001, 11))
    assert all(t.n_histories == 4_000_001 for t in r.tallies)
    print("claims: C2 at 100 mm, gradients and spectra", flush=True)
    w = C.c2_hpge(n_histories=1, distance=100.0)
    G.load_workload(ctx, w)
    over_schedules(G, ctx, lambda: ctx.run_grad(w.source, [122.0, 1332.5], 3_000_000, 12,
                                                np.ones(6, np.float32), spectrum=(4096, 0.5)))
    print("claims: pooled kernel", flush=True)
    ctx.set_option(G.OPT_POOL, 1)
    try:
        over_schedules(G, ctx, lambda: ctx.run(w.source, [661.7], 2_000_000, 13))
    finally:
        ctx.set_option(G.OPT_POOL, 0)


def test_claims_do_not_change_results_small_and_empty(G, ctx):
    w = C.c2_hpge(n_histories=1, distance=100.0)
    G.load_workload(ctx, w)
    print("claims: tiny runs (1, 63, 65 histories)", flush=True)
    for n in (1, 63, 65):
        r = over_schedules(G, ctx, lambda: ctx.run(w.source, [661.7, 59.5], n, 14))
        assert all(t.n_histories == n for t in r.tallies)


def test_claims_do_not_change_results_noalloc(G, ctx):
    w = C.c2_hpge(n_histories=1, distance=100.0)
    G.load_workload(ctx, w)
    print("claims: no-allocation entry point", flush=True)
    over_schedules(G, ctx, lambda: ctx.run_noalloc(w.source, [122.0, 661.7, 1332.5], 2_000_003, 15))
