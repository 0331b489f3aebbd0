"""gadep_run_noalloc (the entry point that allocates no device memory) against
gadep_run on the same inputs, through the C interface: every tally and every
spectrum channel bit for bit, on two calls in a row, the second one smaller,
and size limits rejected on the host."""
import numpy as np
import pytest

from workloads import configs as C

pytestmark = pytest.mark.gpu

FIELDS = ("n_histories", "n_absorbed", "n_fep", "n_escape", "n_uncollided", "n_lost", "n_killed",
          "n_glitch", "n_source_fail", "edep_active_keV", "edep_total_keV", "e_escape_keV",
          "e_source_keV", "spectrum_overflow")


@pytest.fixture(scope="module")
def G():
    from paper_2605_25963_amd import gadep
    gadep.lib()
    return gadep


def same(a, b):
    assert len(a.tallies) == len(b.tallies)
    for ta, tb in zip(a.tallies, b.tallies):
        for f in FIELDS:
            assert getattr(ta, f) == getattr(tb, f), f
    if a.spectra is not None or b.spectra is not None:
        assert np.array_equal(a.spectra, b.spectra)


def test_noalloc_equals_run_on_two_calls(G):
    w = C.c2_hpge(distance=100.0)
    with G.Context(0) as ctx:
        G.load_workload(ctx, w)
        energies = [59.5, 661.7, 1332.5]
        spec = (8192, 0.25)
        print("noalloc: C2 at 100 mm, 3 energies x 400000, spectra", flush=True)
        a = ctx.run_noalloc(w.source, energies, 400_000, seed=1234, spectrum=spec)
        b = ctx.run(w.source, energies, 400_000, seed=1234, spectrum=spec)
        same(a, b)
        assert a.tallies[1].n_fep > 0 and a.spectra.sum() > 0
        # a second, smaller call: the array still holds the first call's contents
        print("noalloc: second call, 1 energy x 50000, no spectra", flush=True)
        a2 = ctx.run_noalloc(w.source, [122.06], 50_000, seed=77, first_history=9)
        b2 = ctx.run(w.source, [122.06], 50_000, seed=77, first_history=9)
        same(a2, b2)
        assert a2.tallies[0].n_histories == 50_000


def test_noalloc_volume_source_and_lines(G):
    w = C.c4_grad()
    with G.Context(0) as ctx:
        G.load_workload(ctx, w)
        print("noalloc: C4 volume source, 2 energies x 100000", flush=True)
        a = ctx.run_noalloc(w.source, [88.0, 1173.2], 100_000, seed=5)
        b = ctx.run(w.source, [88.0, 1173.2], 100_000, seed=5)
        same(a, b)
        src = G.make_source(G.SRC_POINT, (0.0, 0.0, 120.0), lines_keV=[59.5, 661.7, 1173.2],
                            lines_prob=[1.0, 2.0, 0.5])
        print("noalloc: point source with 3 lines x 100000", flush=True)
        a = ctx.run_noalloc(src, None, 100_000, seed=6, spectrum=(4096, 0.5))
        b = ctx.run(src, None, 100_000, seed=6, spectrum=(4096, 0.5))
        same(a, b)


def test_noalloc_rejects_sizes_beyond_the_scratch(G):
    w = C.c1_bare()
    with G.Context(0) as ctx:
        G.load_workload(ctx, w)
        with pytest.raises(G.GadepError) as e:
            ctx.run_noalloc(w.source, np.linspace(100, 200, 257), 10, seed=1)
        assert e.value.name == "GADEP_E_ARG"
        with pytest.raises(G.GadepError) as e:
            ctx.run_noalloc(w.source, np.linspace(100, 200, 100), 10, seed=1,
                            spectrum=(8192, 0.25))
        assert e.value.name == "GADEP_E_ARG" and "scratch" in str(e.value)
        # within the limits it still runs after the rejected calls
        a = ctx.run_noalloc(w.source, [661.7], 20_000, seed=3)
        b = ctx.run(w.source, [661.7], 20_000, seed=3)
        same(a, b)


def test_noalloc_cone_electrons_and_pairs(G):
    """The other kernel variants through the no-allocation entry: a cone
    source (general variant, with its weight), electron tracks, and pair
    production, each equal to gadep_run bit for bit."""
    w = C.c2_hpge(n_histories=1, distance=100.0)
    with G.Context(0) as ctx:
        G.load_workload(ctx, w)
        cone = C.Source(C.KIND_CONE, pos=w.source.pos)
        print("noalloc: cone source", flush=True)
        a = ctx.run_noalloc(cone, [661.7, 1332.5], 200_000, seed=21, spectrum=(4096, 0.5))
        b = ctx.run(cone, [661.7, 1332.5], 200_000, seed=21, spectrum=(4096, 0.5))
        same(a, b)
        assert np.array_equal(a.weights(), b.weights()) and np.all(a.weights() < 1.0)
        print("noalloc: electron tracks", flush=True)
        ctx.set_option(G.OPT_ELECTRONS, 1)
        try:
            a = ctx.run_noalloc(w.source, [661.7, 2000.0], 200_000, seed=22)
            b = ctx.run(w.source, [661.7, 2000.0], 200_000, seed=22)
        finally:
            ctx.set_option(G.OPT_ELECTRONS, 0)
        same(a, b)
        print("noalloc: pair production", flush=True)
        w.tables, w.grid = C._tables_for(w.materials, coherent=False, pair=True)
        G.load_workload(ctx, w)
        a = ctx.run_noalloc(w.source, [2000.0], 200_000, seed=23)
        b = ctx.run(w.source, [2000.0], 200_000, seed=23)
        same(a, b)
        assert a.tallies[0].n_fep > 0
