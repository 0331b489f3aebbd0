"""ctypes front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product package.  It
shares nothing with the HIP path except the input arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
MAX_GROUPS = 8
POINT, BEAM, CYL = 0, 1, 2


def build(verbose=False):
    """Compile oracle.c into liboracle.so with gcc."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-o", LIB_PATH, os.path.join(HERE, "oracle.c"), "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)


class Tally(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "n_histories", "n_absorbed", "n_fep", "n_uncollided", "n_escape", "n_lost", "n_killed",
        "n_source_fail", "n_balance_fail", "n_segments", "n_crossings", "n_photo", "n_compton",
        "n_coherent", "n_pair", "n_electrons", "spectrum_overflow")] + [
        ("edep_active", C.c_double), ("edep_total", C.c_double), ("e_escape", C.c_double),
        ("sum_score", C.c_double * MAX_GROUPS), ("sum_fep_score", C.c_double * MAX_GROUPS),
        ("sum_fep_score2", C.c_double * MAX_GROUPS)]


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos", C.c_double * 3), ("dir", C.c_double * 3),
                ("r_in", C.c_double), ("r_out", C.c_double), ("h", C.c_double),
                ("region", C.c_int32), ("n_lines", C.c_int32),
                ("line_keV", C.POINTER(C.c_double)), ("line_prob", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_scene_create.restype = C.c_void_p
        L.orc_scene_create.argtypes = [C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.c_int64, C.c_int32, C.c_int32]
        L.orc_scene_destroy.argtypes = [C.c_void_p]
        L.orc_set_region.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_int32]
        L.orc_set_xs.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_int32, dp, dp, dp,
                                 dp]
        L.orc_locate.restype = C.c_int32
        L.orc_locate.argtypes = [C.c_void_p, dp]
        L.orc_closest_hit.restype = C.c_int32
        L.orc_closest_hit.argtypes = [C.c_void_p, dp, dp, C.c_int64, dp, C.POINTER(C.c_int64)]
        L.orc_mu.argtypes = [C.c_void_p, C.c_int32, C.c_double, dp, C.c_int32, dp]
        for f in ("orc_kn_integral", "orc_kn_sigma", "orc_kn_sample", "orc_thomson_sample"):
            getattr(L, f).restype = C.c_double
        L.orc_kn_integral.argtypes = [C.c_double, C.c_double]
        L.orc_kn_sigma.argtypes = [C.c_double]
        L.orc_kn_sample.argtypes = [C.c_double, C.c_double]
        L.orc_thomson_sample.argtypes = [C.c_double]
        L.orc_run.restype = C.c_int32
        L.orc_run.argtypes = [C.c_void_p, C.POINTER(Source), C.c_double, C.c_int64, C.c_int64,
                              C.c_uint64, C.c_uint32, dp, C.c_int32, C.c_int32, C.c_double,
                              C.POINTER(C.c_uint64), C.c_int32, C.c_int32, C.POINTER(Tally)]
        L.orc_broaden.argtypes = [dp, C.c_int32, C.c_double, C.c_double, C.c_double, dp]
        L.orc_rotate.argtypes = [dp, C.c_double, C.c_double, dp]
        L.orc_set_electrons.argtypes = [C.c_void_p, C.c_int32]
        L.orc_csda_range.restype = C.c_double
        L.orc_csda_range.argtypes = [C.c_double]
        L.orc_csda_energy.restype = C.c_double
        L.orc_csda_energy.argtypes = [C.c_double]
        L.orc_emission.restype = C.c_int32
        L.orc_emission.argtypes = [C.c_void_p, C.POINTER(Source), C.c_uint64, C.c_uint32, C.c_int64,
                                   dp, dp, C.POINTER(C.c_int32)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def kn_integral(k, eps):
    return lib().orc_kn_integral(k, eps)


def kn_sigma(k):
    return lib().orc_kn_sigma(k)


def kn_sample(k, u):
    return lib().orc_kn_sample(k, u)


def thomson_sample(u):
    return lib().orc_thomson_sample(u)


def rotate(d, ct, phi):
    """Direction after a scattering of polar cosine ct and azimuth phi about unit d."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_rotate(_dp(d), float(ct), float(phi), _dp(out))
    return out


def broaden(spectrum, channel_keV, a, b):
    x = np.ascontiguousarray(spectrum, dtype=np.float64)
    out = np.zeros_like(x)
    lib().orc_broaden(_dp(x), len(x), channel_keV, a, b, _dp(out))
    return out


@dataclass
class Result:
    tally: Tally
    spectrum: np.ndarray | None
    n: int

    def fepe(self):
        return self.tally.n_fep / max(1, self.tally.n_histories)

    def fepe_sigma(self):
        p = self.fepe()
        return (p * (1 - p) / max(1, self.tally.n_histories)) ** 0.5

    def grad(self, n_groups):
        n = self.tally.n_histories
        return np.array([self.tally.sum_fep_score[g] / n for g in range(n_groups)])

    def grad_sigma(self, n_groups):
        n = self.tally.n_histories
        m1 = self.grad(n_groups)
        m2 = np.array([self.tally.sum_fep_score2[g] / n for g in range(n_groups)])
        return np.sqrt(np.maximum(m2 - m1 * m1, 0.0) / n)


class Scene:
    """Oracle-side scene: mesh, region table and cross sections."""

    def __init__(self, xyz, tri, tri_region, n_regions, use_bvh=True):
        xyz = np.ascontiguousarray(xyz, dtype=np.float32)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        reg = np.ascontiguousarray(tri_region, dtype=np.int32)
        self._keep = (xyz, tri, reg)
        self.h = lib().orc_scene_create(
            xyz.ctypes.data_as(C.POINTER(C.c_float)), len(xyz),
            tri.ctypes.data_as(C.POINTER(C.c_int32)), reg.ctypes.data_as(C.POINTER(C.c_int32)),
            len(tri), int(n_regions), 1 if use_bvh else 0)
        if not self.h:
            raise ValueError("oracle: bad scene arrays")
        self.n_regions = int(n_regions)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.orc_scene_destroy(h)
            self.h = None

    def set_region(self, r, material, density, group=-1, active=False):
        rc = lib().orc_set_region(self.h, r, material, float(density), int(group), 1 if active else 0)
        if rc:
            raise ValueError(f"oracle: set_region({r}) -> {rc}")

    def set_xs(self, material, grid, photo, compton, coherent=None, pair=None):
        lnE0, dlnE, n = grid
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
                for a in (photo, compton, coherent, pair)]
        ptrs = [None if a is None else _dp(a) for a in arrs]
        rc = lib().orc_set_xs(self.h, material, lnE0, dlnE, n, *ptrs)
        if rc:
            raise ValueError(f"oracle: set_xs({material}) -> {rc}")

    def locate(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        return lib().orc_locate(self.h, _dp(p))

    def set_electrons(self, on):
        """Secondary electrons as straight CSDA tracks (1) or local deposits (0)."""
        lib().orc_set_electrons(self.h, 1 if on else 0)

    def closest_hit(self, o, d, exclude=-1):
        o = np.ascontiguousarray(o, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        t = C.c_double()
        f = C.c_int64()
        ok = lib().orc_closest_hit(self.h, _dp(o), _dp(d), exclude, C.byref(t), C.byref(f))
        return (t.value, f.value) if ok else (np.inf, -1)

    def mu(self, region, E, scales=None):
        """(photo, Compton, coherent, pair) linear attenuation [1/mm]."""
        out = np.zeros(4)
        sc = None if scales is None else np.ascontiguousarray(scales, dtype=np.float64)
        lib().orc_mu(self.h, region, E, None if sc is None else _dp(sc),
                     0 if sc is None else len(sc), _dp(out))
        return out

    def emission(self, source, seed, history, unit=0):
        """(energy, point, tries) of one history's emission step as transport draws it
        (energy 0 for a mono-energetic source; tries 0: every rejection try failed)."""
        E = C.c_double()
        p = np.zeros(3)
        tries = C.c_int32()
        src, keep = _make_source(source)
        rc = lib().orc_emission(self.h, C.byref(src), int(seed), int(unit), int(history), C.byref(E),
                                _dp(p), C.byref(tries))
        del keep
        if rc:
            raise ValueError(f"oracle: emission -> {rc}")
        return E.value, p, tries.value

    def run(self, source, E0, n, seed, unit=0, first=0, scales=None, n_channels=0,
            channel_keV=0.25, max_steps=10000, threads=None):
        if threads is None:
            threads = os.cpu_count() or 1
        n_groups = 0 if scales is None else len(scales)
        sc = np.ascontiguousarray(scales if scales is not None else [1.0], dtype=np.float64)
        spec = np.zeros(n_channels, dtype=np.uint64) if n_channels > 0 else None
        t = Tally()
        src, keep = _make_source(source)
        rc = lib().orc_run(self.h, C.byref(src), float(E0), int(n), int(first), int(seed), int(unit),
                           _dp(sc), n_groups, int(n_channels), float(channel_keV),
                           spec.ctypes.data_as(C.POINTER(C.c_uint64)) if spec is not None else None,
                           int(max_steps), int(threads), C.byref(t))
        del keep
        if rc:
            raise ValueError(f"oracle: run -> {rc}")
        return Result(t, spec, int(n))


def _make_source(s):
    """Accepts a workloads.configs.Source (duck-typed)."""
    src = Source()
    src.kind = int(s.kind)
    src.pos = (C.c_double * 3)(*s.pos)
    d = np.asarray(s.direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    src.dir = (C.c_double * 3)(*d)
    src.r_in, src.r_out, src.h = float(s.r_in), float(s.r_out), float(s.h)
    src.region = int(s.region)
    keep = []
    if s.lines_keV:
        le = np.ascontiguousarray(s.lines_keV, dtype=np.float64)
        lp = np.ascontiguousarray(s.lines_prob, dtype=np.float64)
        keep = [le, lp]
        src.n_lines = len(le)
        src.line_keV = _dp(le)
        src.line_prob = _dp(lp)
    return src, keep


def scene_from_workload(w, use_bvh=True):
    """Oracle scene loaded with a workloads.configs.Workload's arrays."""
    sc = w.scene
    s = Scene(sc.xyz, sc.tri, sc.tri_region, sc.n_regions, use_bvh=use_bvh)
    mat, rho, grp, act = w.region_arrays()
    for r in range(sc.n_regions):
        s.set_region(r, int(mat[r]), float(rho[r]), int(grp[r]), bool(act[r]))
    for m, tab in w.tables.items():
        s.set_xs(m, w.grid, *tab)
    return s
