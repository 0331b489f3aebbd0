"""ctypes binding of libgadep.so (include/gadep.h).

Argument marshalling only: every step of the transport runs in the library's
HIP kernels.  Method names follow the C functions without the ``gadep_``
prefix (``Context.run`` is ``gadep_run``); module-level ``gadep_*`` aliases
are provided as well.  There is no fallback: if the library is missing the
import of this module's functions raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgadep.so")

MAX_REGIONS = 64
MAX_GROUPS = 8
ACTIVE = 1
SRC_POINT, SRC_BEAM, SRC_CYL, SRC_CONE = 0, 1, 2, 3

OPT_MAX_STEPS, OPT_BLOCK, OPT_PERIOD, OPT_CLAIM, OPT_VALIDATE, OPT_MIN_GAP_NM, OPT_GRAPHS, \
    OPT_COUNTERS, OPT_GRID, OPT_EXIT_PLANES, OPT_SPLIT_PCT, OPT_SCREEN, OPT_POOL, \
    OPT_ELECTRONS, OPT_GUIDE = range(1, 16)

STATUS = {
    0: "GADEP_OK", -1: "GADEP_E_ARG", -2: "GADEP_E_MESH_OPEN", -3: "GADEP_E_MESH_ORIENT",
    -4: "GADEP_E_MESH_OVERLAP", -5: "GADEP_E_XS", -6: "GADEP_E_STATE", -7: "GADEP_E_HIP",
    -8: "GADEP_E_OOM", -9: "GADEP_E_TOPOLOGY", -10: "GADEP_E_MESH_DEGENERATE",
}


class GadepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class Region(C.Structure):
    _fields_ = [("material", C.c_int32), ("density_g_cm3", C.c_float),
                ("scale_group", C.c_int32), ("flags", C.c_uint32)]


class Source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos_mm", C.c_float * 3), ("dir", C.c_float * 3),
                ("r_in_mm", C.c_float), ("r_out_mm", C.c_float), ("h_mm", C.c_float),
                ("region", C.c_int32), ("n_lines", C.c_int32),
                ("line_keV", C.POINTER(C.c_float)), ("line_prob", C.POINTER(C.c_float))]


class Tally(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "n_histories", "n_absorbed", "n_fep", "n_escape", "n_uncollided", "n_lost", "n_killed",
        "n_glitch", "n_source_fail")] + [
        ("edep_active_keV", C.c_double), ("edep_total_keV", C.c_double),
        ("e_escape_keV", C.c_double), ("e_source_keV", C.c_double),
        ("spectrum", C.POINTER(C.c_uint64)), ("n_channels", C.c_int32),
        ("channel_keV", C.c_float), ("spectrum_overflow", C.c_uint64), ("weight", C.c_double)]


class Job(C.Structure):
    _fields_ = [("src", Source), ("energies_keV", C.POINTER(C.c_double)),
                ("n_energies", C.c_int32), ("n_histories", C.c_int64),
                ("first_history", C.c_int64), ("scales", C.POINTER(C.c_float)),
                ("n_scales", C.c_int32), ("scene", C.c_int32), ("stream", C.c_uint32),
                ("region_material_override", C.POINTER(C.c_int32)),
                ("region_density_override", C.POINTER(C.c_float))]


class Counters(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "segments", "crossings", "node_visits", "tri_tests", "photo", "compton", "coherent",
        "rng_calls", "locates", "emissions", "plane_tests", "iterations", "iterations_node",
        "iterations_facet", "passes", "cycles_outcome", "cycles_refill", "cycles_launch",
        "cycles_setup", "cycles_traversal", "box_tests", "pair", "electrons", "wavefronts",
        "wave_cycles", "cone_tests")]


class Detector(C.Structure):
    """gadep_detector: Table 2 parameter groups [mm] plus discretisation."""
    _fields_ = ([(n, C.c_double) for n in ("d1", "d2", "d3", "d4", "d5", "d6", "d7", "d8", "d9",
                                           "d10", "D1", "D2", "D3", "D4", "D5", "D6", "D7")] +
                [("n_theta", C.c_int32), ("n_phi", C.c_int32), ("z_slices", C.c_int32),
                 ("eps_mm", C.c_double), ("cup_gap_mm", C.c_double), ("cup_rim_mm", C.c_double),
                 ("pin_radius_mm", C.c_double), ("pin_length_mm", C.c_double),
                 ("finger_radius_mm", C.c_double), ("world_half_mm", C.c_double)])


DM_REGIONS = ["world", "air", "housing", "window", "vacuum", "cup", "crystal", "active",
              "contact", "bore", "pin", "finger"]


class MeshInfo(C.Structure):
    _fields_ = [("n_shells", C.c_int32), ("genus_max", C.c_int32), ("n_nodes", C.c_int64),
                ("depth", C.c_int32), ("sah_cost", C.c_double), ("n_slots", C.c_int64),
                ("min_gap_mm", C.c_double), ("convex_exit", C.c_int32),
                ("n_exit_planes", C.c_int32), ("region_root", C.c_int32 * (MAX_REGIONS + 1))]


EXPORTS = [
    "gadep_create", "gadep_destroy", "gadep_last_error", "gadep_set_option", "gadep_get_option",
    "gadep_load_mesh", "gadep_load_scene", "gadep_set_xs", "gadep_set_scales", "gadep_run",
    "gadep_run_grad", "gadep_run_batch", "gadep_autotune", "gadep_get_counters",
    "gadep_broaden_dev", "gadep_raycast", "gadep_locate", "gadep_mesh_prepare",
    "gadep_get_last_launch_ms", "gadep_detmesh", "gadep_write_vrml", "gadep_philox",
    "gadep_run_noalloc", "gadep_get_last_clock_mhz", "gadep_load_overlay",
]

_lib = None


def lib():
    """The loaded library; raises if it has not been built.

    torch (when installed) is imported first: it carries its own HIP runtime
    under the same soname, and loading it before libgadep.so makes the library
    bind to that runtime, so one process has one HIP runtime and torch tensors
    and streams can be handed to the library.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    p, i32, i64, u64, f32p, i32p, dp = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint64,
                                        C.POINTER(C.c_float), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double))
    sig = {
        "gadep_create": (i32, [C.c_int, p, C.POINTER(p)]),
        "gadep_destroy": (None, [p]),
        "gadep_last_error": (C.c_char_p, [p]),
        "gadep_set_option": (i32, [p, i32, i64]),
        "gadep_get_option": (i32, [p, i32, C.POINTER(i64)]),
        "gadep_load_mesh": (i32, [p, f32p, i64, i32p, i32p, i64, C.POINTER(Region), i32]),
        "gadep_load_scene": (i32, [p, i32, f32p, i64, i32p, i32p, i64, C.POINTER(Region), i32]),
        "gadep_load_overlay": (i32, [p, i32, i32, i32, f32p, i64, i32p, i32p, i64,
                                     C.POINTER(Region), i32]),
        "gadep_set_xs": (i32, [p, i32, C.c_double, C.c_double, i32, f32p, f32p, f32p, f32p]),
        "gadep_set_scales": (i32, [p, f32p, i32]),
        "gadep_run": (i32, [p, C.POINTER(Source), dp, i32, i64, u64, i64, C.POINTER(Tally)]),
        "gadep_run_noalloc": (i32, [p, C.POINTER(Source), dp, i32, i64, u64, i64,
                                    C.POINTER(Tally)]),
        "gadep_run_grad": (i32, [p, C.POINTER(Source), dp, i32, i64, u64, i64, f32p, i32,
                                 C.POINTER(Tally), dp, dp]),
        "gadep_run_batch": (i32, [p, C.POINTER(Job), i32, u64, C.POINTER(Tally), dp, dp]),
        "gadep_autotune": (i32, [p, C.POINTER(Job), i32, i64, i32p, i32p, i32p]),
        "gadep_get_counters": (i32, [p, C.POINTER(Counters)]),
        "gadep_get_last_launch_ms": (i32, [p, C.POINTER(C.c_double)]),
        "gadep_get_last_clock_mhz": (i32, [p, C.POINTER(C.c_double)]),
        "gadep_broaden_dev": (i32, [p, p, p, i32, i32, C.c_double, C.c_double, C.c_double]),
        "gadep_raycast": (i32, [p, i32, f32p, f32p, i32p, i64, f32p, i32p, i32p]),
        "gadep_locate": (i32, [p, i32, f32p, i64, i32p]),
        "gadep_philox": (i32, [p, C.POINTER(C.c_uint32), u64, i64, C.POINTER(C.c_uint32)]),
        "gadep_mesh_prepare": (i32, [f32p, i64, i32p, i32p, i64, i32, C.c_double, i32, i32,
                                     C.c_double, i32p, i32p, p, i64, i32p, i64,
                                     C.POINTER(MeshInfo), C.c_char_p, i32]),
        "gadep_detmesh": (i32, [C.POINTER(Detector), f32p, i64, i32p, i32p, i64,
                                C.POINTER(C.c_int64), C.POINTER(C.c_int64), i32p, C.c_char_p, i32]),
        "gadep_write_vrml": (i32, [C.c_char_p, f32p, i64, i32p, i32p, i64, i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


def make_source(kind=SRC_POINT, pos=(0, 0, 0), direction=(0, 0, -1), r_in=0.0, r_out=0.0, h=0.0,
                region=-1, lines_keV=None, lines_prob=None):
    """gadep_source plus the arrays it points to (kept alive by the returned object)."""
    s = Source()
    s.kind = int(kind)
    s.pos_mm = (C.c_float * 3)(*[float(x) for x in pos])
    s.dir = (C.c_float * 3)(*[float(x) for x in direction])
    s.r_in_mm, s.r_out_mm, s.h_mm = float(r_in), float(r_out), float(h)
    s.region = int(region)
    s._keep = []
    if lines_keV is not None and len(lines_keV):
        le, lp = _f32(lines_keV), _f32(lines_prob)
        s._keep = [le, lp]
        s.n_lines = len(le)
        s.line_keV = _ptr(le, C.c_float)
        s.line_prob = _ptr(lp, C.c_float)
    return s


def source_from(src):
    """gadep_source from any object with the fields of workloads.configs.Source."""
    return make_source(src.kind, src.pos, src.direction, src.r_in, src.r_out, src.h, src.region,
                       src.lines_keV, src.lines_prob)


@dataclass
class Result:
    """Per-unit tallies (and spectra, gradients) of one run."""

    tallies: list
    spectra: np.ndarray | None = None
    grad: np.ndarray | None = None
    grad_var: np.ndarray | None = None
    _keep: list = field(default_factory=list)

    def weights(self):
        """Photons each history stands for (1, or Omega/4pi for a cone source)."""
        return np.array([t.weight for t in self.tallies])

    def fepe(self):
        return np.array([t.weight * t.n_fep / max(1, t.n_histories) for t in self.tallies])

    def fepe_sigma(self):
        w = self.weights()
        q = np.array([t.n_fep / max(1, t.n_histories) for t in self.tallies])
        n = np.array([max(1, t.n_histories) for t in self.tallies], dtype=np.float64)
        return w * np.sqrt(q * (1 - q) / n)

    def field(self, name):
        return np.array([getattr(t, name) for t in self.tallies])


class Context:
    """One library context (device buffers, scenes, tables) on one stream."""

    def __init__(self, device=0, stream=None):
        L = lib()
        h = C.c_void_p()
        s = None
        if stream is not None:
            s = C.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
        rc = L.gadep_create(int(device), s, C.byref(h))
        if rc:
            raise GadepError(rc, "gadep_create failed (no HIP device?)")
        self.h = h
        self._scene_regions = {}

    def close(self):
        if getattr(self, "h", None):
            lib().gadep_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc:
            raise GadepError(rc, lib().gadep_last_error(self.h).decode(errors="replace"))

    # -- options
    def set_option(self, opt, value):
        self._check(lib().gadep_set_option(self.h, int(opt), int(value)))

    def get_option(self, opt):
        v = C.c_int64()
        self._check(lib().gadep_get_option(self.h, int(opt), C.byref(v)))
        return v.value

    # -- geometry and tables
    def load_scene(self, scene, xyz, tri, tri_region, regions):
        xyz, tri, reg = _f32(xyz, (-1, 3)), _i32(tri).reshape(-1, 3), _i32(tri_region)
        rs = (Region * len(regions))()
        for i, r in enumerate(regions):
            rs[i].material, rs[i].density_g_cm3, rs[i].scale_group, rs[i].flags = \
                int(r[0]), float(r[1]), int(r[2]), int(r[3])
        self._check(lib().gadep_load_scene(self.h, int(scene), _ptr(xyz, C.c_float), len(xyz),
                                           _ptr(tri, C.c_int32), _ptr(reg, C.c_int32), len(tri),
                                           rs, len(regions)))
        self._scene_regions[int(scene)] = len(regions)

    def load_overlay(self, scene, base_scene, host_region, xyz, tri, tri_region, regions):
        """gadep_load_overlay: per-job shells on the detector in base_scene; regions[0]
        (the host) is ignored, overlay region k is region n_base + k - 1 of the scene."""
        xyz, tri, reg = _f32(xyz, (-1, 3)), _i32(tri).reshape(-1, 3), _i32(tri_region)
        rs = (Region * len(regions))()
        for i, r in enumerate(regions):
            rs[i].material, rs[i].density_g_cm3, rs[i].scale_group, rs[i].flags = \
                int(r[0]), float(r[1]), int(r[2]), int(r[3])
        self._check(lib().gadep_load_overlay(self.h, int(scene), int(base_scene), int(host_region),
                                             _ptr(xyz, C.c_float), len(xyz), _ptr(tri, C.c_int32),
                                             _ptr(reg, C.c_int32), len(tri), rs, len(regions)))
        self._scene_regions[int(scene)] = self._scene_regions.get(int(base_scene), 0) + len(regions) - 1

    def load_mesh(self, xyz, tri, tri_region, regions):
        self.load_scene(0, xyz, tri, tri_region, regions)

    def set_xs(self, material, grid, photo, compton, coherent=None, pair=None):
        lnE0, dlnE, n = grid
        arrs = [None if a is None else _f32(a) for a in (photo, compton, coherent, pair)]
        self._check(lib().gadep_set_xs(self.h, int(material), float(lnE0), float(dlnE), int(n),
                                       *[_ptr(a, C.c_float) for a in arrs]))

    def set_scales(self, scales):
        s = _f32(scales)
        self._check(lib().gadep_set_scales(self.h, _ptr(s, C.c_float), len(s)))

    # -- transport
    @staticmethod
    def _tallies(n_units, spectrum):
        out = (Tally * n_units)()
        spec = None
        if spectrum is not None:
            nch, w = spectrum
            spec = np.zeros((n_units, nch), dtype=np.uint64)
            for u in range(n_units):
                out[u].spectrum = spec[u].ctypes.data_as(C.POINTER(C.c_uint64))
                out[u].n_channels = int(nch)
                out[u].channel_keV = float(w)
        return out, spec

    def run(self, source, energies, n_histories, seed, first_history=0, spectrum=None):
        src = source if isinstance(source, Source) else source_from(source)
        e = np.ascontiguousarray(energies if energies is not None else [0.0], dtype=np.float64)
        nu = len(e)
        out, spec = self._tallies(nu, spectrum)
        self._check(lib().gadep_run(self.h, C.byref(src), None if src.n_lines else _ptr(e, C.c_double),
                                    nu, int(n_histories), int(seed), int(first_history), out))
        return Result(list(out), spec)

    def run_noalloc(self, source, energies, n_histories, seed, first_history=0, spectrum=None):
        """gadep_run_noalloc: gadep_run without device allocations (fixed scratch)."""
        src = source if isinstance(source, Source) else source_from(source)
        e = np.ascontiguousarray(energies if energies is not None else [0.0], dtype=np.float64)
        nu = len(e)
        out, spec = self._tallies(nu, spectrum)
        self._check(lib().gadep_run_noalloc(self.h, C.byref(src),
                                            None if src.n_lines else _ptr(e, C.c_double), nu,
                                            int(n_histories), int(seed), int(first_history), out))
        return Result(list(out), spec)

    def run_grad(self, source, energies, n_histories, seed, scales, first_history=0,
                 spectrum=None):
        src = source if isinstance(source, Source) else source_from(source)
        e = np.ascontiguousarray(energies if energies is not None else [0.0], dtype=np.float64)
        nu = len(e)
        sc = _f32(scales)
        out, spec = self._tallies(nu, spectrum)
        g = np.zeros((nu, len(sc)))
        gv = np.zeros((nu, len(sc)))
        self._check(lib().gadep_run_grad(self.h, C.byref(src),
                                         None if src.n_lines else _ptr(e, C.c_double), nu,
                                         int(n_histories), int(seed), int(first_history),
                                         _ptr(sc, C.c_float), len(sc), out, _ptr(g, C.c_double),
                                         _ptr(gv, C.c_double)))
        return Result(list(out), spec, g, gv)

    def make_jobs(self, jobs):
        """jobs: list of dicts with keys source, energies, n_histories and optional
        first_history, scales, scene, stream, material_override, density_override."""
        arr = (Job * len(jobs))()
        keep = []
        for i, j in enumerate(jobs):
            src = j["source"] if isinstance(j["source"], Source) else source_from(j["source"])
            keep.append(src)
            arr[i].src = src
            if src.n_lines:
                arr[i].energies_keV = None
                arr[i].n_energies = 1
            else:
                e = np.ascontiguousarray(j["energies"], dtype=np.float64)
                keep.append(e)
                arr[i].energies_keV = _ptr(e, C.c_double)
                arr[i].n_energies = len(e)
            arr[i].n_histories = int(j["n_histories"])
            arr[i].first_history = int(j.get("first_history", 0))
            if j.get("scales") is not None:
                s = _f32(j["scales"])
                keep.append(s)
                arr[i].scales = _ptr(s, C.c_float)
                arr[i].n_scales = len(s)
            arr[i].scene = int(j.get("scene", 0))
            arr[i].stream = int(j.get("stream", i))
            if j.get("material_override") is not None:
                m = _i32(j["material_override"])
                keep.append(m)
                arr[i].region_material_override = _ptr(m, C.c_int32)
            if j.get("density_override") is not None:
                d = _f32(j["density_override"])
                keep.append(d)
                arr[i].region_density_override = _ptr(d, C.c_float)
        return arr, keep

    def run_batch(self, jobs, seed, grad=False, spectrum=None):
        arr, keep = self.make_jobs(jobs)
        nu = sum(a.n_energies for a in arr)
        out, spec = self._tallies(nu, spectrum)
        g = np.zeros((nu, MAX_GROUPS)) if grad else None
        gv = np.zeros((nu, MAX_GROUPS)) if grad else None
        self._check(lib().gadep_run_batch(self.h, arr, len(arr), int(seed), out,
                                          _ptr(g, C.c_double), _ptr(gv, C.c_double)))
        return Result(list(out), spec, g, gv, keep)

    def autotune(self, jobs, pilot_histories):
        arr, keep = self.make_jobs(jobs)
        b, p, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib().gadep_autotune(self.h, arr, len(arr), int(pilot_histories),
                                         C.byref(b), C.byref(p), C.byref(c)))
        return b.value, p.value, c.value

    def get_last_launch_ms(self):
        v = C.c_double()
        self._check(lib().gadep_get_last_launch_ms(self.h, C.byref(v)))
        return v.value

    def get_last_clock_mhz(self):
        v = C.c_double()
        self._check(lib().gadep_get_last_clock_mhz(self.h, C.byref(v)))
        return v.value

    def get_counters(self):
        c = Counters()
        self._check(lib().gadep_get_counters(self.h, C.byref(c)))
        return {n: getattr(c, n) for n, _ in Counters._fields_}

    # -- device checks of the geometry
    def raycast(self, o, d, region=None, scene=0):
        o, d = _f32(o, (-1, 3)), _f32(d, (-1, 3))
        n = len(o)
        r = None if region is None else _i32(region)
        t = np.zeros(n, np.float32)
        tri = np.zeros(n, np.int32)
        ra = np.zeros(n, np.int32)
        self._check(lib().gadep_raycast(self.h, int(scene), _ptr(o, C.c_float), _ptr(d, C.c_float),
                                        _ptr(r, C.c_int32), n, _ptr(t, C.c_float),
                                        _ptr(tri, C.c_int32), _ptr(ra, C.c_int32)))
        return t, tri, ra

    def locate(self, p, scene=0):
        p = _f32(p, (-1, 3))
        out = np.zeros(len(p), np.int32)
        self._check(lib().gadep_locate(self.h, int(scene), _ptr(p, C.c_float), len(p),
                                       _ptr(out, C.c_int32)))
        return out

    def philox(self, counters, key):
        """Philox4x32-10 blocks on the device: counters [n][4] uint32, key uint64."""
        c = np.ascontiguousarray(np.asarray(counters, np.uint32).reshape(-1, 4))
        out = np.zeros_like(c)
        self._check(lib().gadep_philox(self.h, _ptr(c, C.c_uint32), C.c_uint64(int(key)), len(c),
                                       _ptr(out, C.c_uint32)))
        return out

    def broaden_dev(self, in_ptr, out_ptr, n_spectra, n_channels, channel_keV, a, b):
        """in_ptr/out_ptr: device addresses (e.g. torch tensor .data_ptr()) of FP64 arrays."""
        self._check(lib().gadep_broaden_dev(self.h, C.c_void_p(in_ptr), C.c_void_p(out_ptr),
                                            int(n_spectra), int(n_channels), float(channel_keV),
                                            float(a), float(b)))


def mesh_prepare(xyz, tri, tri_region, n_regions, min_gap_mm=1e-4, validate=True, bvh_method=0,
                 want_nodes=False, split_budget=1.0):
    """Host-only validation/topology/BVH (gadep_mesh_prepare).  bvh_method 2
    returns the transport BVH (spatial splits) instead of the plain one."""
    L = lib()
    xyz, tri, reg = _f32(xyz, (-1, 3)), _i32(tri).reshape(-1, 3), _i32(tri_region)
    nt = len(tri)
    outside = np.zeros(nt, np.int32)
    shell = np.zeros(nt, np.int32)
    info = MeshInfo()
    err = C.create_string_buffer(512)

    def call(nodes, cap_nodes, order, cap_slots):
        return L.gadep_mesh_prepare(
            _ptr(xyz, C.c_float), len(xyz), _ptr(tri, C.c_int32), _ptr(reg, C.c_int32), nt,
            int(n_regions), float(min_gap_mm), 1 if validate else 0, int(bvh_method),
            float(split_budget), _ptr(outside, C.c_int32), _ptr(shell, C.c_int32),
            None if nodes is None else nodes.ctypes.data_as(C.c_void_p), cap_nodes,
            None if order is None else _ptr(order, C.c_int32), cap_slots, C.byref(info), err, 512)

    rc = call(None, 0, None, 0)
    if rc:
        raise GadepError(rc, err.value.decode(errors="replace"))
    order = np.zeros(info.n_slots, np.int32)
    nodes = np.zeros((info.n_nodes, 16), np.int32) if want_nodes else None
    rc = call(nodes, info.n_nodes, order, info.n_slots)
    if rc:
        raise GadepError(rc, err.value.decode(errors="replace"))
    res = dict(outside=outside, shell=shell, order=order, n_shells=info.n_shells,
               genus_max=info.genus_max, n_nodes=info.n_nodes, depth=info.depth,
               sah_cost=info.sah_cost, n_slots=info.n_slots, min_gap_mm=info.min_gap_mm,
               convex_exit=bool(info.convex_exit), n_exit_planes=info.n_exit_planes,
               region_root=np.array(info.region_root, np.int64))
    if nodes is not None:
        res["nodes"] = nodes
    return res


def detmesh(params=None, **kw):
    """gadep_detmesh: (xyz [nv, 3] float32, tri [nt, 3] int32, tri_region [nt] int32,
    region_parent [GADEP_DM_N] int32) of a coaxial HPGe detector; params is a
    Detector or keyword fields of one."""
    d = params if params is not None else Detector(**kw)
    L = lib()
    nv, nt = C.c_int64(), C.c_int64()
    parent = np.zeros(len(DM_REGIONS), np.int32)
    err = C.create_string_buffer(512)
    rc = L.gadep_detmesh(C.byref(d), None, 0, None, None, 0, C.byref(nv), C.byref(nt),
                         _ptr(parent, C.c_int32), err, 512)
    if rc:
        raise GadepError(rc, err.value.decode(errors="replace"))
    xyz = np.zeros((nv.value, 3), np.float32)
    tri = np.zeros((nt.value, 3), np.int32)
    reg = np.zeros(nt.value, np.int32)
    rc = L.gadep_detmesh(C.byref(d), _ptr(xyz, C.c_float), nv.value, _ptr(tri, C.c_int32),
                         _ptr(reg, C.c_int32), nt.value, C.byref(nv), C.byref(nt),
                         _ptr(parent, C.c_int32), err, 512)
    if rc:
        raise GadepError(rc, err.value.decode(errors="replace"))
    return xyz, tri, reg, parent


def write_vrml(path, xyz, tri, tri_region, n_regions):
    """gadep_write_vrml: the mesh as VRML 2.0, one IndexedFaceSet per region."""
    xyz, tri, reg = _f32(xyz, (-1, 3)), _i32(tri).reshape(-1, 3), _i32(tri_region)
    rc = lib().gadep_write_vrml(os.fsencode(path), _ptr(xyz, C.c_float), len(xyz),
                                _ptr(tri, C.c_int32), _ptr(reg, C.c_int32), len(tri), int(n_regions))
    if rc:
        raise GadepError(rc, f"write_vrml({path}) failed")


def load_workload(ctx, w, scene=0):
    """Loads a workload-like object (scene arrays, region table, xs tables) into ctx."""
    mat, rho, grp, act = w.region_arrays()
    regions = [(int(mat[r]), float(rho[r]), int(grp[r]), ACTIVE if act[r] else 0)
               for r in range(len(mat))]
    sc = w.scene
    for m, tab in w.tables.items():
        ctx.set_xs(m, w.grid, *tab)
    ctx.load_scene(scene, sc.xyz, sc.tri, sc.tri_region, regions)
    return regions


# module-level aliases with the C names
def gadep_create(device=0, stream=None):
    return Context(device, stream)


def gadep_destroy(ctx):
    ctx.close()


gadep_set_option = Context.set_option
gadep_get_option = Context.get_option
gadep_load_mesh = Context.load_mesh
gadep_load_scene = Context.load_scene
gadep_load_overlay = Context.load_overlay
gadep_set_xs = Context.set_xs
gadep_set_scales = Context.set_scales
gadep_run = Context.run
gadep_run_noalloc = Context.run_noalloc
gadep_run_grad = Context.run_grad
gadep_run_batch = Context.run_batch
gadep_autotune = Context.autotune
gadep_get_counters = Context.get_counters
gadep_get_last_launch_ms = Context.get_last_launch_ms
gadep_get_last_clock_mhz = Context.get_last_clock_mhz
gadep_raycast = Context.raycast
gadep_locate = Context.locate
gadep_philox = Context.philox
gadep_broaden_dev = Context.broaden_dev
gadep_mesh_prepare = mesh_prepare
