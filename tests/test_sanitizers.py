"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code, on
the CPU: the library's mesh validation, parity topology and BVH builders,
the parametric detector generator and VRML writer (built with g++ from their
sources, no device code), and the oracle (gcc), each driven over the
workloads' meshes; any sanitizer report fails the test."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from workloads import configs as C
from workloads import meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all", "-pthread"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc/g++")


def _run(cmd, timeout=600):
    p = subprocess.run(cmd, capture_output=True, text=True, env=ENV, timeout=timeout)
    report = "AddressSanitizer" in p.stderr or "runtime error" in p.stderr \
        or "LeakSanitizer" in p.stderr
    assert p.returncode == 0 and not report, (cmd, p.returncode, p.stdout[-2000:], p.stderr[-4000:])
    return p.stdout


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    host = str(d / "host_driver")
    orc = str(d / "oracle_driver")
    csrc = os.path.join(ROOT, "paper_2605_25963_amd", "csrc")
    p1 = subprocess.Popen(["g++", "-std=c++17", *SAN, "-I" + os.path.join(ROOT, "include"),
                           "-I" + csrc, os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                           os.path.join(csrc, "mesh_prep.cpp"), os.path.join(csrc, "detmesh.cpp"),
                           "-o", host], stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    p2 = subprocess.Popen(["gcc", "-std=c11", *SAN, "-I" + os.path.join(ROOT, "oracle"),
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", orc],
                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    for p in (p1, p2):
        out, _ = p.communicate(timeout=600)
        assert p.returncode == 0, out.decode(errors="replace")[-3000:]
    return host, orc, d


def write_mesh(path, xyz, tri, reg, n_regions):
    xyz = np.ascontiguousarray(xyz, np.float32)
    tri = np.ascontiguousarray(tri, np.int32).reshape(-1, 3)
    reg = np.ascontiguousarray(reg, np.int32)
    with open(path, "wb") as f:
        f.write(struct.pack("<qqii", len(xyz), len(tri), int(n_regions), 0))
        f.write(xyz.tobytes())
        f.write(tri.tobytes())
        f.write(reg.tobytes())


def write_setup(path, w, e0):
    mat, rho, grp, act = w.region_arrays()
    lnE0, dlnE, n = w.grid
    with open(path, "wb") as f:
        f.write(struct.pack("<ii", len(mat), 0))
        for r in range(len(mat)):
            f.write(struct.pack("<iiiid", int(mat[r]), int(grp[r]), int(act[r]), 0, float(rho[r])))
        f.write(struct.pack("<iidd", len(w.materials), int(n), float(lnE0), float(dlnE)))
        for m in range(len(w.materials)):
            tab = list(w.tables[m]) + [None] * (4 - len(w.tables[m]))
            for part in tab[:4]:
                a = np.zeros(n) if part is None else np.asarray(part, np.float64)
                f.write(a.astype("<f8").tobytes())
        s = w.source
        lines = list(zip(s.lines_keV or [], s.lines_prob or []))
        f.write(struct.pack("<iiii", int(s.kind), int(s.region), len(lines), 0))
        d = np.asarray(s.direction, np.float64)
        d = d / np.linalg.norm(d)
        f.write(struct.pack("<12d", *s.pos, *d, s.r_in, s.r_out, s.h, float(e0), 0.0, 0.0))
        for k, p in lines:
            f.write(struct.pack("<dd", float(k), float(p)))


WORKLOADS = {
    "c1": lambda: (C.c1_bare(), 661.7),
    "c2_small": lambda: (C.c2_hpge(n_histories=1, n_seg=32, n_phi=4, distance=20.0), 200.0),
    "c3_bottle": lambda: (C.c3_job_workload(C.c3_jobs(4)[1]), 300.0),
    "c5_small": lambda: (C.c5_stress(n_histories=1, n_seg=32, n_phi=4, z_slices=1), 0.0),
}


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_host_preparation_under_sanitizers(drivers, name):
    host, orc, d = drivers
    w, e0 = WORKLOADS[name]()
    sc = w.scene
    mesh = str(d / f"{name}.mesh")
    write_mesh(mesh, sc.xyz, sc.tri, sc.tri_region, sc.n_regions)
    out = _run([host, "mesh", mesh])
    assert "method 2" in out
    # an open shell (one facet removed) is rejected without a report
    keep = np.ones(len(sc.tri), bool)
    keep[len(sc.tri) // 2] = False
    bad = str(d / f"{name}_open.mesh")
    write_mesh(bad, sc.xyz, np.asarray(sc.tri)[keep], np.asarray(sc.tri_region)[keep], sc.n_regions)
    assert "rejected" in _run([host, "badmesh", bad])


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_oracle_under_sanitizers(drivers, name):
    host, orc, d = drivers
    w, e0 = WORKLOADS[name]()
    sc = w.scene
    mesh = str(d / f"{name}_o.mesh")
    setup = str(d / f"{name}.setup")
    write_mesh(mesh, sc.xyz, sc.tri, sc.tri_region, sc.n_regions)
    write_setup(setup, w, e0)
    out = _run([orc, mesh, setup, "3000"])
    assert out.count("pass") == 2 and "balance 0" in out


def test_generator_under_sanitizers(drivers):
    from paper_2605_25963_amd import gadep as G
    host, orc, d = drivers
    cases = [C.DETMESH_C2, C.table1_detmesh("#1 GMX45P4-76", n_theta=32, n_phi=4),
             C.table1_detmesh("#3 GEM-C50P4", n_theta=32, n_phi=4)]
    bad = dict(C.DETMESH_C2)
    bad["D4"] = 40.0  # a dead layer thicker than the crystal's radius: rejected
    cases.append(bad)
    for i, p in enumerate(cases):
        f = str(d / f"det{i}.bin")
        with open(f, "wb") as fh:
            fh.write(bytes(G.Detector(**p)))
        out = _run([host, "detmesh", f, str(d / f"det{i}.wrl")])
        assert ("rejected" in out) == (i == 3), out
