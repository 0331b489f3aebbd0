"""DetMesh-style parametric detector meshes (gadep_detmesh, gadep_write_vrml),
host only: the Table 2 parameter groups turned into closed shells that the
validator accepts, nested as declared, with Eq. 1-4 vertices and the Eq. 6
active volume; the 20236-facet coaxial detector's parameters reproduce the independently
written fixture generator shell for shell; Table 1's crystals; VRML output."""
import math
import os

import numpy as np
import pytest

from workloads import configs as C
from workloads import meshgen as mg


@pytest.fixture(scope="module")
def G():
    from paper_2605_25963_amd import gadep
    gadep.lib()
    return gadep


C2 = C.DETMESH_C2
TABLE1 = C.TABLE1
table1_params = C.table1_detmesh


def shells(xyz, tri, reg):
    for k in np.unique(reg):
        yield int(k), tri[reg == k]


def test_c2_parameters_reproduce_the_fixture(G):
    xyz, tri, reg, parent = G.detmesh(**C2)
    sc = C.c2_hpge(n_histories=1).scene
    assert len(tri) == len(sc.tri) == 20236
    names = {"air": "air", "housing": "endcap", "window": "window", "vacuum": "interior",
             "cup": "cup", "crystal": "dead", "active": "active", "bore": "bore",
             "finger": "coldfinger"}
    fx_names = [r["name"] for r in sc.regions]
    for k, F in shells(xyz, tri, reg):
        name = G.DM_REGIONS[k]
        if name not in names:
            continue
        mine = np.unique(xyz[np.unique(F)], axis=0)
        j = fx_names.index(names[name])
        sel = np.asarray(sc.tri_region) == j
        ref = np.unique(np.asarray(sc.xyz, np.float32)[np.unique(np.asarray(sc.tri)[sel])], axis=0)
        assert mine.shape == ref.shape and np.abs(mine - ref).max() < 1e-5, name
        assert len(F) == int(sel.sum()), name


def test_shells_are_closed_valid_and_nested_as_declared(G):
    for p in (C2, table1_params("#3 GEM-C50P4"), table1_params("#1 GMX45P4-76")):
        xyz, tri, reg, parent = G.detmesh(**p)
        V = xyz.astype(np.float64)
        for k, F in shells(xyz, tri, reg):
            assert mg.euler_characteristic(F) == 2, k  # genus 0
            assert mg.signed_volume(V, F) > 0, k       # Eq. 5 normals point out
        r = G.mesh_prepare(xyz, tri, reg, len(G.DM_REGIONS))
        outside = r["outside"]
        for k, F in shells(xyz, tri, reg):
            assert set(outside[reg == k].tolist()) == {int(parent[k])}, (k, parent[k])


def test_eq1_to_eq4_vertices_and_eq6_active_volume(G):
    xyz, tri, reg, parent = G.detmesh(**C2)
    V = xyz.astype(np.float64)
    n, nphi, R, L, Rc, D4 = 128, 20, 32.0, 60.0, 3.0, 0.7
    crystal = np.unique(tri[reg == 6])
    P = V[crystal]
    rho = np.hypot(P[:, 0], P[:, 1])
    # Eq. 1-2: off-axis vertices lie at the angles 2 pi i / N
    th = np.arctan2(P[:, 1], P[:, 0])[rho > 1e-6]
    k = th / (2 * math.pi / n)
    assert np.abs(k - np.round(k)).max() < 1e-4
    # Eq. 3-4: one ring per phi_j on the rounded edge
    for j in range(1, nphi):
        phi = 0.5 * math.pi * j / nphi
        rj = (R - Rc) + Rc * math.cos(phi)
        zj = -Rc * (1 - math.sin(phi))
        on = (np.abs(P[:, 2] - zj) < 2e-5) & (np.abs(rho - rj) < 2e-5)
        assert on.sum() == n, j
    # Eq. 6: active radius D2 - D4, front face at -D4, rounding Rc - D4
    A = V[np.unique(tri[reg == 7])]
    assert np.hypot(A[:, 0], A[:, 1]).max() == pytest.approx(R - D4, abs=2e-5)
    assert A[:, 2].max() == pytest.approx(-D4, abs=1e-6)
    assert A[:, 2].min() == pytest.approx(-L + 1e-3, abs=1e-5)
    # the end-cap is an inscribed 128-gon prism: (N/2) r^2 sin(2 pi / N) h
    F = tri[reg == 2]
    vol = mg.signed_volume(V, F)
    assert vol == pytest.approx(0.5 * n * 38.0 ** 2 * math.sin(2 * math.pi / n) * 105.5, rel=1e-5)


@pytest.mark.parametrize("name", sorted(TABLE1))
def test_table1_detectors(G, name):
    p = table1_params(name)
    xyz, tri, reg, parent = G.detmesh(**p)
    dia, length, hdia, hdepth, outer, inner = TABLE1[name]
    present = set(np.unique(reg).tolist())
    # a 0.3 um layer is thinner than the separation: no shell of its own
    assert (6 in present) == (outer >= 4e-3)
    assert (8 in present) == (inner >= 4e-3)
    assert 7 in present and 9 in present
    r = G.mesh_prepare(xyz, tri, reg, len(G.DM_REGIONS))
    assert r["n_shells"] == len(present)


def test_parameters_that_do_not_fit_are_rejected(G):
    for bad in (dict(d8=50.0), dict(D3=40.0), dict(D5=70.0), dict(d7=60.0), dict(d1=50.0),
                dict(cup_rim_mm=6.0), dict(n_theta=2)):
        p = dict(C2)
        p.update(bad)
        with pytest.raises(G.GadepError):
            G.detmesh(**p)


def test_vrml_export(G, tmp_path):
    xyz, tri, reg, parent = G.detmesh(**table1_params("#2 GEM-C50-LB-C", n_theta=16, n_phi=4))
    path = os.path.join(tmp_path, "det.wrl")
    G.write_vrml(path, xyz, tri, reg, len(G.DM_REGIONS))
    text = open(path).read()
    assert text.startswith("#VRML V2.0 utf8")
    shapes = text.split("DEF region_")[1:]
    assert len(shapes) == len(np.unique(reg))
    for sh in shapes:
        k = int(sh.split(" ", 1)[0])
        idx = sh.split("coordIndex [", 1)[1].split("]", 1)[0]
        faces = [f for f in idx.split("-1,") if f.strip()]
        assert len(faces) == int((reg == k).sum())
        first = [int(x) for x in faces[0].replace(",", " ").split()]
        assert first == tri[reg == k][0].tolist()
        pts = sh.split("point [", 1)[1].split("]", 1)[0].replace(",", " ").split()
        assert len(pts) == 3 * len(xyz)
    with pytest.raises(G.GadepError):
        G.write_vrml(os.path.join(tmp_path, "no", "such", "dir.wrl"), xyz, tri, reg, len(G.DM_REGIONS))
