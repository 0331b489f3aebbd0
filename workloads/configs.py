"""Synthetic workloads shaped like the paper's HPGe calibration runs.

Every input is seeded and deterministic.  The detectors are synthetic
stand-ins for the paper's ORTEC detectors (Table 1): dimensions follow a
p-type coaxial crystal of about 64 mm diameter and 60 mm length with a
0.7 mm outer dead layer, a 5 mm-radius bore with a hemispherical tip, an Al
cup, a 1 mm Al end-cap and a 0.5 mm Al window (Sec. 2.1, Sec. 2.3).

Coincident surfaces are separated inside-out by EPS (Sec. 2.4.2, Fig. 6).
All lengths in mm, energies in keV, densities in g/cm^3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import meshgen as mg
from . import xsgen

EPS = 1.0e-3  # inside-out separation of otherwise coincident faces [mm]

# photon lines of the paper's calibration nuclides (Table 3)
TABLE3_LINES_KEV = [59.54, 81.00, 121.78, 244.70, 344.28, 356.02, 411.13,
                    443.97, 778.90, 964.06, 1112.09, 1332.49, 1408.02]

KIND_POINT, KIND_BEAM, KIND_CYL, KIND_CONE = 0, 1, 2, 3


def log_energies(n, e0=40.0, e1=2000.0):
    return [e0 * (e1 / e0) ** (i / (n - 1)) for i in range(n)]


@dataclass
class Source:
    kind: int = KIND_POINT
    pos: tuple = (0.0, 0.0, 0.0)       # point / beam origin; base centre for CYL
    direction: tuple = (0.0, 0.0, -1.0)  # BEAM only
    r_in: float = 0.0                  # CYL: annulus radii and height along +z
    r_out: float = 0.0
    h: float = 0.0
    region: int = -1                   # CYL: region the emission point must lie in
    lines_keV: list = None             # optional line spectrum (replaces mono energy)
    lines_prob: list = None


@dataclass
class Workload:
    name: str
    scene: mg.Scene
    materials: list                    # material names; index = material id
    tables: dict                       # material id -> (photo, compton, coherent) arrays
    grid: tuple                        # (lnE0, dlnE, n)
    source: Source
    energies: list
    n_histories: int
    seed: int
    groups: list = field(default_factory=list)   # scale-group names, index = group id
    extra: dict = field(default_factory=dict)

    def region_arrays(self):
        """(material id, density, group, active flag) per region."""
        mat = np.array([self.materials.index(r["material"]) for r in self.scene.regions], np.int32)
        rho = np.array([r["density"] for r in self.scene.regions], np.float32)
        grp = np.array([r["group"] for r in self.scene.regions], np.int32)
        act = np.array([1 if r["active"] else 0 for r in self.scene.regions], np.int32)
        return mat, rho, grp, act


def _tables_for(materials, coherent=True, overrides=None, pair=False):
    lnE0, dlnE, n = xsgen.grid()
    tabs = {}
    for i, name in enumerate(materials):
        if overrides and name in overrides:
            tabs[i] = overrides[name]
        else:
            tabs[i] = xsgen.material_table(name, lnE0, dlnE, n, coherent=coherent, pair=pair)
    return tabs, (lnE0, dlnE, n)


# ----------------------------------------------------------------------------
# detectors

def bare_crystal(n_seg=64):
    """Bare active Ge prism r 30, z in [-60, 0], in vacuum (256 facets at N=64)."""
    b = mg.SceneBuilder("vacuum", 0.0)
    b.add("crystal", "Ge", 5.32, mg.cylinder(30.0, -60.0, 0.0, n_seg), group=0, active=True)
    return b


HPGE_GROUPS = ["dead", "crystal", "window", "endcap", "cup"]


def hpge_detector(n_seg=128, n_phi=20, z_slices=1, world_half=500.0, builder=None):
    """p-type coaxial HPGe detector in an air box (region ids in add order).

    Front face of the end-cap at z = 5.5; crystal front face at z = 0.
    """
    b = builder or mg.SceneBuilder("vacuum", 0.0)
    g = {name: i for i, name in enumerate(HPGE_GROUPS)}
    h = world_half
    b.add("air", "air", 1.205e-3, mg.box((-h, -h, -h), (h, h, h)))
    b.add("endcap", "Al", 2.699, mg.cylinder(38.0, -100.0, 5.5, n_seg, z_slices), group=g["endcap"])
    b.add("window", "Al", 2.699, mg.cylinder(37.0, 5.0, 5.5 - EPS, n_seg), group=g["window"])
    b.add("interior", "vacuum", 0.0, mg.cylinder(37.0, -99.0, 5.0 - EPS, n_seg, z_slices))
    b.add("cup", "Al", 2.699, mg.cup(33.5, 32.5, -62.0, -1.0, 1.0, n_seg, z_slices), group=g["cup"])
    b.add("dead", "Ge", 5.32, mg.rounded_cylinder(32.0, -60.0, 0.0, 3.0, n_seg, n_phi, z_slices),
          group=g["dead"])
    # Eq. 6: active radius and length shrink by the dead-layer thickness D4
    d4 = 0.7
    b.add("active", "Ge", 5.32,
          mg.rounded_cylinder(32.0 - d4, -60.0 + EPS, 0.0 - d4, 3.0 - d4, n_seg, n_phi, z_slices),
          group=g["crystal"], active=True)
    b.add("bore", "vacuum", 0.0, mg.capsule_top(5.0, -60.0 + 2 * EPS, -15.0, n_seg, n_phi, z_slices))
    b.add("pin", "Cu", 8.96, mg.cylinder(1.0, -59.0, -25.0, n_seg, z_slices))
    b.add("coldfinger", "Cu", 8.96, mg.cylinder(5.0, -98.0, -62.5, n_seg, z_slices))
    return b


def add_bottle(b, r, h, z_base, matrix, density, n_seg=64, wall=1.5, group=-1):
    """PP container (closed, wall thickness `wall`) around a matrix cylinder."""
    b.add("container", "PP", 0.90,
          mg.cylinder(r + wall, z_base, z_base + h + 2 * wall, n_seg))
    return b.add("matrix", matrix, density,
                 mg.cylinder(r, z_base + wall, z_base + wall + h, n_seg), group=group)


def bottle_overlay(r, h, z_base, matrix, density, n_seg=64, wall=1.5, group=-1):
    """A PP bottle and its matrix alone, as an overlay mesh (regions: the host,
    container, matrix) for a detector scene; the same shells add_bottle puts
    into a full scene."""
    b = mg.SceneBuilder("vacuum", 0.0)
    add_bottle(b, r, h, z_base, matrix, density, n_seg=n_seg, wall=wall, group=group)
    return b.build()


def overlay_regions(scene, materials):
    """Region tuples (material id, density, group, ACTIVE flag) of an overlay scene."""
    return [(materials.index(r["material"]), float(r["density"]), int(r["group"]),
             1 if r["active"] else 0) for r in scene.regions]


# ----------------------------------------------------------------------------
# the five calibration workloads

def c1_bare(n_histories=100_000, seed=1001):
    b = bare_crystal(64)
    scene = b.build()
    mats = ["vacuum", "Ge"]
    tabs, grid = _tables_for(mats, coherent=False)
    return Workload("c1_bare_ge_256tri", scene, mats, tabs, grid,
                    Source(KIND_POINT, pos=(0.0, 0.0, 100.0)), [661.7], n_histories, seed,
                    groups=["crystal"])


def c2_hpge(n_histories=100_000_000, seed=1002, n_seg=128, n_phi=20, distance=250.0):
    b = hpge_detector(n_seg, n_phi)
    scene = b.build()
    mats = ["vacuum", "air", "Al", "Ge", "Cu"]
    tabs, grid = _tables_for(mats, coherent=False)
    return Workload("c2_hpge_20k_tri_point250", scene, mats, tabs, grid,
                    Source(KIND_POINT, pos=(0.0, 0.0, 5.5 + distance)),
                    log_energies(12), n_histories, seed, groups=list(HPGE_GROUPS))


def c3_jobs(n_jobs=64, seed=3003):
    """Per-job bottle geometry, matrix, density and history count (64 bottle jobs on the 256-facet crystal)."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(n_jobs):
        r = float(rng.uniform(20.0, 60.0))
        h = float(rng.uniform(10.0, 80.0))
        rho = float(rng.uniform(0.8, 1.6))
        n_total = int(round(10.0 ** rng.uniform(6.0, 8.0)))
        jobs.append(dict(r=r, h=h, density=rho, matrix="water" if j % 2 == 0 else "soil",
                         n_total=n_total))
    return jobs


def c3_job_workload(job, seed=1003, n_energies=20):
    b = bare_crystal(64)
    m = add_bottle(b, job["r"], job["h"], 2.0, job["matrix"], job["density"], group=1)
    scene = b.build()
    mats = ["vacuum", "Ge", "PP", "water", "soil"]
    tabs, grid = _tables_for(mats, coherent=False)
    src = Source(KIND_CYL, pos=(0.0, 0.0, 2.0 + 1.5), r_in=0.0, r_out=job["r"], h=job["h"], region=m)
    per_e = max(1, job["n_total"] // n_energies)
    return Workload("c3_bottle_on_bare_ge", scene, mats, tabs, grid, src,
                    log_energies(n_energies), per_e, seed, groups=["crystal", "matrix"])


def c4_grad(n_histories=100_000_000, seed=1004, n_seg=128, n_phi=20):
    b = hpge_detector(n_seg, n_phi)
    m = add_bottle(b, 35.0, 40.0, 5.5 + 2.0, "water", 1.0, group=len(HPGE_GROUPS))
    scene = b.build()
    mats = ["vacuum", "air", "Al", "Ge", "Cu", "PP", "water"]
    tabs, grid = _tables_for(mats, coherent=False)
    src = Source(KIND_CYL, pos=(0.0, 0.0, 5.5 + 2.0 + 1.5), r_in=0.0, r_out=35.0, h=40.0, region=m)
    return Workload("c4_hpge_water_sample_grad", scene, mats, tabs, grid, src,
                    log_energies(20), n_histories, seed, groups=list(HPGE_GROUPS) + ["matrix"])


def c5_stress(n_histories=125_000_000, seed=1005, n_seg=1024, n_phi=48, z_slices=24,
              matrix="water", density=1.0):
    b = hpge_detector(n_seg, n_phi, z_slices)
    # Marinelli beaker: PP inverted cup around an inverted-cup matrix that
    # wraps the end-cap side and covers the window with a 20 mm layer
    b.add("beaker", "PP", 0.90, mg.inverted_cup(71.5, 38.5, -61.5, 29.0, 23.0, n_seg, z_slices))
    m = b.add("matrix", matrix, density, mg.inverted_cup(70.0, 40.0, -60.0, 27.5, 20.0, n_seg, z_slices),
              group=len(HPGE_GROUPS))
    scene = b.build()
    mats = ["vacuum", "air", "Al", "Ge", "Cu", "PP", "water", "soil"]
    tabs, grid = _tables_for(mats, coherent=True)
    p = [1.0 / len(TABLE3_LINES_KEV)] * len(TABLE3_LINES_KEV)
    src = Source(KIND_CYL, pos=(0.0, 0.0, -60.0), r_in=0.0, r_out=70.0, h=87.5, region=m,
                 lines_keV=list(TABLE3_LINES_KEV), lines_prob=p)
    return Workload("c5_marinelli_1m_tri", scene, mats, tabs, grid, src, [0.0], n_histories, seed,
                    groups=list(HPGE_GROUPS) + ["matrix"])


# ----------------------------------------------------------------------------
# closed-form fixtures

def slab(thickness, mu_photo, mu_compton=0.0, mu_coherent=0.0, half=50.0, density=1.0,
         active=True, mu_pair=None):
    """Box slab z in [-thickness, 0] in vacuum with constant synthetic partials.

    The partials are mass attenuation coefficients [cm^2/g]; with density 1
    the linear coefficient is 0.1 * value [1/mm].  mu_pair (optional) is a
    constant pair-production partial, which transport applies above 2 m_e c^2
    only.
    """
    b = mg.SceneBuilder("vacuum", 0.0)
    b.add("slab", "synthetic", density, mg.box((-half, -half, -thickness), (half, half, 0.0)),
          group=0, active=active)
    scene = b.build()
    lnE0, dlnE, n = xsgen.grid()
    mats = ["vacuum", "synthetic"]
    tabs = {0: xsgen.constant_table(n=n),
            1: xsgen.constant_table(mu_photo, mu_compton, mu_coherent, n, pair=mu_pair)}
    return scene, mats, tabs, (lnE0, dlnE, n)


def nested_spheres(radii=(10.0, 20.0, 30.0), n_seg=48, n_rings=24):
    """Concentric spheres, region i+1 inside radius radii[i] (innermost first)."""
    b = mg.SceneBuilder("vacuum", 0.0)
    for i, r in enumerate(sorted(radii, reverse=True)):
        b.add(f"shell{i}", "Ge", 5.32, mg.uv_sphere(r, n_seg, n_rings))
    return b.build()


# ----------------------------------------------------------------------------
# parameter sets for the parametric detector generator (gadep_detmesh)

# The 20236-facet coaxial HPGe detector in Table 2 terms: end-cap r 38 on z in [-100, 5.5] (wall d3,
# window d2 = 0.5 at d5 = 5 above the crystal), cup wall d4 = 1 with a 0.5 mm
# gap, crystal r 32 x 60 with R_c 3, 0.7 mm dead layer, 5 mm bore 45 mm deep,
# pin and cold finger.
DETMESH_C2 = dict(d1=37.0, d2=0.5, d3=1.0, d4=1.0, d5=5.0, d6=3.5, d7=100.0, d8=62.0, d9=1.0,
                  d10=1.0, D1=60.0, D2=32.0, D3=3.0, D4=0.7, D5=45.0, D6=5.0, D7=0.0003,
                  n_theta=128, n_phi=20, z_slices=1, eps_mm=1e-3, cup_gap_mm=0.5,
                  cup_rim_mm=-1.0, pin_radius_mm=1.0, pin_length_mm=34.0, finger_radius_mm=5.0,
                  world_half_mm=500.0)

# Table 1 crystals: diameter, length, hole diameter, hole depth, outer / inner
# dead layer [mm] (the paper's QA numbers)
TABLE1 = {
    "#1 GMX45P4-76": (61.8, 61.9, 8.3, 60.0, 0.0003, 0.7),
    "#2 GEM-C50-LB-C": (68.1, 63.3, 10.1, 50.2, 0.7, 0.0003),
    "#3 GEM-C50P4": (67.9, 65.6, 8.5, 52.5, 0.7, 0.0003),
    "#4 GEM-C50P4": (68.7, 65.6, 8.6, 52.0, 0.7, 0.0003),
    "#5 GEM-C50P4": (68.5, 65.0, 8.7, 52.2, 0.7, 0.0003),
    "#6 GMX50P4-83": (68.8, 65.8, 8.6, 52.2, 0.0003, 0.7),
}

# material of each gadep_detmesh region (world, air, housing, window, vacuum,
# cup, crystal, active, contact, bore, pin, finger)
DETMESH_MATERIALS = ["vacuum", "air", "Al", "Al", "vacuum", "Al", "Ge", "Ge", "Ge", "vacuum",
                     "Cu", "Cu"]


def table1_detmesh(name, n_theta=64, n_phi=10):
    """gadep_detmesh parameters for a Table 1 crystal in the housing of the 20236-facet detector,
    widened to fit (the paper gives no housing numbers for these)."""
    dia, length, hdia, hdepth, outer, inner = TABLE1[name]
    D2 = dia / 2
    p = dict(DETMESH_C2)
    p.update(D1=length, D2=D2, D3=3.0, D4=outer, D5=hdepth, D6=hdia / 2, D7=inner,
             d1=D2 + 5.0, d6=3.5, d8=length + 2.0, d7=length + 40.0,
             n_theta=n_theta, n_phi=n_phi, pin_length_mm=hdepth - hdia / 2 - 8.0)
    return p

