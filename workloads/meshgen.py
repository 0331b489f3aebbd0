"""Closed, outward-oriented triangle shells for synthetic HPGe detector scenes.

This module only builds seeded, deterministic *inputs* (vertex and facet
arrays); it holds none of the transport arithmetic.  It serves both the HIP
path and the CPU oracle.

Conventions (paper Sec. 2.2.2):
  * ring vertices of a body of revolution sit at the angularly equidistant
    angles theta_i = 2*pi*i/N_theta, i = 0..N_theta-1 (Eq. 1), with
    x = R cos(theta_i), y = R sin(theta_i) (Eq. 2);
  * the rounded front edge of a crystal is sampled at phi_j = (pi/2) j/N_phi,
    j = 0..N_phi (Eq. 3), with rho_j = (R - Rc) + Rc cos(phi_j) and the height
    offset Rc (1 - sin(phi_j)) (Eq. 4).  The paper writes the rounded face at
    the low-z end of a local frame; here it is mirrored so that it faces +z,
    toward the source;
  * every facet is wound counter-clockwise when seen from outside, so that
    the Eq. 5 normal (v1 - v0) x (v2 - v0) points out of the enclosed volume.

Caps are triangle fans around a centre vertex, so a plain N-segment
cylinder has 4N facets.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Shell:
    """One closed, consistently oriented triangle surface."""

    V: np.ndarray  # [nv, 3] float64, mm
    F: np.ndarray  # [nf, 3] int64, CCW seen from outside

    def translated(self, dx=0.0, dy=0.0, dz=0.0) -> "Shell":
        return Shell(self.V + np.array([dx, dy, dz]), self.F.copy())


class _Builder:
    def __init__(self):
        self.verts: list = []
        self.faces: list = []

    def vert(self, x, y, z) -> int:
        self.verts.append((x, y, z))
        return len(self.verts) - 1

    def ring(self, rho, z, n) -> list:
        """Eq. 1-2: N angularly equidistant vertices of radius rho at height z."""
        idx = []
        for i in range(n):
            th = 2.0 * math.pi * i / n
            idx.append(self.vert(rho * math.cos(th), rho * math.sin(th), z))
        return idx

    def band(self, lo, hi, outward=True):
        """Quad strip between two rings; lower ring `lo`, upper ring `hi`.

        With outward=True the normal of a vertical band points away from the
        axis (theta_hat x z_hat = r_hat); outward=False reverses it.
        """
        n = len(lo)
        for i in range(n):
            j = (i + 1) % n
            a0, a1, b0, b1 = lo[i], lo[j], hi[i], hi[j]
            if outward:
                self.faces.append((a0, a1, b1))
                self.faces.append((a0, b1, b0))
            else:
                self.faces.append((a0, b1, a1))
                self.faces.append((a0, b0, b1))

    def fan(self, centre, ring, up=True):
        """Cap fan: normal +z when up, -z otherwise."""
        n = len(ring)
        for i in range(n):
            j = (i + 1) % n
            if up:
                self.faces.append((centre, ring[i], ring[j]))
            else:
                self.faces.append((centre, ring[j], ring[i]))

    def annulus(self, inner, outer, up=True):
        """Flat annulus between two rings at the same height."""
        n = len(inner)
        for i in range(n):
            j = (i + 1) % n
            if up:
                self.faces.append((inner[i], outer[i], outer[j]))
                self.faces.append((inner[i], outer[j], inner[j]))
            else:
                self.faces.append((inner[i], outer[j], outer[i]))
                self.faces.append((inner[i], inner[j], outer[j]))

    def shell(self) -> Shell:
        return Shell(np.asarray(self.verts, dtype=np.float64),
                     np.asarray(self.faces, dtype=np.int64))


def _zlevels(z0, z1, slices):
    return [z0 + (z1 - z0) * k / slices for k in range(slices + 1)]


def cylinder(r, z0, z1, n_seg, z_slices=1) -> Shell:
    """Closed right circular prism (inscribed N-gon), axis z, z in [z0, z1]."""
    assert z1 > z0 and r > 0 and n_seg >= 3 and z_slices >= 1
    b = _Builder()
    rings = [b.ring(r, z, n_seg) for z in _zlevels(z0, z1, z_slices)]
    for k in range(z_slices):
        b.band(rings[k], rings[k + 1])
    b.fan(b.vert(0.0, 0.0, z0), rings[0], up=False)
    b.fan(b.vert(0.0, 0.0, z1), rings[-1], up=True)
    return b.shell()


def rounded_cylinder(r, z0, z1, rc, n_seg, n_phi, z_slices=1) -> Shell:
    """Cylinder whose top (+z) edge is rounded with radius rc (Eq. 3-4).

    The arc rings j = 0..n_phi run from (rho = r, z = z1 - rc), which is the
    top ring of the side wall, to (rho = r - rc, z = z1), the rim of the flat
    front face.
    """
    assert 0 < rc < r and z1 - z0 > rc and n_phi >= 1
    b = _Builder()
    side_top = z1 - rc
    rings = [b.ring(r, z, n_seg) for z in _zlevels(z0, side_top, z_slices)]
    for k in range(z_slices):
        b.band(rings[k], rings[k + 1])
    prev = rings[-1]
    for j in range(1, n_phi + 1):
        phi = 0.5 * math.pi * j / n_phi
        rho = (r - rc) + rc * math.cos(phi)
        z = z1 - rc * (1.0 - math.sin(phi))
        if j == n_phi:  # exact end values
            rho, z = r - rc, z1
        cur = b.ring(rho, z, n_seg)
        b.band(prev, cur)
        prev = cur
    b.fan(b.vert(0.0, 0.0, z0), rings[0], up=False)
    b.fan(b.vert(0.0, 0.0, z1), prev, up=True)
    return b.shell()


def capsule_top(r, z0, z_apex, n_seg, n_phi, z_slices=1) -> Shell:
    """Cylinder with a hemispherical top tip ending in an apex at z_apex.

    Used for the borehole: flat bottom at z0, side wall up to z_apex - r, then
    a hemisphere of radius r sampled at n_phi polar steps; the last ring
    collapses into the single apex vertex, so no redundant geometry sits at
    the apex.
    """
    assert z_apex - r > z0 and n_phi >= 2
    b = _Builder()
    zc = z_apex - r
    rings = [b.ring(r, z, n_seg) for z in _zlevels(z0, zc, z_slices)]
    for k in range(z_slices):
        b.band(rings[k], rings[k + 1])
    prev = rings[-1]
    for j in range(1, n_phi):
        phi = 0.5 * math.pi * j / n_phi
        cur = b.ring(r * math.cos(phi), zc + r * math.sin(phi), n_seg)
        b.band(prev, cur)
        prev = cur
    b.fan(b.vert(0.0, 0.0, z_apex), prev, up=True)
    b.fan(b.vert(0.0, 0.0, z0), rings[0], up=False)
    return b.shell()


def cup(r_out, r_in, z0, z1, floor, n_seg, z_slices=1) -> Shell:
    """Genus-0 cup solid open at +z: outer wall r_out on [z0, z1], cavity of
    radius r_in down to the floor at z0 + floor."""
    assert r_out > r_in > 0 and z1 - z0 > floor > 0
    b = _Builder()
    zf = z0 + floor
    outer = [b.ring(r_out, z, n_seg) for z in _zlevels(z0, z1, z_slices)]
    inner = [b.ring(r_in, z, n_seg) for z in _zlevels(zf, z1, z_slices)]
    for k in range(z_slices):
        b.band(outer[k], outer[k + 1], outward=True)
        b.band(inner[k], inner[k + 1], outward=False)
    b.fan(b.vert(0.0, 0.0, z0), outer[0], up=False)
    b.annulus(inner[-1], outer[-1], up=True)
    b.fan(b.vert(0.0, 0.0, zf), inner[0], up=True)
    return b.shell()


def inverted_cup(r_out, r_in, z0, z1, roof, n_seg, z_slices=1) -> Shell:
    """Genus-0 cup solid open at -z (a Marinelli-type shape): outer wall r_out
    on [z0, z1], cavity of radius r_in from z0 up to z1 - roof."""
    s = cup(r_out, r_in, -z1, -z0, roof, n_seg, z_slices)
    V = s.V.copy()
    V[:, 2] = -V[:, 2]
    # mirroring z reverses orientation; swap two vertices of each facet
    F = s.F[:, [0, 2, 1]].copy()
    return Shell(V, F)


def box(lo, hi) -> Shell:
    """Axis-aligned box, 12 facets."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    V = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], dtype=np.float64)
    F = np.array([
        [0, 2, 1], [0, 3, 2],  # z0, normal -z
        [4, 5, 6], [4, 6, 7],  # z1, normal +z
        [0, 1, 5], [0, 5, 4],  # y0, normal -y
        [3, 7, 6], [3, 6, 2],  # y1, normal +y
        [0, 4, 7], [0, 7, 3],  # x0, normal -x
        [1, 2, 6], [1, 6, 5],  # x1, normal +x
    ], dtype=np.int64)
    return Shell(V, F)


def uv_sphere(R, n_seg, n_rings) -> Shell:
    """Sphere from n_rings-1 latitude rings plus two pole vertices."""
    b = _Builder()
    south = b.vert(0.0, 0.0, -R)
    rings = []
    for k in range(1, n_rings):
        lat = -0.5 * math.pi + math.pi * k / n_rings
        rings.append(b.ring(R * math.cos(lat), R * math.sin(lat), n_seg))
    for k in range(len(rings) - 1):
        b.band(rings[k], rings[k + 1])
    b.fan(south, rings[0], up=False)
    b.fan(b.vert(0.0, 0.0, R), rings[-1], up=True)
    return b.shell()


# ----------------------------------------------------------------------------
# checks on the generator itself (used by tests; not part of any transport)

def signed_volume(V, F) -> float:
    """Sum over facets of v0 . (v1 x v2) / 6."""
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def euler_characteristic(F) -> int:
    """V - E + F over the vertices and edges actually referenced by F."""
    verts = np.unique(F)
    e = np.sort(np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]), axis=1)
    edges = np.unique(e, axis=0)
    return int(len(verts) - len(edges) + len(F))


# ----------------------------------------------------------------------------
# scenes

@dataclass
class Scene:
    """Region-tagged triangle soup plus the region table.

    Region 0 is the world (everything outside every shell).  Each shell is
    tagged with the region it encloses.
    """

    xyz: np.ndarray            # [nv, 3] float32
    tri: np.ndarray            # [nt, 3] int32
    tri_region: np.ndarray     # [nt] int32
    regions: list              # list of dicts: name, material, density, group, active
    shells: list = field(default_factory=list)  # (name, first_tri, n_tri)

    @property
    def n_regions(self) -> int:
        return len(self.regions)

    def region_id(self, name) -> int:
        for i, r in enumerate(self.regions):
            if r["name"] == name:
                return i
        raise KeyError(name)


class SceneBuilder:
    def __init__(self, world_material="vacuum", world_density=0.0):
        self.regions = [dict(name="world", material=world_material,
                             density=world_density, group=-1, active=False)]
        self._V, self._F, self._R = [], [], []
        self._nv = 0
        self.shells = []

    def add_region(self, name, material, density, group=-1, active=False) -> int:
        self.regions.append(dict(name=name, material=material, density=float(density),
                                 group=int(group), active=bool(active)))
        return len(self.regions) - 1

    def add_shell(self, region: int, shell: Shell, name=None):
        nt0 = sum(len(f) for f in self._F)
        self._V.append(shell.V)
        self._F.append(shell.F + self._nv)
        self._R.append(np.full(len(shell.F), region, dtype=np.int32))
        self._nv += len(shell.V)
        self.shells.append((name or self.regions[region]["name"], nt0, len(shell.F)))

    def add(self, name, material, density, shell, group=-1, active=False) -> int:
        r = self.add_region(name, material, density, group, active)
        self.add_shell(r, shell, name)
        return r

    def build(self) -> Scene:
        V = np.concatenate(self._V).astype(np.float32)
        F = np.concatenate(self._F).astype(np.int32)
        R = np.concatenate(self._R).astype(np.int32)
        return Scene(V, F, R, [dict(r) for r in self.regions], list(self.shells))
