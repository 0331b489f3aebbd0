// DetMesh-style parametric detector meshes (Sec. 2.2 and 2.3): a single-ended
// coaxial HPGe detector from the Table 2 parameter groups, built inside-out as
// closed, outward-oriented triangle shells, one per region, plus a VRML 2.0
// writer (Sec. 2.2.3).
//
// Bodies of revolution sample N_theta equidistant angles (Eq. 1-2); the
// rounded front edge of the crystal samples N_phi polar steps (Eq. 3-4) and
// faces +z, toward a source in front of the detector; the active volume
// shrinks by the dead-layer thickness (Eq. 6).  Nested shells that would
// touch are separated inside-out by eps (Sec. 2.4.2).  Facets are wound
// counter-clockwise seen from outside, so the Eq. 5 normal points out.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "gadep.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Mesh {
  std::vector<double> v;   // xyz
  std::vector<int32_t> f;  // 3 per facet
  std::vector<int32_t> reg;
};

// One closed shell under construction, appended to a Mesh with its region.
class Shell {
 public:
  Shell(Mesh& m, int32_t region) : m_(m), region_(region) {}

  int32_t vert(double x, double y, double z) {
    m_.v.push_back(x);
    m_.v.push_back(y);
    m_.v.push_back(z);
    return static_cast<int32_t>(m_.v.size() / 3 - 1);
  }
  // Eq. 1-2: n angularly equidistant vertices of radius rho at height z
  std::vector<int32_t> ring(double rho, double z, int n) {
    std::vector<int32_t> r(n);
    for (int i = 0; i < n; ++i) {
      const double th = 2.0 * kPi * i / n;
      r[i] = vert(rho * cos(th), rho * sin(th), z);
    }
    return r;
  }
  // quad strip between a lower and an upper ring; outward: normal away from the axis
  void band(const std::vector<int32_t>& lo, const std::vector<int32_t>& hi, bool outward) {
    const int n = static_cast<int>(lo.size());
    for (int i = 0; i < n; ++i) {
      const int j = (i + 1) % n;
      if (outward) {
        face(lo[i], lo[j], hi[j]);
        face(lo[i], hi[j], hi[i]);
      } else {
        face(lo[i], hi[j], lo[j]);
        face(lo[i], hi[i], hi[j]);
      }
    }
  }
  // cap fan around a centre vertex; up: normal +z
  void fan(int32_t c, const std::vector<int32_t>& r, bool up) {
    const int n = static_cast<int>(r.size());
    for (int i = 0; i < n; ++i) {
      const int j = (i + 1) % n;
      if (up)
        face(c, r[i], r[j]);
      else
        face(c, r[j], r[i]);
    }
  }
  // flat annulus between two rings at one height; up: normal +z
  void annulus(const std::vector<int32_t>& in, const std::vector<int32_t>& out, bool up) {
    const int n = static_cast<int>(in.size());
    for (int i = 0; i < n; ++i) {
      const int j = (i + 1) % n;
      if (up) {
        face(in[i], out[i], out[j]);
        face(in[i], out[j], in[j]);
      } else {
        face(in[i], out[j], out[i]);
        face(in[i], in[j], out[j]);
      }
    }
  }

 private:
  void face(int32_t a, int32_t b, int32_t c) {
    m_.f.push_back(a);
    m_.f.push_back(b);
    m_.f.push_back(c);
    m_.reg.push_back(region_);
  }
  Mesh& m_;
  int32_t region_;
};

std::vector<double> levels(double z0, double z1, int slices) {
  std::vector<double> z(slices + 1);
  for (int k = 0; k <= slices; ++k) z[k] = z0 + (z1 - z0) * k / slices;
  return z;
}

void cylinder(Mesh& m, int32_t region, double r, double z0, double z1, int n, int slices) {
  Shell s(m, region);
  std::vector<std::vector<int32_t>> rings;
  for (double z : levels(z0, z1, slices)) rings.push_back(s.ring(r, z, n));
  for (int k = 0; k < slices; ++k) s.band(rings[k], rings[k + 1], true);
  s.fan(s.vert(0, 0, z0), rings.front(), false);
  s.fan(s.vert(0, 0, z1), rings.back(), true);
}

// cylinder whose +z edge is rounded with radius rc (Eq. 3-4): the arc runs
// from the side wall's top ring (rho = r, z = z1 - rc) to the rim of the flat
// front face (rho = r - rc, z = z1)
void rounded_cylinder(Mesh& m, int32_t region, double r, double z0, double z1, double rc, int n,
                      int n_phi, int slices) {
  if (!(rc > 0)) {
    cylinder(m, region, r, z0, z1, n, slices);
    return;
  }
  Shell s(m, region);
  std::vector<std::vector<int32_t>> rings;
  for (double z : levels(z0, z1 - rc, slices)) rings.push_back(s.ring(r, z, n));
  for (int k = 0; k < slices; ++k) s.band(rings[k], rings[k + 1], true);
  std::vector<int32_t> prev = rings.back();
  for (int j = 1; j <= n_phi; ++j) {
    const double phi = 0.5 * kPi * j / n_phi;  // Eq. 3
    double rho = (r - rc) + rc * cos(phi);     // Eq. 4
    double z = z1 - rc * (1.0 - sin(phi));
    if (j == n_phi) rho = r - rc, z = z1;
    std::vector<int32_t> cur = s.ring(rho, z, n);
    s.band(prev, cur, true);
    prev = cur;
  }
  s.fan(s.vert(0, 0, z0), rings.front(), false);
  s.fan(s.vert(0, 0, z1), prev, true);
}

// cylinder with a hemispherical +z tip ending at z_apex (a borehole)
void capsule(Mesh& m, int32_t region, double r, double z0, double z_apex, int n, int n_phi,
             int slices) {
  Shell s(m, region);
  const double zc = z_apex - r;
  std::vector<std::vector<int32_t>> rings;
  for (double z : levels(z0, zc, slices)) rings.push_back(s.ring(r, z, n));
  for (int k = 0; k < slices; ++k) s.band(rings[k], rings[k + 1], true);
  std::vector<int32_t> prev = rings.back();
  for (int j = 1; j < n_phi; ++j) {
    const double phi = 0.5 * kPi * j / n_phi;
    std::vector<int32_t> cur = s.ring(r * cos(phi), zc + r * sin(phi), n);
    s.band(prev, cur, true);
    prev = cur;
  }
  s.fan(s.vert(0, 0, z_apex), prev, true);
  s.fan(s.vert(0, 0, z0), rings.front(), false);
}

// genus-0 cup solid open at +z: outer wall r_out on [z0, z1], cavity of radius
// r_in down to the floor at z0 + floor
void cup(Mesh& m, int32_t region, double r_out, double r_in, double z0, double z1, double floor,
         int n, int slices) {
  Shell s(m, region);
  const double zf = z0 + floor;
  std::vector<std::vector<int32_t>> outer, inner;
  for (double z : levels(z0, z1, slices)) outer.push_back(s.ring(r_out, z, n));
  for (double z : levels(zf, z1, slices)) inner.push_back(s.ring(r_in, z, n));
  for (int k = 0; k < slices; ++k) {
    s.band(outer[k], outer[k + 1], true);
    s.band(inner[k], inner[k + 1], false);
  }
  s.fan(s.vert(0, 0, z0), outer.front(), false);
  s.annulus(inner.back(), outer.back(), true);
  s.fan(s.vert(0, 0, zf), inner.front(), true);
}

// axis-aligned cube [-h, h]^3 (a world box), 12 facets
void box(Mesh& m, int32_t region, double h) {
  const int32_t base = static_cast<int32_t>(m.v.size() / 3);
  for (int k = 0; k < 8; ++k) {  // vertex k: x, y, z = +h where bit 0, 1, 2 is set
    m.v.push_back((k & 1) ? h : -h);
    m.v.push_back((k & 2) ? h : -h);
    m.v.push_back((k & 4) ? h : -h);
  }
  // faces -z, +z, -y, +y, -x, +x, each counter-clockwise seen from outside
  static const int q[6][4] = {{0, 2, 3, 1}, {4, 5, 7, 6}, {0, 1, 5, 4},
                              {2, 6, 7, 3}, {0, 4, 6, 2}, {1, 3, 7, 5}};
  for (const auto& k : q) {
    m.f.insert(m.f.end(), {base + k[0], base + k[1], base + k[2], base + k[0], base + k[2], base + k[3]});
    m.reg.push_back(region);
    m.reg.push_back(region);
  }
}

int fail(char* err, int32_t len, int code, const std::string& msg) {
  if (err && len > 0) {
    strncpy(err, msg.c_str(), static_cast<size_t>(len) - 1);
    err[len - 1] = 0;
  }
  return code;
}

}  // namespace

extern "C" {

gadep_status gadep_detmesh(const gadep_detector* p, float* xyz, int64_t cap_vertices,
                           int32_t* tri_vertices, int32_t* tri_region, int64_t cap_facets,
                           int64_t* n_vertices, int64_t* n_facets, int32_t* region_parent,
                           char* err, int32_t err_len) {
  if (!p || !n_vertices || !n_facets) return static_cast<gadep_status>(fail(err, err_len, GADEP_E_ARG, "detmesh: null argument"));
  const int n = p->n_theta, nphi = p->n_phi, zs = p->z_slices;
  const double e = p->eps_mm;
  auto bad = [&](const std::string& m) {
    return static_cast<gadep_status>(fail(err, err_len, GADEP_E_ARG, "detmesh: " + m));
  };
  if (n < 3 || nphi < 2 || zs < 1 || !(e > 0)) return bad("n_theta >= 3, n_phi >= 2, z_slices >= 1, eps > 0");
  const double D1 = p->D1, D2 = p->D2, D3 = p->D3, D4 = p->D4, D5 = p->D5, D6 = p->D6, D7 = p->D7;
  if (!(D1 > 0 && D2 > 0 && D3 >= 0 && D4 >= 0 && D5 >= 0 && D6 >= 0 && D7 >= 0))
    return bad("crystal parameters must be positive (D3..D7 >= 0)");
  if (!(D3 < D2 && D3 < D1)) return bad("rounding radius D3 must be below the crystal radius and length");
  // outer dead layer: a shell of its own only when it is clearly thicker than
  // the separation (an implanted contact of a fraction of a micrometre is not)
  const bool dead = D4 >= 4.0 * e;
  const double Ra = dead ? D2 - D4 : D2, Ztop_a = dead ? -D4 : 0.0;
  const double Rca = dead ? (D3 > D4 ? D3 - D4 : 0.0) : D3;
  const double zbot_a = dead ? -D1 + e : -D1;
  const bool hole = D5 > 0 && D6 > 0;
  const bool contact = hole && D7 >= 4.0 * e;
  if (hole) {
    // the borehole (with its contact layer) stays within the flat-fronted
    // core of the active volume, clear of its front face
    if (!(D6 + (contact ? D7 : 0.0) + 2 * e < Ra - Rca)) return bad("borehole (with contact layer) wider than the active volume");
    if (!(-D1 + D5 + (contact ? D7 : 0.0) < Ztop_a - 2 * e)) return bad("borehole reaches the front face");
    if (!(D5 > D6 + 4 * e)) return bad("borehole length must exceed its radius");
  }
  const double d1 = p->d1, d2 = p->d2, d3 = p->d3, d4 = p->d4, d5 = p->d5, d6 = p->d6, d7 = p->d7,
               d8 = p->d8, d9 = p->d9, d10 = p->d10;
  if (!(d1 > 0 && d2 > 0 && d3 > 0 && d4 > 0 && d5 > 0 && d6 > 0 && d7 > 0 && d8 > 0 && d9 > 0 && d10 > 0))
    return bad("external parameters d1..d10 must be positive");
  // crystal cup around the crystal: cavity radius D2 + gap, wall d4, floor d10,
  // from z = -d8 up to its rim
  const double gap = p->cup_gap_mm, rim = p->cup_rim_mm;
  if (!(gap > 0)) return bad("cup_gap_mm must be positive");
  const double r_cav = D2 + gap, r_cup = r_cav + d4;
  if (!(-d8 + d10 < -D1 - e)) return bad("crystal cup too short for the crystal (d8 - d10 <= D1)");
  if (!(rim > -D1 && rim < d5 - e)) return bad("cup rim must lie between the crystal back and the window");
  // vacuum housing: inner radius over the side vacuum d6, wall d3; its front
  // wall is the window plane (thickness d2) at top vacuum d5 above the crystal
  const double R_in = r_cup + d6, R_out = R_in + d3;
  if (!(d1 <= R_in)) return bad("window radius d1 exceeds the housing's inner radius");
  const double z_win0 = d5, z_top = d5 + d2, z_hbot = -d7, z_vbot = -d7 + d9;
  // adaptive assembly: the vacuum reaches from the housing floor to just
  // below the window, whatever the crystal's distance to the window
  if (!(z_vbot < -d8 - e)) return bad("housing too short for the crystal cup (d7 - d9 <= d8)");
  const double world = p->world_half_mm;
  if (world > 0 && !(world > R_out + e && world > z_top + e && world > d7 + e))
    return bad("world box smaller than the housing");

  Mesh m;
  std::vector<int32_t> parent(GADEP_DM_N, -1);
  parent[GADEP_DM_WORLD] = -1;
  const int32_t outside = world > 0 ? GADEP_DM_AIR : GADEP_DM_WORLD;
  if (world > 0) {
    box(m, GADEP_DM_AIR, world);
    parent[GADEP_DM_AIR] = GADEP_DM_WORLD;
  }
  // housing (end-cap) and the window disk in its front wall
  cylinder(m, GADEP_DM_HOUSING, R_out, z_hbot, z_top, n, zs);
  parent[GADEP_DM_HOUSING] = outside;
  cylinder(m, GADEP_DM_WINDOW, d1, z_win0, z_top - e, n, 1);
  parent[GADEP_DM_WINDOW] = GADEP_DM_HOUSING;
  cylinder(m, GADEP_DM_VACUUM, R_in, z_vbot, z_win0 - e, n, zs);
  parent[GADEP_DM_VACUUM] = GADEP_DM_HOUSING;
  cup(m, GADEP_DM_CUP, r_cup, r_cav, -d8, rim, d10, n, zs);
  parent[GADEP_DM_CUP] = GADEP_DM_VACUUM;
  // crystal: outer dead layer and active volume (Eq. 6)
  const int32_t crystal_region = dead ? GADEP_DM_CRYSTAL : GADEP_DM_ACTIVE;
  rounded_cylinder(m, crystal_region, D2, -D1, 0.0, D3, n, nphi, zs);
  parent[crystal_region] = GADEP_DM_VACUUM;
  if (dead) {
    rounded_cylinder(m, GADEP_DM_ACTIVE, Ra, zbot_a, Ztop_a, Rca, n, nphi, zs);
    parent[GADEP_DM_ACTIVE] = GADEP_DM_CRYSTAL;
  }
  // borehole from the back face, positioned by the crystal's place in the cup;
  // the contact layer lines it inside the active volume
  if (hole) {
    double zb = zbot_a + e;
    int32_t host = GADEP_DM_ACTIVE;
    if (contact) {
      capsule(m, GADEP_DM_CONTACT, D6 + D7, zb, -D1 + D5 + D7, n, nphi, zs);
      parent[GADEP_DM_CONTACT] = host;
      host = GADEP_DM_CONTACT;
      zb += e;
    }
    capsule(m, GADEP_DM_BORE, D6, zb, -D1 + D5, n, nphi, zs);
    parent[GADEP_DM_BORE] = host;
    const double pr = p->pin_radius_mm, pl = p->pin_length_mm;
    if (pr > 0 && pl > 0) {
      if (!(pr + e < D6 && zb + 1.0 + pl < -D1 + D5 - D6 - e)) return bad("pin does not fit in the borehole");
      cylinder(m, GADEP_DM_PIN, pr, zb + 1.0, zb + 1.0 + pl, n, 1);
      parent[GADEP_DM_PIN] = GADEP_DM_BORE;
    }
  }
  // cold finger between the cup floor and the housing floor
  const double fr = p->finger_radius_mm;
  if (fr > 0) {
    const double f0 = z_vbot + 1.0, f1 = -d8 - 0.5;
    if (!(fr < r_cup && f1 - f0 > 1.0)) return bad("no room for the cold finger");
    cylinder(m, GADEP_DM_FINGER, fr, f0, f1, n, zs);
    parent[GADEP_DM_FINGER] = GADEP_DM_VACUUM;
  }

  const int64_t nv = static_cast<int64_t>(m.v.size() / 3), nt = static_cast<int64_t>(m.reg.size());
  *n_vertices = nv;
  *n_facets = nt;
  if (region_parent) memcpy(region_parent, parent.data(), sizeof(int32_t) * GADEP_DM_N);
  if (xyz || tri_vertices || tri_region) {
    if (cap_vertices < nv || cap_facets < nt)
      return static_cast<gadep_status>(fail(err, err_len, GADEP_E_ARG, "detmesh: output capacity too small"));
    if (xyz)
      for (int64_t i = 0; i < 3 * nv; ++i) xyz[i] = static_cast<float>(m.v[i]);
    if (tri_vertices) memcpy(tri_vertices, m.f.data(), sizeof(int32_t) * 3 * nt);
    if (tri_region) memcpy(tri_region, m.reg.data(), sizeof(int32_t) * nt);
  }
  return GADEP_OK;
}

gadep_status gadep_write_vrml(const char* path, const float* xyz, int64_t n_vertices,
                              const int32_t* tri_vertices, const int32_t* tri_region,
                              int64_t n_tri, int32_t n_regions) {
  if (!path || !xyz || !tri_vertices || !tri_region || n_vertices < 3 || n_tri < 1 || n_regions < 1)
    return GADEP_E_ARG;
  for (int64_t f = 0; f < n_tri; ++f) {
    if (tri_region[f] < 0 || tri_region[f] >= n_regions) return GADEP_E_ARG;
    for (int k = 0; k < 3; ++k)
      if (tri_vertices[3 * f + k] < 0 || tri_vertices[3 * f + k] >= n_vertices) return GADEP_E_ARG;
  }
  FILE* fp = fopen(path, "w");
  if (!fp) return GADEP_E_ARG;
  fprintf(fp, "#VRML V2.0 utf8\n# %lld facets in %d regions\n", static_cast<long long>(n_tri), n_regions);
  // one Shape with an IndexedFaceSet per region; all regions share the vertex list
  for (int32_t r = 0; r < n_regions; ++r) {
    int64_t count = 0;
    for (int64_t f = 0; f < n_tri; ++f) count += tri_region[f] == r;
    if (count == 0) continue;
    const double hue = 0.61803398875 * r - floor(0.61803398875 * r);
    fprintf(fp, "DEF region_%d Shape {\n  appearance Appearance { material Material { diffuseColor %.3f %.3f %.3f transparency 0.5 } }\n",
            r, 0.3 + 0.7 * hue, 0.3 + 0.7 * (1.0 - hue), 0.6);
    fprintf(fp, "  geometry IndexedFaceSet {\n    solid FALSE\n    coord Coordinate { point [\n");
    for (int64_t i = 0; i < n_vertices; ++i)
      fprintf(fp, "      %.9g %.9g %.9g,\n", xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
    fprintf(fp, "    ] }\n    coordIndex [\n");
    for (int64_t f = 0; f < n_tri; ++f)
      if (tri_region[f] == r)
        fprintf(fp, "      %d, %d, %d, -1,\n", tri_vertices[3 * f], tri_vertices[3 * f + 1],
                tri_vertices[3 * f + 2]);
    fprintf(fp, "    ]\n  }\n}\n");
  }
  const bool ok = ferror(fp) == 0;
  fclose(fp);
  return ok ? GADEP_OK : GADEP_E_ARG;
}

}  // extern "C"
