// Host-only driver for the AddressSanitizer / UndefinedBehaviorSanitizer
// build of the library's CPU code (mesh validation, parity topology, BVH
// builders, parametric detector generator, VRML writer).  Reads meshes and
// detector parameter blocks written by the test and runs every host path on
// them; any sanitizer report makes the process fail.
//
// usage: host_driver mesh <file> | detmesh <file> <vrml-out> | badmesh <file>
// mesh file: int64 nv, int64 nt, int32 n_regions, int32 pad, float xyz[3 nv],
//            int32 tri[3 nt], int32 tri_region[nt]
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "gadep.h"

static bool read_all(const char* path, std::vector<char>& buf) {
  FILE* f = fopen(path, "rb");
  if (!f) return false;
  char tmp[65536];
  size_t n;
  while ((n = fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + n);
  fclose(f);
  return true;
}

struct Mesh {
  int64_t nv = 0, nt = 0;
  int32_t n_regions = 0;
  std::vector<float> xyz;
  std::vector<int32_t> tri, reg;
};

static bool load_mesh(const char* path, Mesh& m) {
  std::vector<char> b;
  if (!read_all(path, b) || b.size() < 24) return false;
  memcpy(&m.nv, b.data(), 8);
  memcpy(&m.nt, b.data() + 8, 8);
  memcpy(&m.n_regions, b.data() + 16, 4);
  const size_t need = 24 + 12 * m.nv + 12 * m.nt + 4 * m.nt;
  if (b.size() != need) return false;
  m.xyz.resize(3 * m.nv);
  m.tri.resize(3 * m.nt);
  m.reg.resize(m.nt);
  memcpy(m.xyz.data(), b.data() + 24, 12 * m.nv);
  memcpy(m.tri.data(), b.data() + 24 + 12 * m.nv, 12 * m.nt);
  memcpy(m.reg.data(), b.data() + 24 + 12 * m.nv + 12 * m.nt, 4 * m.nt);
  return true;
}

static int prepare_all(const Mesh& m, double split) {
  for (int method = 0; method <= 2; ++method) {
    gadep_mesh_info info;
    char err[256];
    gadep_status s = gadep_mesh_prepare(m.xyz.data(), m.nv, m.tri.data(), m.reg.data(), m.nt,
                                        m.n_regions, 1e-4, 1, method, split, nullptr, nullptr,
                                        nullptr, 0, nullptr, 0, &info, err, sizeof err);
    if (s != GADEP_OK) {
      fprintf(stderr, "prepare method %d: %d %s\n", method, s, err);
      return 1;
    }
    std::vector<int32_t> outside(m.nt), shell(m.nt), order(info.n_slots);
    std::vector<uint32_t> nodes(16 * info.n_nodes);
    s = gadep_mesh_prepare(m.xyz.data(), m.nv, m.tri.data(), m.reg.data(), m.nt, m.n_regions,
                           1e-4, 1, method, split, outside.data(), shell.data(), nodes.data(),
                           info.n_nodes, order.data(), info.n_slots, &info, err, sizeof err);
    if (s != GADEP_OK) {
      fprintf(stderr, "prepare method %d (outputs): %d %s\n", method, s, err);
      return 1;
    }
    printf("method %d: shells %d nodes %lld depth %d slots %lld\n", method, info.n_shells,
           (long long)info.n_nodes, info.depth, (long long)info.n_slots);
  }
  return 0;
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  if (!strcmp(argv[1], "mesh")) {
    Mesh m;
    if (!load_mesh(argv[2], m)) return 3;
    return prepare_all(m, 1.0);
  }
  if (!strcmp(argv[1], "badmesh")) {
    // the mesh has a defect: every validation path must reject it cleanly
    Mesh m;
    if (!load_mesh(argv[2], m)) return 3;
    gadep_mesh_info info;
    char err[256];
    gadep_status s = gadep_mesh_prepare(m.xyz.data(), m.nv, m.tri.data(), m.reg.data(), m.nt,
                                        m.n_regions, 1e-4, 1, 0, 1.0, nullptr, nullptr, nullptr,
                                        0, nullptr, 0, &info, err, sizeof err);
    printf("rejected: %d %s\n", s, err);
    return s == GADEP_OK ? 1 : 0;
  }
  if (!strcmp(argv[1], "detmesh") && argc >= 4) {
    std::vector<char> b;
    if (!read_all(argv[2], b) || b.size() != sizeof(gadep_detector)) return 3;
    gadep_detector d;
    memcpy(&d, b.data(), sizeof d);
    int64_t nv = 0, nt = 0;
    int32_t parent[64];
    char err[256];
    gadep_status s = gadep_detmesh(&d, nullptr, 0, nullptr, nullptr, 0, &nv, &nt, parent, err,
                                   sizeof err);
    if (s != GADEP_OK) {
      printf("detmesh rejected: %d %s\n", s, err);
      return 0;  // parameters that do not fit are an expected outcome
    }
    Mesh m;
    m.nv = nv;
    m.nt = nt;
    m.xyz.resize(3 * nv);
    m.tri.resize(3 * nt);
    m.reg.resize(nt);
    s = gadep_detmesh(&d, m.xyz.data(), nv, m.tri.data(), m.reg.data(), nt, &nv, &nt, parent, err,
                      sizeof err);
    if (s != GADEP_OK) return 4;
    m.n_regions = 0;
    for (int32_t r : m.reg) m.n_regions = r + 1 > m.n_regions ? r + 1 : m.n_regions;
    if (gadep_write_vrml(argv[3], m.xyz.data(), m.nv, m.tri.data(), m.reg.data(), m.nt,
                         m.n_regions) != GADEP_OK)
      return 5;
    printf("detmesh: %lld vertices %lld facets\n", (long long)nv, (long long)nt);
    return prepare_all(m, 1.0);
  }
  return 2;
}
