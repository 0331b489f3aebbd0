/* Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * oracle (test infrastructure): loads a mesh, its regions, cross sections and
 * a source written by the test, and runs the oracle's localisation, closest
 * hit, emission, transport (two threads, spectrum, scores) and broadening on
 * them.  Any sanitizer report makes the process fail.
 *
 * usage: oracle_driver <mesh file> <setup file> <histories>
 * mesh file: as the host driver's.  setup file: int32 n_regions, int32 pad, then per
 * region {int32 material, group, active, pad; double density}; int32 n_mat,
 * n_e; double lnE0, dlnE; per material 4 partials of n_e doubles (all zero =
 * absent); source {int32 kind, region, n_lines, pad; double pos[3], dir[3],
 * r_in, r_out, h, E0}; n_lines pairs {double keV, weight}. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static char* slurp(const char* path, long* len) {
  FILE* f = fopen(path, "rb");
  if (!f) return NULL;
  fseek(f, 0, SEEK_END);
  *len = ftell(f);
  fseek(f, 0, SEEK_SET);
  char* b = (char*)malloc((size_t)*len);
  if (b && fread(b, 1, (size_t)*len, f) != (size_t)*len) {
    free(b);
    b = NULL;
  }
  fclose(f);
  return b;
}

#define TAKE(dst, n)                         \
  do {                                       \
    if (off + (long)(n) > len) return 3;     \
    memcpy((dst), buf + off, (size_t)(n));   \
    off += (long)(n);                        \
  } while (0)

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  long len = 0, off = 0;
  char* buf = slurp(argv[1], &len);
  if (!buf) return 3;
  int64_t nv, nt;
  int32_t n_regions, pad;
  TAKE(&nv, 8);
  TAKE(&nt, 8);
  TAKE(&n_regions, 4);
  TAKE(&pad, 4);
  float* xyz = (float*)malloc(12 * (size_t)nv);
  int32_t* tri = (int32_t*)malloc(12 * (size_t)nt);
  int32_t* reg = (int32_t*)malloc(4 * (size_t)nt);
  TAKE(xyz, 12 * nv);
  TAKE(tri, 12 * nt);
  TAKE(reg, 4 * nt);
  free(buf);

  buf = slurp(argv[2], &len);
  off = 0;
  if (!buf) return 3;
  int32_t nr, pad2;
  TAKE(&nr, 4);
  TAKE(&pad2, 4);  /* keeps the doubles that follow 8-byte aligned */
  if (nr != n_regions) return 4;
  int rc = 0;
  for (int pass = 0; pass < 2 && rc == 0; ++pass) {
    /* pass 0: brute force; pass 1: the oracle's own BVH */
    orc_scene* s = orc_scene_create(xyz, nv, tri, reg, nt, n_regions, pass);
    if (!s) return 5;
    long o2 = off;
    for (int32_t r = 0; r < n_regions; ++r) {
      int32_t hdr[4];
      double rho;
      memcpy(hdr, buf + o2, 16);
      memcpy(&rho, buf + o2 + 16, 8);
      o2 += 24;
      if (orc_set_region(s, r, hdr[0], rho, hdr[1], hdr[2])) return 6;
    }
    int32_t n_mat, n_e;
    double lnE0, dlnE;
    memcpy(&n_mat, buf + o2, 4);
    memcpy(&n_e, buf + o2 + 4, 4);
    memcpy(&lnE0, buf + o2 + 8, 8);
    memcpy(&dlnE, buf + o2 + 16, 8);
    o2 += 24;
    for (int32_t m = 0; m < n_mat; ++m) {
      const double* part[4];
      for (int i = 0; i < 4; ++i) {
        const double* p = (const double*)(buf + o2);
        int any = 0;
        for (int32_t k = 0; k < n_e; ++k) any |= p[k] != 0.0;
        part[i] = any ? p : NULL;
        o2 += 8L * n_e;
      }
      if (orc_set_xs(s, m, lnE0, dlnE, n_e, part[0], part[1], part[2], part[3])) return 7;
    }
    int32_t sh[4];
    double sd[12];
    memcpy(sh, buf + o2, 16);
    memcpy(sd, buf + o2 + 16, 96);
    o2 += 112;
    orc_source src;
    memset(&src, 0, sizeof src);
    src.kind = sh[0];
    src.region = sh[1];
    src.n_lines = sh[2];
    for (int a = 0; a < 3; ++a) {
      src.pos[a] = sd[a];
      src.dir[a] = sd[3 + a];
    }
    src.r_in = sd[6];
    src.r_out = sd[7];
    src.h = sd[8];
    const double E0 = sd[9];
    double* lk = NULL;
    double* lp = NULL;
    if (src.n_lines > 0) {
      lk = (double*)malloc(8 * (size_t)src.n_lines);
      lp = (double*)malloc(8 * (size_t)src.n_lines);
      for (int32_t i = 0; i < src.n_lines; ++i) {
        memcpy(&lk[i], buf + o2, 8);
        memcpy(&lp[i], buf + o2 + 8, 8);
        o2 += 16;
      }
      src.line_keV = lk;
      src.line_prob = lp;
    }
    /* geometry queries */
    for (int i = 0; i < 200; ++i) {
      const double p[3] = {-40.0 + 0.4 * i, 7.0 - 0.05 * i, -50.0 + 0.6 * i};
      const double d[3] = {0.48, 0.37, 0.7929};
      double t;
      int64_t f;
      (void)orc_locate(s, p);
      (void)orc_closest_hit(s, p, d, -1, &t, &f);
    }
    double E, pt[3];
    int32_t att;
    for (int64_t h = 0; h < 100; ++h)
      if (orc_emission(s, &src, 17, 0, h, &E, pt, &att)) rc = 8;
    /* transport with spectrum and scores */
    const int32_t nch = 4096;
    uint64_t* spec = (uint64_t*)calloc(nch, 8);
    double scales[ORC_MAX_GROUPS];
    for (int g = 0; g < ORC_MAX_GROUPS; ++g) scales[g] = 1.0 + 0.01 * g;
    orc_tally t;
    if (orc_run(s, &src, E0, atol(argv[3]), 5, 99, 3, scales, ORC_MAX_GROUPS, nch, 0.5, spec, 10000,
                2, &t))
      rc = 9;
    printf("pass %d: histories %llu fep %llu lost %llu balance %llu\n", pass,
           (unsigned long long)t.n_histories, (unsigned long long)t.n_fep,
           (unsigned long long)t.n_lost, (unsigned long long)t.n_balance_fail);
    double* in = (double*)calloc(nch, 8);
    double* out = (double*)calloc(nch, 8);
    for (int32_t c = 0; c < nch; ++c) in[c] = (double)spec[c];
    orc_broaden(in, nch, 0.5, 0.64, 0.0018, out);
    free(in);
    free(out);
    free(spec);
    free(lk);
    free(lp);
    orc_scene_destroy(s);
  }
  free(buf);
  free(xyz);
  free(tri);
  free(reg);
  return rc;
}
