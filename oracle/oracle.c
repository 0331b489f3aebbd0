/*
 * oracle.c -- plain FP64 CPU reference for analog photon transport through a
 * closed, region-tagged triangle mesh.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for clarity, not speed:
 * every history re-derives its region from scratch with the ray-parity rule
 * (paper Sec. 2.4.2) after each boundary crossing, so the per-facet
 * inside/outside bookkeeping of a fast path is never trusted here.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846
#define MEC2 510.99895           /* electron rest energy [keV] */
#define R_E 2.8179403262e-13     /* classical electron radius [cm] */
#define MAX_MATERIALS 64
#define LEAF_MAX 4
#define STEP_PAST 1.0e-6         /* mm along the flight, past a crossed facet */
#define STEP_NORMAL 1.0e-7       /* mm along the facet normal: keeps grazing crossings
                                    clear of the facet's degenerate band */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: a 4x32-bit counter is enciphered with a 2x32-bit key by ten
 * rounds; each round multiplies words 0 and 2 by fixed odd constants, swaps
 * and xors the high halves with the other words and the round key, and the
 * key is advanced by the Weyl increments between rounds. */

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  memcpy(out, c, sizeof c);
}

/* Stream of doubles in (0,1) for one history: counter = (draw, h_lo, h_hi, unit). */
typedef struct {
  uint32_t key[2];
  uint32_t ctr[4];
  double buf[2];
  int left;
} orc_rng;

static void rng_init(orc_rng* g, uint64_t seed, uint64_t history, uint32_t unit) {
  g->key[0] = (uint32_t)seed;
  g->key[1] = (uint32_t)(seed >> 32);
  g->ctr[0] = 0;
  g->ctr[1] = (uint32_t)history;
  g->ctr[2] = (uint32_t)(history >> 32);
  g->ctr[3] = unit;
  g->left = 0;
}

static double rng_uniform(orc_rng* g) {
  if (g->left == 0) {
    uint32_t x[4];
    orc_philox4x32_10(g->ctr, g->key, x);
    g->ctr[0] += 1;
    /* 53 random bits per double, offset by half an ulp so 0 and 1 never occur */
    g->buf[0] = ((double)(x[0] >> 5) * 67108864.0 + (double)(x[1] >> 6) + 0.5) / 9007199254740992.0;
    g->buf[1] = ((double)(x[2] >> 5) * 67108864.0 + (double)(x[3] >> 6) + 0.5) / 9007199254740992.0;
    g->left = 2;
  }
  g->left -= 1;
  return g->buf[1 - g->left];
}

/* ------------------------------------------------------------------------ */
/* scene */

typedef struct {
  double lo[3], hi[3];
  int64_t left, right; /* children, or -1 for a leaf */
  int64_t first, count;
} onode;

typedef struct {
  int present[4];
  double* lnval[4]; /* ln(mu/rho) per grid point, per partial (photo, Compton,
                       coherent, pair production) */
} omat;

struct orc_scene {
  int64_t nt;
  int32_t nreg;
  double* v;       /* [nt][9] vertices */
  int32_t* reg;    /* [nt] region enclosed by the facet's shell */
  int use_bvh;
  onode* nodes;
  int64_t nnodes;
  int64_t* order;  /* facet order of the BVH leaves */
  double ext;      /* bounding-box diagonal: scale for tolerances */
  int32_t mat[ORC_MAX_REGIONS];
  double rho[ORC_MAX_REGIONS];
  int32_t grp[ORC_MAX_REGIONS];
  int32_t act[ORC_MAX_REGIONS];
  omat mats[MAX_MATERIALS];
  int grid_set;
  double lnE0, dlnE;
  int32_t nE;
  int electrons; /* 1: secondary electrons run straight CSDA tracks (see electron_track) */
};

static const double* V(const orc_scene* s, int64_t t) { return s->v + 9 * t; }

static double centroid(const orc_scene* s, int64_t t, int a) {
  const double* w = V(s, t);
  return (w[a] + w[3 + a] + w[6 + a]) / 3.0;
}

static int g_sort_axis;
static const orc_scene* g_sort_scene;
static int cmp_centroid(const void* A, const void* B) {
  double a = centroid(g_sort_scene, *(const int64_t*)A, g_sort_axis);
  double b = centroid(g_sort_scene, *(const int64_t*)B, g_sort_axis);
  return (a > b) - (a < b);
}

/* Median-split hierarchy: sort by centroid along the widest axis, halve. */
static int64_t build_node(orc_scene* s, int64_t first, int64_t count) {
  int64_t id = s->nnodes++;
  onode* nd = &s->nodes[id];
  for (int a = 0; a < 3; ++a) {
    nd->lo[a] = INFINITY;
    nd->hi[a] = -INFINITY;
  }
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = first; i < first + count; ++i) {
    const double* w = V(s, s->order[i]);
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 3; ++a) {
        if (w[3 * k + a] < nd->lo[a]) nd->lo[a] = w[3 * k + a];
        if (w[3 * k + a] > nd->hi[a]) nd->hi[a] = w[3 * k + a];
      }
    for (int a = 0; a < 3; ++a) {
      double c = centroid(s, s->order[i], a);
      if (c < clo[a]) clo[a] = c;
      if (c > chi[a]) chi[a] = c;
    }
  }
  nd->first = first;
  nd->count = count;
  nd->left = nd->right = -1;
  if (count <= LEAF_MAX) return id;
  int axis = 0;
  for (int a = 1; a < 3; ++a)
    if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
  g_sort_axis = axis;
  g_sort_scene = s;
  qsort(s->order + first, (size_t)count, sizeof(int64_t), cmp_centroid);
  int64_t half = count / 2;
  int64_t l = build_node(s, first, half);
  int64_t r = build_node(s, first + half, count - half);
  s->nodes[id].left = l;
  s->nodes[id].right = r;
  return id;
}

orc_scene* orc_scene_create(const float* xyz, int64_t nv, const int32_t* tri,
                            const int32_t* tri_region, int64_t nt, int32_t n_regions,
                            int32_t use_bvh) {
  if (nt <= 0 || n_regions < 1 || n_regions > ORC_MAX_REGIONS) return NULL;
  orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
  s->nt = nt;
  s->nreg = n_regions;
  s->v = (double*)malloc(sizeof(double) * 9 * (size_t)nt);
  s->reg = (int32_t*)malloc(sizeof(int32_t) * (size_t)nt);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t t = 0; t < nt; ++t) {
    for (int k = 0; k < 3; ++k) {
      int64_t vi = tri[3 * t + k];
      if (vi < 0 || vi >= nv) {
        orc_scene_destroy(s);
        return NULL;
      }
      for (int a = 0; a < 3; ++a) {
        double x = (double)xyz[3 * vi + a];
        s->v[9 * t + 3 * k + a] = x;
        if (x < lo[a]) lo[a] = x;
        if (x > hi[a]) hi[a] = x;
      }
    }
    s->reg[t] = tri_region[t];
  }
  s->ext = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                (hi[2] - lo[2]) * (hi[2] - lo[2]));
  for (int r = 0; r < ORC_MAX_REGIONS; ++r) s->grp[r] = -1;
  s->use_bvh = use_bvh;
  s->order = (int64_t*)malloc(sizeof(int64_t) * (size_t)nt);
  for (int64_t t = 0; t < nt; ++t) s->order[t] = t;
  if (use_bvh) {
    s->nodes = (onode*)malloc(sizeof(onode) * (size_t)(2 * nt + 1));
    s->nnodes = 0;
    build_node(s, 0, nt);
  }
  return s;
}

void orc_scene_destroy(orc_scene* s) {
  if (!s) return;
  free(s->v);
  free(s->reg);
  free(s->nodes);
  free(s->order);
  for (int m = 0; m < MAX_MATERIALS; ++m)
    for (int i = 0; i < 4; ++i) free(s->mats[m].lnval[i]);
  free(s);
}

int32_t orc_set_region(orc_scene* s, int32_t r, int32_t material, double density, int32_t group,
                       int32_t active) {
  if (r < 0 || r >= s->nreg || material < 0 || material >= MAX_MATERIALS) return -1;
  if (group >= ORC_MAX_GROUPS || density < 0) return -1;
  s->mat[r] = material;
  s->rho[r] = density;
  s->grp[r] = group;
  s->act[r] = active;
  return 0;
}

int32_t orc_set_xs(orc_scene* s, int32_t m, double lnE0, double dlnE, int32_t n,
                   const double* photo, const double* compton, const double* coherent,
                   const double* pair) {
  if (m < 0 || m >= MAX_MATERIALS || n < 2 || !(dlnE > 0)) return -1;
  if (s->grid_set && (lnE0 != s->lnE0 || dlnE != s->dlnE || n != s->nE)) return -2;
  s->grid_set = 1;
  s->lnE0 = lnE0;
  s->dlnE = dlnE;
  s->nE = n;
  const double* src[4] = {photo, compton, coherent, pair};
  for (int i = 0; i < 4; ++i) {
    free(s->mats[m].lnval[i]);
    s->mats[m].lnval[i] = NULL;
    s->mats[m].present[i] = 0;
    if (!src[i]) continue;
    int npos = 0;
    for (int k = 0; k < n; ++k) {
      if (!(src[i][k] >= 0) || isinf(src[i][k])) return -3;
      npos += src[i][k] > 0;
    }
    if (npos == 0) continue;
    if (npos != n) return -3;
    s->mats[m].lnval[i] = (double*)malloc(sizeof(double) * (size_t)n);
    for (int k = 0; k < n; ++k) s->mats[m].lnval[i][k] = log(src[i][k]);
    s->mats[m].present[i] = 1;
  }
  return 0;
}

/* mu/rho interpolated linearly in ln E on ln(mu/rho), per partial; pair
 * production exists only above 2 m_e c^2 (Sec. 2.4.1 lists it among the
 * photon interactions). */
static void mass_atten(const orc_scene* s, int32_t m, double E, double out[4]) {
  double x = (log(E) - s->lnE0) / s->dlnE;
  int64_t k = (int64_t)floor(x);
  if (k < 0) k = 0;
  if (k > s->nE - 2) k = s->nE - 2;
  double w = x - (double)k;
  if (w < 0) w = 0;
  if (w > 1) w = 1;
  for (int i = 0; i < 4; ++i) {
    if (!s->mats[m].present[i] || (i == 3 && E <= 2.0 * MEC2)) {
      out[i] = 0.0;
      continue;
    }
    const double* L = s->mats[m].lnval[i];
    out[i] = exp(L[k] + w * (L[k + 1] - L[k]));
  }
}

void orc_mu(const orc_scene* s, int32_t r, double E, const double* scales, int32_t n_scales,
            double out[4]) {
  double mr[4];
  mass_atten(s, s->mat[r], E, mr);
  double f = 0.1 * s->rho[r];
  if (scales && s->grp[r] >= 0 && s->grp[r] < n_scales) f *= scales[s->grp[r]];
  for (int i = 0; i < 4; ++i) out[i] = f * mr[i];
}

/* ------------------------------------------------------------------------ */
/* ray-facet intersection, Moller-Trumbore in FP64 */

enum { MISS = 0, HIT = 1, DEGENERATE = 2 };

static void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

/* Classifies the crossing of the line o + t d (t > 0) with facet f.  A crossing
 * within 1e-12 (relative) of an edge or vertex, a ray lying in the facet plane
 * or a hit at t ~ 0 is DEGENERATE: its parity contribution is ambiguous. */
static int ray_facet(const orc_scene* s, int64_t f, const double* o, const double* d, double* t_out,
                     double* d_dot_n) {
  const double* w = V(s, f);
  double e1[3], e2[3], p[3], q[3], so[3];
  sub3(w + 3, w, e1);
  sub3(w + 6, w, e2);
  cross3(d, e2, p);
  double det = dot3(e1, p);
  double n[3];
  cross3(e1, e2, n);
  double nn = norm3(n);
  if (fabs(det) <= 1e-14 * norm3(e1) * norm3(e2)) {
    sub3(o, w, so);
    if (fabs(dot3(so, n)) <= 1e-12 * nn * s->ext) return DEGENERATE; /* in-plane ray */
    return MISS;
  }
  double inv = 1.0 / det;
  sub3(o, w, so);
  double u = dot3(so, p) * inv;
  cross3(so, e1, q);
  double v = dot3(d, q) * inv;
  double bw = 1.0 - u - v;
  const double tol = 1e-12;
  if (u < -tol || v < -tol || bw < -tol) return MISS;
  double t = dot3(e2, q) * inv;
  if (t < -1e-12 * s->ext) return MISS;
  *t_out = t;
  *d_dot_n = dot3(d, n);
  if (u < tol || v < tol || bw < tol || t <= 1e-12 * s->ext) return DEGENERATE;
  return HIT;
}

/* slab test against an axis-aligned box widened by a small margin */
static int ray_box(const onode* nd, const double* o, const double* d, double tmax, double* tenter) {
  double t0 = 0.0, t1 = tmax;
  for (int a = 0; a < 3; ++a) {
    double lo = nd->lo[a] - 1e-9, hi = nd->hi[a] + 1e-9;
    if (d[a] == 0.0) {
      if (o[a] < lo || o[a] > hi) return 0;
      continue;
    }
    double ta = (lo - o[a]) / d[a], tb = (hi - o[a]) / d[a];
    if (ta > tb) {
      double x = ta;
      ta = tb;
      tb = x;
    }
    if (ta > t0) t0 = ta;
    if (tb < t1) t1 = tb;
    if (t0 > t1) return 0;
  }
  *tenter = t0;
  return 1;
}

/* Visits the facets of every leaf whose box the ray touches within [0, *tmax];
 * visit() returns a new tmax (closest-hit shrinks it; all-hits keeps it). */
typedef double (*visit_fn)(const orc_scene*, int64_t facet, void* ctx, double tmax);

static void for_candidates(const orc_scene* s, const double* o, const double* d, double tmax,
                           visit_fn visit, void* ctx) {
  if (!s->use_bvh) {
    for (int64_t f = 0; f < s->nt; ++f) tmax = visit(s, f, ctx, tmax);
    return;
  }
  int64_t stack[256];
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const onode* nd = &s->nodes[stack[--sp]];
    double te;
    if (!ray_box(nd, o, d, tmax, &te)) continue;
    if (nd->left < 0) {
      for (int64_t i = nd->first; i < nd->first + nd->count; ++i) tmax = visit(s, s->order[i], ctx, tmax);
    } else {
      stack[sp++] = nd->right;
      stack[sp++] = nd->left;
    }
  }
}

typedef struct {
  const double *o, *d;
  int64_t exclude, best;
  double tbest;
} closest_ctx;

static double visit_closest(const orc_scene* s, int64_t f, void* vc, double tmax) {
  closest_ctx* c = (closest_ctx*)vc;
  if (f == c->exclude) return tmax;
  double t, dn;
  int r = ray_facet(s, f, c->o, c->d, &t, &dn);
  if (r == MISS || !(t > 0.0)) return tmax;
  if (t < c->tbest || (t == c->tbest && f < c->best)) {
    c->tbest = t;
    c->best = f;
  }
  return c->tbest < tmax ? c->tbest : tmax;
}

int32_t orc_closest_hit(const orc_scene* s, const double o[3], const double d[3], int64_t exclude,
                        double* t, int64_t* tri) {
  closest_ctx c = {o, d, exclude, -1, INFINITY};
  for_candidates(s, o, d, INFINITY, visit_closest, &c);
  if (c.best < 0) return 0;
  *t = c.tbest;
  *tri = c.best;
  return 1;
}

typedef struct {
  const double *o, *d;
  int degenerate;
  unsigned char parity[ORC_MAX_REGIONS];
  double first[ORC_MAX_REGIONS];
} parity_ctx;

static double visit_parity(const orc_scene* s, int64_t f, void* vc, double tmax) {
  parity_ctx* c = (parity_ctx*)vc;
  if (c->degenerate) return tmax;
  double t, dn;
  int r = ray_facet(s, f, c->o, c->d, &t, &dn);
  if (r == MISS) return tmax;
  if (r == DEGENERATE) {
    c->degenerate = 1;
    return tmax;
  }
  int32_t g = s->reg[f];
  c->parity[g] ^= 1;
  if (t < c->first[g]) c->first[g] = t;
  return tmax;
}

/* fixed, irrational-looking probe directions (normalised at use) */
static const double PROBE[8][3] = {
    {0.5773502691896257, 0.3826834323650898, 0.7213475204444817},
    {-0.4472135954999579, 0.8164965809277260, 0.3651483716701107},
    {0.2672612419124244, -0.5345224838248488, -0.8017837257372732},
    {-0.7071067811865476, -0.4082482904638631, 0.5773502691896258},
    {0.1301889109703266, 0.9176629354822471, -0.3754345426502468},
    {0.8660254037844386, -0.2886751345948129, 0.4082482904638630},
    {-0.2357022603955158, -0.9428090415820634, -0.2357022603955158},
    {0.6324555320336759, 0.3162277660168379, -0.7071067811865476},
};

int32_t orc_locate(const orc_scene* s, const double p[3]) {
  for (int k = 0; k < 8; ++k) {
    double d[3] = {PROBE[k][0], PROBE[k][1], PROBE[k][2]};
    double nd = norm3(d);
    d[0] /= nd;
    d[1] /= nd;
    d[2] /= nd;
    parity_ctx c;
    c.o = p;
    c.d = d;
    c.degenerate = 0;
    memset(c.parity, 0, sizeof c.parity);
    for (int r = 0; r < ORC_MAX_REGIONS; ++r) c.first[r] = INFINITY;
    for_candidates(s, p, d, INFINITY, visit_parity, &c);
    if (c.degenerate) continue;
    /* odd count => inside; the odd geometry crossed first contains p;
     * exact ties resolve to the smaller region id */
    int32_t best = 0;
    double tb = INFINITY;
    for (int32_t r = 1; r < s->nreg; ++r)
      if (c.parity[r] && c.first[r] < tb) {
        tb = c.first[r];
        best = r;
      }
    return best;
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Klein-Nishina and Thomson sampling by inverse CDF */

/* With eps = E'/E and t = (1/eps - 1)/k = 1 - cos(theta), the KN density is
 * proportional to f(eps) = 1/eps + eps - 2t + t^2 on [1/(1+2k), 1]; this is
 * its antiderivative. */
double orc_kn_integral(double k, double eps) {
  double le = log(eps);
  return le + 0.5 * eps * eps - (2.0 / k) * (le - eps) + (1.0 / (k * k)) * (-1.0 / eps - 2.0 * le + eps);
}

/* d sigma / d eps = (pi r_e^2 / k) f(eps) */
double orc_kn_sigma(double k) {
  double e0 = 1.0 / (1.0 + 2.0 * k);
  return PI * R_E * R_E / k * (orc_kn_integral(k, 1.0) - orc_kn_integral(k, e0));
}

double orc_kn_sample(double k, double u) {
  double e0 = 1.0 / (1.0 + 2.0 * k);
  double F0 = orc_kn_integral(k, e0);
  double target = F0 + u * (orc_kn_integral(k, 1.0) - F0);
  double lo = e0, hi = 1.0;
  for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
    double mid = 0.5 * (lo + hi);
    if (orc_kn_integral(k, mid) < target)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* cos(theta) with density 3/8 (1 + mu^2): CDF (mu^3 + 3 mu + 4) / 8 */
double orc_thomson_sample(double u) {
  double lo = -1.0, hi = 1.0;
  for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
    double mid = 0.5 * (lo + hi);
    if ((mid * mid * mid + 3.0 * mid + 4.0) / 8.0 < u)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* New direction at polar angle theta (cos ct) and azimuth phi about the
 * unit direction d, by the classic direction-cosine formula
 *   d' = d ct + st (cos phi (w d - z) + sin phi (z x d)) / sqrt(1 - w^2)
 * about the coordinate axis z; the frame is relabelled so that this axis
 * is the one d is least aligned with (|w| <= 1/sqrt 3), where the formula is
 * well conditioned, so no direction is ever treated as lying on an axis. */
static void rotate(double* d, double ct, double phi) {
  double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  double cp = cos(phi), sp = sin(phi);
  /* axis of the formula: the smallest component of d; (a, b, c) is a cyclic
   * relabelling of (x, y, z) that puts it last */
  int c = 2;
  if (fabs(d[0]) <= fabs(d[1]) && fabs(d[0]) <= fabs(d[2]))
    c = 0;
  else if (fabs(d[1]) <= fabs(d[2]))
    c = 1;
  int a = (c + 1) % 3, b = (c + 2) % 3;
  double u = d[a], v = d[b], w = d[c];
  double q = sqrt(1.0 - w * w);
  double nu = u * ct + st * (u * w * cp - v * sp) / q;
  double nv = v * ct + st * (v * w * cp + u * sp) / q;
  double nw = w * ct - st * cp * q;
  double nn = sqrt(nu * nu + nv * nv + nw * nw);
  d[a] = nu / nn;
  d[b] = nv / nn;
  d[c] = nw / nn;
}

void orc_rotate(const double d[3], double ct, double phi, double out[3]) {
  double v[3] = {d[0], d[1], d[2]};
  rotate(v, ct, phi);
  memcpy(out, v, sizeof v);
}

/* ------------------------------------------------------------------------ */
/* secondary electrons (a synthetic reading of the electron transport the
 * paper couples to its photons, Sec. 2.4.1): each electron set in motion by
 * a photoelectric absorption, a Compton scattering or a pair production runs
 * a straight track in the continuous-slowing-down approximation, with the
 * mass range of Katz and Penfold (1952), and leaves in every region it
 * crosses the energy it loses there.  Electrons below ELEC_TMIN deposit at
 * once.  Ranges use the regions' nominal densities (not the density scales),
 * so the score-function derivative keeps its form. */

#define ELEC_TMIN 10.0 /* keV: the lower end of the range relation's validity */

/* Katz-Penfold mass range [g/cm^2] of an electron of kinetic energy T [keV] */
static double csda_range(double T) {
  const double t = T * 1e-3;
  if (t > 2.5) return 0.530 * t - 0.106;
  if (!(t > 0.0)) return 0.0;
  return 0.412 * pow(t, 1.265 - 0.0954 * log(t));
}

double orc_csda_range(double T_keV) { return csda_range(T_keV); }

/* kinetic energy [keV] whose range is R [g/cm^2]: bisection (the range grows
 * monotonically with the energy) */
static double csda_energy(double R) {
  if (!(R > 0.0)) return 0.0;
  double lo = 0.0, hi = 4000.0;
  for (int i = 0; i < 100; ++i) {
    const double m = 0.5 * (lo + hi);
    if (csda_range(m) < R)
      lo = m;
    else
      hi = m;
  }
  return 0.5 * (lo + hi);
}

double orc_csda_energy(double R) { return csda_energy(R); }

typedef struct {
  double act, tot, esc; /* energy left in ACTIVE regions, in all regions, carried out */
  int lost;
} etrack;

/* An electron of kinetic energy T from p along the unit direction e, in
 * `region`: straight, region by region (the region past each crossing by the
 * parity rule, as for photons); in a region of density rho it can run
 * 10 R / rho mm on its remaining range R; it stops where that range is spent,
 * or leaves the world through void. */
static etrack electron_track(const orc_scene* s, const double* p0, const double* e, double T,
                             int32_t region) {
  etrack out = {0.0, 0.0, 0.0, 0};
  double p[3] = {p0[0], p0[1], p0[2]};
  double R = csda_range(T), Tcur = T;
  int64_t last = -1;
  for (int steps = 0; steps < 100000; ++steps) {
    const double rho = s->rho[region];
    const double smax = rho > 0.0 ? 10.0 * R / rho : INFINITY;
    double th;
    int64_t tri;
    const int hit = orc_closest_hit(s, p, e, last, &th, &tri);
    if (hit && th < smax) {
      const double Rn = fmax(0.0, R - rho * th / 10.0);
      const double Tn = csda_energy(Rn);
      const double dep = Tcur - Tn;
      out.tot += dep;
      if (s->act[region]) out.act += dep;
      Tcur = Tn;
      R = Rn;
      for (int a = 0; a < 3; ++a) p[a] += th * e[a];
      const double* fv = V(s, tri);
      double e1[3], e2[3], fn[3];
      sub3(fv + 3, fv, e1);
      sub3(fv + 6, fv, e2);
      cross3(e1, e2, fn);
      const double fl = norm3(fn);
      const double side = dot3(e, fn) >= 0.0 ? STEP_NORMAL / fl : -STEP_NORMAL / fl;
      double q[3];
      for (int a = 0; a < 3; ++a) q[a] = p[a] + STEP_PAST * e[a] + side * fn[a];
      region = orc_locate(s, q);
      last = tri;
      if (region < 0) {
        out.lost = 1;
        return out;
      }
      continue;
    }
    if (rho > 0.0) { /* the range ends inside this region */
      out.tot += Tcur;
      if (s->act[region]) out.act += Tcur;
      return out;
    }
    /* void and no facet ahead: out of the world (or lost inside a void shell) */
    out.esc = Tcur;
    out.lost = region != 0;
    return out;
  }
  out.lost = 1;
  return out;
}

int32_t orc_set_electrons(orc_scene* s, int32_t on) {
  if (!s) return -1;
  s->electrons = on ? 1 : 0;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* transport */

typedef struct {
  const orc_scene* s;
  const orc_source* src;
  double E0;
  int64_t first, n;
  uint64_t seed;
  uint32_t unit;
  const double* scales;
  int32_t ngroups;
  int32_t nch;
  double chw;
  uint64_t* spectrum; /* this worker's private copy */
  int32_t max_steps;
  int32_t src_region;
  orc_tally tally;
} worker;

/* Energy of a line source: line i with probability line_prob[i] / sum. */
static double draw_line(const orc_source* src, orc_rng* g) {
  double tot = 0;
  for (int i = 0; i < src->n_lines; ++i) tot += src->line_prob[i];
  double x = rng_uniform(g) * tot, c = 0;
  int pick = src->n_lines - 1;
  for (int i = 0; i < src->n_lines; ++i) {
    c += src->line_prob[i];
    if (x < c) {
      pick = i;
      break;
    }
  }
  return src->line_keV[pick];
}

/* A point uniform in the source's cylindrical annulus r_in <= r <= r_out,
 * 0 <= z <= h (the area element r dr makes r^2 uniform), kept only when the
 * parity rule puts it in the source region: the accepted points are uniform
 * in the faceted region.  Returns the number of tries used, 0 when all 1000
 * failed. */
static int volume_point(const orc_scene* s, const orc_source* src, orc_rng* g, double p[3]) {
  for (int attempt = 1; attempt <= 1000; ++attempt) {
    double r2lo = src->r_in * src->r_in, r2hi = src->r_out * src->r_out;
    double r = sqrt(r2lo + rng_uniform(g) * (r2hi - r2lo));
    double ph = 2.0 * PI * rng_uniform(g);
    p[0] = src->pos[0] + r * cos(ph);
    p[1] = src->pos[1] + r * sin(ph);
    p[2] = src->pos[2] + rng_uniform(g) * src->h;
    if (orc_locate(s, p) == src->region) return attempt;
  }
  return 0;
}

static void isotropic(orc_rng* g, double* d) {
  double ct = 2.0 * rng_uniform(g) - 1.0;
  double ph = 2.0 * PI * rng_uniform(g);
  double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  d[0] = st * cos(ph);
  d[1] = st * sin(ph);
  d[2] = ct;
}

static void one_history(worker* w, int64_t h) {
  const orc_scene* s = w->s;
  const orc_source* src = w->src;
  orc_tally* T = &w->tally;
  orc_rng g;
  rng_init(&g, w->seed, (uint64_t)h, w->unit);
  T->n_histories++;

  double p[3], d[3], E;
  int32_t region;
  /* energy */
  E = src->n_lines > 0 ? draw_line(src, &g) : w->E0;
  const double E0 = E;
  /* position, direction, region */
  if (src->kind == ORC_CYL) {
    if (volume_point(s, src, &g, p) == 0) {
      T->n_source_fail++;
      return;
    }
    region = src->region;
    isotropic(&g, d);
  } else {
    memcpy(p, src->pos, sizeof p);
    region = w->src_region;
    if (src->kind == ORC_BEAM)
      memcpy(d, src->dir, sizeof d);
    else
      isotropic(&g, d);
  }

  double tau = -log(rng_uniform(&g));
  double edep_act = 0.0, edep_tot = 0.0;
  int clean = 1, interacted = 0, absorbed = 0, escaped = 0;
  double e_esc = 0.0; /* energy carried out of the world by this history's photons */
  /* the second annihilation photon of a pair event waits here until the first
   * one is done (a 511 keV photon cannot make a pair, so one slot is enough) */
  int pending = 0, broken = 0; /* broken: lost or killed */
  double p2[3], d2[3];
  int32_t region2 = 0;
  double tau0[ORC_MAX_GROUPS] = {0};
  int nint[ORC_MAX_GROUPS] = {0};
  int64_t last = -1;
  const double Ecut = exp(s->lnE0);

#define DEPOSIT(x, reg)          \
  do {                           \
    edep_tot += (x);             \
    if (s->act[(reg)])           \
      edep_act += (x);           \
    else                         \
      clean = 0;                 \
  } while (0)

/* kinetic energy x given to an electron at p along direction ed in region
 * reg: a CSDA track, or a local deposit below ELEC_TMIN or without electrons */
#define ELECTRON(x, ed, reg)                                             \
  do {                                                                   \
    if (s->electrons && (x) >= ELEC_TMIN) {                              \
      const etrack et = electron_track(s, p, (ed), (x), (reg));          \
      edep_tot += et.tot;                                                \
      edep_act += et.act;                                                \
      if (et.tot > et.act || et.esc > 0.0) clean = 0;                    \
      if (et.esc > 0.0) {                                                \
        e_esc += et.esc;                                                 \
        T->e_escape += et.esc;                                           \
      }                                                                  \
      if (et.lost) {                                                     \
        T->n_lost++;                                                     \
        broken = 1;                                                      \
      }                                                                  \
      T->n_electrons++;                                                  \
    } else {                                                             \
      DEPOSIT((x), (reg));                                               \
    }                                                                    \
  } while (0)

/* the current photon is done (absorbed or escaped): go on with the waiting
 * annihilation photon, if there is one */
#define NEXT_PHOTON()                    \
  if (pending) {                         \
    memcpy(p, p2, sizeof p);             \
    memcpy(d, d2, sizeof d);             \
    region = region2;                    \
    E = MEC2;                            \
    last = -1;                           \
    pending = 0;                         \
    tau = -log(rng_uniform(&g));         \
    continue;                            \
  }

  int steps = 0;
  for (;;) {
    if (++steps > w->max_steps) {
      T->n_killed++;
      clean = 0;
      broken = 1;
      break;
    }
    T->n_segments++;
    double mu4[4];
    orc_mu(s, region, E, w->scales, w->ngroups, mu4);
    double mu = mu4[0] + mu4[1] + mu4[2] + mu4[3];
    int32_t gidx = s->grp[region];
    double mu0 = 0.0; /* unscaled total attenuation of the region */
    if (gidx >= 0 && gidx < w->ngroups) {
      double m0[4];
      orc_mu(s, region, E, NULL, 0, m0);
      mu0 = m0[0] + m0[1] + m0[2] + m0[3];
    }
    double th;
    int64_t tri;
    int hit = orc_closest_hit(s, p, d, last, &th, &tri);
    if (hit && (mu == 0.0 || mu * th < tau)) {
      /* boundary crossing: move, spend optical depth, re-locate */
      tau -= mu * th;
      if (gidx >= 0 && gidx < w->ngroups) tau0[gidx] += mu0 * th;
      for (int a = 0; a < 3; ++a) p[a] += th * d[a];
      /* probe point just past the crossed facet, on the side the flight goes to */
      const double* fv = V(s, tri);
      double e1[3], e2[3], fn[3];
      sub3(fv + 3, fv, e1);
      sub3(fv + 6, fv, e2);
      cross3(e1, e2, fn);
      const double fl = norm3(fn);
      const double side = dot3(d, fn) >= 0.0 ? STEP_NORMAL / fl : -STEP_NORMAL / fl;
      double q[3];
      for (int a = 0; a < 3; ++a) q[a] = p[a] + STEP_PAST * d[a] + side * fn[a];
      region = orc_locate(s, q);
      last = tri;
      T->n_crossings++;
      if (region < 0) {
        T->n_lost++;
        clean = 0;
        broken = 1;
        break;
      }
      continue;
    }
    if (mu > 0.0) {
      double sflight = tau / mu;
      if (gidx >= 0 && gidx < w->ngroups) tau0[gidx] += mu0 * sflight;
      for (int a = 0; a < 3; ++a) p[a] += sflight * d[a];
      last = -1;
      interacted = 1;
      if (gidx >= 0 && gidx < w->ngroups) nint[gidx]++;
      double x = rng_uniform(&g) * mu;
      if (x < mu4[0]) {
        T->n_photo++;
        if (s->electrons && E >= ELEC_TMIN) {
          /* the photoelectron leaves isotropically (synthetic reading) */
          double ed[3];
          isotropic(&g, ed);
          ELECTRON(E, ed, region);
        } else {
          DEPOSIT(E, region);
        }
        if (broken) break;
        NEXT_PHOTON();
        absorbed = !escaped;
        break;
      } else if (x < mu4[0] + mu4[1]) {
        T->n_compton++;
        double k = E / MEC2;
        double eps = orc_kn_sample(k, rng_uniform(&g));
        double ct = 1.0 - (1.0 / eps - 1.0) / k;
        double ph = 2.0 * PI * rng_uniform(&g);
        double Ep = eps * E;
        if (s->electrons && E - Ep >= ELEC_TMIN) {
          /* the recoil electron: in the scattering plane, on the other side,
           * at cot(theta_e) = (1 + k) tan(theta / 2) from the incoming photon */
          const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
          const double a = (1.0 + k) * st, b = 1.0 + ct;
          const double cte = a / sqrt(a * a + b * b);
          double ed[3] = {d[0], d[1], d[2]};
          rotate(ed, cte, ph + PI);
          ELECTRON(E - Ep, ed, region);
          if (broken) break;
        } else {
          DEPOSIT(E - Ep, region);
        }
        rotate(d, ct, ph);
        E = Ep;
        if (E < Ecut) {
          DEPOSIT(E, region);
          NEXT_PHOTON();
          absorbed = !escaped;
          break;
        }
      } else if (x < mu4[0] + mu4[1] + mu4[2]) {
        T->n_coherent++;
        double ct = orc_thomson_sample(rng_uniform(&g));
        double ph = 2.0 * PI * rng_uniform(&g);
        rotate(d, ct, ph);
      } else {
        /* pair production: the photon is gone; the pair's kinetic energy
         * E - 2 m_e c^2 is deposited here and the positron annihilates at
         * rest into two 511 keV photons flying apart along a random axis */
        T->n_pair++;
        /* the pair's kinetic energy as one track along the photon (reading) */
        ELECTRON(E - 2.0 * MEC2, d, region);
        if (broken) break;
        double a[3];
        isotropic(&g, a);
        memcpy(p2, p, sizeof p2);
        for (int k = 0; k < 3; ++k) {
          d[k] = a[k];
          d2[k] = -a[k];
        }
        region2 = region;
        pending = 1;
        E = MEC2;
      }
      tau = -log(rng_uniform(&g));
      continue;
    }
    /* vacuum and no facet ahead */
    if (region == 0) {
      escaped = 1;
      clean = 0;
      e_esc += E;
      T->e_escape += E;
      if (!interacted) T->n_uncollided++;
      NEXT_PHOTON();
    } else {
      T->n_lost++;
      clean = 0;
      broken = 1;
    }
    break;
  }
#undef DEPOSIT
#undef ELECTRON
#undef NEXT_PHOTON

  if (escaped && !broken) T->n_escape++;
  if (absorbed) T->n_absorbed++;
  int fep = absorbed && clean;
  if (fep) T->n_fep++;
  T->edep_active += edep_act;
  T->edep_total += edep_tot;
  double bal = edep_tot + e_esc;
  if (!broken && fabs(bal - E0) > 1e-9 * E0) T->n_balance_fail++;
  if (edep_act > 0.0 && w->spectrum) {
    double c = floor(edep_act / w->chw);
    if (c < (double)w->nch)
      w->spectrum[(int64_t)c]++;
    else
      T->spectrum_overflow++;
  }
  for (int gi = 0; gi < w->ngroups; ++gi) {
    double sc = (double)nint[gi] / w->scales[gi] - tau0[gi];
    T->sum_score[gi] += sc;
    if (fep) {
      T->sum_fep_score[gi] += sc;
      T->sum_fep_score2[gi] += sc * sc;
    }
  }
}

int32_t orc_emission(const orc_scene* s, const orc_source* src, uint64_t seed, uint32_t unit,
                     int64_t history, double* E, double p[3], int32_t* attempts) {
  if (!s || !src || !E || !p || !attempts || history < 0) return -1;
  orc_rng g;
  rng_init(&g, seed, (uint64_t)history, unit);
  *E = src->n_lines > 0 ? draw_line(src, &g) : 0.0;
  if (src->kind == ORC_CYL) {
    *attempts = volume_point(s, src, &g, p);
  } else {
    memcpy(p, src->pos, 3 * sizeof(double));
    *attempts = 1;
  }
  return 0;
}

static void* worker_main(void* arg) {
  worker* w = (worker*)arg;
  for (int64_t i = 0; i < w->n; ++i) one_history(w, w->first + i);
  return NULL;
}

int32_t orc_run(const orc_scene* s, const orc_source* src, double E0, int64_t n, int64_t first,
                uint64_t seed, uint32_t unit, const double* scales, int32_t n_groups,
                int32_t n_channels, double channel_keV, uint64_t* spectrum, int32_t max_steps,
                int32_t n_threads, orc_tally* out) {
  if (!s || !src || !out || n < 0 || n_groups < 0 || n_groups > ORC_MAX_GROUPS) return -1;
  if (!s->grid_set) return -2;
  if (n_groups > 0 && !scales) return -1;
  for (int g = 0; g < n_groups; ++g)
    if (!(scales[g] > 0)) return -1;
  double emax = exp(s->lnE0 + s->dlnE * (s->nE - 1)), emin = exp(s->lnE0);
  if (src->n_lines > 0) {
    for (int i = 0; i < src->n_lines; ++i)
      if (src->line_keV[i] < emin || src->line_keV[i] > emax) return -3;
  } else if (!(E0 >= emin && E0 <= emax)) {
    return -3;
  }
  if (n_threads < 1) n_threads = 1;
  if (max_steps <= 0) max_steps = 10000;
  int32_t src_region = 0;
  if (src->kind != ORC_CYL) {
    src_region = orc_locate(s, src->pos);
    if (src_region < 0) return -4;
  }
  memset(out, 0, sizeof *out);
  if (spectrum) memset(spectrum, 0, sizeof(uint64_t) * (size_t)n_channels);
  worker* ws = (worker*)calloc((size_t)n_threads, sizeof(worker));
  pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
  for (int i = 0; i < n_threads; ++i) {
    worker* w = &ws[i];
    int64_t a = n * i / n_threads, b = n * (i + 1) / n_threads;
    w->s = s;
    w->src = src;
    w->E0 = E0;
    w->first = first + a;
    w->n = b - a;
    w->seed = seed;
    w->unit = unit;
    w->scales = scales;
    w->ngroups = n_groups;
    w->nch = n_channels;
    w->chw = channel_keV;
    w->spectrum = spectrum ? (uint64_t*)calloc((size_t)n_channels, sizeof(uint64_t)) : NULL;
    w->max_steps = max_steps;
    w->src_region = src_region;
    pthread_create(&th[i], NULL, worker_main, w);
  }
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
  for (int i = 0; i < n_threads; ++i) {
    orc_tally* t = &ws[i].tally;
    out->n_histories += t->n_histories;
    out->n_absorbed += t->n_absorbed;
    out->n_fep += t->n_fep;
    out->n_uncollided += t->n_uncollided;
    out->n_escape += t->n_escape;
    out->n_lost += t->n_lost;
    out->n_killed += t->n_killed;
    out->n_source_fail += t->n_source_fail;
    out->n_balance_fail += t->n_balance_fail;
    out->n_segments += t->n_segments;
    out->n_crossings += t->n_crossings;
    out->n_photo += t->n_photo;
    out->n_compton += t->n_compton;
    out->n_coherent += t->n_coherent;
    out->n_pair += t->n_pair;
    out->n_electrons += t->n_electrons;
    out->spectrum_overflow += t->spectrum_overflow;
    out->edep_active += t->edep_active;
    out->edep_total += t->edep_total;
    out->e_escape += t->e_escape;
    for (int g = 0; g < ORC_MAX_GROUPS; ++g) {
      out->sum_score[g] += t->sum_score[g];
      out->sum_fep_score[g] += t->sum_fep_score[g];
      out->sum_fep_score2[g] += t->sum_fep_score2[g];
    }
    if (spectrum) {
      for (int c = 0; c < n_channels; ++c) spectrum[c] += ws[i].spectrum[c];
      free(ws[i].spectrum);
    }
  }
  free(ws);
  free(th);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Gaussian broadening: each channel's count is spread by the normal law of
 * standard deviation FWHM/(2 sqrt(2 ln 2)) centred on the channel centre,
 * integrated over each receiving channel within 5 sigma. */

static double Phi(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

void orc_broaden(const double* in, int32_t n, double w, double a, double b, double* out) {
  for (int c = 0; c < n; ++c) out[c] = 0.0;
  for (int cp = 0; cp < n; ++cp) {
    if (in[cp] == 0.0) continue;
    double Ec = (cp + 0.5) * w;
    double sigma = sqrt(a + b * Ec) / (2.0 * sqrt(2.0 * log(2.0)));
    for (int c = 0; c < n; ++c) {
      double centre = (c + 0.5) * w;
      if (fabs(centre - Ec) > 5.0 * sigma) continue;
      out[c] += in[cp] * (Phi(((c + 1) * w - Ec) / sigma) - Phi((c * w - Ec) / sigma));
    }
  }
}
