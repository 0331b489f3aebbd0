/*
 * oracle.h -- plain, slow, FP64 CPU reference for the photon-transport path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant with the HIP path: both read the same input arrays and nothing
 * else.
 *
 * What it computes (paper Sec. 2.4):
 *   - analog photon histories through a closed, region-tagged triangle
 *     mesh, with the region of a point found by the ray-parity rule of
 *     Sec. 2.4.2 (odd crossing count => inside; among odd geometries the one
 *     with the nearest first crossing contains the point; none odd => world),
 *     applied after EVERY boundary crossing;
 *   - free flights sampled in mean free paths and carried across boundaries
 *     (reading of the "partial cross-section" step sampling, Sec. 2.4.1);
 *   - photoelectric absorption, free-electron Klein-Nishina Compton
 *     scattering (inverse-CDF sampling by bisection of the closed-form
 *     integral) and Thomson-law coherent scattering (bisection of its CDF),
 *     local deposition of electron energy, 1 keV (table minimum) cut-off;
 *   - full-energy-peak (FEP) flag, pulse-height spectrum, and the
 *     score-function estimate of dFEPE/ds_g for per-region density scales.
 *
 * Units: mm, keV, g/cm^3, cm^2/g; mu [1/mm] = 0.1 * rho * s_g * (mu/rho).
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_GROUPS 8
#define ORC_MAX_REGIONS 256

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

typedef struct orc_scene orc_scene;

/* Copies the arrays.  use_bvh = 0: brute force over all facets. */
orc_scene* orc_scene_create(const float* xyz, int64_t n_vertices, const int32_t* tri,
                            const int32_t* tri_region, int64_t n_tri, int32_t n_regions,
                            int32_t use_bvh);
void orc_scene_destroy(orc_scene* s);
int32_t orc_set_region(orc_scene* s, int32_t region, int32_t material, double density,
                       int32_t group, int32_t active);
/* Partial mu/rho [cm^2/g] on the grid ln E_k = lnE0 + k dlnE; any pointer may be
 * NULL (that partial is zero).  A partial must be all-zero or all-positive.  The
 * pair-production partial counts only above its threshold 2 m_e c^2 (zero at and
 * below it, whatever the table holds there). */
int32_t orc_set_xs(orc_scene* s, int32_t material, double lnE0, double dlnE, int32_t n,
                   const double* photo, const double* compton, const double* coherent,
                   const double* pair);

/* Secondary electrons (synthetic reading of Sec. 2.4.1's electron transport):
 * on = 1 makes every electron of at least 10 keV set in motion by a photo-
 * electric absorption (isotropic), a Compton scattering (recoil direction
 * from two-body kinematics) or a pair production (the pair's kinetic energy
 * as one track along the photon) run a straight continuous-slowing-down track
 * with the Katz-Penfold (1952) mass range, leaving in each region the energy
 * it loses there and carrying the rest out of the world through void; 0
 * (default) deposits their energy at the interaction point. */
int32_t orc_set_electrons(orc_scene* s, int32_t on);
double orc_csda_range(double T_keV);   /* g/cm^2 */
double orc_csda_energy(double R);      /* keV */

/* Ray-parity localization (Sec. 2.4.2).  Returns region id, or -1 if every
 * probe direction was degenerate. */
int32_t orc_locate(const orc_scene* s, const double p[3]);
/* Nearest facet with t > 0 along o + t d, skipping facet `exclude`.
 * Returns 1 and fills t, tri on a hit, else 0. */
int32_t orc_closest_hit(const orc_scene* s, const double o[3], const double d[3],
                        int64_t exclude, double* t, int64_t* tri);
/* Linear attenuation coefficients [1/mm] (photo, compton, coherent, pair) of
 * region r at E; scales[n_scales] multiply regions whose group is below n_scales. */
void orc_mu(const orc_scene* s, int32_t region, double E, const double* scales, int32_t n_scales,
            double out[4]);

/* Klein-Nishina pieces: k = E / m_e c^2, eps = E'/E. */
double orc_kn_integral(double k, double eps);    /* antiderivative of the bracket */
double orc_kn_sigma(double k);                   /* total, cm^2 per electron */
double orc_kn_sample(double k, double u);        /* inverse CDF, u in (0,1) */
double orc_thomson_sample(double u);             /* cos(theta) from 3/8 (1 + mu^2) */
/* The direction after a scattering of polar cosine ct and azimuth phi about
 * the unit direction d (the rotation used by transport). */
void orc_rotate(const double d[3], double ct, double phi, double out[3]);

enum { ORC_POINT = 0, ORC_BEAM = 1, ORC_CYL = 2 };
typedef struct {
  int32_t kind;
  double pos[3];        /* point/beam origin; CYL: base centre */
  double dir[3];        /* BEAM direction (unit) */
  double r_in, r_out, h;/* CYL: annulus radii, height along +z */
  int32_t region;       /* CYL: the region an emission point must lie in */
  int32_t n_lines;      /* > 0: energy drawn from lines (E0 ignored) */
  const double* line_keV;
  const double* line_prob;
} orc_source;

typedef struct {
  uint64_t n_histories, n_absorbed, n_fep, n_uncollided, n_escape, n_lost, n_killed,
      n_source_fail, n_balance_fail;
  uint64_t n_segments, n_crossings, n_photo, n_compton, n_coherent, n_pair, n_electrons;
  uint64_t spectrum_overflow;
  double edep_active, edep_total, e_escape;
  double sum_score[ORC_MAX_GROUPS];
  double sum_fep_score[ORC_MAX_GROUPS];
  double sum_fep_score2[ORC_MAX_GROUPS];
} orc_tally;

/* The emission step of history `history` of unit `unit` exactly as transport
 * draws it: the line energy (E = 0 for a mono-energetic source) and the
 * emission point; for a CYL source the number of rejection tries used
 * (0: all 1000 failed), else 1.  Returns 0, or -1 on bad arguments. */
int32_t orc_emission(const orc_scene* s, const orc_source* src, uint64_t seed, uint32_t unit,
                     int64_t history, double* E, double p[3], int32_t* attempts);

/* Histories first .. first+n-1 of unit `unit`.  scales[n_groups] multiply the
 * density of every region in the group.  spectrum (nullable) has n_channels
 * bins of channel_keV.  Returns 0, or <0 on bad arguments. */
int32_t orc_run(const orc_scene* s, const orc_source* src, double E0, int64_t n, int64_t first,
                uint64_t seed, uint32_t unit, const double* scales, int32_t n_groups,
                int32_t n_channels, double channel_keV, uint64_t* spectrum, int32_t max_steps,
                int32_t n_threads, orc_tally* out);

/* Gaussian broadening of a spectrum, FWHM(E)^2 = a + b E (keV), each count
 * spread over the channels within 5 sigma of its channel centre. */
void orc_broaden(const double* in, int32_t n, double channel_keV, double a, double b,
                 double* out);

#ifdef __cplusplus
}
#endif
#endif
