/*
 * gadep.h -- C interface of the MI355X photon-transport library.
 *
 * Analog photon transport through a closed, region-tagged triangle mesh for
 * HPGe full-energy-peak efficiency (FEPE) calibration, after DetMesh-Gadep
 * (arXiv 2605.25963), Sec. 2.2-2.4:
 *   - the CPU prepares the geometry and initialises the engine, the GPU
 *     transports the histories, the CPU scores the tallies (Sec. 2.4, Fig. 4);
 *   - facets arrive as in-memory arrays, no file I/O (Sec. 2.2.3);
 *   - each facet carries its enclosed ("inner") region; the region on its
 *     other side is derived here with the ray-parity rule of Sec. 2.4.2, so
 *     callers never declare nesting (Sec. 2.4.2, Fig. 5);
 *   - facets are wound counter-clockwise seen from outside, i.e. the Eq. (5)
 *     normal (v1-v0)x(v2-v0) points out of the enclosed volume.
 *
 * Conventions
 *   Units: mm, keV, g/cm^3, cm^2/g.  Linear attenuation of region r in scale
 *   group g: mu = 0.1 * rho_r * s_g * (mu/rho)(E)  [1/mm].
 *   Region 0 is the world: everything outside every shell.
 *   Every call returns gadep_status (0 = OK, < 0 = error); no exception or
 *   signal crosses the interface.  On error, gadep_last_error(ctx) returns a
 *   message that stays valid until the next call on that context.
 *   Pointers are host pointers unless the name ends in _dev.  Inputs are
 *   borrowed for the duration of the call only (copied, validated, uploaded);
 *   outputs are caller-allocated.  The context owns every device buffer it
 *   allocates and frees them in gadep_destroy.
 *   Calls on one context are serialised by the caller (one context per host
 *   thread); all device work of a context is ordered on its stream.
 */
#ifndef GADEP_H
#define GADEP_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct gadep_ctx gadep_ctx;

typedef enum {
  GADEP_OK = 0,
  GADEP_E_ARG = -1,             /* bad argument (null, size, range, NaN)                */
  GADEP_E_MESH_OPEN = -2,       /* a shell is not a closed 2-manifold                   */
  GADEP_E_MESH_ORIENT = -3,     /* inconsistent winding, or a shell wound inward        */
  GADEP_E_MESH_OVERLAP = -4,    /* shells intersect, coincide, or lie closer than min gap */
  GADEP_E_XS = -5,              /* bad cross-section table, or energy outside the grid  */
  GADEP_E_STATE = -6,           /* call out of order, e.g. run before load_mesh/set_xs  */
  GADEP_E_HIP = -7,             /* HIP runtime failure                                  */
  GADEP_E_OOM = -8,             /* device allocation failed                             */
  GADEP_E_TOPOLOGY = -9,        /* shell nesting could not be derived (parity rule)     */
  GADEP_E_MESH_DEGENERATE = -10 /* zero-area facet or non-finite vertex                 */
} gadep_status;

#define GADEP_MAX_REGIONS 64     /* per scene, world included */
#define GADEP_MAX_GROUPS 8       /* density-scale groups */
#define GADEP_MAX_SCENES 4096
#define GADEP_ACTIVE 1u          /* gadep_region.flags: tallied detector volume */

/* ----------------------------------------------------------------------------
 * context */

/* Creates a context on HIP device `device`.  hip_stream may be NULL (the
 * context creates its own stream) or a caller's hipStream_t (for example
 * torch.cuda.current_stream().cuda_stream), which the context then uses and
 * never destroys. */
gadep_status gadep_create(int device, void* hip_stream, gadep_ctx** out);
void gadep_destroy(gadep_ctx* ctx);
const char* gadep_last_error(const gadep_ctx* ctx);

/* Tunables and switches (gadep_set_option / gadep_get_option). */
typedef enum {
  GADEP_OPT_MAX_STEPS = 1,    /* per-history segment limit (watchdog), default 10000   */
  GADEP_OPT_BLOCK = 2,        /* threads per block of the transport kernel: 64..256,
                                 a multiple of 64 (256)                                 */
  GADEP_OPT_PERIOD = 3,       /* park threshold: lanes of a wavefront that finish their
                                 traversal wait until this many (1..64) have, then the
                                 wavefront runs physics, scoring and new histories for
                                 all of them together; 0 = default (24)                */
  GADEP_OPT_CLAIM = 4,        /* histories per lane taken by one work claim, the least
                                 one when claims shrink (16)                          */
  GADEP_OPT_VALIDATE = 5,     /* 1 = validate meshes at load (default); 0 skips the
                                 closed/orientation/overlap checks (fault-injection
                                 tests only: results are undefined on a bad mesh)      */
  GADEP_OPT_MIN_GAP_NM = 6,   /* smallest allowed distance between shells, nm (100)    */
  GADEP_OPT_GRAPHS = 7,       /* 1 = replay captured HIP graphs for repeated runs (1)  */
  GADEP_OPT_COUNTERS = 8,     /* 1 = count events (segments, node visits, ...) (0)     */
  GADEP_OPT_GRID = 9,         /* blocks of the persistent grid, 0 = from occupancy     */
  GADEP_OPT_EXIT_PLANES = 10, /* 1 = leave a convex outermost shell through its planes
                                 when the world is void (1); 0 = through its facets   */
  GADEP_OPT_SPLIT_PCT = 11,   /* extra facet slots the transport BVH may add by spatial
                                 splits, % of its facets (400); 0 = no spatial splits;
                                 applies to meshes loaded afterwards                  */
  GADEP_OPT_SCREEN = 12,      /* 1 = first-flight screening (1): with exit planes and a
                                 point or beam source in the outermost shell's region,
                                 each wavefront follows 64 new histories at a time to
                                 the end of their first flight, tallies those that
                                 leave through the planes without nearing the inner
                                 shells, and transports the rest in full.  Tallies
                                 are identical either way                             */
  GADEP_OPT_POOL = 13,        /* 1 = pooled transport kernel: each wavefront keeps 96
                                 photons in LDS for its 64 lanes, steps rays with full
                                 lanes while set-up rays last, and runs outcomes, new
                                 histories and set-up 64 photons at a time
                                 (GADEP_OPT_PERIOD: lanes still traversing when such a
                                 round starts, default 32; GADEP_OPT_BLOCK is unused);
                                 0 = per-lane kernel (0; the faster one on MI355X: the
                                 pooled kernel's LDS and registers allow 2 wavefronts
                                 per SIMD against 3).  Tallies are the same either way */
  GADEP_OPT_ELECTRONS = 14,   /* 1 = secondary electrons run straight tracks (a
                                 synthetic reading of the electron transport of
                                 Sec. 2.4.1; 0 = their energy is deposited where they
                                 start, the default): every electron of at least 10
                                 keV set in motion by a photoelectric absorption
                                 (isotropic), a Compton scattering (two-body recoil
                                 direction) or a pair production (the pair's kinetic
                                 energy, along the photon) runs a continuous-slowing-
                                 down track with the Katz-Penfold (1952) mass range
                                 at the regions' nominal densities; each region it
                                 crosses keeps the energy it loses there, and one
                                 that reaches the void world carries the rest out
                                 (the history is then not full-energy).  Per-lane
                                 kernel only (GADEP_E_ARG with GADEP_OPT_POOL = 1) */
  GADEP_OPT_GUIDE = 15        /* shrinking work claims (16): claims on an energy come
                                 in batches, one claim per wavefront of the energy's
                                 share of the grid, and each claim of a batch takes
                                 1/(this value x that count) of the histories the
                                 earlier batches left, down to 64 x GADEP_OPT_CLAIM
                                 (factoring: large claims first, small ones at the
                                 end); 0 = every claim takes 64 x GADEP_OPT_CLAIM.
                                 Histories keep their counter-keyed random numbers,
                                 so tallies do not depend on it (0..16) */
} gadep_option;
gadep_status gadep_set_option(gadep_ctx* ctx, int32_t option, int64_t value);
gadep_status gadep_get_option(const gadep_ctx* ctx, int32_t option, int64_t* value);

/* ----------------------------------------------------------------------------
 * geometry (Sec. 2.2.3, Sec. 2.4.2) */

typedef struct {
  int32_t material;      /* material id given to gadep_set_xs                   */
  float density_g_cm3;   /* >= 0                                                 */
  int32_t scale_group;   /* density-scale group 0..GADEP_MAX_GROUPS-1, -1 = none */
  uint32_t flags;        /* GADEP_ACTIVE: energy deposited here is tallied       */
} gadep_region;

/* Loads scene 0: vertices xyz_mm[n_vertices][3]; facets tri_vertices[n_tri][3]
 * (counter-clockwise seen from outside); tri_region[n_tri] = region whose
 * closed boundary the facet belongs to (1..n_regions-1); regions[n_regions]
 * with regions[0] the world.  Validates (closed consistently-oriented shells,
 * positive signed volume, no intersecting/coincident shells, gap >= min gap),
 * derives each shell's outside region by the parity rule, builds a SAH BVH and
 * uploads.  Errors: GADEP_E_ARG, _MESH_*, _TOPOLOGY, _HIP, _OOM. */
gadep_status gadep_load_mesh(gadep_ctx* ctx, const float* xyz_mm, int64_t n_vertices,
                             const int32_t* tri_vertices, const int32_t* tri_region,
                             int64_t n_tri, const gadep_region* regions, int32_t n_regions);
/* Same, into scene slot `scene` (0..GADEP_MAX_SCENES-1); a batch job picks its
 * scene, e.g. the detector together with a per-job sample container. */
gadep_status gadep_load_scene(gadep_ctx* ctx, int32_t scene, const float* xyz_mm,
                              int64_t n_vertices, const int32_t* tri_vertices,
                              const int32_t* tri_region, int64_t n_tri,
                              const gadep_region* regions, int32_t n_regions);

/* Two-level geometry for batches of calibration jobs (Sec. 1, Sec. 3.2: many
 * sample containers and matrices in front of one detector): loads a per-job
 * overlay -- closed shells such as a sample container and its matrix -- into
 * scene slot `scene`, on top of the detector in slot `base_scene`.  The
 * overlay's mesh (xyz, tri, tri_region as for gadep_load_mesh, facets tagged
 * 1..n_regions-1) lies inside region `host_region` of the detector and
 * crosses none of its shells; its regions[0] is ignored (it is the host
 * region).  The combined scene numbers the detector's regions 0..nb-1 and
 * overlay region k >= 1 as nb + k - 1 (job overrides, volume-source regions
 * and tallies use these numbers), and its facets as the detector's followed
 * by the overlay's.  The detector's BVHs and facet records are stored once
 * for all its overlays; the overlay's are added to the same device arrays,
 * and a photon in a region bounded by both meshes searches both BVHs and
 * keeps the nearest hit.  Validation (GADEP_OPT_VALIDATE) checks the two
 * meshes together: closed, oriented, apart, and each outermost overlay shell
 * directly inside host_region (else GADEP_E_TOPOLOGY).  Reloading the
 * detector's slot invalidates its overlays.  Errors: GADEP_E_ARG,
 * GADEP_E_STATE (no detector in base_scene), _MESH_*, _TOPOLOGY, _HIP, _OOM. */
gadep_status gadep_load_overlay(gadep_ctx* ctx, int32_t scene, int32_t base_scene,
                                int32_t host_region, const float* xyz_mm, int64_t n_vertices,
                                const int32_t* tri_vertices, const int32_t* tri_region,
                                int64_t n_tri, const gadep_region* regions, int32_t n_regions);

/* ----------------------------------------------------------------------------
 * cross sections (Sec. 2.4.1) */

/* Partial mass attenuation coefficients mu/rho [cm^2/g] of `material` on the
 * grid ln E_k = lnE0_keV + k dlnE, k = 0..n_E-1 (the same grid for every
 * material): photoelectric, incoherent (Klein-Nishina), coherent (Thomson) and
 * pair production (Sec. 2.4.1).  Interpolation is linear in ln E of ln(mu/rho),
 * per partial.  Any partial may be NULL (absent); a present partial must be
 * all-positive or all-zero.  The pair partial counts only above 2 m_e c^2 =
 * 1021.998 keV (zero at and below it, whatever the table holds there); a pair
 * event deposits E - 2 m_e c^2 where it happens and starts two 511 keV photons
 * back to back along a random axis, which the history then follows in turn.  The lowest grid energy is the photon cut-off: below it the
 * remaining energy is deposited locally.  Source energies must lie on the
 * grid and below 65536 keV (energy tallies count 2^-16 keV units).
 * Errors: GADEP_E_ARG, GADEP_E_XS. */
gadep_status gadep_set_xs(gadep_ctx* ctx, int32_t material, double lnE0_keV, double dlnE,
                          int32_t n_E, const float* mu_rho_photo, const float* mu_rho_compton,
                          const float* mu_rho_coherent, const float* mu_rho_pair);

/* Density scales s_g used by gadep_run (default 1).  scales[n_scales]. */
gadep_status gadep_set_scales(gadep_ctx* ctx, const float* scales, int32_t n_scales);

/* ----------------------------------------------------------------------------
 * sources and tallies */

/* GADEP_SRC_CONE: an isotropic point source of which only the directions that
 * can meet the inner shells are followed (variance reduction for distant
 * sources; not a step of the paper): every history starts in the cone that
 * subtends the bounding sphere of the shells inside the outermost one (of all
 * shells when the outermost is not a convex exit shell) and stands for the
 * weight w = (1 - cos theta_c) / 2 = Omega / 4 pi of the emitted photons,
 * reported in gadep_tally.weight (FEPE = weight * n_fep / n_histories).  The
 * photons it leaves out cross only the region around the source, so FEPE is
 * unchanged as long as that region has no coherent partial (an elastic
 * scatter there could send such a photon into the detector with its full
 * energy): a source in a region whose material has one is rejected
 * (GADEP_E_ARG).  Spectra and efficiencies other than FEPE lose the photons
 * scattered into the detector from outside the cone.  A source inside that
 * sphere emits into 4 pi (weight 1). */
typedef enum { GADEP_SRC_POINT = 0, GADEP_SRC_BEAM = 1, GADEP_SRC_CYL = 2,
               GADEP_SRC_CONE = 3 } gadep_source_kind;
typedef struct {
  int32_t kind;          /* gadep_source_kind                                      */
  float pos_mm[3];       /* POINT/BEAM/CONE: origin.  CYL: centre of the base face */
  float dir[3];          /* BEAM: direction (normalised here)                      */
  float r_in_mm, r_out_mm, h_mm; /* CYL: uniform in r_in <= r <= r_out, 0 <= z <= h
                                    (axis +z); points outside `region` rejected    */
  int32_t region;        /* CYL: region every emission point must lie in           */
  int32_t n_lines;       /* > 0: each history draws its energy from the lines     */
  const float* line_keV; /* [n_lines]                                              */
  const float* line_prob;/* [n_lines], relative weights                            */
} gadep_source;

/* Per (job, energy) unit.  A history is FEP when it ends by absorption with
 * every deposit inside ACTIVE regions (its ACTIVE deposit equals its source
 * energy).  n_escape = n_histories - n_absorbed - n_lost - n_killed
 * - n_source_fail. */
typedef struct {
  uint64_t n_histories, n_absorbed, n_fep, n_escape, n_uncollided, n_lost, n_killed, n_glitch,
      n_source_fail;
  double edep_active_keV, edep_total_keV, e_escape_keV, e_source_keV;
  uint64_t* spectrum;        /* in: nullable caller buffer [n_channels] of ACTIVE
                                deposit counts, channel = floor(E_dep/channel_keV) */
  int32_t n_channels;        /* in */
  float channel_keV;         /* in */
  uint64_t spectrum_overflow;/* out: histories with E_dep >= n_channels*channel_keV */
  double weight;             /* out: emitted photons each history stands for (1, or
                                Omega / 4 pi for GADEP_SRC_CONE)                   */
} gadep_tally;

/* ----------------------------------------------------------------------------
 * transport (Sec. 2.4: the host prepares geometry and tables and scores, the
 * device transports; Sec. 2.4.1: photon physics and the free path by partial
 * cross sections; Sec. 2.4.2: region at each crossing; Sec. 2.4.3: BVH) */

/* FEPE calibration run (Sec. 3.2: an on-axis point source and FEPE per
 * energy; Table 4 counts particles per energy).
 * n_histories histories (numbers first_history..) at each of the energies,
 * point/beam/volume source, seed for the counter-based generator
 * (Philox4x32-10 keyed by seed, counter = (draw, history, unit)).  Results are
 * a pure function of (inputs, seed, history numbers): disjoint history ranges
 * add up exactly, and launch shape never changes a tally.
 * out[n_energies]; for a line source pass energies_keV = NULL, n_energies = 1. */
gadep_status gadep_run(gadep_ctx* ctx, const gadep_source* src, const double* energies_keV,
                       int32_t n_energies, int64_t n_histories, uint64_t seed,
                       int64_t first_history, gadep_tally* out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gadep_run on the mesh of
 * scene 0 at the context's density scales, with the same arguments, results
 * (bit for bit) and errors, that allocates no device memory.  Its tables,
 * cursors, tally rows and spectra live in one fixed 4 MiB device array per GPU
 * (kept until the process ends); the mesh and cross sections must already be
 * on the device (gadep_load_mesh, gadep_set_xs).  Limits: n_energies <= 256,
 * n_lines <= 256, n_energies * n_channels <= 501280 spectrum words; larger
 * inputs return GADEP_E_ARG.  Like gadep_run it returns when the tallies are
 * in `out`.  Every call on one GPU shares that GPU's array, from any
 * context: calls that overlap in time on one GPU race and must not be made. */
gadep_status gadep_run_noalloc(gadep_ctx* ctx, const gadep_source* src,
                               const double* energies_keV, int32_t n_energies,
                               int64_t n_histories, uint64_t seed, int64_t first_history,
                               gadep_tally* out);

/* Not a step of the paper: FEPE is most sensitive to the dead layer and the
 * crystal at low energies (Sec. 1, Sec. 4), and this gives the derivative a
 * fit of those densities needs.
 * As gadep_run at density scales `scales[n_scales]`, also returning the
 * score-function derivative of FEPE with respect to each scale,
 * dfepe_ds[n_energies][n_scales] = mean over histories of
 * 1_FEP * (n_g / s_g - sum over path segments in group g of mu0 * l),
 * and the variance of that mean, dfepe_ds_var (same shape, nullable). */
gadep_status gadep_run_grad(gadep_ctx* ctx, const gadep_source* src, const double* energies_keV,
                            int32_t n_energies, int64_t n_histories, uint64_t seed,
                            int64_t first_history, const float* scales, int32_t n_scales,
                            gadep_tally* out, double* dfepe_ds, double* dfepe_ds_var);

/* Many calibration jobs of uneven size in one persistent launch: sourceless
 * calibration evaluates many energies, source geometries and matrices for
 * one detector (Sec. 1, Sec. 3.2). */
typedef struct {
  gadep_source src;
  const double* energies_keV;  /* [n_energies]; NULL for a line source (n_energies 1) */
  int32_t n_energies;
  int64_t n_histories;         /* per energy */
  int64_t first_history;
  const float* scales;         /* nullable [n_scales]: all 1 */
  int32_t n_scales;
  int32_t scene;               /* scene slot */
  uint32_t stream;             /* random stream id: identical (stream, seed, histories)
                                  give identical results, batched or not */
  const int32_t* region_material_override; /* nullable [n_regions of the scene]     */
  const float* region_density_override;    /* nullable [n_regions of the scene]     */
} gadep_job;

/* out[sum of n_energies] in job order.  grads (nullable) receives
 * dFEPE/ds [unit][GADEP_MAX_GROUPS] and grads_var (nullable) its variance. */
gadep_status gadep_run_batch(gadep_ctx* ctx, const gadep_job* jobs, int32_t n_jobs,
                             uint64_t seed, gadep_tally* out, double* grads, double* grads_var);

/* Launch tuning (no counterpart in the paper, whose kernel runs on one
 * RTX 4090 configuration, Sec. 3.3).
 * Times short pilot launches of `jobs` (scaled down to about pilot_histories
 * in total) over block sizes, park thresholds (GADEP_OPT_PERIOD) and claim
 * sizes, keeps the fastest in the context and returns it (any output pointer
 * may be NULL).  The result is cached in the process, keyed by the GPU's
 * architecture, the kernel (GADEP_OPT_POOL) and the class of the job mix
 * (log2 of the largest scene's facet count, of the number of jobs and of
 * units, the source kinds): a later call with the same key returns it
 * without timing.  Tallies never depend on these settings. */
gadep_status gadep_autotune(gadep_ctx* ctx, const gadep_job* jobs, int32_t n_jobs,
                            int64_t pilot_histories, int32_t* block, int32_t* period,
                            int32_t* claim);

/* Event counts of the last run with GADEP_OPT_COUNTERS = 1 (the work the
 * performance comparison of Sec. 3.3 / Table 4 rests on, per event). */
typedef struct {
  uint64_t segments, crossings, node_visits, tri_tests, photo, compton, coherent, rng_calls,
      locates, emissions;
  uint64_t plane_tests; /* exit-plane evaluations (see gadep_mesh_info.n_exit_planes) */
  /* per wavefront: traversal-loop iterations, those in which some lane took a
   * node step / a facet test, and passes of the batched per-segment work
   * (outcomes, new histories, set-up) */
  uint64_t iterations, iterations_node, iterations_facet, passes;
  /* per wavefront, shader-clock cycles spent in: outcomes of finished
   * segments, handing out new histories (with screening), drawing emission
   * directions, segment set-up, traversal steps */
  uint64_t cycles_outcome, cycles_refill, cycles_launch, cycles_setup, cycles_traversal;
  /* histories that first-flight screening settled with a ray set-up and one
   * box test: their flight certainly outlasts the outermost shell, so neither
   * the attenuation nor the exit planes are evaluated (no segment is counted) */
  uint64_t box_tests;
  uint64_t pair;        /* pair-production events */
  uint64_t electrons;   /* electron tracks (GADEP_OPT_ELECTRONS) */
  /* wavefronts launched, and the sum of their lifetimes in shader-clock
   * cycles: over wavefronts x launch duration x shader clock, the share of
   * the launch the grid was busy (the rest is the tail of the work claims) */
  uint64_t wavefronts, wave_cycles;
  /* screened histories settled by their direction alone (it misses the sphere
   * around the inner shells' box), without the box test */
  uint64_t cone_tests;
} gadep_counters;
gadep_status gadep_get_counters(const gadep_ctx* ctx, gadep_counters* out);

/* Timing as in Sec. 3.3 (kernel time per run).
 * Duration of the last transport launch, from HIP events recorded on the
 * context's stream right before and after it (the graph replay, when graphs
 * are on, which adds two tiny set-up kernels to the transport kernel). */
gadep_status gadep_get_last_launch_ms(const gadep_ctx* ctx, double* ms);

/* Shader clock [MHz] the last transport launch ran at: each wavefront reads
 * the shader-clock counter (s_memtime) and the constant-rate counter
 * (s_memrealtime) when it starts and when it ends; the ratio of the summed
 * differences times the constant counter's rate.  For scaling the ALU peak
 * of the roofline to the clock actually sustained (the kernel time of Sec.
 * 3.3 depends on it). */
gadep_status gadep_get_last_clock_mhz(const gadep_ctx* ctx, double* mhz);

/* Pulse-height spectrum post-processing (the detector resolution the paper
 * leaves to the analysis after transport, Sec. 2.4 scoring on the host side).
 * Gaussian broadening of spectra on the device: FWHM(E)^2 = a + b E (keV^2,
 * E = channel centre), counts spread over the channels within 5 sigma,
 * each receiving channel taking the integral of the normal law over its
 * width.  in_dev / out_dev: device arrays [n_spectra][n_channels], FP64. */
gadep_status gadep_broaden_dev(gadep_ctx* ctx, const double* in_dev, double* out_dev,
                               int32_t n_spectra, int32_t n_channels, double channel_keV,
                               double a, double b);

/* ----------------------------------------------------------------------------
 * geometry queries on the device (checks of the boundary handling) */

/* Nearest-hit query of Sec. 2.4.2 (the facet ahead and the material behind
 * it) on the BVH of Sec. 2.4.3.
 * Closest facet hit for rays o[n][3] + t d[n][3], t > 0, from region
 * region[n] (nullable: no region-consistency filter).  Returns t[n]
 * (INFINITY on a miss), tri[n] (caller's facet index, -1 on a miss) and
 * region_after[n] (region entered across the hit facet). */
gadep_status gadep_raycast(gadep_ctx* ctx, int32_t scene, const float* o, const float* d,
                           const int32_t* region, int64_t n, float* t, int32_t* tri,
                           int32_t* region_after);
/* Region of points p[n][3] by the ray-parity rule (Sec. 2.4.2); -1 when every
 * probe ray was degenerate. */
gadep_status gadep_locate(gadep_ctx* ctx, int32_t scene, const float* p, int64_t n,
                          int32_t* region);

/* The transport kernel's random-number generator, Philox4x32-10 (Salmon et
 * al., SC'11), run on the device for
 * given counters: counters[n][4] (host, read only), key = k0 | k1 << 32,
 * out[n][4] (host, written).  The kernel keys each block with the run's
 * seed and counts (draw, history lo, history hi, unit stream). */
gadep_status gadep_philox(gadep_ctx* ctx, const uint32_t* counters, uint64_t key, int64_t n,
                          uint32_t* out);

/* ----------------------------------------------------------------------------
 * host-only mesh preparation (no device needed) */

typedef struct {
  int32_t n_shells;       /* connected closed surfaces */
  int32_t genus_max;      /* largest shell genus, from the Euler characteristic */
  int64_t n_nodes;        /* nodes of the returned BVH (each holds two children) */
  int32_t depth;          /* its depth = traversal stack needed */
  double sah_cost;        /* its SAH cost, unit traversal and intersection costs */
  int64_t n_slots;        /* its facet slots (more than n_tri when facets are split) */
  double min_gap_mm;      /* smallest distance found between different shells */
  int32_t convex_exit;    /* 1: the world borders a single convex shell, so a photon
                             leaving it into a void world escapes at once */
  int32_t n_exit_planes;  /* > 0: that shell has this many distinct facet planes (at
                             most 32); with a void world, a photon inside it then
                             searches a BVH over the other shells only and leaves
                             the outermost shell's own region through its planes */
  int32_t region_root[GADEP_MAX_REGIONS + 1]; /* bvh_method 2 only (else -1): root
                             node of region r's transport BVH (-1: no facets bound
                             r); entry n_regions: the outer region's without the
                             outermost shell, when n_exit_planes > 0 */
} gadep_mesh_info;

/* Validation + topology + BVH on the host, as gadep_load_mesh does, without
 * a context.  tri_outside[n_tri] (nullable) receives the region outside each
 * facet, tri_shell[n_tri] (nullable) its shell index.  bvh_method selects the
 * BVH returned in nodes_out / tri_order and described by info: 0 = binned SAH
 * over every facet (the one used for parity counts and geometry queries),
 * 1 = object-median split, 2 = the transport BVHs (binned SAH with spatial
 * splits, Stich et al. 2009), one per region over the facets that bound it
 * (inside or outside that region), concatenated, with their roots in
 * info->region_root (split_budget = extra slots each may add, as a
 * fraction of its facets).  nodes_out (nullable, [cap_nodes][16] 32-bit
 * words, the device layout: two child boxes as 12 floats, then two child
 * links as int32 -- >= 0 a node, < 0 a leaf ~(first_slot << 3 | count) --
 * then 2 words of padding) and tri_order (nullable, [cap_slots]: caller facet
 * index of each slot).  A capacity below info->n_nodes or info->n_slots
 * returns GADEP_E_ARG with info filled. */
gadep_status gadep_mesh_prepare(const float* xyz_mm, int64_t n_vertices,
                                const int32_t* tri_vertices, const int32_t* tri_region,
                                int64_t n_tri, int32_t n_regions, double min_gap_mm,
                                int32_t validate, int32_t bvh_method, double split_budget,
                                int32_t* tri_outside, int32_t* tri_shell, void* nodes_out,
                                int64_t cap_nodes, int32_t* tri_order, int64_t cap_slots,
                                gadep_mesh_info* info, char* err, int32_t err_len);

/* ----------------------------------------------------------------------------
 * parametric detector meshes (Sec. 2.2, 2.3) */

/* A single-ended coaxial HPGe detector by the Table 2 parameter groups [mm].
 * Frame: axis z, crystal front face at z = 0 facing +z (toward the source),
 * crystal z in [-D1, 0].  Readings of the parameters:
 *   crystal radius D2, length D1, front-edge rounding D3 (Eq. 3-4);
 *   outer dead layer D4: the active volume has radius D2 - D4, front face at
 *     -D4, rounding D3 - D4 (Eq. 6); below 4 eps it gets no shell of its own
 *     (an implanted contact of 0.3 um: the crystal shell is then the active one);
 *   borehole radius D6, length D5 from the back face, hemispherical tip; the
 *     contact layer D7 lines it (a shell of its own when >= 4 eps);
 *   crystal cup: cavity radius D2 + cup_gap_mm, wall d4, floor d10, from
 *     z = -d8 up to its rim at z = cup_rim_mm (open toward the window);
 *   vacuum housing: side vacuum d6 outside the cup, wall d3, floor d9 at
 *     z = -d7; its front wall is the window plane, d5 (top vacuum) above the
 *     crystal, d2 thick, with the window (radius d1) as a region of its own;
 *   optional electrode pin in the borehole and cold finger below the cup;
 *   world_half_mm > 0: an air box of that half-size around the housing.
 * Nested shells that would touch are separated inside-out by eps_mm (Sec.
 * 2.4.2).  Discretisation: n_theta angles (Eq. 1-2), n_phi rounding steps
 * (Eq. 3), z_slices side bands. */
typedef struct {
  double d1, d2, d3, d4, d5, d6, d7, d8, d9, d10;
  double D1, D2, D3, D4, D5, D6, D7;
  int32_t n_theta, n_phi, z_slices;
  double eps_mm;
  double cup_gap_mm, cup_rim_mm;
  double pin_radius_mm, pin_length_mm;
  double finger_radius_mm;
  double world_half_mm;
} gadep_detector;

/* Region ids of gadep_detmesh (a region may have no facets: no air box, no
 * separate dead layer, no contact layer, pin or finger). */
enum {
  GADEP_DM_WORLD = 0, GADEP_DM_AIR, GADEP_DM_HOUSING, GADEP_DM_WINDOW, GADEP_DM_VACUUM,
  GADEP_DM_CUP, GADEP_DM_CRYSTAL, GADEP_DM_ACTIVE, GADEP_DM_CONTACT, GADEP_DM_BORE,
  GADEP_DM_PIN, GADEP_DM_FINGER, GADEP_DM_N
};

/* Builds the detector's shells (Eq. 5 orientation, CCW seen from outside).
 * n_vertices / n_facets receive the counts; xyz[3 * n_vertices],
 * tri_vertices[3 * n_facets] and tri_region[n_facets] (each nullable) receive
 * the mesh when the capacities suffice (call once with NULL to size);
 * region_parent[GADEP_DM_N] (nullable) the enclosing region of each region
 * (-1: the world, or no facets).  The arrays feed gadep_load_mesh /
 * gadep_load_scene directly (in memory, Sec. 2.4).  Errors: GADEP_E_ARG with
 * a message for parameters that do not fit together. */
gadep_status gadep_detmesh(const gadep_detector* params, float* xyz, int64_t cap_vertices,
                           int32_t* tri_vertices, int32_t* tri_region, int64_t cap_facets,
                           int64_t* n_vertices, int64_t* n_facets, int32_t* region_parent,
                           char* err, int32_t err_len);

/* Writes a mesh as VRML 2.0 (Sec. 2.2.3): one Shape with an IndexedFaceSet per
 * region that has facets, all sharing the vertex list.  GADEP_E_ARG on bad
 * arrays or an unwritable path. */
gadep_status gadep_write_vrml(const char* path, const float* xyz, int64_t n_vertices,
                              const int32_t* tri_vertices, const int32_t* tri_region,
                              int64_t n_tri, int32_t n_regions);

#ifdef __cplusplus
}
#endif
#endif /* GADEP_H */
