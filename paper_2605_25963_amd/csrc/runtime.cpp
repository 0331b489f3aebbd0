// Runtime behind the C interface: contexts, scenes, tables, unit tables,
// persistent launches, graph replay, tally conversion and the autotuner.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "gadep.h"
#include "gadep_internal.h"

namespace gadep {
// kernels.hip
size_t transport_smem(int block, int depth, bool grad, bool pair);
hipError_t transport_launch(const TransportParams& P, int variant, int grid, int block,
                            hipStream_t s);
hipError_t transport_occupancy(int variant, int block, int depth, int pair, int* blocks_per_cu);
hipError_t fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t locate_units(UnitRec* units, int n_units, const SceneRec* scenes,
                        const SourceRec* sources, int depth, hipStream_t s);
hipError_t raycast(const SceneRec& sc, const float* o, const float* d, const int32_t* region,
                   int64_t n, float* t, int32_t* tri, int32_t* region_after, hipStream_t s);
hipError_t locate(const SceneRec& sc, const float* p, int64_t n, int32_t* region, hipStream_t s);
hipError_t philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out,
                  hipStream_t s);
hipError_t scratch_address(int device, void** out);
hipError_t pool_launch(const TransportParams& P, int variant, int grid, hipStream_t s);
hipError_t pool_occupancy(int variant, int depth, int pair, int* blocks_per_cu);
hipError_t broaden(const double* in, double* out, int n_spectra, int n, double w, double a,
                   double b, hipStream_t s);
}  // namespace gadep

using namespace gadep;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Scene {
  bool loaded = false;
  int32_t n_regions = 0;
  std::vector<gadep_region> regions;
  int32_t depth = 0;
  int64_t n_tri = 0;
  int64_t n_nodes = 0;
  bool convex_exit = false;
  int32_t n_planes = 0;
  int32_t outer_root = kDone;
  int32_t outer_region = 0;
  float trans_lo[3] = {0, 0, 0}, trans_hi[3] = {0, 0, 0};
  float outer_lo[3] = {0, 0, 0}, outer_hi[3] = {0, 0, 0};
  // box of the shells inside a convex exit shell (of all shells without one):
  // the target of cone emission
  double inner_lo[3] = {0, 0, 0}, inner_hi[3] = {0, 0, 0};
  void* d_nodes = nullptr;
  void* d_tris = nullptr;
  void* d_planes = nullptr;
  void* d_roots = nullptr;
  void* d_slots = nullptr;
  // A detector scene keeps its mesh on the host and the element counts of its
  // device arrays, which the overlays loaded on it extend (its BVHs and facet
  // records are stored once for all of them).
  std::vector<float> h_xyz;
  std::vector<int32_t> h_tri, h_reg, h_roots;
  int64_t arena_nodes = 0, arena_slots = 0, arena_tris = 0;
  // An overlay (a per-job mesh, e.g. a sample container, on a detector scene):
  // the detector's slot, its own second root per combined region and the root
  // of its plain BVH; its node, slot and facet records live in the detector's
  // arrays.
  int32_t base = -1;
  void* d_roots2 = nullptr;
  int32_t root_all2 = -1;
};

void fill_scene_rec(const std::vector<std::unique_ptr<Scene>>& scenes, const Scene& sc,
                    SceneRec& sr) {
  const Scene& arr = sc.base >= 0 ? *scenes[sc.base] : sc;
  sr.nodes = static_cast<const BvhNode*>(arr.d_nodes);
  sr.tris = static_cast<const TriRec*>(arr.d_tris);
  sr.slots = static_cast<const int32_t*>(arr.d_slots);
  sr.planes = static_cast<const float*>(arr.d_planes);
  sr.roots2 = static_cast<const int32_t*>(sc.d_roots2);
  sr.root_all2 = sc.root_all2;
  sr.n_regions = sc.n_regions;
  sr.depth = sc.depth;
  sr.roots = static_cast<const int32_t*>(sc.d_roots);
  sr.n_planes = sc.n_planes;
  sr.outer_root = sc.outer_root;
  sr.root_all = 0;
  sr.outer_region = sc.outer_region;
  for (int a = 0; a < 3; ++a) {
    sr.trans_lo[a] = sc.trans_lo[a];
    sr.trans_hi[a] = sc.trans_hi[a];
    sr.outer_lo[a] = sc.outer_lo[a];
    sr.outer_hi[a] = sc.outer_hi[a];
  }
}

// Host side of a no-allocation run: the tables uploaded into the device
// scratch array, and the tally rows read back from it.
struct NoAllocHost {
  UnitRec units[kScratchUnits];
  int64_t chunk_begin[kScratchUnits + 1];
  SceneRec scene;
  SourceRec source;
  float lines[2 * kScratchLines];
  RegionRec regions[kMaxRegions];
  unsigned long long tally[static_cast<size_t>(kScratchUnits) * kT_Slots];
};

// Byte offsets of those tables in the device scratch array; the spectra take
// the rest.
constexpr size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }
constexpr size_t kNaUnits = 0;
constexpr size_t kNaChunks = align256(kNaUnits + kScratchUnits * sizeof(UnitRec));
constexpr size_t kNaScene = align256(kNaChunks + (kScratchUnits + 1) * sizeof(int64_t));
constexpr size_t kNaSource = align256(kNaScene + sizeof(SceneRec));
constexpr size_t kNaLines = align256(kNaSource + sizeof(SourceRec));
constexpr size_t kNaRegions = align256(kNaLines + 2 * kScratchLines * sizeof(float));
constexpr size_t kNaCursor = align256(kNaRegions + kMaxRegions * sizeof(RegionRec));
constexpr size_t kNaTally = align256(kNaCursor + kScratchUnits * sizeof(unsigned long long));
constexpr size_t kNaSpectra =
    align256(kNaTally + static_cast<size_t>(kScratchUnits) * kT_Slots * sizeof(unsigned long long));
constexpr size_t kNaSpectraWords = (kScratchBytes - kNaSpectra) / sizeof(unsigned long long);
static_assert(kNaSpectra + (size_t(1) << 16) <= kScratchBytes, "scratch layout");

struct Material {
  bool set = false;
  std::vector<float> ln[4];  // ln(mu/rho) per grid point; -200 for an absent partial
  bool pair = false;         // has a pair-production partial
};

}  // namespace

struct gadep_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n_cu = 0;
  std::string err;

  std::vector<std::unique_ptr<Scene>> scenes;

  bool grid_set = false;
  double lnE0 = 0, dlnE = 0;
  int32_t nE = 0;
  std::vector<Material> mats;
  bool xs_dirty = false;
  DevBuf xs;

  std::vector<float> scales = std::vector<float>(GADEP_MAX_GROUPS, 1.0f);

  int64_t max_steps = 10000;
  int64_t block = 256;
  int64_t period = 0;
  int64_t claim = 16;
  int64_t validate = 1;
  int64_t min_gap_nm = 100;
  int64_t graphs = 1;
  int64_t counters = 0;
  int64_t grid = 0;
  int64_t exit_planes = 1;
  int64_t split_pct = 400;
  int64_t screen = 1;
  int64_t pool = 0;
  int64_t guide = 16;
  int64_t electrons = 0;

  DevBuf units, chunk_begin, scene_tab, sources, lines, regions, tally, spectra, cursor;
  void* h_tally = nullptr;  // pinned
  size_t h_tally_cap = 0;
  gadep_counters last_counters{};
  bool have_counters = false;
  double last_ms = -1.0;
  double last_sclk_mhz = -1.0;  // shader clock of the last transport launch
  double ref_clock_khz = 100000.0;  // rate of the constant clock the kernels read
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  // graph cache
  hipGraphExec_t graph = nullptr;
  std::vector<uint8_t> graph_key;

  // gadep_run_noalloc: the device's fixed scratch array (its address on this
  // context's device) and host staging of the same tables, set up at create
  void* scratch = nullptr;
  std::unique_ptr<NoAllocHost> na;
};

namespace {

gadep_status set_err(gadep_ctx* c, gadep_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

gadep_status hip_err(gadep_ctx* c, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return set_err(c, GADEP_E_OOM, std::string(what) + ": " + hipGetErrorString(e));
  return set_err(c, GADEP_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                      \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_err(ctx, e_, what); \
  } while (0)

gadep_status ensure(gadep_ctx* ctx, DevBuf& b, size_t bytes, const char* what) {
  if (bytes == 0) bytes = 16;
  if (b.cap >= bytes) return GADEP_OK;
  if (b.p) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  size_t cap = bytes + bytes / 4;
  HIP_TRY(hipMalloc(&b.p, cap), what);
  b.cap = cap;
  // cached graphs refer to the old buffer
  if (ctx->graph) {
    (void)hipGraphExecDestroy(ctx->graph);
    ctx->graph = nullptr;
    ctx->graph_key.clear();
  }
  return GADEP_OK;
}

void free_buf(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

gadep_status upload(gadep_ctx* ctx, DevBuf& b, const void* src, size_t bytes, const char* what) {
  gadep_status s = ensure(ctx, b, bytes, what);
  if (s) return s;
  if (bytes) HIP_TRY(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, ctx->stream), what);
  return GADEP_OK;
}

gadep_status sync_xs(gadep_ctx* ctx) {
  if (!ctx->xs_dirty) return GADEP_OK;
  const size_t nm = ctx->mats.size();
  std::vector<float> host(nm * ctx->nE * 4, -200.0f);
  for (size_t m = 0; m < nm; ++m) {
    if (!ctx->mats[m].set) continue;
    for (int32_t k = 0; k < ctx->nE; ++k)
      for (int i = 0; i < 4; ++i) host[(m * ctx->nE + k) * 4 + i] = ctx->mats[m].ln[i][k];
  }
  gadep_status s = upload(ctx, ctx->xs, host.data(), host.size() * sizeof(float), "upload xs");
  if (s) return s;
  HIP_TRY(hipStreamSynchronize(ctx->stream), "upload xs");
  ctx->xs_dirty = false;
  return GADEP_OK;
}

// ---------------------------------------------------------------------------
// run planning

struct Plan {
  std::vector<UnitRec> units;
  std::vector<int64_t> chunk_begin;
  std::vector<SourceRec> sources;
  std::vector<float> lines;
  std::vector<RegionRec> regions;
  std::vector<double> unit_energy;  // for reporting
  std::vector<double> unit_weight;  // photons each history stands for (cone emission)
  bool spectrum = false;
  int32_t n_channels = 0;
  float channel_keV = 0;
  bool grad = false;
  int32_t depth = 1;
};

gadep_status check_source(gadep_ctx* ctx, const gadep_source& s, const Scene& sc) {
  if (s.kind < GADEP_SRC_POINT || s.kind > GADEP_SRC_CONE)
    return set_err(ctx, GADEP_E_ARG, "source: unknown kind");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(s.pos_mm[a])) return set_err(ctx, GADEP_E_ARG, "source: non-finite position");
  if (s.kind == GADEP_SRC_BEAM) {
    double n = 0;
    for (int a = 0; a < 3; ++a) n += double(s.dir[a]) * s.dir[a];
    if (!(n > 0) || !std::isfinite(n)) return set_err(ctx, GADEP_E_ARG, "source: bad beam direction");
  }
  if (s.kind == GADEP_SRC_CYL) {
    if (!(s.r_in_mm >= 0) || !(s.r_out_mm > s.r_in_mm) || !(s.h_mm > 0))
      return set_err(ctx, GADEP_E_ARG, "source: bad cylinder dimensions");
    if (s.region < 0 || s.region >= sc.n_regions)
      return set_err(ctx, GADEP_E_ARG, "source: region out of range");
  }
  if (s.n_lines < 0) return set_err(ctx, GADEP_E_ARG, "source: n_lines < 0");
  if (s.n_lines > 0) {
    if (!s.line_keV || !s.line_prob) return set_err(ctx, GADEP_E_ARG, "source: null line arrays");
    double tot = 0;
    for (int i = 0; i < s.n_lines; ++i) {
      if (!(s.line_prob[i] >= 0)) return set_err(ctx, GADEP_E_ARG, "source: negative line weight");
      tot += s.line_prob[i];
    }
    if (!(tot > 0)) return set_err(ctx, GADEP_E_ARG, "source: line weights sum to zero");
  }
  return GADEP_OK;
}

gadep_status check_energy(gadep_ctx* ctx, double E) {
  const double lo = exp(ctx->lnE0), hi = exp(ctx->lnE0 + ctx->dlnE * (ctx->nE - 1));
  if (!(E >= lo * (1 - 1e-12) && E <= hi * (1 + 1e-12)))
    return set_err(ctx, GADEP_E_XS, "energy " + std::to_string(E) + " keV outside the table grid");
  if (!(E < 65536.0))  // energy tallies count 2^-16 keV units in 32 bits per history
    return set_err(ctx, GADEP_E_ARG, "energy " + std::to_string(E) + " keV: at most 65536 keV");
  return GADEP_OK;
}

// Cone emission of a GADEP_SRC_CONE source towards the scene's inner box:
// axis (unit, from the source to the centre of the box's bounding sphere),
// cosine of the half-angle (-1: the whole sphere) and the weight Omega/4pi.
// The sphere's radius is raised by 1e-4 relative so that rounding of the
// sampled directions can never exclude one that meets the box.
gadep_status cone_setup(gadep_ctx* ctx, const Scene& sc, const gadep_source& src,
                        const RegionRec* regions, SourceRec& sr, double& weight) {
  weight = 1.0;
  sr.cone_cos = -1.0f;
  if (src.kind != GADEP_SRC_CONE) return GADEP_OK;
  double c[3], r2 = 0, d2 = 0;
  for (int a = 0; a < 3; ++a) {
    c[a] = 0.5 * (sc.inner_lo[a] + sc.inner_hi[a]);
    const double h = 0.5 * (sc.inner_hi[a] - sc.inner_lo[a]);
    r2 += h * h;
    d2 += (src.pos_mm[a] - c[a]) * (src.pos_mm[a] - c[a]);
  }
  const double R = sqrt(r2) * (1.0 + 1e-4), D = sqrt(d2);
  // the region around the source must not scatter elastically (see gadep.h)
  for (int32_t r = 0; r < sc.n_regions; ++r) {
    if (r != 0 && r != sc.outer_region) continue;
    const RegionRec& rr = regions[r];
    if (rr.mult > 0.0f && ctx->mats[rr.material].ln[2][0] > -200.0f)
      return set_err(ctx, GADEP_E_ARG, "cone source: the region around it has a coherent partial");
  }
  if (!(D > R)) return GADEP_OK;  // inside the sphere: the whole sphere
  for (int a = 0; a < 3; ++a) sr.dir[a] = static_cast<float>((c[a] - src.pos_mm[a]) / D);
  const double cc = sqrt(1.0 - (R / D) * (R / D));
  sr.cone_cos = static_cast<float>(cc);
  // the weight of the directions the kernel samples: those with cos >= the
  // FP32 cosine it is given
  weight = 0.5 * (1.0 - static_cast<double>(sr.cone_cos));
  return GADEP_OK;
}

gadep_status plan_jobs(gadep_ctx* ctx, const gadep_job* jobs, int32_t n_jobs,
                       const gadep_tally* out, bool grad, Plan& P) {
  if (!jobs || n_jobs <= 0) return set_err(ctx, GADEP_E_ARG, "no jobs");
  if (!ctx->grid_set) return set_err(ctx, GADEP_E_STATE, "run before gadep_set_xs");
  P = Plan();
  P.grad = grad;
  const int64_t chunk = 64 * ctx->claim;
  int64_t chunks = 0;
  int32_t unit_index = 0;
  for (int32_t j = 0; j < n_jobs; ++j) {
    const gadep_job& J = jobs[j];
    if (J.scene < 0 || J.scene >= static_cast<int32_t>(ctx->scenes.size()) || !ctx->scenes[J.scene] ||
        !ctx->scenes[J.scene]->loaded)
      return set_err(ctx, GADEP_E_STATE, "job " + std::to_string(j) + ": scene not loaded");
    const Scene& sc = *ctx->scenes[J.scene];
    gadep_status s = check_source(ctx, J.src, sc);
    if (s) return s;
    if (J.n_histories < 0 || J.first_history < 0)
      return set_err(ctx, GADEP_E_ARG, "job: negative history count or first history");
    if (J.n_energies < 1 || J.n_energies > 65536)
      return set_err(ctx, GADEP_E_ARG, "job: n_energies must be in [1, 65536]");
    if (J.src.n_lines == 0 && !J.energies_keV)
      return set_err(ctx, GADEP_E_ARG, "job: energies_keV is NULL for a mono-energetic source");
    if (J.src.n_lines > 0 && J.n_energies != 1)
      return set_err(ctx, GADEP_E_ARG, "job: a line source takes n_energies = 1");
    if (J.stream > 0xFFFFu) return set_err(ctx, GADEP_E_ARG, "job: stream id above 65535");
    if (J.n_scales < 0 || J.n_scales > GADEP_MAX_GROUPS || (J.n_scales > 0 && !J.scales))
      return set_err(ctx, GADEP_E_ARG, "job: bad scales");
    float sc8[GADEP_MAX_GROUPS];
    for (int g = 0; g < GADEP_MAX_GROUPS; ++g) sc8[g] = 1.0f;
    for (int g = 0; g < J.n_scales; ++g) {
      if (!(J.scales[g] > 0) || !std::isfinite(J.scales[g]))
        return set_err(ctx, GADEP_E_ARG, "job: scales must be positive");
      sc8[g] = J.scales[g];
    }
    // region table of this job
    const int32_t roff = static_cast<int32_t>(P.regions.size());
    for (int32_t r = 0; r < sc.n_regions; ++r) {
      gadep_region R = sc.regions[r];
      if (J.region_material_override) R.material = J.region_material_override[r];
      if (J.region_density_override) R.density_g_cm3 = J.region_density_override[r];
      if (R.material < 0 || R.material >= static_cast<int32_t>(ctx->mats.size()) ||
          !ctx->mats[R.material].set)
        return set_err(ctx, GADEP_E_STATE,
                       "region " + std::to_string(r) + ": material has no cross sections");
      if (!(R.density_g_cm3 >= 0) || !std::isfinite(R.density_g_cm3))
        return set_err(ctx, GADEP_E_ARG, "region density must be finite and >= 0");
      if (R.scale_group < -1 || R.scale_group >= GADEP_MAX_GROUPS)
        return set_err(ctx, GADEP_E_ARG, "region scale group out of range");
      const float s = R.scale_group >= 0 ? sc8[R.scale_group] : 1.0f;
      RegionRec rr;
      rr.mult = static_cast<float>(0.1 * R.density_g_cm3 * s);
      rr.inv_scale = 1.0f / s;
      rr.material = R.material;
      rr.bits = (R.scale_group >= 0 ? R.scale_group : 0xFF) | ((R.flags & GADEP_ACTIVE) ? 0x100 : 0);
      P.regions.push_back(rr);
    }
    // source
    SourceRec sr{};
    sr.kind = J.src.kind;
    for (int a = 0; a < 3; ++a) sr.pos[a] = J.src.pos_mm[a];
    if (J.src.kind == GADEP_SRC_BEAM) {
      double n = sqrt(double(J.src.dir[0]) * J.src.dir[0] + double(J.src.dir[1]) * J.src.dir[1] +
                      double(J.src.dir[2]) * J.src.dir[2]);
      for (int a = 0; a < 3; ++a) sr.dir[a] = static_cast<float>(J.src.dir[a] / n);
    }
    sr.r_in = J.src.r_in_mm;
    sr.r_out = J.src.r_out_mm;
    sr.h = J.src.h_mm;
    sr.region = J.src.region;
    sr.n_lines = J.src.n_lines;
    sr.line_off = static_cast<int32_t>(P.lines.size() / 2);
    if (J.src.n_lines > 0) {
      double tot = 0;
      for (int i = 0; i < J.src.n_lines; ++i) tot += J.src.line_prob[i];
      double cum = 0;
      for (int i = 0; i < J.src.n_lines; ++i) {
        gadep_status es = check_energy(ctx, J.src.line_keV[i]);
        if (es) return es;
        cum += J.src.line_prob[i];
        P.lines.push_back(J.src.line_keV[i]);
        P.lines.push_back(static_cast<float>(i == J.src.n_lines - 1 ? 2.0 : cum / tot));
      }
    }
    double weight = 1.0;
    if ((s = cone_setup(ctx, sc, J.src, P.regions.data() + roff, sr, weight))) return s;
    const int32_t src_idx = static_cast<int32_t>(P.sources.size());
    P.sources.push_back(sr);
    P.depth = std::max(P.depth, sc.depth);
    for (int32_t e = 0; e < J.n_energies; ++e) {
      UnitRec u{};
      u.n = J.n_histories;
      u.first = J.first_history;
      double E = J.src.n_lines > 0 ? 0.0 : J.energies_keV[e];
      if (J.src.n_lines == 0) {
        gadep_status es = check_energy(ctx, E);
        if (es) return es;
      }
      u.energy = static_cast<float>(E);
      u.source = src_idx;
      u.scene = J.scene;
      u.region_off = roff;
      u.stream = (J.stream << 16) | static_cast<uint32_t>(e);
      u.src_region = 0;
      u.n_groups = grad ? GADEP_MAX_GROUPS : 0;
      u.flags = 0;
      if (sc.convex_exit && P.regions[roff].mult == 0.0f)
        u.flags = kUnitExitEscapes | (sc.n_planes > 0 && ctx->exit_planes ? kUnitExitPlanes : 0);
      P.units.push_back(u);
      P.unit_energy.push_back(E);
      P.unit_weight.push_back(weight);
      P.chunk_begin.push_back(chunks);
      chunks += (u.n + chunk - 1) / chunk;
      if (out) {
        const gadep_tally& t = out[unit_index];
        if (t.spectrum) {
          if (t.n_channels <= 0 || !(t.channel_keV > 0))
            return set_err(ctx, GADEP_E_ARG, "tally: spectrum needs n_channels > 0 and channel_keV > 0");
          if (P.spectrum && (t.n_channels != P.n_channels || t.channel_keV != P.channel_keV))
            return set_err(ctx, GADEP_E_ARG, "tally: all spectra of one run share their binning");
          P.spectrum = true;
          P.n_channels = t.n_channels;
          P.channel_keV = t.channel_keV;
        }
      }
      ++unit_index;
    }
  }
  P.chunk_begin.push_back(chunks);
  return GADEP_OK;
}

void to_tally(const unsigned long long* T, gadep_tally& t) {
  t.n_histories = T[kT_Hist];
  t.n_absorbed = T[kT_Absorbed];
  t.n_fep = T[kT_Fep];
  t.n_lost = T[kT_Lost];
  t.n_killed = T[kT_Killed];
  t.n_glitch = T[kT_Glitch];
  t.n_source_fail = T[kT_SrcFail];
  t.n_escape = T[kT_Hist] - T[kT_Absorbed] - T[kT_Lost] - T[kT_Killed] - T[kT_SrcFail];
  t.n_uncollided = t.n_escape - T[kT_CollEscape];
  t.edep_active_keV = static_cast<double>(static_cast<int64_t>(T[kT_EdepAct])) / kEnergyFix;
  t.edep_total_keV = static_cast<double>(static_cast<int64_t>(T[kT_EdepTot])) / kEnergyFix;
  t.e_escape_keV = static_cast<double>(static_cast<int64_t>(T[kT_EEsc])) / kEnergyFix;
  t.e_source_keV = static_cast<double>(static_cast<int64_t>(T[kT_ESrc])) / kEnergyFix;
  t.spectrum_overflow = T[kT_SpecOvf];
}

// The transport kernel the context's options select: the pooled kernel (one
// wavefront per block) or the per-lane one (ctx->block threads).  grid <= 0:
// from the occupancy of the kernel on every compute unit.
hipError_t pick_grid(const gadep_ctx* ctx, int variant, int depth, int pair, int* grid) {
  if (ctx->grid > 0) {
    *grid = static_cast<int>(ctx->grid);
    return hipSuccess;
  }
  int per_cu = 0;
  hipError_t e = ctx->pool ? pool_occupancy(variant, depth, pair, &per_cu)
                           : transport_occupancy(variant, static_cast<int>(ctx->block), depth, pair,
                                                 &per_cu);
  if (e != hipSuccess) return e;
  *grid = per_cu * ctx->n_cu;
  return hipSuccess;
}

hipError_t launch_transport(const gadep_ctx* ctx, const TransportParams& K, int variant, int grid,
                            hipStream_t s) {
  return ctx->pool ? pool_launch(K, variant, grid, s)
                   : transport_launch(K, variant, grid, static_cast<int>(ctx->block), s);
}

// shader clock of the launch whose tally rows are T[n_units][kT_Slots]
void note_clock(gadep_ctx* ctx, const unsigned long long* T, int32_t n_units) {
  double core = 0, ref = 0;
  for (int32_t u = 0; u < n_units; ++u) {
    core += static_cast<double>(T[static_cast<int64_t>(u) * kT_Slots + kT_ClkCore]);
    ref += static_cast<double>(T[static_cast<int64_t>(u) * kT_Slots + kT_ClkRef]);
  }
  ctx->last_sclk_mhz = ref > 0 ? core / ref * ctx->ref_clock_khz * 1e-3 : -1.0;
}

gadep_status execute(gadep_ctx* ctx, Plan& P, uint64_t seed, gadep_tally* out, double* grads,
                     double* grads_var, int32_t n_grad_cols, float* elapsed_ms = nullptr) {
  gadep_status s = sync_xs(ctx);
  if (s) return s;
  const int32_t nu = static_cast<int32_t>(P.units.size());
  // scene table
  std::vector<SceneRec> st(ctx->scenes.size());
  for (size_t i = 0; i < ctx->scenes.size(); ++i) {
    if (!ctx->scenes[i] || !ctx->scenes[i]->loaded) continue;
    fill_scene_rec(ctx->scenes, *ctx->scenes[i], st[i]);
  }
  if ((s = upload(ctx, ctx->scene_tab, st.data(), st.size() * sizeof(SceneRec), "scene table"))) return s;
  if ((s = upload(ctx, ctx->units, P.units.data(), P.units.size() * sizeof(UnitRec), "unit table"))) return s;
  if ((s = upload(ctx, ctx->chunk_begin, P.chunk_begin.data(), P.chunk_begin.size() * sizeof(int64_t),
                  "chunk table")))
    return s;
  if ((s = upload(ctx, ctx->sources, P.sources.data(), P.sources.size() * sizeof(SourceRec), "sources"))) return s;
  if ((s = upload(ctx, ctx->lines, P.lines.data(), P.lines.size() * sizeof(float), "lines"))) return s;
  if ((s = upload(ctx, ctx->regions, P.regions.data(), P.regions.size() * sizeof(RegionRec), "regions"))) return s;
  const int64_t tally_words = static_cast<int64_t>(nu) * kT_Slots;
  const int64_t spec_words = P.spectrum ? static_cast<int64_t>(nu) * P.n_channels : 0;
  if ((s = ensure(ctx, ctx->tally, tally_words * 8, "tally"))) return s;
  if ((s = ensure(ctx, ctx->spectra, std::max<int64_t>(spec_words, 1) * 8, "spectra"))) return s;
  if ((s = ensure(ctx, ctx->cursor, std::max<int64_t>(nu, 8) * 8, "cursor"))) return s;

  TransportParams K{};
  K.units = static_cast<const UnitRec*>(ctx->units.p);
  K.chunk_begin = static_cast<const int64_t*>(ctx->chunk_begin.p);
  K.n_units = nu;
  K.chunk = static_cast<int32_t>(64 * ctx->claim);
  K.total_h = 0;
  for (const UnitRec& u : P.units) K.total_h += u.n;
  K.guide = static_cast<int32_t>(ctx->guide);
  K.scenes = static_cast<const SceneRec*>(ctx->scene_tab.p);
  K.sources = static_cast<const SourceRec*>(ctx->sources.p);
  K.lines = static_cast<const float*>(ctx->lines.p);
  K.regions = static_cast<const RegionRec*>(ctx->regions.p);
  K.xs = static_cast<const float*>(ctx->xs.p);
  K.n_e = ctx->nE;
  K.ln_e0 = static_cast<float>(ctx->lnE0);
  K.inv_dlne = static_cast<float>(1.0 / ctx->dlnE);
  K.e_cut = static_cast<float>(exp(ctx->lnE0));
  K.tally = static_cast<unsigned long long*>(ctx->tally.p);
  K.spectra = P.spectrum ? static_cast<unsigned long long*>(ctx->spectra.p) : nullptr;
  K.n_channels = P.n_channels;
  K.inv_channel_kev = P.spectrum ? 1.0f / P.channel_keV : 0.0f;
  K.cursor = static_cast<unsigned long long*>(ctx->cursor.p);
  K.seed_lo = static_cast<uint32_t>(seed);
  K.seed_hi = static_cast<uint32_t>(seed >> 32);
  K.max_steps = static_cast<int32_t>(ctx->max_steps);
  K.stack_depth = P.depth;
  K.period = static_cast<int32_t>(ctx->period);
  K.screen = static_cast<int32_t>(ctx->screen);
  K.pair = 0;
  for (const Material& m : ctx->mats)
    if (m.set && m.pair) K.pair = 1;
  if (ctx->electrons && ctx->pool)
    return set_err(ctx, GADEP_E_ARG, "electron tracks run with the per-lane kernel (GADEP_OPT_POOL = 0)");

  // the general kernel variant: volume or cone sources, or a unit whose scene
  // has overlays
  bool gen = false;
  for (const SourceRec& sr : P.sources) gen = gen || sr.kind == kCyl || sr.kind == kCone;
  for (const UnitRec& u : P.units) gen = gen || st[u.scene].roots2 != nullptr;
  const int variant =
      (P.grad ? 1 : 0) | (P.spectrum ? 2 : 0) | (ctx->counters ? 4 : 0) | (gen ? 8 : 0) |
      (K.pair ? 16 : 0) | (ctx->electrons ? 32 : 0);
  const int block = ctx->pool ? 64 : static_cast<int>(ctx->block);
  int grid = 0;
  HIP_TRY(pick_grid(ctx, variant, P.depth, K.pair, &grid), "occupancy");
  if (grid < 1) return set_err(ctx, GADEP_E_ARG, "block size does not fit (LDS or registers)");

  // graph key: everything baked into the captured launches
  std::vector<uint8_t> key(sizeof(TransportParams) + 5 * sizeof(int64_t));
  memcpy(key.data(), &K, sizeof K);
  int64_t extra[5] = {variant, grid, block, static_cast<int64_t>(tally_words + spec_words), ctx->pool};
  memcpy(key.data() + sizeof K, extra, sizeof extra);

  if (!ctx->ev0) HIP_TRY(hipEventCreate(&ctx->ev0), "event");
  if (!ctx->ev1) HIP_TRY(hipEventCreate(&ctx->ev1), "event");
  auto enqueue = [&]() -> hipError_t {
    hipError_t e = fill_u64(K.tally, tally_words, 0, ctx->stream);
    if (e == hipSuccess && spec_words) e = fill_u64(K.spectra, spec_words, 0, ctx->stream);
    if (e == hipSuccess) e = fill_u64(K.cursor, nu, 0, ctx->stream);
    if (e == hipSuccess)
      e = locate_units(static_cast<UnitRec*>(ctx->units.p), nu,
                       static_cast<const SceneRec*>(ctx->scene_tab.p),
                       static_cast<const SourceRec*>(ctx->sources.p), P.depth, ctx->stream);
    if (e == hipSuccess) e = launch_transport(ctx, K, variant, grid, ctx->stream);
    return e;
  };
  // the enqueue below is wrapped by two events: the launch duration
  if (!ctx->graphs) {
    hipError_t e = fill_u64(K.tally, tally_words, 0, ctx->stream);
    if (e == hipSuccess && spec_words) e = fill_u64(K.spectra, spec_words, 0, ctx->stream);
    if (e == hipSuccess) e = fill_u64(K.cursor, nu, 0, ctx->stream);
    if (e == hipSuccess)
      e = locate_units(static_cast<UnitRec*>(ctx->units.p), nu,
                       static_cast<const SceneRec*>(ctx->scene_tab.p),
                       static_cast<const SourceRec*>(ctx->sources.p), P.depth, ctx->stream);
    HIP_TRY(e, "set-up kernels");
  }
  HIP_TRY(hipEventRecord(ctx->ev0, ctx->stream), "event");
  if (ctx->graphs) {
    if (!ctx->graph || ctx->graph_key != key) {
      if (ctx->graph) {
        (void)hipGraphExecDestroy(ctx->graph);
        ctx->graph = nullptr;
      }
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal), "capture");
      hipError_t ce = enqueue();
      hipError_t ee = hipStreamEndCapture(ctx->stream, &g);
      if (ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_err(ctx, ce, "capture transport");
      }
      HIP_TRY(ee, "end capture");
      hipError_t ie = hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIP_TRY(ie, "graph instantiate");
      ctx->graph_key = key;
    }
    HIP_TRY(hipGraphLaunch(ctx->graph, ctx->stream), "graph launch");
  } else {
    HIP_TRY(launch_transport(ctx, K, variant, grid, ctx->stream), "transport launch");
  }
  HIP_TRY(hipEventRecord(ctx->ev1, ctx->stream), "event");

  // read back
  const size_t need = static_cast<size_t>(tally_words) * 8;
  if (ctx->h_tally_cap < need) {
    if (ctx->h_tally) (void)hipHostFree(ctx->h_tally);
    ctx->h_tally = nullptr;
    HIP_TRY(hipHostMalloc(&ctx->h_tally, need), "pinned tally");
    ctx->h_tally_cap = need;
  }
  HIP_TRY(hipMemcpyAsync(ctx->h_tally, K.tally, need, hipMemcpyDeviceToHost, ctx->stream), "tally D2H");
  std::vector<unsigned long long> spec;
  if (spec_words) {
    spec.resize(static_cast<size_t>(spec_words));
    HIP_TRY(hipMemcpyAsync(spec.data(), K.spectra, spec_words * 8, hipMemcpyDeviceToHost, ctx->stream),
            "spectra D2H");
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream), "transport");
  {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1), "event time");
    ctx->last_ms = ms;
    if (elapsed_ms) *elapsed_ms = ms;
  }

  const unsigned long long* T = static_cast<const unsigned long long*>(ctx->h_tally);
  note_clock(ctx, T, nu);
  gadep_counters cnt{};
  cnt.wavefronts = static_cast<uint64_t>(grid) * (block / 64);
  for (int32_t u = 0; u < nu; ++u) {
    const unsigned long long* Tu = T + static_cast<int64_t>(u) * kT_Slots;
    cnt.wave_cycles += Tu[kT_ClkCore];
    if (out) {
      gadep_tally& t = out[u];
      to_tally(Tu, t);
      t.weight = P.unit_weight[u];
      if (t.spectrum && spec_words)
        memcpy(t.spectrum, spec.data() + static_cast<int64_t>(u) * P.n_channels, P.n_channels * 8);
    }
    if (P.grad && (grads || grads_var)) {
      const double n = static_cast<double>(Tu[kT_Hist]);
      for (int32_t g = 0; g < n_grad_cols; ++g) {
        const double m1 = n > 0 ? static_cast<double>(static_cast<int64_t>(Tu[kT_FepScore + g])) / kScoreFix / n : 0.0;
        const double q = static_cast<double>(Tu[kT_FepScore2 + g]) +
                         static_cast<double>(Tu[kT_FepScore2Lo + g]) / (1 << kScore2LoBits);
        const double m2 = n > 0 ? q / kScore2Fix / n : 0.0;
        if (grads) grads[static_cast<int64_t>(u) * n_grad_cols + g] = m1;
        if (grads_var) grads_var[static_cast<int64_t>(u) * n_grad_cols + g] = n > 1 ? std::max(0.0, m2 - m1 * m1) / n : 0.0;
      }
    }
    const unsigned long long* ev = Tu + kT_Ev;
    cnt.segments += ev[kEv_Segments];
    cnt.crossings += ev[kEv_Crossings];
    cnt.node_visits += ev[kEv_NodeVisits];
    cnt.tri_tests += ev[kEv_TriTests];
    cnt.photo += ev[kEv_Photo];
    cnt.compton += ev[kEv_Compton];
    cnt.coherent += ev[kEv_Coherent];
    cnt.rng_calls += ev[kEv_Rng];
    cnt.locates += ev[kEv_Locates];
    cnt.emissions += ev[kEv_Emissions];
    cnt.plane_tests += ev[kEv_PlaneTests];
    cnt.iterations += ev[kEv_Iters];
    cnt.iterations_node += ev[kEv_ItersNode];
    cnt.iterations_facet += ev[kEv_ItersTri];
    cnt.passes += ev[kEv_Passes];
    cnt.cycles_outcome += ev[kEv_CycOutcome];
    cnt.cycles_refill += ev[kEv_CycRefill];
    cnt.cycles_launch += ev[kEv_CycLaunch];
    cnt.cycles_setup += ev[kEv_CycSetup];
    cnt.cycles_traversal += ev[kEv_CycTrav];
    cnt.box_tests += ev[kEv_BoxTests];
    cnt.pair += ev[kEv_Pair];
    cnt.electrons += ev[kEv_Electrons];
    cnt.cone_tests += ev[kEv_ConeTests];
  }
  if (ctx->counters) {
    ctx->last_counters = cnt;
    ctx->have_counters = true;
  }
  return GADEP_OK;
}

gadep_job single_job(const gadep_source* src, const double* energies, int32_t n_energies,
                     int64_t n, int64_t first, const float* scales, int32_t n_scales) {
  gadep_job j{};
  j.src = *src;
  j.energies_keV = energies;
  j.n_energies = n_energies;
  j.n_histories = n;
  j.first_history = first;
  j.scales = scales;
  j.n_scales = n_scales;
  j.scene = 0;
  j.stream = 0;
  return j;
}

}  // namespace

// ============================================================================
// C interface

extern "C" {

gadep_status gadep_create(int device, void* hip_stream, gadep_ctx** out) {
  if (!out) return GADEP_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return GADEP_E_HIP;
  if (device < 0 || device >= n) return GADEP_E_ARG;
  auto* ctx = new gadep_ctx();
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return GADEP_E_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete ctx;
    return GADEP_E_HIP;
  }
  ctx->n_cu = prop.multiProcessorCount;
  {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
      ctx->ref_clock_khz = khz;
  }
  // the no-allocation run's scratch: this device's copy of the array (the
  // device is current), and its host staging
  if (scratch_address(device, &ctx->scratch) != hipSuccess) ctx->scratch = nullptr;
  ctx->na = std::make_unique<NoAllocHost>();
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&ctx->stream) != hipSuccess) {
      delete ctx;
      return GADEP_E_HIP;
    }
    ctx->own_stream = true;
  }
  *out = ctx;
  return GADEP_OK;
}

void gadep_destroy(gadep_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
  for (auto& sc : ctx->scenes)
    if (sc) {
      if (sc->d_nodes) (void)hipFree(sc->d_nodes);
      if (sc->d_tris) (void)hipFree(sc->d_tris);
      if (sc->d_planes) (void)hipFree(sc->d_planes);
      if (sc->d_roots) (void)hipFree(sc->d_roots);
      if (sc->d_slots) (void)hipFree(sc->d_slots);
      if (sc->d_roots2) (void)hipFree(sc->d_roots2);
    }
  for (DevBuf* b : {&ctx->xs, &ctx->units, &ctx->chunk_begin, &ctx->scene_tab, &ctx->sources,
                    &ctx->lines, &ctx->regions, &ctx->tally, &ctx->spectra, &ctx->cursor})
    free_buf(*b);
  if (ctx->h_tally) (void)hipHostFree(ctx->h_tally);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* gadep_last_error(const gadep_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gadep_status gadep_set_option(gadep_ctx* ctx, int32_t option, int64_t v) {
  if (!ctx) return GADEP_E_ARG;
  switch (option) {
    case GADEP_OPT_MAX_STEPS:
      if (v < 1 || v > (1 << 30)) return set_err(ctx, GADEP_E_ARG, "max_steps out of range");
      ctx->max_steps = v;
      return GADEP_OK;
    case GADEP_OPT_BLOCK:
      if (v < 64 || v > 256 || v % 64) return set_err(ctx, GADEP_E_ARG, "block must be 64, 128, 192 or 256");
      ctx->block = v;
      return GADEP_OK;
    case GADEP_OPT_PERIOD:
      if (v < 0 || v > 64) return set_err(ctx, GADEP_E_ARG, "park threshold must be in [0, 64]");
      ctx->period = v;
      return GADEP_OK;
    case GADEP_OPT_CLAIM:
      if (v < 1 || v > (1 << 20)) return set_err(ctx, GADEP_E_ARG, "claim out of range");
      ctx->claim = v;
      return GADEP_OK;
    case GADEP_OPT_VALIDATE:
      ctx->validate = v ? 1 : 0;
      return GADEP_OK;
    case GADEP_OPT_MIN_GAP_NM:
      if (v < 0) return set_err(ctx, GADEP_E_ARG, "min gap must be >= 0");
      ctx->min_gap_nm = v;
      return GADEP_OK;
    case GADEP_OPT_GRAPHS:
      ctx->graphs = v ? 1 : 0;
      return GADEP_OK;
    case GADEP_OPT_COUNTERS:
      ctx->counters = v ? 1 : 0;
      return GADEP_OK;
    case GADEP_OPT_GRID:
      if (v < 0 || v > (1 << 20)) return set_err(ctx, GADEP_E_ARG, "grid out of range");
      ctx->grid = v;
      return GADEP_OK;
    case GADEP_OPT_EXIT_PLANES:
      ctx->exit_planes = v ? 1 : 0;
      return GADEP_OK;
    case GADEP_OPT_SPLIT_PCT:
      if (v < 0 || v > 1600) return set_err(ctx, GADEP_E_ARG, "split budget must be in [0, 1600] %");
      ctx->split_pct = v;
      return GADEP_OK;
    case GADEP_OPT_SCREEN:
      ctx->screen = v ? 1 : 0;
      return GADEP_OK;
    case GADEP_OPT_POOL:
      ctx->pool = v ? 1 : 0;
      return GADEP_OK;
    case GADEP_OPT_ELECTRONS:
      ctx->electrons = v ? 1 : 0;
      return GADEP_OK;
    case GADEP_OPT_GUIDE:
      if (v < 0 || v > 16) return set_err(ctx, GADEP_E_ARG, "guide must be in [0, 16]");
      ctx->guide = v;
      return GADEP_OK;
    default:
      return set_err(ctx, GADEP_E_ARG, "unknown option");
  }
}

gadep_status gadep_get_option(const gadep_ctx* ctx, int32_t option, int64_t* v) {
  if (!ctx || !v) return GADEP_E_ARG;
  switch (option) {
    case GADEP_OPT_MAX_STEPS: *v = ctx->max_steps; return GADEP_OK;
    case GADEP_OPT_BLOCK: *v = ctx->block; return GADEP_OK;
    case GADEP_OPT_PERIOD: *v = ctx->period; return GADEP_OK;
    case GADEP_OPT_CLAIM: *v = ctx->claim; return GADEP_OK;
    case GADEP_OPT_VALIDATE: *v = ctx->validate; return GADEP_OK;
    case GADEP_OPT_MIN_GAP_NM: *v = ctx->min_gap_nm; return GADEP_OK;
    case GADEP_OPT_GRAPHS: *v = ctx->graphs; return GADEP_OK;
    case GADEP_OPT_COUNTERS: *v = ctx->counters; return GADEP_OK;
    case GADEP_OPT_GRID: *v = ctx->grid; return GADEP_OK;
    case GADEP_OPT_EXIT_PLANES: *v = ctx->exit_planes; return GADEP_OK;
    case GADEP_OPT_SPLIT_PCT: *v = ctx->split_pct; return GADEP_OK;
    case GADEP_OPT_SCREEN: *v = ctx->screen; return GADEP_OK;
    case GADEP_OPT_POOL: *v = ctx->pool; return GADEP_OK;
    case GADEP_OPT_GUIDE: *v = ctx->guide; return GADEP_OK;
    case GADEP_OPT_ELECTRONS: *v = ctx->electrons; return GADEP_OK;
    default: return GADEP_E_ARG;
  }
}

gadep_status gadep_load_scene(gadep_ctx* ctx, int32_t scene, const float* xyz, int64_t nv,
                              const int32_t* tri, const int32_t* tri_region, int64_t nt,
                              const gadep_region* regions, int32_t n_regions) {
  if (!ctx) return GADEP_E_ARG;
  if (scene < 0 || scene >= GADEP_MAX_SCENES) return set_err(ctx, GADEP_E_ARG, "scene slot out of range");
  if (!regions) return set_err(ctx, GADEP_E_ARG, "regions is NULL");
  for (int32_t r = 0; r < n_regions; ++r) {
    const gadep_region& R = regions[r];
    if (R.material < 0 || !(R.density_g_cm3 >= 0) || !std::isfinite(R.density_g_cm3) ||
        R.scale_group < -1 || R.scale_group >= GADEP_MAX_GROUPS)
      return set_err(ctx, GADEP_E_ARG, "region " + std::to_string(r) + ": bad material, density or group");
  }
  PreparedMesh pm;
  std::string err;
  int rc = prepare_mesh(xyz, nv, tri, tri_region, nt, n_regions, ctx->min_gap_nm * 1e-6,
                        ctx->validate != 0, 0, ctx->split_pct * 0.01, pm, err);
  if (rc != GADEP_OK) return set_err(ctx, static_cast<gadep_status>(rc), err);
  if (static_cast<int32_t>(ctx->scenes.size()) <= scene) ctx->scenes.resize(scene + 1);
  if (!ctx->scenes[scene]) ctx->scenes[scene].reset(new Scene());
  Scene& sc = *ctx->scenes[scene];
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "sync");
  if (sc.d_nodes) (void)hipFree(sc.d_nodes);
  if (sc.d_tris) (void)hipFree(sc.d_tris);
  if (sc.d_planes) (void)hipFree(sc.d_planes);
  if (sc.d_roots) (void)hipFree(sc.d_roots);
  if (sc.d_slots) (void)hipFree(sc.d_slots);
  if (sc.d_roots2) (void)hipFree(sc.d_roots2);
  sc.d_nodes = sc.d_tris = sc.d_planes = sc.d_roots = sc.d_slots = sc.d_roots2 = nullptr;
  sc.loaded = false;
  sc.base = -1;
  sc.root_all2 = -1;
  // overlays loaded on this slot referred to the arrays just freed
  for (auto& o : ctx->scenes)
    if (o && o->base == scene) o->loaded = false;
  // the transport BVHs follow the plain one, their indices shifted to match
  std::vector<BvhNode> nodes = pm.nodes;
  const int32_t n_plain = static_cast<int32_t>(pm.nodes.size());
  for (BvhNode nd : pm.trans_nodes) {
    for (int c = 0; c < 2; ++c) {
      if (nd.child[c] >= 0) {
        nd.child[c] += n_plain;
      } else {
        const int32_t x = ~nd.child[c];
        nd.child[c] = leaf_code((x >> 3) + nt, x & 7);
      }
    }
    nodes.push_back(nd);
  }
  // one record per facet (caller order); the slots of every BVH name them
  std::vector<TriRec> tris(static_cast<size_t>(nt));
  for (const TriRec& r : pm.tris) tris[r.orig] = r;
  std::vector<int32_t> slots(pm.order);
  for (const TriRec& r : pm.trans_tris) slots.push_back(r.orig);
  std::vector<int32_t> roots(static_cast<size_t>(n_regions), kDone);
  for (int32_t r = 0; r < n_regions; ++r)
    if (pm.trans_root[r] >= 0) roots[r] = pm.trans_root[r] + n_plain;
  const int32_t n_planes = static_cast<int32_t>(pm.planes.size() / 4);
  HIP_TRY(hipMalloc(&sc.d_nodes, nodes.size() * sizeof(BvhNode)), "alloc nodes");
  HIP_TRY(hipMalloc(&sc.d_tris, tris.size() * sizeof(TriRec)), "alloc facets");
  HIP_TRY(hipMemcpy(sc.d_nodes, nodes.data(), nodes.size() * sizeof(BvhNode), hipMemcpyHostToDevice),
          "upload nodes");
  HIP_TRY(hipMemcpy(sc.d_tris, tris.data(), tris.size() * sizeof(TriRec), hipMemcpyHostToDevice),
          "upload facets");
  HIP_TRY(hipMalloc(&sc.d_slots, slots.size() * sizeof(int32_t)), "alloc slots");
  HIP_TRY(hipMemcpy(sc.d_slots, slots.data(), slots.size() * sizeof(int32_t), hipMemcpyHostToDevice),
          "upload slots");
  HIP_TRY(hipMalloc(&sc.d_roots, roots.size() * sizeof(int32_t)), "alloc roots");
  HIP_TRY(hipMemcpy(sc.d_roots, roots.data(), roots.size() * sizeof(int32_t), hipMemcpyHostToDevice),
          "upload roots");
  if (n_planes > 0) {
    HIP_TRY(hipMalloc(&sc.d_planes, pm.planes.size() * sizeof(float)), "alloc planes");
    HIP_TRY(hipMemcpy(sc.d_planes, pm.planes.data(), pm.planes.size() * sizeof(float),
                      hipMemcpyHostToDevice),
            "upload planes");
  }
  sc.n_planes = n_planes;
  sc.outer_root = n_planes > 0 && pm.trans_root[n_regions] >= 0 ? pm.trans_root[n_regions] + n_plain
                                                                : kDone;
  sc.outer_region = pm.outer_region;
  for (int a = 0; a < 3; ++a) {
    sc.trans_lo[a] = pm.trans_lo[a];
    sc.trans_hi[a] = pm.trans_hi[a];
    sc.outer_lo[a] = pm.outer_lo[a];
    sc.outer_hi[a] = pm.outer_hi[a];
  }
  if (n_planes > 0 && pm.trans_lo[0] <= pm.trans_hi[0]) {
    for (int a = 0; a < 3; ++a) {
      sc.inner_lo[a] = pm.trans_lo[a];
      sc.inner_hi[a] = pm.trans_hi[a];
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      sc.inner_lo[a] = INFINITY;
      sc.inner_hi[a] = -INFINITY;
    }
    for (int64_t f = 0; f < 3 * nt; ++f) {
      const float* v = xyz + 3 * static_cast<int64_t>(tri[f]);
      for (int a = 0; a < 3; ++a) {
        sc.inner_lo[a] = std::min<double>(sc.inner_lo[a], v[a]);
        sc.inner_hi[a] = std::max<double>(sc.inner_hi[a], v[a]);
      }
    }
  }
  sc.regions.assign(regions, regions + n_regions);
  sc.n_regions = n_regions;
  sc.depth = std::max(pm.depth, pm.trans_depth);
  sc.n_tri = nt;
  sc.n_nodes = static_cast<int64_t>(pm.nodes.size());
  sc.convex_exit = pm.convex_exit;
  sc.h_xyz.assign(xyz, xyz + 3 * nv);
  sc.h_tri.assign(tri, tri + 3 * nt);
  sc.h_reg.assign(tri_region, tri_region + nt);
  sc.h_roots = roots;
  sc.arena_nodes = static_cast<int64_t>(nodes.size());
  sc.arena_slots = static_cast<int64_t>(slots.size());
  sc.arena_tris = nt;
  sc.loaded = true;
  if (ctx->graph) {
    (void)hipGraphExecDestroy(ctx->graph);
    ctx->graph = nullptr;
    ctx->graph_key.clear();
  }
  return GADEP_OK;
}

gadep_status gadep_load_overlay(gadep_ctx* ctx, int32_t scene, int32_t base_scene,
                                int32_t host_region, const float* xyz, int64_t nv,
                                const int32_t* tri, const int32_t* tri_region, int64_t nt,
                                const gadep_region* regions, int32_t n_regions) {
  if (!ctx) return GADEP_E_ARG;
  if (scene < 0 || scene >= GADEP_MAX_SCENES || base_scene < 0 || base_scene >= GADEP_MAX_SCENES ||
      scene == base_scene)
    return set_err(ctx, GADEP_E_ARG, "overlay: scene slots out of range or equal");
  if (base_scene >= static_cast<int32_t>(ctx->scenes.size()) || !ctx->scenes[base_scene] ||
      !ctx->scenes[base_scene]->loaded || ctx->scenes[base_scene]->base >= 0)
    return set_err(ctx, GADEP_E_STATE, "overlay: the base scene is not a loaded detector scene");
  if (!xyz || !tri || !tri_region || !regions || nv <= 0 || nt <= 0 || n_regions < 2)
    return set_err(ctx, GADEP_E_ARG, "overlay: empty mesh or region table");
  Scene& B = *ctx->scenes[base_scene];
  const int32_t nb = B.n_regions;
  const int32_t n_comb = nb + n_regions - 1;
  if (host_region < 0 || host_region >= nb)
    return set_err(ctx, GADEP_E_ARG, "overlay: host region out of range");
  if (n_comb > kMaxRegions)
    return set_err(ctx, GADEP_E_ARG, "overlay: more than 64 regions with the base scene's");
  for (int32_t r = 1; r < n_regions; ++r) {
    const gadep_region& R = regions[r];
    if (R.material < 0 || !(R.density_g_cm3 >= 0) || !std::isfinite(R.density_g_cm3) ||
        R.scale_group < -1 || R.scale_group >= GADEP_MAX_GROUPS)
      return set_err(ctx, GADEP_E_ARG, "overlay region " + std::to_string(r) + ": bad material, density or group");
  }
  for (int64_t f = 0; f < nt; ++f)
    if (tri_region[f] < 1 || tri_region[f] >= n_regions)
      return set_err(ctx, GADEP_E_ARG, "overlay: facet region out of range (1..n_regions-1)");
  // overlay region k >= 1 is region nb + k - 1 of the combined scene; its
  // region 0 (outside every overlay shell) is the base's host region
  auto comb = [&](int32_t k) { return k == 0 ? host_region : nb + k - 1; };
  PreparedMesh po;
  std::string err;
  int rc = prepare_mesh(xyz, nv, tri, tri_region, nt, n_regions, ctx->min_gap_nm * 1e-6, false, 0,
                        ctx->split_pct * 0.01, po, err);
  if (rc != GADEP_OK) return set_err(ctx, static_cast<gadep_status>(rc), "overlay: " + err);
  if (ctx->validate) {
    // the detector and the overlay together: closed, oriented, apart from each
    // other, and each outermost overlay shell directly inside the host region
    const int64_t nvb = static_cast<int64_t>(B.h_xyz.size() / 3), ntb = B.n_tri;
    std::vector<float> cx(B.h_xyz);
    cx.insert(cx.end(), xyz, xyz + 3 * nv);
    std::vector<int32_t> ct(B.h_tri), cr(B.h_reg);
    for (int64_t i = 0; i < 3 * nt; ++i) ct.push_back(tri[i] + static_cast<int32_t>(nvb));
    for (int64_t f = 0; f < nt; ++f) cr.push_back(comb(tri_region[f]));
    PreparedMesh pc;
    rc = prepare_mesh(cx.data(), nvb + nv, ct.data(), cr.data(), ntb + nt, n_comb,
                      ctx->min_gap_nm * 1e-6, true, 0, 0.0, pc, err);
    if (rc != GADEP_OK) return set_err(ctx, static_cast<gadep_status>(rc), "overlay on the detector: " + err);
    for (int64_t f = 0; f < nt; ++f)
      if (pc.outside[ntb + f] != comb(po.outside[f]))
        return set_err(ctx, GADEP_E_TOPOLOGY, "overlay: its shells do not lie in region " +
                                                  std::to_string(host_region) + " of the base scene");
  }
  // the overlay's records, placed after the detector's in its arrays
  const int64_t NO = B.arena_nodes, SO = B.arena_slots, TO = B.arena_tris;
  const int32_t n_plain = static_cast<int32_t>(po.nodes.size());
  if (SO + nt + static_cast<int64_t>(po.trans_tris.size()) >= (int64_t(1) << 28) ||
      NO + n_plain + static_cast<int64_t>(po.trans_nodes.size()) >= (int64_t(1) << 30))
    return set_err(ctx, GADEP_E_ARG, "overlay: the detector's arrays are full");
  std::vector<BvhNode> nodes;
  nodes.reserve(po.nodes.size() + po.trans_nodes.size());
  for (BvhNode nd : po.nodes) {
    for (int c = 0; c < 2; ++c) {
      if (nd.child[c] >= 0) {
        nd.child[c] += static_cast<int32_t>(NO);
      } else {
        const int32_t x = ~nd.child[c];
        nd.child[c] = leaf_code((x >> 3) + SO, x & 7);
      }
    }
    nodes.push_back(nd);
  }
  for (BvhNode nd : po.trans_nodes) {
    for (int c = 0; c < 2; ++c) {
      if (nd.child[c] >= 0) {
        nd.child[c] += static_cast<int32_t>(NO) + n_plain;
      } else {
        const int32_t x = ~nd.child[c];
        nd.child[c] = leaf_code((x >> 3) + SO + nt, x & 7);
      }
    }
    nodes.push_back(nd);
  }
  std::vector<TriRec> tris(static_cast<size_t>(nt));
  for (TriRec r : po.tris) {
    const int32_t in = static_cast<int32_t>(r.regions & 0xFFFFu), out = static_cast<int32_t>(r.regions >> 16);
    r.regions = static_cast<uint32_t>(comb(in)) | (static_cast<uint32_t>(comb(out)) << 16);
    const int32_t f = r.orig;
    r.orig = static_cast<int32_t>(B.n_tri) + f;  // the facet's number in the combined scene
    tris[f] = r;
  }
  std::vector<int32_t> slots;
  slots.reserve(nt + po.trans_tris.size());
  for (int32_t f : po.order) slots.push_back(static_cast<int32_t>(TO) + f);
  for (const TriRec& r : po.trans_tris) slots.push_back(static_cast<int32_t>(TO) + r.orig);
  std::vector<int32_t> roots(B.h_roots), roots2(static_cast<size_t>(n_comb), kDone);
  for (int32_t k = 1; k < n_regions; ++k)
    roots.push_back(po.trans_root[k] >= 0 ? po.trans_root[k] + static_cast<int32_t>(NO) + n_plain : kDone);
  if (po.trans_root[0] >= 0) roots2[host_region] = po.trans_root[0] + static_cast<int32_t>(NO) + n_plain;

  HIP_TRY(hipSetDevice(ctx->device), "set device");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "sync");
  // grow the detector's arrays by the overlay's records
  auto grow = [&](void*& d, int64_t old_count, size_t elem, const void* add, int64_t add_count,
                  const char* what) -> gadep_status {
    void* n = nullptr;
    HIP_TRY(hipMalloc(&n, (old_count + add_count) * elem), what);
    if (old_count) {
      hipError_t e = hipMemcpy(n, d, old_count * elem, hipMemcpyDeviceToDevice);
      if (e != hipSuccess) {
        (void)hipFree(n);
        return hip_err(ctx, e, what);
      }
    }
    hipError_t e = hipMemcpy(static_cast<char*>(n) + old_count * elem, add, add_count * elem,
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(n);
      return hip_err(ctx, e, what);
    }
    (void)hipFree(d);
    d = n;
    return GADEP_OK;
  };
  gadep_status st;
  if ((st = grow(B.d_nodes, NO, sizeof(BvhNode), nodes.data(), static_cast<int64_t>(nodes.size()), "overlay nodes")))
    return st;
  B.arena_nodes = NO + static_cast<int64_t>(nodes.size());
  if ((st = grow(B.d_tris, TO, sizeof(TriRec), tris.data(), nt, "overlay facets"))) return st;
  B.arena_tris = TO + nt;
  if ((st = grow(B.d_slots, SO, sizeof(int32_t), slots.data(), static_cast<int64_t>(slots.size()), "overlay slots")))
    return st;
  B.arena_slots = SO + static_cast<int64_t>(slots.size());

  if (static_cast<int32_t>(ctx->scenes.size()) <= scene) ctx->scenes.resize(scene + 1);
  if (!ctx->scenes[scene]) ctx->scenes[scene].reset(new Scene());
  Scene& O = *ctx->scenes[scene];
  if (O.d_nodes) (void)hipFree(O.d_nodes);
  if (O.d_tris) (void)hipFree(O.d_tris);
  if (O.d_planes) (void)hipFree(O.d_planes);
  if (O.d_slots) (void)hipFree(O.d_slots);
  if (O.d_roots) (void)hipFree(O.d_roots);
  if (O.d_roots2) (void)hipFree(O.d_roots2);
  O = Scene();
  for (auto& o : ctx->scenes)
    if (o && o->base == scene) o->loaded = false;
  HIP_TRY(hipMalloc(&O.d_roots, roots.size() * sizeof(int32_t)), "overlay roots");
  HIP_TRY(hipMemcpy(O.d_roots, roots.data(), roots.size() * sizeof(int32_t), hipMemcpyHostToDevice), "overlay roots");
  HIP_TRY(hipMalloc(&O.d_roots2, roots2.size() * sizeof(int32_t)), "overlay roots");
  HIP_TRY(hipMemcpy(O.d_roots2, roots2.data(), roots2.size() * sizeof(int32_t), hipMemcpyHostToDevice), "overlay roots");
  O.base = base_scene;
  O.root_all2 = static_cast<int32_t>(NO);
  O.regions = B.regions;
  for (int32_t k = 1; k < n_regions; ++k) O.regions.push_back(regions[k]);
  O.n_regions = n_comb;
  O.depth = std::max(B.depth, std::max(po.depth, po.trans_depth));
  O.n_tri = B.n_tri + nt;
  O.n_nodes = static_cast<int64_t>(nodes.size());
  // an overlay in the world takes the world's single convex neighbour away
  const bool keep_exit = host_region != 0;
  O.convex_exit = keep_exit && B.convex_exit;
  O.n_planes = keep_exit ? B.n_planes : 0;
  O.outer_root = keep_exit ? B.outer_root : kDone;
  O.outer_region = B.outer_region;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < 3 * nt; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min<double>(lo[a], xyz[3 * static_cast<int64_t>(tri[i]) + a]);
      hi[a] = std::max<double>(hi[a], xyz[3 * static_cast<int64_t>(tri[i]) + a]);
    }
  for (int a = 0; a < 3; ++a) {
    O.outer_lo[a] = B.outer_lo[a];
    O.outer_hi[a] = B.outer_hi[a];
    const bool tb = B.trans_lo[0] <= B.trans_hi[0];
    O.trans_lo[a] = tb ? std::min<float>(B.trans_lo[a], static_cast<float>(lo[a])) : static_cast<float>(lo[a]);
    O.trans_hi[a] = tb ? std::max<float>(B.trans_hi[a], static_cast<float>(hi[a])) : static_cast<float>(hi[a]);
    O.inner_lo[a] = std::min(B.inner_lo[a], lo[a]);
    O.inner_hi[a] = std::max(B.inner_hi[a], hi[a]);
  }
  O.loaded = true;
  if (ctx->graph) {
    (void)hipGraphExecDestroy(ctx->graph);
    ctx->graph = nullptr;
    ctx->graph_key.clear();
  }
  return GADEP_OK;
}

gadep_status gadep_load_mesh(gadep_ctx* ctx, const float* xyz, int64_t nv, const int32_t* tri,
                             const int32_t* tri_region, int64_t nt, const gadep_region* regions,
                             int32_t n_regions) {
  return gadep_load_scene(ctx, 0, xyz, nv, tri, tri_region, nt, regions, n_regions);
}

gadep_status gadep_set_xs(gadep_ctx* ctx, int32_t material, double lnE0, double dlnE, int32_t nE,
                          const float* photo, const float* compton, const float* coherent,
                          const float* pair) {
  if (!ctx) return GADEP_E_ARG;
  if (material < 0 || material >= 1024) return set_err(ctx, GADEP_E_ARG, "material id out of range");
  if (nE < 2 || !(dlnE > 0) || !std::isfinite(lnE0) || !std::isfinite(dlnE))
    return set_err(ctx, GADEP_E_XS, "bad energy grid");
  if (ctx->grid_set && (lnE0 != ctx->lnE0 || dlnE != ctx->dlnE || nE != ctx->nE))
    return set_err(ctx, GADEP_E_XS, "every material must use the same energy grid");
  Material m;
  const float* src[4] = {photo, compton, coherent, pair};
  for (int i = 0; i < 4; ++i) {
    m.ln[i].assign(nE, -200.0f);
    if (!src[i]) continue;
    int npos = 0;
    for (int32_t k = 0; k < nE; ++k) {
      if (!(src[i][k] >= 0) || !std::isfinite(src[i][k]))
        return set_err(ctx, GADEP_E_XS, "cross sections must be finite and >= 0");
      npos += src[i][k] > 0;
    }
    if (npos == 0) continue;
    if (npos != nE) return set_err(ctx, GADEP_E_XS, "a partial must be all-positive or all-zero");
    for (int32_t k = 0; k < nE; ++k) m.ln[i][k] = logf(src[i][k]);
    if (i == 3) m.pair = true;
  }
  m.set = true;
  if (static_cast<int32_t>(ctx->mats.size()) <= material) ctx->mats.resize(material + 1);
  ctx->mats[material] = std::move(m);
  ctx->grid_set = true;
  ctx->lnE0 = lnE0;
  ctx->dlnE = dlnE;
  ctx->nE = nE;
  ctx->xs_dirty = true;
  // uploaded now, so that a run that cannot allocate finds them on the device
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  return sync_xs(ctx);
}

gadep_status gadep_set_scales(gadep_ctx* ctx, const float* scales, int32_t n) {
  if (!ctx) return GADEP_E_ARG;
  if (n < 0 || n > GADEP_MAX_GROUPS || (n > 0 && !scales)) return set_err(ctx, GADEP_E_ARG, "bad scales");
  for (int32_t g = 0; g < n; ++g)
    if (!(scales[g] > 0) || !std::isfinite(scales[g])) return set_err(ctx, GADEP_E_ARG, "scales must be > 0");
  for (int32_t g = 0; g < GADEP_MAX_GROUPS; ++g) ctx->scales[g] = g < n ? scales[g] : 1.0f;
  return GADEP_OK;
}

gadep_status gadep_run(gadep_ctx* ctx, const gadep_source* src, const double* energies,
                       int32_t n_energies, int64_t n, uint64_t seed, int64_t first, gadep_tally* out) {
  if (!ctx) return GADEP_E_ARG;
  if (!src || !out) return set_err(ctx, GADEP_E_ARG, "null source or output");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  gadep_job j = single_job(src, energies, n_energies, n, first, ctx->scales.data(), GADEP_MAX_GROUPS);
  Plan P;
  gadep_status s = plan_jobs(ctx, &j, 1, out, false, P);
  if (s) return s;
  return execute(ctx, P, seed, out, nullptr, nullptr, 0);
}

gadep_status gadep_run_noalloc(gadep_ctx* ctx, const gadep_source* src, const double* energies,
                               int32_t n_energies, int64_t n, uint64_t seed, int64_t first,
                               gadep_tally* out) {
  if (!ctx) return GADEP_E_ARG;
  if (!src || !out) return set_err(ctx, GADEP_E_ARG, "null source or output");
  if (!ctx->scratch || !ctx->na) return set_err(ctx, GADEP_E_STATE, "no device scratch on this device");
  if (!ctx->grid_set || ctx->xs_dirty) return set_err(ctx, GADEP_E_STATE, "run before gadep_set_xs");
  if (ctx->scenes.empty() || !ctx->scenes[0] || !ctx->scenes[0]->loaded)
    return set_err(ctx, GADEP_E_STATE, "run before gadep_load_mesh");
  if (n_energies < 1 || n_energies > kScratchUnits)
    return set_err(ctx, GADEP_E_ARG, "run_noalloc: n_energies must be in [1, 256]");
  if (n < 0 || first < 0) return set_err(ctx, GADEP_E_ARG, "negative history count or first history");
  if (src->n_lines > kScratchLines)
    return set_err(ctx, GADEP_E_ARG, "run_noalloc: at most 256 source lines");
  if (src->n_lines == 0 && !energies)
    return set_err(ctx, GADEP_E_ARG, "energies_keV is NULL for a mono-energetic source");
  if (src->n_lines > 0 && n_energies != 1)
    return set_err(ctx, GADEP_E_ARG, "a line source takes n_energies = 1");
  const Scene& sc = *ctx->scenes[0];
  gadep_status s = check_source(ctx, *src, sc);
  if (s) return s;
  NoAllocHost& H = *ctx->na;

  // spectra: one binning for all units, within the scratch array
  bool spectrum = false;
  int32_t n_channels = 0;
  float channel_keV = 0.0f;
  for (int32_t u = 0; u < n_energies; ++u) {
    const gadep_tally& t = out[u];
    if (!t.spectrum) continue;
    if (t.n_channels <= 0 || !(t.channel_keV > 0))
      return set_err(ctx, GADEP_E_ARG, "tally: spectrum needs n_channels > 0 and channel_keV > 0");
    if (spectrum && (t.n_channels != n_channels || t.channel_keV != channel_keV))
      return set_err(ctx, GADEP_E_ARG, "tally: all spectra of one run share their binning");
    spectrum = true;
    n_channels = t.n_channels;
    channel_keV = t.channel_keV;
  }
  const int64_t spec_words = spectrum ? static_cast<int64_t>(n_energies) * n_channels : 0;
  if (spec_words > static_cast<int64_t>(kNaSpectraWords))
    return set_err(ctx, GADEP_E_ARG, "run_noalloc: n_energies * n_channels above the scratch "
                                     "capacity of " + std::to_string(kNaSpectraWords) +
                                     " spectrum words");

  // region table at the context's density scales
  for (int32_t r = 0; r < sc.n_regions; ++r) {
    const gadep_region& R = sc.regions[r];
    if (R.material < 0 || R.material >= static_cast<int32_t>(ctx->mats.size()) ||
        !ctx->mats[R.material].set)
      return set_err(ctx, GADEP_E_STATE, "a region's material has no cross sections");
    const float sg = R.scale_group >= 0 ? ctx->scales[R.scale_group] : 1.0f;
    RegionRec& rr = H.regions[r];
    rr.mult = static_cast<float>(0.1 * R.density_g_cm3 * sg);
    rr.inv_scale = 1.0f / sg;
    rr.material = R.material;
    rr.bits = (R.scale_group >= 0 ? R.scale_group : 0xFF) | ((R.flags & GADEP_ACTIVE) ? 0x100 : 0);
  }
  // source and its lines (cumulative weights, the last one past 1)
  SourceRec& sr = H.source;
  sr = SourceRec{};
  sr.kind = src->kind;
  for (int a = 0; a < 3; ++a) sr.pos[a] = src->pos_mm[a];
  if (src->kind == GADEP_SRC_BEAM) {
    const double nn = sqrt(double(src->dir[0]) * src->dir[0] + double(src->dir[1]) * src->dir[1] +
                           double(src->dir[2]) * src->dir[2]);
    for (int a = 0; a < 3; ++a) sr.dir[a] = static_cast<float>(src->dir[a] / nn);
  }
  sr.r_in = src->r_in_mm;
  sr.r_out = src->r_out_mm;
  sr.h = src->h_mm;
  sr.region = src->region;
  sr.n_lines = src->n_lines;
  sr.line_off = 0;
  double weight = 1.0;
  if ((s = cone_setup(ctx, sc, *src, H.regions, sr, weight))) return s;
  if (src->n_lines > 0) {
    double tot = 0, cum = 0;
    for (int i = 0; i < src->n_lines; ++i) tot += src->line_prob[i];
    for (int i = 0; i < src->n_lines; ++i) {
      if ((s = check_energy(ctx, src->line_keV[i]))) return s;
      cum += src->line_prob[i];
      H.lines[2 * i] = src->line_keV[i];
      H.lines[2 * i + 1] = static_cast<float>(i == src->n_lines - 1 ? 2.0 : cum / tot);
    }
  }
  // units and their chunks
  const int64_t chunk = 64 * ctx->claim;
  int64_t chunks = 0;
  for (int32_t e = 0; e < n_energies; ++e) {
    UnitRec& u = H.units[e];
    u = UnitRec{};
    u.n = n;
    u.first = first;
    const double E = src->n_lines > 0 ? 0.0 : energies[e];
    if (src->n_lines == 0 && (s = check_energy(ctx, E))) return s;
    u.energy = static_cast<float>(E);
    u.source = 0;
    u.scene = 0;
    u.region_off = 0;
    u.stream = static_cast<uint32_t>(e);
    u.src_region = 0;
    u.n_groups = 0;
    u.flags = 0;
    if (sc.convex_exit && H.regions[0].mult == 0.0f)
      u.flags = kUnitExitEscapes | (sc.n_planes > 0 && ctx->exit_planes ? kUnitExitPlanes : 0);
    H.chunk_begin[e] = chunks;
    chunks += (n + chunk - 1) / chunk;
  }
  H.chunk_begin[n_energies] = chunks;
  fill_scene_rec(ctx->scenes, sc, H.scene);

  HIP_TRY(hipSetDevice(ctx->device), "set device");
  char* base = static_cast<char*>(ctx->scratch);
  auto up = [&](size_t off, const void* p, size_t bytes) {
    return hipMemcpyAsync(base + off, p, bytes, hipMemcpyHostToDevice, ctx->stream);
  };
  HIP_TRY(up(kNaUnits, H.units, n_energies * sizeof(UnitRec)), "upload units");
  HIP_TRY(up(kNaChunks, H.chunk_begin, (n_energies + 1) * sizeof(int64_t)), "upload chunks");
  HIP_TRY(up(kNaScene, &H.scene, sizeof(SceneRec)), "upload scene");
  HIP_TRY(up(kNaSource, &H.source, sizeof(SourceRec)), "upload source");
  if (src->n_lines > 0) HIP_TRY(up(kNaLines, H.lines, 2 * src->n_lines * sizeof(float)), "upload lines");
  HIP_TRY(up(kNaRegions, H.regions, sc.n_regions * sizeof(RegionRec)), "upload regions");

  TransportParams K{};
  K.units = reinterpret_cast<const UnitRec*>(base + kNaUnits);
  K.chunk_begin = reinterpret_cast<const int64_t*>(base + kNaChunks);
  K.n_units = n_energies;
  K.chunk = static_cast<int32_t>(chunk);
  K.total_h = n * static_cast<int64_t>(n_energies);
  K.guide = static_cast<int32_t>(ctx->guide);
  K.scenes = reinterpret_cast<const SceneRec*>(base + kNaScene);
  K.sources = reinterpret_cast<const SourceRec*>(base + kNaSource);
  K.lines = reinterpret_cast<const float*>(base + kNaLines);
  K.regions = reinterpret_cast<const RegionRec*>(base + kNaRegions);
  K.xs = static_cast<const float*>(ctx->xs.p);
  K.n_e = ctx->nE;
  K.ln_e0 = static_cast<float>(ctx->lnE0);
  K.inv_dlne = static_cast<float>(1.0 / ctx->dlnE);
  K.e_cut = static_cast<float>(exp(ctx->lnE0));
  K.tally = reinterpret_cast<unsigned long long*>(base + kNaTally);
  K.spectra = spectrum ? reinterpret_cast<unsigned long long*>(base + kNaSpectra) : nullptr;
  K.n_channels = n_channels;
  K.inv_channel_kev = spectrum ? 1.0f / channel_keV : 0.0f;
  K.cursor = reinterpret_cast<unsigned long long*>(base + kNaCursor);
  K.seed_lo = static_cast<uint32_t>(seed);
  K.seed_hi = static_cast<uint32_t>(seed >> 32);
  K.max_steps = static_cast<int32_t>(ctx->max_steps);
  K.stack_depth = std::max<int32_t>(1, sc.depth);
  K.period = static_cast<int32_t>(ctx->period);
  K.screen = static_cast<int32_t>(ctx->screen);
  K.pair = 0;
  for (const Material& m : ctx->mats)
    if (m.set && m.pair) K.pair = 1;
  if (ctx->electrons && ctx->pool)
    return set_err(ctx, GADEP_E_ARG, "electron tracks run with the per-lane kernel (GADEP_OPT_POOL = 0)");
  const bool gen = src->kind == GADEP_SRC_CYL || src->kind == GADEP_SRC_CONE || H.scene.roots2 != nullptr;
  const int variant = (spectrum ? 2 : 0) | (gen ? 8 : 0) | (K.pair ? 16 : 0) | (ctx->electrons ? 32 : 0);
  int grid = 0;
  HIP_TRY(pick_grid(ctx, variant, K.stack_depth, K.pair, &grid), "occupancy");
  if (grid < 1) return set_err(ctx, GADEP_E_ARG, "block size does not fit (LDS or registers)");
  // the array keeps the last call's contents: clear the tallies, spectra and
  // cursors with a fill kernel
  const int64_t tally_words = static_cast<int64_t>(n_energies) * kT_Slots;
  HIP_TRY(fill_u64(K.tally, tally_words, 0, ctx->stream), "clear tallies");
  if (spec_words) HIP_TRY(fill_u64(K.spectra, spec_words, 0, ctx->stream), "clear spectra");
  HIP_TRY(fill_u64(K.cursor, n_energies, 0, ctx->stream), "clear cursors");
  HIP_TRY(locate_units(reinterpret_cast<UnitRec*>(base + kNaUnits), n_energies,
                       reinterpret_cast<const SceneRec*>(base + kNaScene),
                       reinterpret_cast<const SourceRec*>(base + kNaSource), K.stack_depth,
                       ctx->stream),
          "locate units");
  HIP_TRY(launch_transport(ctx, K, variant, grid, ctx->stream), "transport launch");
  HIP_TRY(hipMemcpyAsync(H.tally, K.tally, tally_words * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, ctx->stream),
          "tally D2H");
  for (int32_t u = 0; u < n_energies && spec_words; ++u)
    if (out[u].spectrum)
      HIP_TRY(hipMemcpyAsync(out[u].spectrum, K.spectra + static_cast<int64_t>(u) * n_channels,
                             n_channels * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             ctx->stream),
              "spectra D2H");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "transport");
  note_clock(ctx, H.tally, n_energies);
  for (int32_t u = 0; u < n_energies; ++u) {
    to_tally(H.tally + static_cast<int64_t>(u) * kT_Slots, out[u]);
    out[u].weight = weight;
  }
  return GADEP_OK;
}

gadep_status gadep_run_grad(gadep_ctx* ctx, const gadep_source* src, const double* energies,
                            int32_t n_energies, int64_t n, uint64_t seed, int64_t first,
                            const float* scales, int32_t n_scales, gadep_tally* out, double* dfepe_ds,
                            double* dfepe_ds_var) {
  if (!ctx) return GADEP_E_ARG;
  if (!src || !out) return set_err(ctx, GADEP_E_ARG, "null source or output");
  if (n_scales < 1 || n_scales > GADEP_MAX_GROUPS || !scales)
    return set_err(ctx, GADEP_E_ARG, "run_grad needs 1..8 scales");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  gadep_job j = single_job(src, energies, n_energies, n, first, scales, n_scales);
  Plan P;
  gadep_status s = plan_jobs(ctx, &j, 1, out, true, P);
  if (s) return s;
  return execute(ctx, P, seed, out, dfepe_ds, dfepe_ds_var, n_scales);
}

gadep_status gadep_run_batch(gadep_ctx* ctx, const gadep_job* jobs, int32_t n_jobs, uint64_t seed,
                             gadep_tally* out, double* grads, double* grads_var) {
  if (!ctx) return GADEP_E_ARG;
  if (!out) return set_err(ctx, GADEP_E_ARG, "null output");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  Plan P;
  const bool grad = grads || grads_var;
  gadep_status s = plan_jobs(ctx, jobs, n_jobs, out, grad, P);
  if (s) return s;
  return execute(ctx, P, seed, out, grads, grads_var, GADEP_MAX_GROUPS);
}

// Settings the autotuner found, per (GPU architecture, kernel, class of the
// job mix): a later call with the same key takes them without timing again.
// The class is what the timing depends on: mesh size (log2 of the largest
// scene's facets), number of jobs and units (log2), source kinds, gradients.
struct TuneKey {
  std::string arch;
  int64_t pool, mesh_class, jobs_class, units_class, kinds, grad;
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, pool, mesh_class, jobs_class, units_class, kinds, grad) <
           std::tie(o.arch, o.pool, o.mesh_class, o.jobs_class, o.units_class, o.kinds, o.grad);
  }
};
struct TuneVal {
  int64_t block, period, claim;
};
std::mutex g_tune_mutex;
std::map<TuneKey, TuneVal> g_tune_cache;

int64_t log2_class(int64_t x) {
  int64_t c = 0;
  while (x > 1) {
    x >>= 1;
    ++c;
  }
  return c;
}

gadep_status gadep_autotune(gadep_ctx* ctx, const gadep_job* jobs, int32_t n_jobs, int64_t pilot,
                            int32_t* block_out, int32_t* period_out, int32_t* claim_out) {
  if (!ctx) return GADEP_E_ARG;
  if (pilot < 1) return set_err(ctx, GADEP_E_ARG, "pilot_histories must be >= 1");
  if (!jobs || n_jobs <= 0) return set_err(ctx, GADEP_E_ARG, "no jobs");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  TuneKey key;
  {
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, ctx->device), "device properties");
    key.arch = prop.gcnArchName;
    int64_t facets = 0, units = 0, kinds = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
      const int32_t sc = jobs[j].scene;
      if (sc >= 0 && sc < static_cast<int32_t>(ctx->scenes.size()) && ctx->scenes[sc])
        facets = std::max(facets, ctx->scenes[sc]->n_tri);
      units += std::max(1, jobs[j].n_energies);
      kinds |= int64_t(1) << std::min(7, std::max(0, jobs[j].src.kind));
    }
    key.pool = ctx->pool;
    key.mesh_class = log2_class(facets);
    key.jobs_class = log2_class(n_jobs);
    key.units_class = log2_class(units);
    key.kinds = kinds;
    key.grad = 0;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      if (!ctx->pool) ctx->block = it->second.block;
      ctx->period = it->second.period;
      ctx->claim = it->second.claim;
      if (block_out) *block_out = static_cast<int32_t>(ctx->pool ? 64 : it->second.block);
      if (period_out) *period_out = static_cast<int32_t>(it->second.period);
      if (claim_out) *claim_out = static_cast<int32_t>(it->second.claim);
      return GADEP_OK;
    }
  }
  std::vector<gadep_job> pj(jobs, jobs + std::max(0, n_jobs));
  int64_t total = 0;
  for (auto& j : pj) total += j.n_histories * std::max(1, j.n_energies);
  // scale every job down to about `pilot` histories in total, keeping the mix
  for (auto& j : pj)
    if (total > pilot) j.n_histories = std::max<int64_t>(1, j.n_histories * pilot / total);
  size_t units = 0;
  for (auto& j : pj) units += std::max(1, j.n_energies);
  std::vector<gadep_tally> out(units);
  const int64_t saved_block = ctx->block, saved_claim = ctx->claim, saved_period = ctx->period,
                saved_graphs = ctx->graphs;
  auto restore = [&]() {
    ctx->block = saved_block;
    ctx->claim = saved_claim;
    ctx->period = saved_period;
    ctx->graphs = saved_graphs;
  };
  ctx->graphs = 0;
  float best = INFINITY;
  int64_t best_block = saved_block, best_claim = saved_claim, best_period = saved_period;
  // block size x claim size x threshold (per-lane kernel: lanes parked before
  // the wavefront runs the batched physics; pooled kernel: lanes still
  // traversing when a housekeeping round starts); tallies depend on none of
  // them.  The pooled kernel always runs one wavefront per block.
  const std::vector<int64_t> blocks = ctx->pool ? std::vector<int64_t>{64} : std::vector<int64_t>{128, 256};
  const int64_t claims[] = {16, 64};
  const std::vector<int64_t> periods =
      ctx->pool ? std::vector<int64_t>{16, 24, 32, 40, 48} : std::vector<int64_t>{16, 24, 32};
  for (int64_t b : blocks)
    for (int64_t c : claims)
      for (int64_t q : periods) {
        if (!ctx->pool) ctx->block = b;
        ctx->claim = c;
        ctx->period = q;
        Plan P;
        gadep_status s = plan_jobs(ctx, pj.data(), static_cast<int32_t>(pj.size()), out.data(), false, P);
        if (s) {
          restore();
          return s;
        }
        float ms = 0, ms2 = 0;
        s = execute(ctx, P, 12345, out.data(), nullptr, nullptr, 0, &ms);  // warm-up
        if (!s) s = execute(ctx, P, 12345, out.data(), nullptr, nullptr, 0, &ms2);
        if (s) {
          restore();
          return s;
        }
        if (ms2 < best) {
          best = ms2;
          best_block = b;
          best_claim = c;
          best_period = q;
        }
      }
  if (!ctx->pool) ctx->block = best_block;
  ctx->claim = best_claim;
  ctx->period = best_period;
  ctx->graphs = saved_graphs;
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[key] = TuneVal{best_block, best_period, best_claim};
  }
  if (block_out) *block_out = static_cast<int32_t>(best_block);
  if (period_out) *period_out = static_cast<int32_t>(ctx->period);
  if (claim_out) *claim_out = static_cast<int32_t>(best_claim);
  return GADEP_OK;
}

gadep_status gadep_get_last_launch_ms(const gadep_ctx* ctx, double* ms) {
  if (!ctx || !ms) return GADEP_E_ARG;
  if (ctx->last_ms < 0) return GADEP_E_STATE;
  *ms = ctx->last_ms;
  return GADEP_OK;
}

gadep_status gadep_get_last_clock_mhz(const gadep_ctx* ctx, double* mhz) {
  if (!ctx || !mhz) return GADEP_E_ARG;
  if (ctx->last_sclk_mhz < 0) return GADEP_E_STATE;
  *mhz = ctx->last_sclk_mhz;
  return GADEP_OK;
}

gadep_status gadep_get_counters(const gadep_ctx* ctx, gadep_counters* out) {
  if (!ctx || !out) return GADEP_E_ARG;
  if (!ctx->have_counters) return GADEP_E_STATE;
  *out = ctx->last_counters;
  return GADEP_OK;
}

gadep_status gadep_broaden_dev(gadep_ctx* ctx, const double* in_dev, double* out_dev,
                               int32_t n_spectra, int32_t n_channels, double w, double a, double b) {
  if (!ctx) return GADEP_E_ARG;
  if (!in_dev || !out_dev || n_spectra < 1 || n_channels < 1 || !(w > 0) || !(a >= 0) || !(b >= 0) ||
      !(a + b > 0))
    return set_err(ctx, GADEP_E_ARG, "broaden: bad arguments");
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  HIP_TRY(broaden(in_dev, out_dev, n_spectra, n_channels, w, a, b, ctx->stream), "broaden");
  HIP_TRY(hipStreamSynchronize(ctx->stream), "broaden");
  return GADEP_OK;
}

static gadep_status scene_rec(gadep_ctx* ctx, int32_t scene, SceneRec& sr) {
  if (scene < 0 || scene >= static_cast<int32_t>(ctx->scenes.size()) || !ctx->scenes[scene] ||
      !ctx->scenes[scene]->loaded)
    return set_err(ctx, GADEP_E_STATE, "scene not loaded");
  fill_scene_rec(ctx->scenes, *ctx->scenes[scene], sr);
  return GADEP_OK;
}

gadep_status gadep_raycast(gadep_ctx* ctx, int32_t scene, const float* o, const float* d,
                           const int32_t* region, int64_t n, float* t, int32_t* tri,
                           int32_t* region_after) {
  if (!ctx) return GADEP_E_ARG;
  if (!o || !d || !t || !tri || !region_after || n < 0) return set_err(ctx, GADEP_E_ARG, "raycast: bad arguments");
  if (n == 0) return GADEP_OK;
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  SceneRec sr;
  gadep_status s = scene_rec(ctx, scene, sr);
  if (s) return s;
  void* buf = nullptr;
  const size_t nb = static_cast<size_t>(n);
  const size_t bytes = nb * (3 + 3 + 1 + 1 + 1 + 1) * 4;
  HIP_TRY(hipMalloc(&buf, bytes), "raycast buffers");
  float* d_o = static_cast<float*>(buf);
  float* d_d = d_o + 3 * nb;
  int32_t* d_r = reinterpret_cast<int32_t*>(d_d + 3 * nb);
  float* d_t = reinterpret_cast<float*>(d_r + nb);
  int32_t* d_tri = reinterpret_cast<int32_t*>(d_t + nb);
  int32_t* d_ra = d_tri + nb;
  hipError_t e = hipMemcpyAsync(d_o, o, 12 * nb, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_d, d, 12 * nb, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && region) e = hipMemcpyAsync(d_r, region, 4 * nb, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = raycast(sr, d_o, d_d, region ? d_r : nullptr, n, d_t, d_tri, d_ra, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(t, d_t, 4 * nb, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(tri, d_tri, 4 * nb, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(region_after, d_ra, 4 * nb, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_err(ctx, e, "raycast");
  return GADEP_OK;
}

gadep_status gadep_philox(gadep_ctx* ctx, const uint32_t* counters, uint64_t key, int64_t n,
                          uint32_t* out) {
  if (!ctx) return GADEP_E_ARG;
  if (!counters || !out || n < 0) return set_err(ctx, GADEP_E_ARG, "philox: bad arguments");
  if (n == 0) return GADEP_OK;
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  void* buf = nullptr;
  const size_t bytes = static_cast<size_t>(n) * 16;
  HIP_TRY(hipMalloc(&buf, 2 * bytes), "philox buffers");
  uint32_t* d_c = static_cast<uint32_t*>(buf);
  uint32_t* d_o = d_c + 4 * static_cast<size_t>(n);
  hipError_t e = hipMemcpyAsync(d_c, counters, bytes, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = philox(d_c, static_cast<uint32_t>(key), static_cast<uint32_t>(key >> 32), n, d_o, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_o, bytes, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_err(ctx, e, "philox");
  return GADEP_OK;
}

gadep_status gadep_locate(gadep_ctx* ctx, int32_t scene, const float* p, int64_t n, int32_t* region) {
  if (!ctx) return GADEP_E_ARG;
  if (!p || !region || n < 0) return set_err(ctx, GADEP_E_ARG, "locate: bad arguments");
  if (n == 0) return GADEP_OK;
  HIP_TRY(hipSetDevice(ctx->device), "set device");
  SceneRec sr;
  gadep_status s = scene_rec(ctx, scene, sr);
  if (s) return s;
  void* buf = nullptr;
  const size_t nb = static_cast<size_t>(n);
  HIP_TRY(hipMalloc(&buf, nb * 16), "locate buffers");
  float* d_p = static_cast<float*>(buf);
  int32_t* d_r = reinterpret_cast<int32_t*>(d_p + 3 * nb);
  hipError_t e = hipMemcpyAsync(d_p, p, 12 * nb, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = locate(sr, d_p, n, d_r, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(region, d_r, 4 * nb, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_err(ctx, e, "locate");
  return GADEP_OK;
}

}  // extern "C"
