// Internal data layouts shared by the host runtime and the gfx950 kernels.
//
// Everything the kernels read lives in device memory in these layouts; the
// host fills them once per mesh / per table / per run.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace gadep {

constexpr int kLeafMax = 4;          // facets per BVH leaf
constexpr int kMaxDepth = 64;        // hard cap on BVH depth (traversal stack)
constexpr int kMaxRegions = 64;      // regions per scene (parity mask is 64-bit)
constexpr int kMaxGroups = 8;        // density-scale groups
constexpr int kMaxExitPlanes = 32;   // distinct facet planes of a convex outermost shell
constexpr float kMec2 = 510.99895f;  // electron rest energy [keV]

// Fixed-point scales of the 64-bit tally accumulators (exact, order-free sums).
constexpr double kEnergyFix = 65536.0;      // keV
constexpr double kScoreFix = 16777216.0;    // score
// score^2 of a history, x = score^2 * 2^16, is kept in two slots: floor(x)
// and the rest of x rounded in units of 2^-24, so that the squares of tiny
// scores (a layer of a few micrometres, such as a separation gap) are not lost
// while the range stays that of floor(x).
constexpr double kScore2Fix = 65536.0;  // score^2, integer part
constexpr int kScore2LoBits = 24;       // fraction bits of the second slot

// node link meaning "no node" (an empty stack, a region without facets)
constexpr int32_t kDone = INT32_MIN;

// Two children per node, each with its box; 64 bytes, read as four 16-byte loads.
struct alignas(16) BvhNode {
  float lmin[3], lmax[3];
  float rmin[3], rmax[3];
  int32_t child[2];  // >= 0: node index; < 0: leaf ~(first_facet << 3 | count)
  int32_t pad[2];
};
static_assert(sizeof(BvhNode) == 64, "node layout");

// Facet record; 48 bytes, read as three 16-byte loads.  Leaves list slots,
// and each slot names a facet, so a facet that several BVHs (or several
// leaves of one) list is stored once.
struct alignas(16) TriRec {
  float v0[3], v1[3], v2[3];
  uint32_t regions;  // inside (low 16 bits) | outside (high 16 bits)
  int32_t orig;      // caller's facet index
  uint32_t pad;
};
static_assert(sizeof(TriRec) == 48, "facet layout");

inline int32_t leaf_code(int64_t first, int32_t count) {
  return ~static_cast<int32_t>((first << 3) | count);
}

// Region as seen by the kernel: mu = mult * (mu/rho)(E); mu0 = mu * inv_scale.
struct alignas(16) RegionRec {
  float mult;        // 0.1 * density * scale
  float inv_scale;   // 1 / scale
  int32_t material;  // xs table index
  int32_t bits;      // group (low 8 bits, 0xFF none) | ACTIVE << 8
};

// A scene's device tables.  Node 0 is the root of the plain BVH over every
// facet (one record per facet), used for parity counts, geometry queries and
// the localisation of volume-source points (root_all); the transport BVHs
// (spatial splits, one per region, their records after the plain ones)
// follow.  A photon in region r searches roots[r], whose facets are exactly
// those that bound r.  When the outermost shell is convex with at most
// kMaxExitPlanes distinct planes, `planes` holds its planes (outward unit
// normal, offset n . x), outer_root is the outer region's BVH without that
// shell and trans_lo/trans_hi bound it.
struct SceneRec {
  const BvhNode* nodes;
  const TriRec* tris;     // one record per facet, in the caller's order
  const int32_t* slots;   // facet of each leaf slot, for every BVH
  const float* planes;  // 4 floats per plane
  const int32_t* roots;  // root node of each region's transport BVH (kDone: none)
  // Two-level scenes (a per-job overlay on a shared detector): a second BVH
  // root per region, searched after the first with the nearest hit kept
  // (null: none), and the root of the overlay's plain BVH (-1: none).
  const int32_t* roots2;
  int32_t root_all2;
  int32_t n_regions;
  int32_t depth;        // deepest of the BVHs
  int32_t n_planes;     // 0: no exit planes
  int32_t outer_root;   // outer region's transport BVH without the outermost shell
  int32_t root_all;
  int32_t outer_region;
  float trans_lo[3], trans_hi[3];
  float outer_lo[3], outer_hi[3];  // box of the outermost shell (with exit planes)
};

// UnitRec.flags
constexpr int32_t kUnitExitEscapes = 1;  // entering the (void) world ends the history
// With kUnitExitEscapes and exit planes: the outer shell's own region is left
// through its planes, and its segments search outer_root (the other shells).
constexpr int32_t kUnitExitPlanes = 2;

enum SourceKind : int32_t { kPoint = 0, kBeam = 1, kCyl = 2, kCone = 3 };

struct SourceRec {
  int32_t kind;
  float pos[3];
  float dir[3];
  float r_in, r_out, h;
  int32_t region;
  int32_t n_lines;
  int32_t line_off;  // into the line table (float2: keV, cumulative probability)
  float cone_cos;    // kCone: directions uniform in the cone of this half-angle cosine about dir
};

struct UnitRec {
  int64_t n;            // histories
  int64_t first;        // number of the first history
  float energy;         // keV (ignored for a line source)
  int32_t source;       // SourceRec index
  int32_t scene;        // SceneRec index
  int32_t region_off;   // first RegionRec of this unit's region table
  uint32_t stream;      // random stream id: counter word 3
  int32_t src_region;   // region of a point/beam origin (set on the device)
  int32_t n_groups;
  int32_t flags;        // kUnit* bits
};

// Per-unit tally slots (uint64 each).
enum TallySlot : int {
  kT_Hist = 0, kT_Absorbed, kT_Fep, kT_CollEscape, kT_Lost, kT_Killed, kT_Glitch, kT_SrcFail,
  kT_SpecOvf, kT_EdepAct, kT_EdepTot, kT_EEsc, kT_ESrc,
  // per wavefront, over its lifetime: shader-clock cycles (s_memtime) and
  // ticks of the constant-rate clock (s_memrealtime); their ratio is the
  // shader clock the launch ran at
  kT_ClkCore, kT_ClkRef,
  kT_Score = 16, kT_FepScore = 24, kT_FepScore2 = 32,
  kT_Ev = 40,  // event counters, up to 32 slots
  kT_FepScore2Lo = 72,  // fractions of the FEP score^2 sums (see kScore2Fix)
  kT_Slots = 80
};
enum EventSlot : int {
  kEv_Segments = 0, kEv_Crossings, kEv_NodeVisits, kEv_TriTests, kEv_Photo, kEv_Compton,
  kEv_Coherent, kEv_Rng, kEv_Locates, kEv_Emissions, kEv_PlaneTests,
  // wavefront-level: loop iterations, those with a node / facet step, passes
  // of the batched per-segment work
  kEv_Iters, kEv_ItersNode, kEv_ItersTri, kEv_Passes,
  // wavefront-level shader-clock cycles per section of the loop
  kEv_CycOutcome, kEv_CycRefill, kEv_CycLaunch, kEv_CycSetup, kEv_CycTrav,
  // screened histories settled by one box test (no attenuation, no exit planes)
  kEv_BoxTests,
  kEv_Pair,  // pair-production events
  kEv_Electrons,  // electron tracks
  // screened histories settled by the direction alone: it misses the sphere
  // around the inner shells' box (no box test)
  kEv_ConeTests,
  kEv_N
};
static_assert(kT_Ev + kEv_N <= kT_FepScore2Lo, "tally slots");

// Fixed device scratch of the no-allocation run (one array per GPU): its size
// and the number of devices whose addresses are kept.
constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int kScratchDevices = 64;
constexpr int32_t kScratchUnits = 256;  // energies per no-allocation run
constexpr int32_t kScratchLines = 256;  // source lines per no-allocation run

struct TransportParams {
  const UnitRec* units;
  const int64_t* chunk_begin;  // [n_units + 1], prefix sums of chunks per unit
  int32_t n_units;
  int32_t chunk;               // histories per claim (the least, when claims shrink)
  int64_t total_h;             // histories of all units
  const SceneRec* scenes;
  const SourceRec* sources;
  const float* lines;          // float2 pairs
  const RegionRec* regions;
  const float* xs;             // float4 per (material, grid point): ln photo, Compton, coherent, pair
  int32_t n_e;
  float ln_e0;
  float inv_dlne;
  float e_cut;
  unsigned long long* tally;   // [n_units][kT_Slots]
  unsigned long long* spectra; // [n_units][n_channels] or null
  int32_t n_channels;
  float inv_channel_kev;
  unsigned long long* cursor;  // [n_units] claims made per unit
  uint32_t seed_lo, seed_hi;
  int32_t max_steps;
  int32_t stack_depth;
  int32_t period;
  int32_t screen;              // 1: first-flight screening where it applies
  int32_t pair;                // 1: some material has a pair-production partial
  int32_t guide;               // > 0: claims shrink by factoring (1/guide of the rest per batch)
};
static_assert(sizeof(TransportParams) % 8 == 0, "no tail padding in the graph key");

// ---------------------------------------------------------------------------
// host preparation (mesh_prep.cpp)

struct PreparedMesh {
  std::vector<TriRec> tris;        // BVH order
  std::vector<BvhNode> nodes;
  std::vector<int32_t> outside;    // per caller facet
  std::vector<int32_t> shell;      // per caller facet
  std::vector<int32_t> order;      // caller facet of each BVH slot
  int32_t depth = 0;
  double sah = 0.0;
  int32_t n_shells = 0;
  int32_t genus_max = 0;
  double min_gap = 0.0;
  // The world borders exactly one shell and that shell is convex: a photon
  // that leaves it into the world can never meet another facet.
  bool convex_exit = false;
  // Set when that shell has at most kMaxExitPlanes distinct planes: its
  // planes, 4 floats each (outward unit normal, offset n . x).
  std::vector<float> planes;
  int32_t outer_region = 0;
  float outer_lo[3] = {0, 0, 0}, outer_hi[3] = {0, 0, 0};  // box of that shell
  // Transport BVHs, built with spatial splits (a facet may have several
  // records), one per region: region r's lists the facets that bound r (inside
  // or outside region r), the only ones a photon in r can cross next.  When
  // `planes` is set, one more (index n_regions) lists those of the outer
  // region without the outermost shell, which the planes replace.  They are
  // concatenated: trans_root[r] is the root node of BVH r (-1: r has no
  // facets); child indices and record slots refer to the concatenation.
  std::vector<BvhNode> trans_nodes;
  std::vector<TriRec> trans_tris;
  std::vector<int32_t> trans_root;
  int32_t trans_depth = 0;
  double trans_sah = 0.0;  // sum over the BVHs, each relative to its own root
  // bounds of the outer region's BVH without the outermost shell (lo > hi:
  // none, or no facets)
  float trans_lo[3] = {0, 0, 0}, trans_hi[3] = {0, 0, 0};
};

// Returns a gadep_status value; fills err on failure.
// split_budget: extra facet records the transport BVH may add, as a fraction
// of its facets (0 = no spatial splits).
int prepare_mesh(const float* xyz, int64_t nv, const int32_t* tri, const int32_t* tri_region,
                 int64_t nt, int32_t n_regions, double min_gap, bool validate, int bvh_method,
                 double split_budget, PreparedMesh& out, std::string& err);

}  // namespace gadep
