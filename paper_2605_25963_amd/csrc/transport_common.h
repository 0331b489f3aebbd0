// Physics and wavefront helpers shared by the transport kernels: cross-section
// interpolation, the scattering rotation, wavefront reductions, fixed-point
// tally conversions, and the per-photon phases and limits of the state
// machines.
#pragma once
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "gadep_internal.h"

namespace gadep {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// physics helpers

struct Xs {
  int k;
  float w;
};

__device__ __forceinline__ Xs xs_index(float E, float ln_e0, float inv_dlne, int n_e) {
  const float x = (hw_log(E) - ln_e0) * inv_dlne;
  int k = static_cast<int>(floorf(x));
  k = k < 0 ? 0 : (k > n_e - 2 ? n_e - 2 : k);
  float w = x - static_cast<float>(k);
  w = fminf(fmaxf(w, 0.0f), 1.0f);
  return {k, w};
}

// partial linear attenuation [1/mm] of a region: log-log interpolation of
// each partial, mu_i = mult * exp(lerp(ln(mu/rho)_i)).  The products are kept
// out of contraction, so that mu = mp + mc + mh comes out the same wherever it
// is formed (screening decides a flight with a per-unit value that must equal
// the set-up's).
__device__ __forceinline__ void xs_mu(const float4* __restrict__ xs, int n_e, const RegionRec& rr,
                                      Xs ix, float& mp, float& mc, float& mh) {
#pragma clang fp contract(off)
  if (rr.mult > 0.0f) {
    const float4 lo = gload(xs, rr.material * n_e + ix.k);
    const float4 hi = gload(xs, rr.material * n_e + ix.k + 1);
    mp = rr.mult * __expf(fmaf(ix.w, hi.x - lo.x, lo.x));
    mc = rr.mult * __expf(fmaf(ix.w, hi.y - lo.y, lo.y));
    mh = rr.mult * __expf(fmaf(ix.w, hi.z - lo.z, lo.z));
  } else {
    mp = mc = mh = 0.0f;
  }
}

// pair-production partial [1/mm]; zero unless `on` (some material has one)
// and E lies above the threshold 2 m_e c^2
__device__ __forceinline__ float xs_pair(const float4* __restrict__ xs, int n_e, const RegionRec& rr,
                                         Xs ix, float E, bool on) {
#pragma clang fp contract(off)
  if (!on || !(E > 2.0f * kMec2) || !(rr.mult > 0.0f)) return 0.0f;
  const float lo = gload(xs, rr.material * n_e + ix.k).w;
  const float hi = gload(xs, rr.material * n_e + ix.k + 1).w;
  return rr.mult * __expf(fmaf(ix.w, hi - lo, lo));
}

// New direction at polar cosine ct and azimuth 2 pi u about (dx, dy, dz), in an
// orthonormal basis built branch-free from the direction (Duff et al., JCGT
// 2017).  sin/cos of 2 pi u come from the hardware sine, which takes
// revolutions.
__device__ __forceinline__ void turn(float& dx, float& dy, float& dz, float ct, float u) {
  const float st = hw_sqrt(fmaxf(0.0f, 1.0f - ct * ct));
  const float cp = __builtin_amdgcn_cosf(u), sp = __builtin_amdgcn_sinf(u);
  const float s = copysignf(1.0f, dz);
  const float a = -1.0f / (s + dz);
  const float b = dx * dy * a;
  const float b1x = 1.0f + s * dx * dx * a, b1y = s * b, b1z = -s * dx;
  const float b2x = b, b2y = s + dy * dy * a, b2z = -dy;
  const float ux = st * cp, uy = st * sp;
  float nx = ct * dx + ux * b1x + uy * b2x;
  float ny = ct * dy + ux * b1y + uy * b2y;
  float nz = ct * dz + ux * b1z + uy * b2z;
  const float inv = rsqrtf(nx * nx + ny * ny + nz * nz);
  dx = nx * inv;
  dy = ny * inv;
  dz = nz * inv;
}

// ---------------------------------------------------------------------------
// wavefront helpers

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int m = 1; m < kWave; m <<= 1) x += __shfl_xor(x, m, kWave);
  return x;
}

__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x >> 32));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// First-flight screening constants of a unit (point or beam source in the
// outermost shell's region, fixed energy).  No point of the outermost shell
// is farther from the source than the farthest corner of its box, so a first
// flight whose optical depth reaches tau (that distance times the outer
// region's attenuation m, with a margin far above rounding) always ends at the
// shell.  A direction whose cosine with (ax, ay, az) is below cos misses the
// sphere around the inner shells' box, so it misses the box as well (radius
// and cosine widened far beyond rounding; cos = -2: no such test).
struct ScreenUnit {
  float tau = INFINITY, far = INFINITY, m = -1.0f;
  float ax = 0.0f, ay = 0.0f, az = 0.0f, cos = -2.0f;
};

__device__ __forceinline__ ScreenUnit screen_unit(const SceneRec& S, const SourceRec& Src,
                                                  const RegionRec& ro, float energy, const float4* xs,
                                                  int n_e, float ln_e0, float inv_dlne, bool pair) {
  ScreenUnit su;
  float d2 = 0.0f;
  for (int a = 0; a < 3; ++a) {
    const float e = fmaxf(fabsf(S.outer_lo[a] - Src.pos[a]), fabsf(S.outer_hi[a] - Src.pos[a]));
    d2 = fmaf(e, e, d2);
  }
  su.far = sqrtf(d2) * 1.0001f;
  float m_p, m_c, m_h;
  const Xs ixu = xs_index(energy, ln_e0, inv_dlne, n_e);
  xs_mu(xs, n_e, ro, ixu, m_p, m_c, m_h);
  su.m = m_p + m_c + m_h + xs_pair(xs, n_e, ro, ixu, energy, pair);
  su.tau = su.m * su.far * 1.0001f;
  if (S.trans_lo[0] <= S.trans_hi[0]) {
    float c[3], r2 = 0.0f, dd = 0.0f;
    for (int a = 0; a < 3; ++a) {
      const float h = 0.5f * (S.trans_hi[a] - S.trans_lo[a]);
      c[a] = 0.5f * (S.trans_hi[a] + S.trans_lo[a]) - Src.pos[a];
      r2 = fmaf(h, h, r2);
      dd = fmaf(c[a], c[a], dd);
    }
    const float r = sqrtf(r2) * 1.001f + 1e-3f, d = sqrtf(dd);
    if (d > 1.01f * r) {
      su.ax = c[0] / d;
      su.ay = c[1] / d;
      su.az = c[2] / d;
      const float sn = r / d;
      su.cos = sqrtf(1.0f - sn * sn) - 1e-4f;
    }
  }
  return su;
}

// Work claims.  cursor[u] counts the claims made on unit u; claim c of a unit
// is a fixed range of its histories.  With `guide` = 0 every claim holds
// `chunk` histories.  Otherwise claims come in batches of B (the number of
// wavefronts the unit's share of the grid holds), and every claim of a batch
// takes 1/(guide x B) of the histories the earlier batches left, rounded down
// to whole wavefronts of histories, until that falls to `chunk` or below;
// from then on claims hold `chunk` (factoring, Hummel, Schonberg & Flynn
// 1992).  Claims start large and shrink toward the end of the unit: few
// device-scope atomics (each one a write past the L2) and a short tail.  The
// ranges depend on c alone, so the schedule cannot change which histories
// run.
//
// A wavefront keeps the batch its last claim fell in (claims on a unit only
// grow), so that finding the batch of the next claim takes a step or two.
struct ClaimBatch {
  int unit = -1;
  int64_t k0 = 0;  // first claim of the batch
  int64_t h = 0;   // its first history
  int64_t R = 0;   // histories the earlier batches left
  int64_t s = 0;   // histories per claim of the batch (<= chunk: fixed from here on)
};

// Returns the first history of the claim on every lane (at or beyond the
// unit's size once the unit is used up) and its end in h1.
__device__ __forceinline__ int64_t claim_histories(const TransportParams& P, int u, int64_t n_w,
                                                   int lane, ClaimBatch& cb, int64_t& h1) {
  const int64_t nu = P.units[u].n;
  unsigned long long c = 0;
  if (lane == 0) c = atomicAdd(P.cursor + u, 1ull);
  const int64_t k = static_cast<int64_t>(uniform_u64(__shfl(c, 0, kWave)));
  const int64_t chunk = P.chunk;
  int64_t h = k * chunk, size = chunk;
  if (P.guide > 0) {
    int64_t B = P.total_h > 0 ? n_w * nu / P.total_h : 1;
    if (B < 1) B = 1;
    const int64_t D = static_cast<int64_t>(P.guide) * B;
    if (cb.unit != u) {
      cb.unit = u;
      cb.k0 = 0;
      cb.h = 0;
      cb.R = nu;
      cb.s = (nu / D) & ~static_cast<int64_t>(kWave - 1);
    }
    while (cb.s > chunk && k - cb.k0 >= B) {
      cb.h += B * cb.s;
      cb.R -= B * cb.s;
      cb.k0 += B;
      cb.s = (cb.R / D) & ~static_cast<int64_t>(kWave - 1);
    }
    if (cb.s > chunk) size = cb.s;
    h = cb.h + (k - cb.k0) * size;
  }
  const int64_t e = h + size;
  h1 = e < nu ? e : nu;
  return h;
}

// Energies in keV (0 <= E < 65536) in units of 2^-16 keV: E * 2^16 is exact in
// FP32, so rounding it to an integer in FP32 gives the same value as FP64.
__device__ __forceinline__ unsigned long long fx_kev(float e) {
  return static_cast<unsigned long long>(__float2uint_rn(e * 65536.0f));
}

__device__ __forceinline__ unsigned long long fx(double v, double scale) {
  return static_cast<unsigned long long>(__double2ll_rn(v * scale));
}

// ---------------------------------------------------------------------------
// closest hit with the region-consistency filter

struct HitOut {
  float t;
  int slot;
  int region_after;
};

// Closest facet with 0 < t <= tmax, skipping slot `exclude`.  A candidate is
// accepted only if it is consistent with the current region: entering
// requires outside == cur, leaving requires inside == cur (cur < 0: accept
// all).  Returns true on a hit; `glitch` is set when a rejected candidate lay
// nearer than the accepted one.
template <bool COUNT>
__device__ __forceinline__ bool closest_hit(const SceneRec& sc, const Ray& r, float ox, float oy,
                                            float oz, float dx, float dy, float dz, float tmax,
                                            int exclude, int cur, int* stack, int stride,
                                            HitOut& h, bool& glitch, uint32_t& nvis,
                                            uint32_t& ntri, int root = 0) {
  float best = tmax;
  int best_slot = -1;
  int best_reg = 0;
  float rejected = INFINITY;
  const TriRec* __restrict__ tris = sc.tris;
  float tm = tmax;
  const uint32_t v = traverse(sc.nodes, r, tm, stack, stride, sc.depth, [&](int first, int count,
                                                                             float tcur) {
    for (int k = 0; k < count; ++k) {
      const int slot = first + k;
      if (COUNT) ntri++;
      if (slot == exclude) continue;
      float4 a, b, c;
      load_tri(tris, gload(sc.slots, slot), a, b, c);
      float t;
      bool enter;
      if (wt_test(r, ox, oy, oz, dx, dy, dz, a, b, c, tcur, t, enter) == kWtMiss) continue;
      const uint32_t regs = __float_as_uint(c.y);
      const int inside = static_cast<int>(regs & 0xFFFFu);
      const int outside = static_cast<int>(regs >> 16);
      if (cur >= 0 && (enter ? outside : inside) != cur) {
        rejected = fminf(rejected, t);
        continue;
      }
      tcur = t;
      best = t;
      best_slot = slot;
      best_reg = enter ? inside : outside;
    }
    return tcur;
  }, root);
  if (COUNT) nvis += v;
  glitch = rejected < best;
  if (best_slot < 0) return false;
  h.t = best;
  h.slot = best_slot;
  h.region_after = best_reg;
  return true;
}

// ---------------------------------------------------------------------------
// secondary electrons (the straight-track reading of the electron transport
// of Sec. 2.4.1): each electron of at least kElecMin set in motion by a
// photoelectric absorption, a Compton scattering or a pair production runs a
// straight continuous-slowing-down track with the Katz-Penfold (1952) mass
// range, and every region it crosses keeps the energy it loses there.

constexpr float kElecMin = 10.0f;  // keV: lower end of the range relation

// mass range [g/cm^2] of an electron of kinetic energy T [keV]
__device__ __forceinline__ float csda_range(float T) {
  const float t = T * 1e-3f;
  if (t > 2.5f) return 0.530f * t - 0.106f;
  if (!(t > 0.0f)) return 0.0f;
  const float lt = __logf(t);
  return 0.412f * __expf((1.265f - 0.0954f * lt) * lt);
}

// kinetic energy [keV] with mass range R: bisection (the range grows with T)
__device__ __forceinline__ float csda_energy(float R) {
  if (!(R > 0.0f)) return 0.0f;
  float lo = 0.0f, hi = 4000.0f;
  for (int i = 0; i < 32; ++i) {
    const float m = 0.5f * (lo + hi);
    if (csda_range(m) < R)
      lo = m;
    else
      hi = m;
  }
  return 0.5f * (lo + hi);
}

struct ElecOut {
  float act, tot, esc;  // energy left in ACTIVE regions, in all regions, carried out of the world
  int lost;             // ended in a void region that is not the world
};

// The track of an electron of kinetic energy T from p along the unit
// direction e in `region`: nearest facets on the plain BVHs (of an overlay
// too) with the region-consistency filter; in a region of nominal density
// rho it runs 10 R / rho mm on its remaining range R.  Out of line: it is
// rare, and its traversal loop would otherwise swell the transport kernel.
// `stack` is the calling lane's LDS column (entries stack[k * stride]), free
// while the lane does the per-segment work.
__device__ __noinline__ ElecOut electron_track(const SceneRec* __restrict__ scene,
                                               const RegionRec* __restrict__ regions, float px,
                                               float py, float pz, float ex, float ey, float ez,
                                               float T, int region, int* stack, int stride) {
  const SceneRec S = *scene;
  ElecOut out{0.0f, 0.0f, 0.0f, 0};
  float R = csda_range(T), Tcur = T;
  int excl = -1;
  uint32_t nv = 0, nt = 0;
  for (int it = 0; it < 4096; ++it) {
    const RegionRec rr = gload(regions, region);
    const float rho10 = rr.mult * rr.inv_scale;  // 0.1 x nominal density: g/cm^2 per mm
    const bool active = (rr.bits >> 8) & 1;
    const float smax = rho10 > 0.0f ? R / rho10 : INFINITY;
    const Ray r = make_ray(px, py, pz, ex, ey, ez);
    HitOut h;
    bool glitch;
    bool hit = closest_hit<false>(S, r, px, py, pz, ex, ey, ez, smax, excl, region, stack, stride,
                                  h, glitch, nv, nt);
    if (S.root_all2 >= 0) {
      HitOut h2;
      if (closest_hit<false>(S, r, px, py, pz, ex, ey, ez, hit ? h.t : smax, excl, region, stack,
                             stride, h2, glitch, nv, nt, S.root_all2)) {
        h = h2;
        hit = true;
      }
    }
    if (hit) {
      const float Rn = fmaxf(0.0f, R - rho10 * h.t);
      const float Tn = csda_energy(Rn);
      const float dep = Tcur - Tn;
      out.tot += dep;
      if (active) out.act += dep;
      Tcur = Tn;
      R = Rn;
      px = fmaf(h.t, ex, px);
      py = fmaf(h.t, ey, py);
      pz = fmaf(h.t, ez, pz);
      region = h.region_after;
      excl = h.slot;
      continue;
    }
    if (rho10 > 0.0f) {  // the range ends in this region
      out.tot += Tcur;
      if (active) out.act += Tcur;
      return out;
    }
    out.esc = Tcur;  // void and no facet ahead
    out.lost = region != 0;
    return out;
  }
  out.lost = 1;
  return out;
}

// Per-photon phases.  kSample: draw a volume-source point; kLaunch: the
// emission point is settled, draw the direction and first flight; kResume: the
// photon is done but a pair event left a second one waiting.
enum Phase : int { kNeed = 0, kTrav = 1, kParked = 2, kSetup = 3, kSample = 4, kLaunch = 5,
                   kResume = 6 };
constexpr int kMaxEmitAttempts = 1000;  // volume-source rejection tries per history
constexpr int kQueue = 128;             // screened histories a wavefront can hold
constexpr int kSlow = 128;              // set-aside short first flights a wavefront can hold
constexpr int kXcds = 8;                // accelerator dies (XCDs) of an MI355X, one L2 each
// probe direction for localising volume-source points (generic: no axis or
// facet plane of the synthetic meshes is parallel to it)
static __constant__ float kLocateDir[3] = {0.4830462f, 0.3714437f, 0.7929236f};
constexpr int kExitPlane = -2;  // best_id of a crossing through an exit plane

}  // namespace gadep
