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

// Energies in keV (0 <= E < 65536) in units of 2^-16 keV: E * 2^16 is exact in
// FP32, so rounding it to an integer in FP32 gives the same value as FP64.
__device__ __forceinline__ unsigned long long fx_kev(float e) {
  return static_cast<unsigned long long>(__float2uint_rn(e * 65536.0f));
}

__device__ __forceinline__ unsigned long long fx(double v, double scale) {
  return static_cast<unsigned long long>(__double2ll_rn(v * scale));
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
