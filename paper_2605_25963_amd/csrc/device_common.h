// Device building blocks for gfx950: counter-based RNG, ray set-up, the
// watertight facet test and BVH traversal.  Wavefronts are 64 lanes wide.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gadep_internal.h"

namespace gadep {

// Loads through pointers fetched from memory are generic (flat) unless told
// otherwise; flat loads wait on the LDS counter too.  These casts make the
// hot fetches plain global loads.
#define GADEP_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T gload(const T* p, int64_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const GADEP_GLOBAL T*)p)[i];
#else
  return p[i];  // host pass of device code: never executed
#endif
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// whose halves are mixed with the other counter words and the round key; the
// key advances by the Weyl constants between rounds.

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // full 64-bit products: one v_mad_u64_u32 each instead of a mul_lo / mul_hi pair
    const uint64_t p0 = static_cast<uint64_t>(c0) * 0xD2511F53u;
    const uint64_t p1 = static_cast<uint64_t>(c2) * 0xCD9E8D57u;
    const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
    const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
    // three-input XORs, one v_bitop3_b32 each (truth table 0x96: odd parity)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Per-history stream: counter = (draw, history lo, history hi, stream id); the
// stream id is the unit's and is passed at each draw.
// Four 32-bit outputs per call are consumed through a shift register.
struct Rng {
  uint32_t b0, b1, b2, b3;
  uint32_t left;
  uint32_t draw;
  uint32_t h_lo, h_hi;
};

__device__ __forceinline__ void rng_start(Rng& g, uint64_t history) {
  g.left = 0;
  g.draw = 0;
  g.h_lo = static_cast<uint32_t>(history);
  g.h_hi = static_cast<uint32_t>(history >> 32);
}

// One Philox block for a history: the four outputs for counter
// (draw, history lo, history hi, stream).  Kept out of line: it is called at
// most once per four uniforms, and inlining it at every draw site would
// multiply the kernel's code.
__device__ __noinline__ uint4 philox_block(uint32_t draw, uint32_t h_lo, uint32_t h_hi,
                                           uint32_t stream, uint32_t k0, uint32_t k1) {
  uint32_t c0 = draw, c1 = h_lo, c2 = h_hi, c3 = stream;
  philox4x32_10(c0, c1, c2, c3, k0, k1);
  return make_uint4(c0, c1, c2, c3);
}

// Hardware square root and natural logarithm (v_sqrt_f32, v_log_f32; about
// 1 ulp).  The sampling code takes them on positive, normal arguments only
// (uniforms in (0, 1), energies in keV, 1 - cos^2), so the IEEE wrappers'
// range reduction for denormals is not needed.
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_log(float x) {
  return __builtin_amdgcn_logf(x) * 0.693147180559945f;
}

// Uniform in (0, 1) from one 32-bit output: 23 random bits, (k + 1/2) 2^-23,
// exact in FP32 so that neither 0 nor 1 can occur.
__device__ __forceinline__ float unit_float(uint32_t x) {
  // 1 + k 2^-23 (k = the top 23 bits) minus (1 - 2^-24): exact (Sterbenz),
  // and equal to (k + 1/2) 2^-23
  return __uint_as_float(0x3F800000u | (x >> 9)) - 0.99999994f;
}

// The next uniform of a history's stream.
template <bool COUNT>
__device__ __forceinline__ float rng_u(Rng& g, uint32_t stream, uint32_t k0, uint32_t k1,
                                      uint32_t& nrng) {
  if (g.left == 0) {
    const uint4 x = philox_block(g.draw, g.h_lo, g.h_hi, stream, k0, k1);
    g.b0 = x.x;
    g.b1 = x.y;
    g.b2 = x.z;
    g.b3 = x.w;
    g.draw += 1;
    g.left = 4;
    if (COUNT) nrng++;
  }
  const uint32_t x = g.b0;
  g.b0 = g.b1;
  g.b1 = g.b2;
  g.b2 = g.b3;
  g.left -= 1;
  return unit_float(x);
}

// ---------------------------------------------------------------------------
// rays

// Per-ray constants; the origin and direction themselves are passed
// alongside (they are the photon's own position and direction).
struct Ray {
  float ix, iy, iz;     // 1/d, zero components replaced by +-2^100 reciprocals
  float oix, oiy, oiz;  // o * (1/d), for one FMA per slab plane
  float sx, sy, sz;     // shear constants
  int k;                // watertight permutation kx | ky << 2 | kz << 4, kz = dominant axis
};

__device__ __forceinline__ float pick3(float x, float y, float z, int k) {
  return k == 0 ? x : (k == 1 ? y : z);
}

// reciprocal of a direction component for the slab tests (hardware rcp, 1
// ulp; the slab test widens the exit distance by more than that)
__device__ __forceinline__ float safe_rcp(float d) {
  const float tiny = 7.8886091e-31f;  // 2^-100
  return __builtin_amdgcn_rcpf(fabsf(d) > tiny ? d : copysignf(tiny, d));
}

__device__ __forceinline__ Ray make_ray(float ox, float oy, float oz, float dx, float dy,
                                        float dz) {
  Ray r;
  r.ix = safe_rcp(dx);
  r.iy = safe_rcp(dy);
  r.iz = safe_rcp(dz);
  r.oix = ox * r.ix;
  r.oiy = oy * r.iy;
  r.oiz = oz * r.iz;
  const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
  int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  const float dkz = pick3(dx, dy, dz, kz);
  if (dkz < 0.0f) {
    const int t = kx;
    kx = ky;
    ky = t;
  }
  r.k = kx | (ky << 2) | (kz << 4);
  // shear constants: any rounding is the same for every facet the ray meets,
  // which is all the watertight test needs
  r.sz = __builtin_amdgcn_rcpf(dkz);
  r.sx = pick3(dx, dy, dz, kx) * r.sz;
  r.sy = pick3(dx, dy, dz, ky) * r.sz;
  return r;
}

// slab test of one child box; returns entry distance or +inf on a miss
__device__ __forceinline__ float slab(const Ray& r, float lx, float ly, float lz, float hx, float hy,
                                      float hz, float tmax) {
  const float t0x = fmaf(lx, r.ix, -r.oix), t1x = fmaf(hx, r.ix, -r.oix);
  const float t0y = fmaf(ly, r.iy, -r.oiy), t1y = fmaf(hy, r.iy, -r.oiy);
  const float t0z = fmaf(lz, r.iz, -r.oiz), t1z = fmaf(hz, r.iz, -r.oiz);
  const float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
  const float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
  // widen the exit distance by a few ulps so rounding never drops a box
  return tn <= tf * 1.0000005f ? tn : INFINITY;
}

__device__ __forceinline__ float edge_fn(float a, float b, float c, float d) {
#pragma clang fp contract(off)
  return a * b - c * d;
}

enum { kWtMiss = 0, kWtHit = 1, kWtDegenerate = 2 };

// Watertight ray-facet test (Woop, Benthin, Wald, JCGT 2013): the facet is
// sheared into a frame where the ray runs along +z from the origin; the 2-D
// edge functions are evaluated without contraction (recomputed in FP64 when
// one is exactly zero), so a ray never slips between facets that share an
// edge.  That decides hit or miss and the side: `entering` is true when the
// ray meets the outward (Eq. 5) side.  The distance itself is taken from the
// facet plane, t = ((v0 - o) . n) / (d . n): on long, thin facets the
// sheared-frame distance T/det loses several digits, the plane form does not.
// Hits must satisfy 0 < t <= tmax.  kWtDegenerate marks a crossing exactly on
// an edge or vertex, or a ray lying in the facet plane.
__device__ __forceinline__ int wt_test(const Ray& r, float ox, float oy, float oz, float dx,
                                       float dy, float dz, const float4 a, const float4 b,
                                       const float4 c, float tmax, float& t, bool& entering) {
  const int kx = r.k & 3, ky = (r.k >> 2) & 3, kz = r.k >> 4;
  const float Ax = a.x - ox, Ay = a.y - oy, Az = a.z - oz;
  const float Bx = a.w - ox, By = b.x - oy, Bz = b.y - oz;
  const float Cx = b.z - ox, Cy = b.w - oy, Cz = c.x - oz;
  const float akz = pick3(Ax, Ay, Az, kz), bkz = pick3(Bx, By, Bz, kz),
              ckz = pick3(Cx, Cy, Cz, kz);
  const float ax = fmaf(-r.sx, akz, pick3(Ax, Ay, Az, kx));
  const float ay = fmaf(-r.sy, akz, pick3(Ax, Ay, Az, ky));
  const float bx = fmaf(-r.sx, bkz, pick3(Bx, By, Bz, kx));
  const float by = fmaf(-r.sy, bkz, pick3(Bx, By, Bz, ky));
  const float cx = fmaf(-r.sx, ckz, pick3(Cx, Cy, Cz, kx));
  const float cy = fmaf(-r.sy, ckz, pick3(Cx, Cy, Cz, ky));
  float U = edge_fn(cx, by, cy, bx);
  float V = edge_fn(ax, cy, ay, cx);
  float W = edge_fn(bx, ay, by, ax);
  bool degenerate = false;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = static_cast<float>((double)cx * (double)by - (double)cy * (double)bx);
    V = static_cast<float>((double)ax * (double)cy - (double)ay * (double)cx);
    W = static_cast<float>((double)bx * (double)ay - (double)by * (double)ax);
    degenerate = (U == 0.0f || V == 0.0f || W == 0.0f);
  }
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return kWtMiss;
  const float det = U + V + W;
  if (det == 0.0f) return (U == 0.0f && V == 0.0f && W == 0.0f) ? kWtDegenerate : kWtMiss;
  // plane distance with the Eq. 5 normal of the facet
  const float e1x = a.w - a.x, e1y = b.x - a.y, e1z = b.y - a.z;  // v1 - v0
  const float e2x = b.z - a.x, e2y = b.w - a.y, e2z = c.x - a.z;  // v2 - v0
  const float nx = e1y * e2z - e1z * e2y;
  const float ny = e1z * e2x - e1x * e2z;
  const float nz = e1x * e2y - e1y * e2x;
  const float num = Ax * nx + Ay * ny + Az * nz;
  const float den = dx * nx + dy * ny + dz * nz;
  const float th = num * __builtin_amdgcn_rcpf(den);
  if (!(th > 0.0f) || !(th <= tmax)) return kWtMiss;
  t = th;
  entering = det > 0.0f;
  return degenerate ? kWtDegenerate : kWtHit;
}

__device__ __forceinline__ void load_node(const BvhNode* nodes, int i, float4& n0, float4& n1,
                                          float4& n2, int4& n3) {
  const float4* p = reinterpret_cast<const float4*>(nodes) + 4 * static_cast<int64_t>(i);
  n0 = gload(p, 0);
  n1 = gload(p, 1);
  n2 = gload(p, 2);
  n3 = gload(reinterpret_cast<const int4*>(p), 3);
}

__device__ __forceinline__ void load_tri(const TriRec* tris, int i, float4& a, float4& b,
                                         float4& c) {
  const float4* p = reinterpret_cast<const float4*>(tris) + 3 * static_cast<int64_t>(i);
  a = gload(p, 0);
  b = gload(p, 1);
  c = gload(p, 2);
}


// Depth-first traversal of the two-child BVH.  The pending-node stack lives in
// LDS, one column per thread (stack[i * stride]), so consecutive lanes touch
// consecutive banks.  visit_leaf(first, count, tmax) tests facets and returns
// the (possibly shrunk) tmax.  Returns the number of nodes visited.
template <class LeafFn>
__device__ __forceinline__ uint32_t traverse(const BvhNode* __restrict__ nodes, const Ray& r,
                                             float& tmax, int* stack, int stride, int cap,
                                             LeafFn&& visit_leaf, int root = 0) {
  uint32_t visits = 0;
  int sp = 0;
  int node = root;
  for (;;) {
    while (node >= 0) {
      ++visits;
      float4 n0, n1, n2;
      int4 n3;
      load_node(nodes, node, n0, n1, n2, n3);
      const float tl = slab(r, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, tmax);
      const float tr = slab(r, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, tmax);
      const bool hl = tl != INFINITY, hr = tr != INFINITY;
      if (hl && hr) {
        const bool lfirst = tl <= tr;
        const int near = lfirst ? n3.x : n3.y;
        const int far = lfirst ? n3.y : n3.x;
        if (sp < cap) {
          stack[sp * stride] = far;
          ++sp;
        }
        node = near;
      } else if (hl) {
        node = n3.x;
      } else if (hr) {
        node = n3.y;
      } else {
        node = sp > 0 ? stack[(--sp) * stride] : kDone;
      }
    }
    if (node == kDone) break;
    const int code = ~node;
    tmax = visit_leaf(code >> 3, code & 7, tmax);
    if (sp == 0) break;
    node = stack[(--sp) * stride];
  }
  return visits;
}

}  // namespace gadep
