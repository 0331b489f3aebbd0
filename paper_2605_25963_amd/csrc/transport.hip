// gfx950 kernels of the photon-transport path.
//
// One persistent grid transports every history of every (job, energy) unit.
// Per lane, a history runs segment by segment (paper Sec. 2.4.1-2.4.3):
//   emission -> free path in mean free paths -> closest boundary on the BVH
//   (watertight FP32 test, region-consistency filter) -> either cross the
//   boundary (region from the facet's inside/outside pair) or interact
//   (photoelectric, Klein-Nishina Compton, Thomson coherent) -> score.
// Work is claimed per wavefront in chunks of consecutive histories of one
// unit (large chunks first, smaller ones toward the end of the unit); a lane
// whose history ends immediately starts the next history of the chunk, and a
// wavefront only drains (waits for its live lanes) when its next chunk
// belongs to another unit.  Tallies are integer (fixed point for sums),
// accumulated per wavefront in LDS and flushed with one global atomic per
// slot, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <mutex>
#include <utility>

#include "device_common.h"
#include "gadep_internal.h"
#include "transport_common.h"

namespace gadep {

// ---------------------------------------------------------------------------
// ray-parity localization (Sec. 2.4.2): count crossings per closed geometry
// along a probe ray; odd => inside; the odd geometry crossed first contains
// the point; none odd => world.  Two traversals: the parity mask, then the
// nearest crossing among odd regions.  A probe touching an edge, vertex or
// facet plane is discarded and the next probe direction is tried.

__constant__ float kProbe[4][3] = {
    {0.4830462f, 0.3714437f, 0.7929236f},
    {-0.6651950f, 0.5306224f, -0.5252790f},
    {0.2079117f, -0.8899187f, 0.4058776f},
    {-0.3550744f, -0.4253337f, -0.8325470f},
};

template <bool COUNT>
__device__ int locate_parity(const SceneRec& sc, float px, float py, float pz, int* stack,
                             int stride, uint32_t& nvis, uint32_t& ntri, int root = 0) {
  const TriRec* __restrict__ tris = sc.tris;
  for (int k = 0; k < 4; ++k) {
    const float qx = kProbe[k][0], qy = kProbe[k][1], qz = kProbe[k][2];
    const Ray r = make_ray(px, py, pz, qx, qy, qz);
    uint64_t parity = 0;
    bool degenerate = false;
    float tm = INFINITY;
    uint32_t v = traverse(sc.nodes, r, tm, stack, stride, sc.depth, [&](int first, int count,
                                                                        float tcur) {
      for (int j = 0; j < count; ++j) {
        float4 a, b, c;
        load_tri(tris, gload(sc.slots, first + j), a, b, c);
        float t;
        bool enter;
        const int w = wt_test(r, px, py, pz, qx, qy, qz, a, b, c, INFINITY, t, enter);
        if (COUNT) ntri++;
        if (w == kWtMiss) continue;
        if (w == kWtDegenerate) degenerate = true;
        parity ^= 1ull << (__float_as_uint(c.y) & 63u);
      }
      return tcur;
    }, root);
    if (COUNT) nvis += v;
    if (degenerate) continue;
    if (parity == 0) return 0;
    float best = INFINITY;
    int best_reg = 0;
    tm = INFINITY;
    v = traverse(sc.nodes, r, tm, stack, stride, sc.depth, [&](int first, int count, float tcur) {
      for (int j = 0; j < count; ++j) {
        float4 a, b, c;
        load_tri(tris, gload(sc.slots, first + j), a, b, c);
        const int reg = static_cast<int>(__float_as_uint(c.y) & 0xFFFFu);
        if (!((parity >> reg) & 1ull)) continue;
        float t;
        bool enter;
        if (COUNT) ntri++;
        if (wt_test(r, px, py, pz, qx, qy, qz, a, b, c, tcur, t, enter) == kWtMiss) continue;
        if (t < best || (t == best && reg < best_reg)) {
          best = t;
          best_reg = reg;
        }
        tcur = t;
      }
      return tcur;
    }, root);
    if (COUNT) nvis += v;
    return best_reg;
  }
  return -1;
}

// Region of a point in a scene that may have two levels: inside an overlay
// shell (by the overlay's own parity), else by the base scene's parity.  The
// overlay's shells lie in one region of the base and cross none of its
// shells, so the two counts never mix.
template <bool COUNT>
__device__ int locate_two_level(const SceneRec& sc, float px, float py, float pz, int* stack,
                                int stride, uint32_t& nvis, uint32_t& ntri) {
  if (sc.root_all2 >= 0) {
    const int r = locate_parity<COUNT>(sc, px, py, pz, stack, stride, nvis, ntri, sc.root_all2);
    if (r != 0) return r;
  }
  return locate_parity<COUNT>(sc, px, py, pz, stack, stride, nvis, ntri, 0);
}

// ---------------------------------------------------------------------------
// transport kernel
//
// Persistent state machine.  Every iteration each lane with an open
// traversal takes one traversal step (one BVH node, or one facet test), so a
// long traversal no longer idles the rest of the wavefront.  A lane whose
// traversal has finished parks; when at least `park` lanes are parked (or no
// lane is traversing), the wavefront runs the segment outcome (boundary
// crossing, interaction, escape, scoring), takes new histories for lanes that
// need one and sets up the next traversals, for all parked lanes at once.


// GRAD: score-function tallies; SPEC: pulse-height spectra; COUNT: event
// counters; GEN: the general sources and scenes -- some unit has a volume
// source (emission points are localised by probe traversals) or a cone
// source, or a scene with overlays (a second BVH root per region); without it
// the kernel handles point and beam sources in one-level scenes; PAIR: some
// material has a pair-production partial (pair events, waiting annihilation
// photons); ELEC: secondary electrons run CSDA tracks.
template <bool GRAD, bool SPEC, bool COUNT, bool GEN, bool PAIR, bool ELEC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3)))
transport_kernel(TransportParams P) {
  extern __shared__ unsigned long long smem[];
  const int lane = static_cast<int>(__lane_id());
  // wave-uniform: its LDS areas (tally, queues) are then addressed from scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int nwaves = static_cast<int>(blockDim.x) / kWave;
  unsigned long long* wt = smem + wave * kT_Slots;  // this wavefront's tally
  int* stack = reinterpret_cast<int*>(smem + nwaves * kT_Slots) + threadIdx.x;
  const int stride = static_cast<int>(blockDim.x);
  // per-history scores of the scale groups, one LDS column per thread
  float* sc = reinterpret_cast<float*>(stack) + P.stack_depth * stride;
  // per-wavefront queues of screened histories: those that need full
  // transport, and short first flights set aside for the exact exit test
  int64_t* const qbase = reinterpret_cast<int64_t*>(
      reinterpret_cast<char*>(smem + nwaves * kT_Slots) +
      static_cast<size_t>(P.stack_depth) * stride * sizeof(int) +
      (GRAD ? static_cast<size_t>(kMaxGroups) * stride * sizeof(float) : 0));
  int64_t* queue = qbase + wave * (kQueue + kSlow);
  int64_t* slow = queue + kQueue;  // (a constant offset from queue: no register of its own)
  // the second annihilation photon of a pair event, waiting for the first to
  // be done: x, y, z, dx, dy, dz (as bits), region (< 0: none); one LDS
  // column per thread (only allocated when some material has a pair partial)
  int* wait = reinterpret_cast<int*>(qbase + nwaves * (kQueue + kSlow)) + threadIdx.x;
  if (PAIR) wait[6 * stride] = -1;
  for (int i = lane; i < kT_Slots; i += kWave) wt[i] = 0;

  const uint64_t clk_core0 = __builtin_amdgcn_s_memtime();
  const uint64_t clk_ref0 = __builtin_amdgcn_s_memrealtime();
  const uint32_t k0 = P.seed_lo, k1 = P.seed_hi;
  const int64_t total_chunks = P.chunk_begin[P.n_units];
  const int park = P.period > 0 ? (P.period > kWave ? kWave : P.period) : 24;

  // wave-uniform claim state.  Each unit has its own chunk cursor; a
  // wavefront starts on the unit that owns its share of all chunks and moves
  // to the next unit only when that one is used up, so it rarely has to
  // drain (let its open histories finish) for a change of unit.
  int claim_unit = 0;
  const int64_t n_w = static_cast<int64_t>(gridDim.x) * nwaves;
  {
    // Workgroups are dealt to the chip's kXcds dies in turn (block b runs on
    // die b % kXcds), and each die has its own L2: number the blocks die by
    // die, so that the waves of one die start on neighbouring units (for a
    // batch of jobs, the same few scenes) and keep that part of the geometry
    // in their L2.
    int64_t blk = blockIdx.x;
    if (gridDim.x % kXcds == 0)
      blk = static_cast<int64_t>(blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
    const int64_t gw = blk * nwaves + wave;
    const int64_t x = (gw * total_chunks + total_chunks / 2) / n_w;
    int lo = 0, hi = P.n_units - 1;  // unit u: chunk_begin[u] <= x < chunk_begin[u+1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (P.chunk_begin[mid] <= x)
        lo = mid;
      else
        hi = mid - 1;
    }
    claim_unit = lo;
  }
  int cur = -1;             // current unit
  int64_t next_h = 0, end_h = 0;
  int pend = -1;            // claimed chunk waiting for a drain
  int64_t pend_h0 = 0, pend_h1 = 0;
  bool exhausted = false;
  ClaimBatch claim_batch;
  UnitRec U{};
  SceneRec S{};
  int sp_cap = 0;  // stack capacity of this scene's BVHs, times the stride
  SourceRec Src{};
  // first-flight screening (see the refill below) and its queue
  bool screen = false;
  int q_head = 0, q_n = 0;
  int s_head = 0, s_n = 0;
  // the screening constants of the current unit (none: every flight is
  // evaluated; attenuation m < 0: per history)
  ScreenUnit scr;

  // lane state: photon
  int phase = kNeed;
  float px = 0, py = 0, pz = 0, dx = 0, dy = 0, dz = 1, E = 0, tau = 0;
  float edep_act = 0, edep_tot = 0;
  int region = 0, last = -1, steps = 0;
  int attempts = 0;  // > 0: localising a volume-source emission point (try number)
  bool clean = true, interacted = false, touched = false;
  bool esc_any = false;  // a photon of this history (pair events: not the last) escaped
  Xs ix{0, 0.0f};
  Rng g{};
  // lane state: current segment and its traversal
  float mu = 0, mp = 0, mc = 0;
  Ray ray{};
  float tbest = 0, trej = INFINITY;
  // sp: depth of the LDS stack times the column stride (its entries are
  // stack[k * stride]), so pushes and pops need no multiply
  int node = kDone, sp = 0, tri_next = 0, tri_end = 0, best_id = -1, best_reg = 0;
  // a leaf met while facets of an earlier one were still pending (kDone: none)
  int leaf2 = kDone;
  // a second BVH root still to search (two-level scenes; kDone: none)
  int node2 = kDone;
  // per-lane accumulators of the per-history (frequent) quantities
  unsigned long long acc_hist = 0, acc_eunc = 0, acc_esrc = 0;
  uint32_t ev[kEv_N];
#pragma unroll
  for (int i = 0; i < kEv_N; ++i) ev[i] = 0;

  auto flush = [&]() {
    if (cur < 0) return;
    const unsigned long long h = wave_sum_u64(acc_hist);
    const unsigned long long eu = wave_sum_u64(acc_eunc);
    const unsigned long long es = wave_sum_u64(acc_esrc);
    unsigned long long evs[kEv_N];
    if (COUNT) {
#pragma unroll
      for (int i = 0; i < kEv_N; ++i) evs[i] = wave_sum_u64(ev[i]);
    }
    if (lane == 0) {
      wt[kT_Hist] += h;
      wt[kT_EEsc] += eu;
      wt[kT_ESrc] += es;
      if (COUNT) {
#pragma unroll
        for (int i = 0; i < kEv_N; ++i) wt[kT_Ev + i] += evs[i];
      }
    }
    __builtin_amdgcn_wave_barrier();
    for (int i = lane; i < kT_Slots; i += kWave) {
      const unsigned long long x = wt[i];
      if (x) atomicAdd(P.tally + static_cast<int64_t>(cur) * kT_Slots + i, x);
      wt[i] = 0;
    }
    __builtin_amdgcn_wave_barrier();
    acc_hist = acc_eunc = acc_esrc = 0;
#pragma unroll
    for (int i = 0; i < kEv_N; ++i) ev[i] = 0;
  };

  auto end_history = [&](bool absorbed, bool escaped, bool lost, bool killed) {
    if (PAIR && (absorbed || escaped) && wait[6 * stride] >= 0) {
      // this photon is done; the history goes on with the waiting one
      if (escaped) {
        esc_any = true;
        atomicAdd(&wt[kT_EEsc], fx_kev(E));
      }
      phase = kResume;
      return;
    }
    phase = kNeed;
    acc_hist += 1;
    if (escaped) {
      if (interacted) {
        atomicAdd(&wt[kT_CollEscape], 1ull);
        atomicAdd(&wt[kT_EEsc], fx_kev(E));
      } else {
        acc_eunc += fx_kev(E);
      }
    } else if (esc_any && !lost && !killed) {
      atomicAdd(&wt[kT_CollEscape], 1ull);  // an earlier photon of the history escaped
    }
    if (esc_any) {
      absorbed = false;
      esc_any = false;
    }
    if (PAIR) wait[6 * stride] = -1;
    const bool fep = absorbed && clean;
    if (absorbed) atomicAdd(&wt[kT_Absorbed], 1ull);
    if (fep) atomicAdd(&wt[kT_Fep], 1ull);
    if (lost) atomicAdd(&wt[kT_Lost], 1ull);
    if (killed) atomicAdd(&wt[kT_Killed], 1ull);
    if (edep_tot > 0.0f) atomicAdd(&wt[kT_EdepTot], fx_kev(edep_tot));
    if (edep_act > 0.0f) {
      atomicAdd(&wt[kT_EdepAct], fx_kev(edep_act));
      if (SPEC) {
        const float ch = floorf(edep_act * P.inv_channel_kev);
        if (ch < static_cast<float>(P.n_channels))
          atomicAdd(P.spectra + static_cast<int64_t>(cur) * P.n_channels + static_cast<int>(ch),
                    1ull);
        else
          atomicAdd(&wt[kT_SpecOvf], 1ull);
      }
    }
    if (GRAD && touched) {
      for (int i = 0; i < U.n_groups; ++i) {
        const float si = sc[i * stride];
        if (si == 0.0f) continue;
        const double s = static_cast<double>(si);
        atomicAdd(&wt[kT_Score + i], fx(s, kScoreFix));
        if (fep) {
          atomicAdd(&wt[kT_FepScore + i], fx(s, kScoreFix));
          const double x = s * s * kScore2Fix;
          const double xi = floor(x);
          atomicAdd(&wt[kT_FepScore2 + i], static_cast<unsigned long long>(xi));
          atomicAdd(&wt[kT_FepScore2Lo + i], fx(x - xi, static_cast<double>(1 << kScore2LoBits)));
        }
      }
    }
  };

  // kinetic energy T given to an electron where the photon is, moving along
  // (ex, ey, ez): a CSDA track when electrons are on (returns true if it
  // ended lost), else deposited in place
  auto electron = [&](float T, float ex, float ey, float ez, bool active) -> bool {
    if (ELEC && T >= kElecMin) {
      if (COUNT) ev[kEv_Electrons]++;
      const ElecOut eo = electron_track(P.scenes + U.scene, P.regions + U.region_off, px, py, pz,
                                        ex, ey, ez, T, region, stack, stride);
      edep_tot += eo.tot;
      edep_act += eo.act;
      if (eo.tot > eo.act || eo.esc > 0.0f) clean = false;
      if (eo.esc > 0.0f) atomicAdd(&wt[kT_EEsc], fx_kev(eo.esc));
      return eo.lost != 0;
    }
    edep_tot += T;
    if (active)
      edep_act += T;
    else
      clean = false;
    return false;
  };

  // a point of a volume source, uniform in its cylindrical annulus
  auto sample_point = [&]() {
    const float r2lo = Src.r_in * Src.r_in, r2hi = Src.r_out * Src.r_out;
    const float rr2 = hw_sqrt(fmaf(rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]), r2hi - r2lo, r2lo));
    const float uphi = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]);
    px = Src.pos[0] + rr2 * __builtin_amdgcn_cosf(uphi);
    py = Src.pos[1] + rr2 * __builtin_amdgcn_sinf(uphi);
    pz = Src.pos[2] + rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]) * Src.h;
  };

  // the emission point is settled (region known): direction, first flight
  auto begin_flight = [&]() {
    acc_esrc += fx_kev(E);
    if (Src.kind == kBeam) {
      dx = Src.dir[0];
      dy = Src.dir[1];
      dz = Src.dir[2];
    } else if (GEN && Src.kind == kCone && Src.cone_cos > -1.0f) {
      // uniform in the cone about the axis: cos theta uniform in [cone_cos, 1]
      const float ct = fmaf(-rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]), 1.0f - Src.cone_cos, 1.0f);
      dx = Src.dir[0];
      dy = Src.dir[1];
      dz = Src.dir[2];
      turn(dx, dy, dz, ct, rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]));
    } else {
      const float ct = fmaf(2.0f, rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]), -1.0f);
      const float st = hw_sqrt(fmaxf(0.0f, 1.0f - ct * ct));
      const float uphi = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]);
      dx = st * __builtin_amdgcn_cosf(uphi);
      dy = st * __builtin_amdgcn_sinf(uphi);
      dz = ct;
    }
    tau = -hw_log(rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]));
    ix = xs_index(E, P.ln_e0, P.inv_dlne, P.n_e);
    edep_act = edep_tot = 0.0f;
    clean = true;
    interacted = touched = false;
    esc_any = false;
    last = -1;
    steps = 0;
    if (GRAD)
      for (int i = 0; i < U.n_groups; ++i) sc[i * stride] = 0.0f;
    phase = kSetup;
  };

  for (;;) {
    const uint64_t trav = __ballot(phase == kTrav);
    if (trav == 0 || __popcll(__ballot(phase == kParked || phase == kNeed)) >= park) {
      // ================= housekeeping for every parked lane =================
      if (COUNT && lane == 0) ev[kEv_Passes]++;
      uint64_t clk = COUNT ? __builtin_amdgcn_s_memtime() : 0;
      auto lap = [&](int slot) {
        if (COUNT) {
          const uint64_t now = __builtin_amdgcn_s_memtime();
          if (lane == 0) ev[slot] += static_cast<uint32_t>(now - clk);
          clk = now;
        }
      };
      if (GEN && phase == kParked && attempts > 0) {
        // ---- a volume-source point was localised: the region on the near
        // side of the first facet along the probe ray (the world if none)
        const int here = best_id != -1 ? (best_reg >> 8) : 0;
        if (here == Src.region) {
          attempts = 0;
          region = here;
          phase = kLaunch;
        } else if (attempts < kMaxEmitAttempts) {
          phase = kSample;
        } else {
          attempts = 0;
          atomicAdd(&wt[kT_SrcFail], 1ull);
          acc_hist += 1;
          phase = kNeed;
        }
      } else if (phase == kParked) {
        // ---- outcome of the finished traversal
        if (trej < tbest) atomicAdd(&wt[kT_Glitch], 1ull);
        const RegionRec rr = gload(P.regions, U.region_off + region);
        const int grp = rr.bits & 0xFF;
        const bool active = (rr.bits >> 8) & 1;
        phase = kSetup;
        if (++steps > P.max_steps) {
          clean = false;
          end_history(false, false, false, true);
        } else if (best_id != -1) {
          // boundary crossing (a facet, or the outermost shell's exit plane)
          if (COUNT) ev[kEv_Crossings]++;
          if (GRAD && grp < kMaxGroups) {
            sc[grp * stride] -= mu * rr.inv_scale * tbest;
            touched = true;
          }
          px = fmaf(tbest, dx, px);
          py = fmaf(tbest, dy, py);
          pz = fmaf(tbest, dz, pz);
          tau = fmaxf(0.0f, fmaf(-mu, tbest, tau));
          region = best_reg & 0xFF;
          last = best_id;
          if (region == 0 && (U.flags & kUnitExitEscapes)) {
            // left the convex outermost shell into the void world: nothing ahead
            clean = false;
            end_history(false, true, false, false);
          }
        } else if (mu > 0.0f) {
          // interaction at the end of the flight
          const float s = tau / mu;
          px = fmaf(s, dx, px);
          py = fmaf(s, dy, py);
          pz = fmaf(s, dz, pz);
          if (GRAD && grp < kMaxGroups) {
            sc[grp * stride] += rr.inv_scale - mu * rr.inv_scale * s;
            touched = true;
          }
          last = -1;
          interacted = true;
          const float x = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]) * mu;
          if (x < mp) {
            if (COUNT) ev[kEv_Photo]++;
            bool lost_e = false;
            if (ELEC && E >= kElecMin) {
              // the photoelectron leaves isotropically (synthetic reading)
              const float ce = fmaf(2.0f, rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]), -1.0f);
              const float se = hw_sqrt(fmaxf(0.0f, 1.0f - ce * ce));
              const float ue = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]);
              lost_e = electron(E, se * __builtin_amdgcn_cosf(ue), se * __builtin_amdgcn_sinf(ue), ce,
                                active);
            } else {
              electron(E, 0.0f, 0.0f, 1.0f, active);
            }
            end_history(!lost_e, false, lost_e, false);
          } else {
            bool absorbed = false;
            if (x < mp + mc) {
              // Klein-Nishina by the composition-rejection of Butcher and Messel
              // (1960): eps = E'/E on [e0, 1] is drawn from the 1/eps or the eps
              // part of (1/eps + eps) with weights ln(1/e0) and (1 - e0^2)/2, and
              // accepted with probability 1 - eps sin^2 / (1 + eps^2).
              if (COUNT) ev[kEv_Compton]++;
              const float k = E * (1.0f / kMec2);
              const float e0 = 1.0f / fmaf(2.0f, k, 1.0f);
              const float e02 = e0 * e0;
              const float a1 = -hw_log(e0);
              const float a2 = 0.5f * (1.0f - e02);
              float eps = 1.0f, t = 0.0f;
              for (int it = 0; it < 64; ++it) {
                const float u1 = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]);
                const float u2 = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]);
                const float u3 = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]);
                float eps2;
                if (u1 * (a1 + a2) < a1) {
                  eps = __expf(-a1 * u2);
                  eps2 = eps * eps;
                } else {
                  eps2 = fmaf(1.0f - e02, u2, e02);
                  eps = hw_sqrt(eps2);
                }
                t = (1.0f - eps) / (k * eps);
                const float sin2 = t * (2.0f - t);
                if (u3 * (1.0f + eps2) <= 1.0f + eps2 - eps * sin2) break;
              }
              const float Ep = eps * E;
              const float dep = E - Ep;
              const float uph = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]);
              bool lost_e = false;
              if (ELEC && dep >= kElecMin) {
                // the recoil electron: in the scattering plane, on the other
                // side, at cot(theta_e) = (1 + k) tan(theta / 2)
                const float ctg = 1.0f - t;
                const float a = (1.0f + k) * hw_sqrt(fmaxf(0.0f, 1.0f - ctg * ctg)), b = 1.0f + ctg;
                float ex = dx, ey = dy, ez = dz;
                turn(ex, ey, ez, a * rsqrtf(fmaf(a, a, b * b)), uph + 0.5f);
                lost_e = electron(dep, ex, ey, ez, active);
              } else {
                electron(dep, 0.0f, 0.0f, 1.0f, active);
              }
              turn(dx, dy, dz, 1.0f - t, uph);
              E = Ep;
              if (lost_e) {
                end_history(false, false, true, false);
                absorbed = true;  // the history is over
              } else if (E < P.e_cut) {
                edep_tot += E;
                if (active)
                  edep_act += E;
                else
                  clean = false;
                end_history(true, false, false, false);
                absorbed = true;
              } else {
                ix = xs_index(E, P.ln_e0, P.inv_dlne, P.n_e);
              }
            } else if (!(PAIR && E > 2.0f * kMec2) ||
                       x < mu - xs_pair(reinterpret_cast<const float4*>(P.xs), P.n_e, rr, ix, E, true)) {
              // coherent: Thomson law 3/8 (1 + mu^2); its CDF (mu^3 + 3 mu + 4)/8
              // inverts in closed form (Cardano): with a = 4u - 2,
              // mu = c - 1/c, c = cbrt(a + sqrt(a^2 + 1)), taken on |a| for accuracy
              if (COUNT) ev[kEv_Coherent]++;
              const float a = fmaf(4.0f, rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]), -2.0f);
              const float c = cbrtf(fabsf(a) + sqrtf(fmaf(a, a, 1.0f)));
              const float ct = copysignf(c - 1.0f / c, a);
              turn(dx, dy, dz, fminf(1.0f, fmaxf(-1.0f, ct)), rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]));
            } else {
              // pair production: the photon is gone; the pair's kinetic energy
              // E - 2 m_e c^2 is deposited here and the positron annihilates at
              // rest into two 511 keV photons flying apart along a random axis.
              // This lane follows the first; the second waits in LDS.
              if (COUNT) ev[kEv_Pair]++;
              const float kin = E - 2.0f * kMec2;
              // the pair's kinetic energy as one track along the photon (reading)
              if (electron(kin, dx, dy, dz, active)) {
                end_history(false, false, true, false);
                absorbed = true;  // the history is over
              } else {
                const float ct = fmaf(2.0f, rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]), -1.0f);
                const float st = hw_sqrt(fmaxf(0.0f, 1.0f - ct * ct));
                const float uphi = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]);
                dx = st * __builtin_amdgcn_cosf(uphi);
                dy = st * __builtin_amdgcn_sinf(uphi);
                dz = ct;
                wait[0] = __float_as_int(px);
                wait[stride] = __float_as_int(py);
                wait[2 * stride] = __float_as_int(pz);
                wait[3 * stride] = __float_as_int(-dx);
                wait[4 * stride] = __float_as_int(-dy);
                wait[5 * stride] = __float_as_int(-dz);
                wait[6 * stride] = region;
                E = kMec2;
                ix = xs_index(E, P.ln_e0, P.inv_dlne, P.n_e);
              }
            }
            if (!absorbed) tau = -hw_log(rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]));
          }
        } else {
          // vacuum and no facet ahead: escape from the world, otherwise lost
          clean = false;
          if (region == 0)
            end_history(false, true, false, false);
          else
            end_history(false, false, true, false);
        }
      }

      if (PAIR && phase == kResume) {
        // the waiting annihilation photon takes over the lane
        px = __int_as_float(wait[0]);
        py = __int_as_float(wait[stride]);
        pz = __int_as_float(wait[2 * stride]);
        dx = __int_as_float(wait[3 * stride]);
        dy = __int_as_float(wait[4 * stride]);
        dz = __int_as_float(wait[5 * stride]);
        region = wait[6 * stride];
        wait[6 * stride] = -1;
        E = kMec2;
        ix = xs_index(E, P.ln_e0, P.inv_dlne, P.n_e);
        last = -1;
        tau = -hw_log(rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]));
        phase = kSetup;
      }
      lap(kEv_CycOutcome);
      // ---- new histories for lanes that need one (chunks of the wave's unit)
      const uint64_t need = __ballot(phase == kNeed);
      if (need) {
        const int n_need = __popcll(need);
        for (;;) {
          if (next_h >= end_h && pend < 0 && !exhausted) {
            // next chunk of the claim unit, else of the units after it in turn
            for (int t = 0; t < P.n_units; ++t) {
              int64_t h1 = 0;
              const int64_t h0 = claim_histories(P, claim_unit, n_w, lane, claim_batch, h1);
              if (h0 < h1) {
                pend = claim_unit;
                pend_h0 = h0;
                pend_h1 = h1;
                break;
              }
              claim_unit = claim_unit + 1 == P.n_units ? 0 : claim_unit + 1;
            }
            if (pend < 0) exhausted = true;
          }
          // a chunk of another unit starts only when no history of this one
          // is open or queued
          if (next_h >= end_h && pend >= 0 &&
              (pend == cur || (q_n == 0 && s_n == 0 && __ballot(phase != kNeed) == 0))) {
            if (pend != cur) {
              flush();
              cur = pend;
              U = P.units[cur];
              S = P.scenes[U.scene];
              sp_cap = S.depth * stride;
              Src = P.sources[U.source];
              const RegionRec ro = gload(P.regions, U.region_off + S.outer_region);
              screen = P.screen && (U.flags & kUnitExitPlanes) && Src.kind != kCyl &&
                       U.src_region == S.outer_region && (!GRAD || (ro.bits & 0xFF) == 0xFF);
              scr = ScreenUnit();
              if (screen && Src.n_lines == 0)
                scr = screen_unit(S, Src, ro, U.energy, reinterpret_cast<const float4*>(P.xs), P.n_e,
                                  P.ln_e0, P.inv_dlne, PAIR);
            }
            next_h = pend_h0;
            end_h = pend_h1;
            pend = -1;
          }
          if (!(screen && q_n < n_need)) break;
          // ---- first-flight screening: every lane takes one of the next 64
          // histories and follows it to the end of its first flight.  Those
          // that leave the outermost shell through its planes without coming
          // near the inner shells (the common case for a distant source) are
          // tallied here; the rest are queued for full transport, which
          // repeats the same draws and arithmetic.  A flight whose optical
          // depth is long enough to cross the whole shell (almost all of them)
          // is settled by one box test; the few shorter ones are set aside in
          // a second queue and settled exactly, by the exit planes, 64 at a
          // time, so that their rare branch runs with full wavefronts.
          const bool exact = s_n >= kWave || (next_h >= end_h && s_n > 0);
          if (!exact && next_h >= end_h) break;
          int64_t h = -1;
          if (exact) {
            if (lane < s_n) h = slow[(s_head + lane) & (kSlow - 1)];
            __builtin_amdgcn_wave_barrier();
            const int taken = s_n < kWave ? s_n : kWave;
            s_head = (s_head + taken) & (kSlow - 1);
            s_n -= taken;
          } else {
            h = next_h + lane < end_h ? next_h + lane : -1;
            next_h = next_h + kWave < end_h ? next_h + kWave : end_h;
          }
          bool survivor = false, defer = false;
          if (h >= 0) {
            const uint64_t hist = static_cast<uint64_t>(U.first + h);
            // the first block of the history's stream, inline: the key and
            // the stream id are wave-uniform, so the round keys stay scalar
            uint32_t c0 = 0u, c1 = static_cast<uint32_t>(hist), c2 = static_cast<uint32_t>(hist >> 32),
                     c3 = U.stream;
            philox4x32_10(c0, c1, c2, c3, k0, k1);
            float u0 = unit_float(c0), u1 = unit_float(c1), u2 = unit_float(c2);
            const float u3 = unit_float(c3);
            float e = U.energy;
            if (Src.n_lines > 0) {
              const float2* L = reinterpret_cast<const float2*>(P.lines) + Src.line_off;
              int pick = Src.n_lines - 1;
              for (int i = 0; i < Src.n_lines; ++i)
                if (u0 < L[i].y) {
                  pick = i;
                  break;
                }
              e = L[pick].x;
              u0 = u1;
              u1 = u2;
              u2 = u3;
            }
            float qx = Src.dir[0], qy = Src.dir[1], qz = Src.dir[2];
            if (GEN && Src.kind == kCone && Src.cone_cos > -1.0f) {
              // the same draws as begin_flight's cone branch
              turn(qx, qy, qz, fmaf(-u0, 1.0f - Src.cone_cos, 1.0f), u1);
              u0 = u2;
            } else if (Src.kind != kBeam) {
              const float ct = fmaf(2.0f, u0, -1.0f);
              const float st = hw_sqrt(fmaxf(0.0f, 1.0f - ct * ct));
              qx = st * __builtin_amdgcn_cosf(u1);
              qy = st * __builtin_amdgcn_sinf(u1);
              qz = ct;
              u0 = u2;
            }
            const float tau0 = -hw_log(u0);
            const float ox = Src.pos[0], oy = Src.pos[1], oz = Src.pos[2];
            bool escapes = false;
            float te = scr.far;
            // the flight outlasts the shell (the common case): no need for
            // the attenuation or the exit distance, only for the box test --
            // and not even that when the direction misses the sphere around
            // the box; the few settled ones that head for the sphere wait for
            // a full batch of such histories and take the box test there
            const bool settled = tau0 >= scr.tau;
            const bool far_off = fmaf(qx, scr.ax, fmaf(qy, scr.ay, qz * scr.az)) < scr.cos;
            if (settled) {
              if (far_off || exact)
                escapes = true;
              else
                defer = true;
            } else if (exact || scr.m < 0.0f) {
              // (with a line spectrum nothing is settled early: no deferral)
              float m = scr.m;  // the unit's, for a fixed energy
              if (m < 0.0f) {
                const RegionRec rr = gload(P.regions, U.region_off + S.outer_region);
                float m_p, m_c, m_h;
                const Xs ixe = xs_index(e, P.ln_e0, P.inv_dlne, P.n_e);
                xs_mu(reinterpret_cast<const float4*>(P.xs), P.n_e, rr, ixe, m_p, m_c, m_h);
                m = m_p + m_c + m_h + xs_pair(reinterpret_cast<const float4*>(P.xs), P.n_e, rr, ixe, e, PAIR);
              }
              const float tfl = m > 0.0f ? tau0 / m : INFINITY;
              te = INFINITY;
              for (int i = 0; i < S.n_planes; ++i) {
                const float4 pl = gload(reinterpret_cast<const float4*>(S.planes), i);
                const float dn = pl.x * qx + pl.y * qy + pl.z * qz;
                const float num = pl.w - (pl.x * ox + pl.y * oy + pl.z * oz);
                if (dn > 0.0f) te = fminf(te, num * __builtin_amdgcn_rcpf(dn));
              }
              te = fmaxf(te, 0.0f);
              escapes = te <= tfl;
            } else {
              defer = true;
            }
            if (escapes && !far_off && S.trans_lo[0] <= S.trans_hi[0]) {
              const Ray r0 = make_ray(ox, oy, oz, qx, qy, qz);
              escapes = slab(r0, S.trans_lo[0], S.trans_lo[1], S.trans_lo[2], S.trans_hi[0],
                             S.trans_hi[1], S.trans_hi[2], te) == INFINITY;
            }
            if (escapes) {
              acc_hist += 1;
              acc_esrc += fx_kev(e);
              acc_eunc += fx_kev(e);
              if (COUNT) {
                // (leaving the world here takes no crossing step: none is counted)
                ev[kEv_Emissions]++;
                ev[kEv_Rng]++;
                if (settled) {
                  ev[far_off ? kEv_ConeTests : kEv_BoxTests]++;
                } else {
                  ev[kEv_Segments]++;
                  ev[kEv_PlaneTests] += S.n_planes;
                }
              }
            } else if (!defer) {
              survivor = true;
            }
          }
          const uint64_t surv = __ballot(survivor);
          if (survivor) {
            const int rank = __popcll(surv & ((1ull << lane) - 1ull));
            queue[(q_head + q_n + rank) & (kQueue - 1)] = h;
          }
          const uint64_t dfr = __ballot(defer);
          if (defer) {
            const int rank = __popcll(dfr & ((1ull << lane) - 1ull));
            slow[(s_head + s_n + rank) & (kSlow - 1)] = h;
          }
          __builtin_amdgcn_wave_barrier();
          q_n += __popcll(surv);
          s_n += __popcll(dfr);
        }
        // hand out histories: from the queue when screening, else in order
        const uint64_t below = need & ((1ull << lane) - 1ull);
        const int rank = __popcll(below);
        int64_t h = -1;
        if (screen) {
          if (phase == kNeed && rank < q_n) h = queue[(q_head + rank) & (kQueue - 1)];
          __builtin_amdgcn_wave_barrier();
          const int taken = n_need < q_n ? n_need : q_n;
          q_head = (q_head + taken) & (kQueue - 1);
          q_n -= taken;
        } else if (next_h < end_h) {
          if (phase == kNeed && next_h + rank < end_h) h = next_h + rank;
          next_h += n_need;
          if (next_h > end_h) next_h = end_h;
        }
        if (phase == kNeed && h >= 0) {
          // ---- emission
          rng_start(g, static_cast<uint64_t>(U.first + h));
          if (COUNT) ev[kEv_Emissions]++;
          if (Src.n_lines > 0) {
            const float x = rng_u<COUNT>(g, U.stream, k0, k1, ev[kEv_Rng]);
            const float2* L = reinterpret_cast<const float2*>(P.lines) + Src.line_off;
            int pick = Src.n_lines - 1;
            for (int i = 0; i < Src.n_lines; ++i)
              if (x < L[i].y) {
                pick = i;
                break;
              }
            E = L[pick].x;
          } else {
            E = U.energy;
          }
          if (GEN && Src.kind == kCyl) {
            // rejection sampling: each point is localised by a probe traversal
            attempts = 0;
            phase = kSample;
          } else {
            px = Src.pos[0];
            py = Src.pos[1];
            pz = Src.pos[2];
            region = U.src_region;
            if (region >= 0) {
              phase = kLaunch;
            } else {
              atomicAdd(&wt[kT_SrcFail], 1ull);
              acc_hist += 1;
            }
          }
        }
      }

      lap(kEv_CycRefill);
      if (GEN && phase == kSample) {
        // next try of a volume-source point
        ++attempts;
        sample_point();
        phase = kSetup;
      }
      if (phase == kLaunch) begin_flight();
      lap(kEv_CycLaunch);

      // ---- set up the next segment: attenuation, flight limit, ray
      if (GEN && phase == kSetup && attempts > 0) {
        // probe ray of a volume-source point.  The point lies in the source
        // region exactly when the nearest facet along the ray that bounds
        // that region is met from its inside, so only the region's own BVH
        // is searched.
        if (COUNT) ev[kEv_Locates]++;
        dx = kLocateDir[0];
        dy = kLocateDir[1];
        dz = kLocateDir[2];
        ray = make_ray(px, py, pz, dx, dy, dz);
        region = -1;
        last = -1;
        mu = 0.0f;
        tbest = INFINITY;
        trej = INFINITY;
        node = gload(S.roots, Src.region);
        node2 = GEN && S.roots2 ? gload(S.roots2, Src.region) : kDone;
        if (node == kDone) {
          node = node2;
          node2 = kDone;
        }
        sp = 0;
        tri_next = tri_end = 0;
        leaf2 = kDone;
        best_id = -1;
        phase = node == kDone ? kParked : kTrav;
      } else if (phase == kSetup) {
        if (COUNT) ev[kEv_Segments]++;
        const RegionRec rr = gload(P.regions, U.region_off + region);
        float mh;
        xs_mu(reinterpret_cast<const float4*>(P.xs), P.n_e, rr, ix, mp, mc, mh);
        mu = mp + mc + mh + xs_pair(reinterpret_cast<const float4*>(P.xs), P.n_e, rr, ix, E, PAIR);
        tbest = mu > 0.0f ? tau / mu : INFINITY;
        ray = make_ray(px, py, pz, dx, dy, dz);
        trej = INFINITY;
        sp = 0;
        tri_next = tri_end = 0;
        leaf2 = kDone;
        best_id = -1;
        // the BVH of the facets that bound this region: no other facet can
        // be crossed next
        if ((U.flags & kUnitExitPlanes) && region == S.outer_region) {
          // the outer shell's own region: its boundary is the nearest of the
          // planes the ray runs towards, and only the shells inside it are
          // searched
          float te = INFINITY;
          for (int i = 0; i < S.n_planes; ++i) {
            const float4 pl = gload(reinterpret_cast<const float4*>(S.planes), i);
            const float dn = pl.x * dx + pl.y * dy + pl.z * dz;
            const float num = pl.w - (pl.x * px + pl.y * py + pl.z * pz);
            if (dn > 0.0f) te = fminf(te, num * __builtin_amdgcn_rcpf(dn));
          }
          if (COUNT) ev[kEv_PlaneTests] += S.n_planes;
          te = fmaxf(te, 0.0f);
          if (te <= tbest) {
            tbest = te;
            best_id = kExitPlane;
            best_reg = 0;
          }
          node = S.outer_root;
          node2 = GEN && S.roots2 ? gload(S.roots2, region) : kDone;
          if (!(S.trans_lo[0] <= S.trans_hi[0]) ||
              slab(ray, S.trans_lo[0], S.trans_lo[1], S.trans_lo[2], S.trans_hi[0], S.trans_hi[1],
                   S.trans_hi[2], tbest) == INFINITY)
            node = node2 = kDone;  // no inner shell ahead within the flight
        } else {
          node = gload(S.roots, region);
          node2 = GEN && S.roots2 ? gload(S.roots2, region) : kDone;
        }
        if (node == kDone) {
          node = node2;
          node2 = kDone;
        }
        phase = node == kDone ? kParked : kTrav;
      }
      lap(kEv_CycSetup);
      if (__ballot(phase != kNeed) == 0 && exhausted && pend < 0 && next_h >= end_h && q_n == 0 &&
          s_n == 0)
        break;
    }

    // ================= one traversal step per traversing lane =================
    // One node and one facet per lane and iteration.  A lane keeps walking the
    // tree while facets of a leaf are still pending (speculative traversal,
    // Aila and Laine 2009): a second leaf it meets waits in `leaf2`, so that
    // node and facet steps overlap instead of alternating.  Nodes are culled
    // with the nearest hit found so far, which can only keep more of them.
    bool did_node = false, did_tri = false;
    const uint64_t clk_trav = COUNT ? __builtin_amdgcn_s_memtime() : 0;
    if (phase == kTrav) {
      const bool busy = tri_next < tri_end;
      if (node < 0 && node != kDone && (!busy || leaf2 == kDone)) {
        // a leaf taken from the stack (or a far child): test it now, or
        // postpone it and keep walking
        const int code = ~node;
        if (!busy) {
          tri_next = code >> 3;
          tri_end = tri_next + (code & 7);
        } else {
          leaf2 = node;
        }
        node = sp > 0 ? stack[sp -= stride] : kDone;
      } else if (node >= 0 && (!busy || leaf2 == kDone)) {
        // one node: both child boxes against [0, tbest]
        if (COUNT) ev[kEv_NodeVisits]++;
        did_node = true;
        float4 n0, n1, n2;
        int4 n3;
        load_node(S.nodes, node, n0, n1, n2, n3);
        const float tl = slab(ray, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, tbest);
        const float tr = slab(ray, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, tbest);
        const bool hl = tl != INFINITY, hr = tr != INFINITY;
        int near = kDone, far = kDone;
        if (hl && hr) {
          const bool lfirst = tl <= tr;
          near = lfirst ? n3.x : n3.y;
          far = lfirst ? n3.y : n3.x;
        } else if (hl) {
          near = n3.x;
        } else if (hr) {
          near = n3.y;
        }
        if (near == kDone) {
          node = sp > 0 ? stack[sp -= stride] : kDone;
        } else if (near < 0) {
          // nearest child is a leaf: test its facets next (or after the
          // pending ones), then go to `far`
          if (!busy) {
            const int code = ~near;
            tri_next = code >> 3;
            tri_end = tri_next + (code & 7);
          } else {
            leaf2 = near;
          }
          node = far != kDone ? far : (sp > 0 ? stack[sp -= stride] : kDone);
        } else {
          if (far != kDone && sp < sp_cap) {
            stack[sp] = far;
            sp += stride;
          }
          node = near;
        }
      }
      if (tri_next >= tri_end && leaf2 != kDone) {
        const int code = ~leaf2;
        tri_next = code >> 3;
        tri_end = tri_next + (code & 7);
        leaf2 = kDone;
      }
      if (tri_next < tri_end) {
        // one facet test, with the region-consistency filter; the facet just
        // crossed is skipped (by its caller id: it may have several slots)
        const int slot = tri_next++;
        if (COUNT) ev[kEv_TriTests]++;
        did_tri = true;
        float4 a, b, c;
        load_tri(S.tris, gload(S.slots, slot), a, b, c);
        const int id = __float_as_int(c.z);
        float t;
        bool enter;
        if (id != last && wt_test(ray, px, py, pz, dx, dy, dz, a, b, c, tbest, t, enter) != kWtMiss) {
          const uint32_t regs = __float_as_uint(c.y);
          const int inside = static_cast<int>(regs & 0xFFFFu);
          const int outside = static_cast<int>(regs >> 16);
          const int before = enter ? outside : inside;
          if (region >= 0 && before != region) {
            trej = fminf(trej, t);
          } else {
            tbest = t;
            best_id = id;
            best_reg = (enter ? inside : outside) | (before << 8);  // after | before << 8
          }
        }
      }
      if (tri_next >= tri_end && node == kDone && leaf2 == kDone) {
        if (GEN && node2 != kDone) {
          // the second level: same ray, nearest hit so far kept
          node = node2;
          node2 = kDone;
        } else {
          phase = kParked;
        }
      }
    }
    if (COUNT) {
      const bool any_node = __ballot(did_node) != 0, any_tri = __ballot(did_tri) != 0;
      const uint64_t now = __builtin_amdgcn_s_memtime();
      if (lane == 0) {
        ev[kEv_CycTrav] += static_cast<uint32_t>(now - clk_trav);
        ev[kEv_Iters]++;
        if (any_node) ev[kEv_ItersNode]++;
        if (any_tri) ev[kEv_ItersTri]++;
      }
    }
  }
  if (lane == 0) {
    wt[kT_ClkCore] += __builtin_amdgcn_s_memtime() - clk_core0;
    wt[kT_ClkRef] += __builtin_amdgcn_s_memrealtime() - clk_ref0;
  }
  __builtin_amdgcn_wave_barrier();
  flush();
}

// ---------------------------------------------------------------------------
// small kernels

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// region of each unit's point/beam origin
__global__ void locate_units_kernel(UnitRec* units, int n_units, const SceneRec* scenes,
                                    const SourceRec* sources, int stack_depth) {
  extern __shared__ int lstack[];
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n_units) return;
  UnitRec& U = units[u];
  const SourceRec s = sources[U.source];
  uint32_t a = 0, b = 0;
  if (s.kind == kCyl) {
    U.src_region = s.region;
  } else {
    U.src_region = locate_two_level<false>(scenes[U.scene], s.pos[0], s.pos[1], s.pos[2],
                                           lstack + threadIdx.x, blockDim.x, a, b);
  }
  (void)stack_depth;
}

// Philox4x32-10 blocks of the transport kernel's generator for given counters
__global__ void philox_kernel(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n,
                              uint32_t* out) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  uint32_t c0 = ctr[4 * i], c1 = ctr[4 * i + 1], c2 = ctr[4 * i + 2], c3 = ctr[4 * i + 3];
  philox4x32_10(c0, c1, c2, c3, k0, k1);
  out[4 * i] = c0;
  out[4 * i + 1] = c1;
  out[4 * i + 2] = c2;
  out[4 * i + 3] = c3;
}

__global__ void raycast_kernel(SceneRec sc, const float* o, const float* d, const int32_t* region,
                               int64_t n, float* t, int32_t* tri, int32_t* region_after) {
  extern __shared__ int lstack[];
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const float ox = o[3 * i], oy = o[3 * i + 1], oz = o[3 * i + 2];
  const float dx = d[3 * i], dy = d[3 * i + 1], dz = d[3 * i + 2];
  const Ray r = make_ray(ox, oy, oz, dx, dy, dz);
  HitOut h;
  bool glitch;
  uint32_t a = 0, b = 0;
  const int cur = region ? region[i] : -1;
  bool hit = closest_hit<false>(sc, r, ox, oy, oz, dx, dy, dz, INFINITY, -1, cur,
                                lstack + threadIdx.x, blockDim.x, h, glitch, a, b);
  if (sc.root_all2 >= 0) {
    HitOut h2;
    if (closest_hit<false>(sc, r, ox, oy, oz, dx, dy, dz, hit ? h.t : INFINITY, -1, cur,
                           lstack + threadIdx.x, blockDim.x, h2, glitch, a, b, sc.root_all2)) {
      h = h2;
      hit = true;
    }
  }
  if (hit) {
    t[i] = h.t;
    // the facet's number in the (combined) scene, from its record
    float4 fa, fb, fc;
    load_tri(sc.tris, gload(sc.slots, h.slot), fa, fb, fc);
    tri[i] = __float_as_int(fc.z);
    region_after[i] = h.region_after;
  } else {
    t[i] = INFINITY;
    tri[i] = -1;
    region_after[i] = -1;
  }
}

__global__ void locate_kernel(SceneRec sc, const float* p, int64_t n, int32_t* region) {
  extern __shared__ int lstack[];
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  uint32_t a = 0, b = 0;
  region[i] = locate_two_level<false>(sc, p[3 * i], p[3 * i + 1], p[3 * i + 2],
                                      lstack + threadIdx.x, blockDim.x, a, b);
}

// Gaussian broadening: one thread per output channel gathers from the input
// channels whose 5-sigma window reaches it.
__global__ void broaden_kernel(const double* in, double* out, int n_spectra, int n, double w,
                               double a, double b, int reach) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= static_cast<int64_t>(n_spectra) * n) return;
  const int s = static_cast<int>(i / n), c = static_cast<int>(i % n);
  const double* src = in + static_cast<int64_t>(s) * n;
  const double centre = (c + 0.5) * w;
  const double k = 1.0 / (2.0 * sqrt(2.0 * log(2.0)));
  double acc = 0.0;
  const int lo = c - reach < 0 ? 0 : c - reach, hi = c + reach >= n ? n - 1 : c + reach;
  for (int cp = lo; cp <= hi; ++cp) {
    const double x = src[cp];
    if (x == 0.0) continue;
    const double Ec = (cp + 0.5) * w;
    const double sigma = sqrt(a + b * Ec) * k;
    if (fabs(centre - Ec) > 5.0 * sigma) continue;
    const double r = 1.0 / (sigma * sqrt(2.0));
    acc += x * 0.5 * (erfc(-((c + 1) * w - Ec) * r) - erfc(-(c * w - Ec) * r));
  }
  out[i] = acc;
}

// ---------------------------------------------------------------------------
// Fixed device scratch for callers that cannot allocate (gadep_run_noalloc):
// the run's unit, chunk, scene, source, line and region tables, the chunk
// cursors, the tally rows and the spectra live in this one array, one copy per
// GPU, held until the process ends.  Host code never uses the array's name
// (a host-side stand-in): it takes the address that hipGetSymbolAddress
// returns for the current device, once per device.

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void** out) {
  static std::mutex m;
  static void* addr[kScratchDevices] = {};
  if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(m);
  if (!addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// launch wrappers (called from the runtime)

using TK = void (*)(TransportParams);

template <int V>
constexpr TK variant_kernel() {
  return transport_kernel<(V & 1) != 0, (V & 2) != 0, (V & 4) != 0, (V & 8) != 0, (V & 16) != 0,
                          (V & 32) != 0>;
}

template <int... V>
static TK pick_from(int variant, std::integer_sequence<int, V...>) {
  static const TK table[] = {variant_kernel<V>()...};
  return table[variant];
}

// variant bits: 1 GRAD, 2 SPEC, 4 COUNT, 8 GEN, 16 PAIR, 32 ELEC
static TK pick(int variant) { return pick_from(variant & 63, std::make_integer_sequence<int, 64>{}); }

// LDS: per-wavefront tallies, the traversal stacks, and (GRAD) the scores
size_t transport_smem(int block, int depth, bool grad, bool pair) {
  return static_cast<size_t>(block / kWave) * kT_Slots * sizeof(unsigned long long) +
         static_cast<size_t>(depth) * block * sizeof(int) +
         (grad ? static_cast<size_t>(kMaxGroups) * block * sizeof(float) : 0) +
         static_cast<size_t>(block / kWave) * (kQueue + kSlow) * sizeof(int64_t) +
         (pair ? static_cast<size_t>(7) * block * sizeof(int) : 0);
}

hipError_t transport_launch(const TransportParams& P, int variant, int grid, int block,
                            hipStream_t s) {
  const size_t smem = transport_smem(block, P.stack_depth, variant & 1, (variant & 16) != 0);
  hipLaunchKernelGGL(pick(variant), dim3(grid), dim3(block), smem, s, P);
  return hipGetLastError();
}

hipError_t transport_occupancy(int variant, int block, int depth, int pair, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, reinterpret_cast<const void*>(pick(variant)), block,
      transport_smem(block, depth, variant & 1, (variant & 16) != 0 || pair != 0));
}

hipError_t fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t locate_units(UnitRec* units, int n_units, const SceneRec* scenes,
                        const SourceRec* sources, int depth, hipStream_t s) {
  const int block = 64;
  const int grid = (n_units + block - 1) / block;
  hipLaunchKernelGGL(locate_units_kernel, dim3(grid), dim3(block), depth * block * sizeof(int), s,
                     units, n_units, scenes, sources, depth);
  return hipGetLastError();
}

hipError_t raycast(const SceneRec& sc, const float* o, const float* d, const int32_t* region,
                   int64_t n, float* t, int32_t* tri, int32_t* region_after, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(raycast_kernel, dim3(static_cast<unsigned>(grid)), dim3(block),
                     sc.depth * block * sizeof(int), s, sc, o, d, region, n, t, tri, region_after);
  return hipGetLastError();
}

hipError_t philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, int64_t n, uint32_t* out,
                  hipStream_t s) {
  const int block = 256;
  const int64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(philox_kernel, dim3(static_cast<unsigned>(grid)), dim3(block), 0, s, ctr,
                     k0, k1, n, out);
  return hipGetLastError();
}

hipError_t locate(const SceneRec& sc, const float* p, int64_t n, int32_t* region, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (n + block - 1) / block;
  hipLaunchKernelGGL(locate_kernel, dim3(static_cast<unsigned>(grid)), dim3(block),
                     sc.depth * block * sizeof(int), s, sc, p, n, region);
  return hipGetLastError();
}

hipError_t broaden(const double* in, double* out, int n_spectra, int n, double w, double a,
                   double b, hipStream_t s) {
  // widest window: 5 sigma at the top channel (sigma grows with E), in channels
  const double emax = n * w;
  const double smax = sqrt(a + b * emax) / (2.0 * sqrt(2.0 * log(2.0)));
  const int reach = static_cast<int>(ceil(5.0 * smax / w)) + 1;
  const int block = 256;
  const int64_t total = static_cast<int64_t>(n_spectra) * n;
  const int64_t grid = (total + block - 1) / block;
  hipLaunchKernelGGL(broaden_kernel, dim3(static_cast<unsigned>(grid)), dim3(block), 0, s, in, out,
                     n_spectra, n, w, a, b, reach);
  return hipGetLastError();
}

}  // namespace gadep
