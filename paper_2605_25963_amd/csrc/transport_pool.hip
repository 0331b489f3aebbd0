// gfx950 transport kernel with a per-wavefront photon pool.
//
// Same method and the same per-history arithmetic as transport_kernel
// (transport.hip): emission, free flight in mean free paths, closest boundary
// on the region's BVH, crossing or interaction, scoring (paper Sec. 2.4.1 -
// 2.4.3).  What changes is how the work meets the wavefront's 64 lanes.
//
// A wavefront (one per workgroup) keeps kPool photon slots in LDS, more than
// it has lanes.  Lanes are workers:
//   * in traversal, each lane steps the ray of one slot; a lane whose ray is
//     done writes the result to the slot, queues the slot for its outcome and
//     at once takes the next set-up ray from the ready ring, so the traversal
//     runs with full lanes while set-up rays last;
//   * when no set-up ray is left and at most `T` lanes still traverse, those
//     rays are paused (their state goes to their slots; their stacks stay in
//     the lanes' LDS columns) and the wavefront runs one housekeeping round on
//     up to 64 slots at once - outcomes, new histories (with first-flight
//     screening), emission and segment set-up - then resumes the paused rays
//     in their own lanes and hands the new ones to the idle lanes.
// Both phases thus run with (nearly) full wavefronts, where the per-lane
// kernel ran its traversal steps with the lanes that still had work and its
// per-segment work with those that had finished.
#include <hip/hip_runtime.h>

#include <utility>

#include "device_common.h"
#include "gadep_internal.h"
#include "transport_common.h"

namespace gadep {

constexpr int kPool = 96;    // photon slots per wavefront
constexpr int kRing = 128;   // capacity of each slot ring (a power of two >= kPool)
constexpr int kNone = -1;    // phase of a housekeeping lane without a slot

// Fields of a photon slot, 32 bits each, stored field-major (pool[f * kPool + slot]).
enum PoolField : int {
  kF_Px = 0, kF_Py, kF_Pz, kF_Dx, kF_Dy, kF_Dz, kF_E, kF_Tau, kF_EdAct, kF_EdTot,
  kF_Mu, kF_Mp, kF_Mc, kF_Tbest, kF_Trej, kF_BestId, kF_BestReg, kF_Misc, kF_Last, kF_Steps,
  kF_HLo, kF_HHi, kF_Draw, kF_Left, kF_B0, kF_B1, kF_B2, kF_Node, kF_Sp, kF_Tri, kF_Leaf2,
  kF_Node2, kF_Att, kF_N
};
// kF_Misc: region + 1 (bits 0-7), clean, interacted, touched, esc_any (bits 8-11)

size_t pool_smem(int depth, bool grad, bool pair) {
  return static_cast<size_t>(kT_Slots) * sizeof(unsigned long long) +
         static_cast<size_t>(kQueue + kSlow) * sizeof(int64_t) +
         static_cast<size_t>(kF_N) * kPool * sizeof(uint32_t) +
         (grad ? static_cast<size_t>(kMaxGroups) * kPool * sizeof(float) : 0) +
         (pair ? static_cast<size_t>(7) * kPool * sizeof(int) : 0) +
         static_cast<size_t>(depth) * kWave * sizeof(int) + 3 * kRing;
}

// GRAD: score-function tallies; SPEC: pulse-height spectra; COUNT: event
// counters; GEN: some unit has a volume or cone source, or a scene with
// overlays; PAIR: some material has a pair-production partial.
template <bool GRAD, bool SPEC, bool COUNT, bool GEN, bool PAIR>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2)))
pool_kernel(TransportParams P) {
  // electron tracks need the lane's LDS stack column, which may hold a paused
  // ray here: the runtime runs them with the per-lane kernel only
  constexpr bool ELEC = false;
  extern __shared__ unsigned long long smem[];
  const int lane = static_cast<int>(__lane_id());
  const uint64_t lanes_below = (1ull << lane) - 1ull;
  unsigned long long* wt = smem;  // this wavefront's tally
  int64_t* queue = reinterpret_cast<int64_t*>(smem + kT_Slots);
  int64_t* slow = queue + kQueue;
  uint32_t* pool = reinterpret_cast<uint32_t*>(slow + kSlow);
  float* scb = reinterpret_cast<float*>(pool + kF_N * kPool);
  int* waitb = reinterpret_cast<int*>(scb + (GRAD ? kMaxGroups * kPool : 0));
  int* stack = waitb + (PAIR ? 7 * kPool : 0) + lane;  // entries stack[k * kWave]
  uint8_t* ring_ready = reinterpret_cast<uint8_t*>(stack - lane + P.stack_depth * kWave);
  uint8_t* ring_done = ring_ready + kRing;
  uint8_t* ring_free = ring_done + kRing;
  // sc / wait columns of the slot a housekeeping lane works on (stride kPool)
  const int stride = kPool;
  float* sc = scb;
  int* wait = waitb;
  for (int i = lane; i < kT_Slots; i += kWave) wt[i] = 0;
  for (int i = lane; i < kPool; i += kWave) {
    ring_free[i] = static_cast<uint8_t>(i);
    if (PAIR) waitb[6 * kPool + i] = -1;
  }
  int rd_head = 0, rd_n = 0, dn_head = 0, dn_n = 0, fr_head = 0, fr_n = kPool;
  __builtin_amdgcn_wave_barrier();

  const uint64_t clk_core0 = __builtin_amdgcn_s_memtime();
  const uint64_t clk_ref0 = __builtin_amdgcn_s_memrealtime();
  const uint32_t k0 = P.seed_lo, k1 = P.seed_hi;
  const int64_t total_chunks = P.chunk_begin[P.n_units];
  // a housekeeping round starts when no set-up ray is left and at most this
  // many lanes still traverse
  const int T = P.period > 0 ? (P.period > kWave - 1 ? kWave - 1 : P.period) : 32;

  // wave-uniform claim state (as in the per-lane kernel)
  int claim_unit = 0;
  const int64_t n_w = static_cast<int64_t>(gridDim.x);
  {
    int64_t blk = blockIdx.x;
    if (gridDim.x % kXcds == 0)
      blk = static_cast<int64_t>(blockIdx.x % kXcds) * (gridDim.x / kXcds) + blockIdx.x / kXcds;
    const int64_t x = (blk * total_chunks + total_chunks / 2) / n_w;
    int lo = 0, hi = P.n_units - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (P.chunk_begin[mid] <= x)
        lo = mid;
      else
        hi = mid - 1;
    }
    claim_unit = lo;
  }
  int cur = -1;  // current unit
  int64_t next_h = 0, end_h = 0;
  int pend = -1;
  int64_t pend_h0 = 0, pend_h1 = 0;
  bool exhausted = false;
  ClaimBatch claim_batch;
  UnitRec U{};
  SceneRec S{};
  int sp_cap = 0;
  SourceRec Src{};
  bool screen = false;
  int q_head = 0, q_n = 0;
  int s_head = 0, s_n = 0;
  ScreenUnit scr;  // the current unit's screening constants

  // photon state of a housekeeping lane, and the ray state of a traversing
  // lane (the same registers: a lane does one or the other at a time)
  int phase = kNone;
  float px = 0, py = 0, pz = 0, dx = 0, dy = 0, dz = 1, E = 0, tau = 0;
  float edep_act = 0, edep_tot = 0;
  int region = 0, last = -1, steps = 0;
  int attempts = 0;
  bool clean = true, interacted = false, touched = false;
  bool esc_any = false;
  Xs ix{0, 0.0f};
  Rng g{};
  float mu = 0, mp = 0, mc = 0;
  Ray ray{};
  float tbest = 0, trej = INFINITY;
  int node = kDone, sp = 0, tri_next = 0, tri_end = 0, best_id = -1, best_reg = 0;
  int leaf2 = kDone;
  // a second BVH root still to search (two-level scenes; kDone: none)
  int node2 = kDone;
  int tslot = -1;  // slot whose ray this lane traverses
  int pslot = -1;  // slot whose ray this lane paused for a housekeeping round
  unsigned long long acc_hist = 0, acc_eunc = 0, acc_esrc = 0;
  uint32_t ev[kEv_N];
#pragma unroll
  for (int i = 0; i < kEv_N; ++i) ev[i] = 0;

  auto fld = [&](int f, int s) -> uint32_t& { return pool[f * kPool + s]; };
  auto fget = [&](int f, int s) -> float { return __uint_as_float(pool[f * kPool + s]); };
  auto fput = [&](int f, int s, float v) { pool[f * kPool + s] = __float_as_uint(v); };

  // the ray of slot s into this lane's traversal registers
  auto load_trav = [&](int s) {
    px = fget(kF_Px, s);
    py = fget(kF_Py, s);
    pz = fget(kF_Pz, s);
    dx = fget(kF_Dx, s);
    dy = fget(kF_Dy, s);
    dz = fget(kF_Dz, s);
    tbest = fget(kF_Tbest, s);
    trej = fget(kF_Trej, s);
    best_id = static_cast<int>(fld(kF_BestId, s));
    best_reg = static_cast<int>(fld(kF_BestReg, s));
    region = static_cast<int>(fld(kF_Misc, s) & 0xFFu) - 1;
    last = static_cast<int>(fld(kF_Last, s));
    node = static_cast<int>(fld(kF_Node, s));
    sp = static_cast<int>(fld(kF_Sp, s));
    const uint32_t t = fld(kF_Tri, s);
    tri_next = static_cast<int>(t >> 3);
    tri_end = tri_next + static_cast<int>(t & 7u);
    leaf2 = static_cast<int>(fld(kF_Leaf2, s));
    node2 = GEN ? static_cast<int>(fld(kF_Node2, s)) : kDone;
    ray = make_ray(px, py, pz, dx, dy, dz);
  };
  // a finished or paused traversal's state into slot s
  auto save_trav = [&](int s, bool paused) {
    fput(kF_Tbest, s, tbest);
    fput(kF_Trej, s, trej);
    fld(kF_BestId, s) = static_cast<uint32_t>(best_id);
    fld(kF_BestReg, s) = static_cast<uint32_t>(best_reg);
    if (paused) {
      fld(kF_Node, s) = static_cast<uint32_t>(node);
      fld(kF_Sp, s) = static_cast<uint32_t>(sp);
      fld(kF_Tri, s) = (static_cast<uint32_t>(tri_next) << 3) | static_cast<uint32_t>(tri_end - tri_next);
      fld(kF_Leaf2, s) = static_cast<uint32_t>(leaf2);
      if (GEN) fld(kF_Node2, s) = static_cast<uint32_t>(node2);
    }
  };
  // the whole photon of slot s into this lane's registers, and back
  auto load_photon = [&](int s) {
    px = fget(kF_Px, s);
    py = fget(kF_Py, s);
    pz = fget(kF_Pz, s);
    dx = fget(kF_Dx, s);
    dy = fget(kF_Dy, s);
    dz = fget(kF_Dz, s);
    E = fget(kF_E, s);
    tau = fget(kF_Tau, s);
    edep_act = fget(kF_EdAct, s);
    edep_tot = fget(kF_EdTot, s);
    mu = fget(kF_Mu, s);
    mp = fget(kF_Mp, s);
    mc = fget(kF_Mc, s);
    tbest = fget(kF_Tbest, s);
    trej = fget(kF_Trej, s);
    best_id = static_cast<int>(fld(kF_BestId, s));
    best_reg = static_cast<int>(fld(kF_BestReg, s));
    const uint32_t m = fld(kF_Misc, s);
    region = static_cast<int>(m & 0xFFu) - 1;
    clean = (m >> 8) & 1u;
    interacted = (m >> 9) & 1u;
    touched = (m >> 10) & 1u;
    esc_any = (m >> 11) & 1u;
    last = static_cast<int>(fld(kF_Last, s));
    steps = static_cast<int>(fld(kF_Steps, s));
    g.h_lo = fld(kF_HLo, s);
    g.h_hi = fld(kF_HHi, s);
    g.draw = fld(kF_Draw, s);
    g.left = fld(kF_Left, s);
    g.b0 = fld(kF_B0, s);
    g.b1 = fld(kF_B1, s);
    g.b2 = fld(kF_B2, s);
    attempts = static_cast<int>(fld(kF_Att, s));
    ix = xs_index(E, P.ln_e0, P.inv_dlne, P.n_e);
  };
  auto store_photon = [&](int s) {
    fput(kF_Px, s, px);
    fput(kF_Py, s, py);
    fput(kF_Pz, s, pz);
    fput(kF_Dx, s, dx);
    fput(kF_Dy, s, dy);
    fput(kF_Dz, s, dz);
    fput(kF_E, s, E);
    fput(kF_Tau, s, tau);
    fput(kF_EdAct, s, edep_act);
    fput(kF_EdTot, s, edep_tot);
    fput(kF_Mu, s, mu);
    fput(kF_Mp, s, mp);
    fput(kF_Mc, s, mc);
    fput(kF_Tbest, s, tbest);
    fput(kF_Trej, s, trej);
    fld(kF_BestId, s) = static_cast<uint32_t>(best_id);
    fld(kF_BestReg, s) = static_cast<uint32_t>(best_reg);
    fld(kF_Misc, s) = static_cast<uint32_t>(region + 1) | (clean ? 1u << 8 : 0u) |
                      (interacted ? 1u << 9 : 0u) | (touched ? 1u << 10 : 0u) |
                      (esc_any ? 1u << 11 : 0u);
    fld(kF_Last, s) = static_cast<uint32_t>(last);
    fld(kF_Steps, s) = static_cast<uint32_t>(steps);
    fld(kF_HLo, s) = g.h_lo;
    fld(kF_HHi, s) = g.h_hi;
    fld(kF_Draw, s) = g.draw;
    fld(kF_Left, s) = g.left;
    fld(kF_B0, s) = g.b0;
    fld(kF_B1, s) = g.b1;
    fld(kF_B2, s) = g.b2;
    fld(kF_Att, s) = static_cast<uint32_t>(attempts);
    fld(kF_Node, s) = static_cast<uint32_t>(node);
    fld(kF_Sp, s) = 0u;
    fld(kF_Tri, s) = 0u;
    fld(kF_Leaf2, s) = static_cast<uint32_t>(kDone);
    if (GEN) fld(kF_Node2, s) = static_cast<uint32_t>(node2);
  };
  // append the slots of the lanes with `pred` to a ring
  auto push = [&](uint8_t* ring, int head, int& n, bool pred, int s) {
    const uint64_t m = __ballot(pred);
    if (pred) ring[(head + n + __popcll(m & lanes_below)) & (kRing - 1)] = static_cast<uint8_t>(s);
    n += __popcll(m);
  };

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

  // kinetic energy T given to an electron where the photon is: deposited in
  // place (the runtime runs electron tracks with the per-lane kernel only: a
  // lane's LDS stack may hold a paused ray here)
  auto electron = [&](float T, float, float, float, bool active) -> bool {
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


  // histories can start (or a claim can be tried) without waiting for a drain
  auto can_start = [&]() -> bool {
    return q_n > 0 || s_n > 0 || next_h < end_h || (pend < 0 && !exhausted) ||
           (pend >= 0 && (pend == cur || fr_n == kPool));
  };

  for (;;) {
    // ================= traversal: full lanes while set-up rays last =========
    for (;;) {
      if (rd_n > 0) {
        // idle lanes take the next set-up rays
        const bool want = tslot < 0;
        const uint64_t m = __ballot(want);
        const int rank = __popcll(m & lanes_below);
        int s = -1;
        if (want && rank < rd_n) s = ring_ready[(rd_head + rank) & (kRing - 1)];
        const int taken = rd_n < __popcll(m) ? rd_n : __popcll(m);
        rd_head = (rd_head + taken) & (kRing - 1);
        rd_n -= taken;
        if (s >= 0) {
          load_trav(s);
          tslot = s;
        }
      }
      const int n_trav = __popcll(__ballot(tslot >= 0));
      if (n_trav == 0) break;
      if (n_trav <= T && rd_n == 0 && (dn_n > 0 || (fr_n > 0 && can_start()))) break;

      // one node and one facet per lane (speculative traversal, as in the
      // per-lane kernel)
      bool did_node = false, did_tri = false;
      const uint64_t clk_trav = COUNT ? __builtin_amdgcn_s_memtime() : 0;
      if (tslot >= 0) {
        const bool busy = tri_next < tri_end;
        if (node < 0 && node != kDone && (!busy || leaf2 == kDone)) {
          const int code = ~node;
          if (!busy) {
            tri_next = code >> 3;
            tri_end = tri_next + (code & 7);
          } else {
            leaf2 = node;
          }
          node = sp > 0 ? stack[sp -= kWave] : kDone;
        } else if (node >= 0 && (!busy || leaf2 == kDone)) {
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
            node = sp > 0 ? stack[sp -= kWave] : kDone;
          } else if (near < 0) {
            if (!busy) {
              const int code = ~near;
              tri_next = code >> 3;
              tri_end = tri_next + (code & 7);
            } else {
              leaf2 = near;
            }
            node = far != kDone ? far : (sp > 0 ? stack[sp -= kWave] : kDone);
          } else {
            if (far != kDone && sp < sp_cap) {
              stack[sp] = far;
              sp += kWave;
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
              best_reg = (enter ? inside : outside) | (before << 8);
            }
          }
        }
      }
      // the second level of a two-level scene: same ray, nearest hit kept
      if (GEN && tslot >= 0 && tri_next >= tri_end && node == kDone && leaf2 == kDone && node2 != kDone) {
        node = node2;
        node2 = kDone;
      }
      // finished rays: their results to the slot, the slot to the done ring
      const bool fin = tslot >= 0 && tri_next >= tri_end && node == kDone && leaf2 == kDone;
      if (fin) save_trav(tslot, false);
      __builtin_amdgcn_wave_barrier();
      push(ring_done, dn_head, dn_n, fin, tslot);
      if (fin) tslot = -1;
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

    // ================= housekeeping round on up to 64 slots ================
    // rays still in flight pause: their state goes to their slots (their
    // stacks stay in these lanes' columns)
    if (tslot >= 0) save_trav(tslot, true);
    pslot = tslot;
    tslot = -1;
    {
      const int n_d = dn_n < kWave ? dn_n : kWave;
      const int n_f = can_start() ? (fr_n < kWave - n_d ? fr_n : kWave - n_d) : 0;
      __builtin_amdgcn_wave_barrier();
      int hs = -1;
      phase = kNone;
      if (lane < n_d) {
        hs = ring_done[(dn_head + lane) & (kRing - 1)];
        phase = kParked;
      } else if (lane < n_d + n_f) {
        hs = ring_free[(fr_head + lane - n_d) & (kRing - 1)];
        phase = kNeed;
      }
      dn_head = (dn_head + n_d) & (kRing - 1);
      dn_n -= n_d;
      fr_head = (fr_head + n_f) & (kRing - 1);
      fr_n -= n_f;
      sc = scb + (hs >= 0 ? hs : 0);
      wait = waitb + (hs >= 0 ? hs : 0);
      if (phase == kParked) load_photon(hs);

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
              (pend == cur || (q_n == 0 && s_n == 0 && kPool - fr_n == __popcll(__ballot(phase == kNeed))))) {
            if (pend != cur) {
              flush();
              cur = pend;
              U = P.units[cur];
              S = P.scenes[U.scene];
              sp_cap = S.depth * kWave;
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
            // the box (as in the per-lane kernel)
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

      // slots back to their rings: set up -> ready, settled without a
      // traversal -> done, no history -> free
      if (hs >= 0 && phase != kNeed) store_photon(hs);
      __builtin_amdgcn_wave_barrier();
      push(ring_ready, rd_head, rd_n, hs >= 0 && phase == kTrav, hs);
      push(ring_done, dn_head, dn_n, hs >= 0 && phase == kParked, hs);
      push(ring_free, fr_head, fr_n, hs >= 0 && phase == kNeed, hs);
      phase = kNone;
    }
    if (fr_n == kPool && exhausted && pend < 0 && next_h >= end_h && q_n == 0 && s_n == 0) break;
    // paused rays resume in their own lanes (their stacks are there)
    __builtin_amdgcn_wave_barrier();
    if (pslot >= 0) {
      load_trav(pslot);
      tslot = pslot;
      pslot = -1;
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
// launch wrappers

using PK = void (*)(TransportParams);

template <int V>
constexpr PK pool_variant() {
  return pool_kernel<(V & 1) != 0, (V & 2) != 0, (V & 4) != 0, (V & 8) != 0, (V & 16) != 0>;
}

template <int... V>
static PK pool_pick_from(int variant, std::integer_sequence<int, V...>) {
  static const PK table[] = {pool_variant<V>()...};
  return table[variant];
}

static PK pool_pick(int variant) {
  return pool_pick_from(variant & 31, std::make_integer_sequence<int, 32>{});
}

hipError_t pool_launch(const TransportParams& P, int variant, int grid, hipStream_t s) {
  const size_t smem = pool_smem(P.stack_depth, variant & 1, (variant & 16) != 0);
  hipLaunchKernelGGL(pool_pick(variant), dim3(grid), dim3(kWave), smem, s, P);
  return hipGetLastError();
}

hipError_t pool_occupancy(int variant, int depth, int pair, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      blocks_per_cu, reinterpret_cast<const void*>(pool_pick(variant)), kWave,
      pool_smem(depth, variant & 1, (variant & 16) != 0 || pair != 0));
}

}  // namespace gadep
