// Plain K-load sweep kernel (the hot loop of the method, Section 3 "The
// axis K" and Section 4.2).
//
// One wavefront-iteration issues K independent loads - each one contiguous,
// coalesced 64-lane segment of 64*V bytes, adjacent to each other or (the
// strided layout) Q segments apart - into K distinct register sets,
// and only then folds them, oldest first; nothing from the next iteration is
// in flight meanwhile, so a wave has at most K loads outstanding.  The loop
// itself never stores: the sinks leave the kernel in one record per wave.
#include <array>
#include <utility>

#include "device.hpp"
#include "kernels.hpp"

namespace ilp {

template <int K, int V, int POL>
__global__ __launch_bounds__(kPlainWgThreads) void plain_kload(PlainArgs a) {
  const uint64_t t0 = wall_ticks();
  const uint32_t lane = lane_id();
  const uint32_t wid = blockIdx.x * (kPlainWgThreads / kWave) + wave_in_wg();
  const uint32_t n_waves = gridDim.x * (kPlainWgThreads / kWave);

  uint32_t s = 0, x = 0;
  // this wave's groups: [q0, q1) in steps of qs (wave-uniform scalars)
  uint64_t q0 = wid, q1 = a.Q, qs = n_waves;
  if (a.order == SWEEP_ORDER_BLOCKED) {
    q0 = (uint64_t)wid * a.G;
    q1 = q0 + a.G < a.Q ? q0 + a.G : a.Q;
    qs = 1;
  }
  // start vector of the first group, advanced by `stride` per iteration,
  // both modulo the buffer's vector count
  uint64_t p = (q0 * a.gstep) % a.n_vec;
#pragma unroll 1
  for (uint64_t q = q0; q < q1; q += qs) {
    typename Vec<V>::T v[K];
    uint64_t pj = p;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      v[j] = load_seg<V, POL>(a.buf + pj * V, lane);
      pj += a.jstep;
      if (pj >= a.n_vec) pj -= a.n_vec;
    }
    // all K loads are issued before the first is consumed: without this
    // barrier the scheduler may refill registers early to raise occupancy
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < K; ++j) fold(v[j], s, x);
    p += a.stride;
    if (p >= a.n_vec) p -= a.n_vec;
  }
  const uint64_t t1 = wall_ticks();
  wave_epilogue(s, x, t0, t1, wid, a.rec, a.lane_out);
}

namespace {

typedef void (*PlainFn)(PlainArgs);

template <int V, int POL, int... Ks>
constexpr std::array<PlainFn, sizeof...(Ks)> row(std::integer_sequence<int, Ks...>) {
  return {&plain_kload<Ks + 1, V, POL>...};
}

template <int V, int POL>
constexpr auto kRow = row<V, POL>(std::make_integer_sequence<int, kMaxK>{});

// [vector width index][policy][K-1]
const PlainFn* table(int vi, int pol) {
  static const std::array<PlainFn, kMaxK> t[3][kNumPolicies] = {
      {kRow<4, 0>, kRow<4, 1>, kRow<4, 2>, kRow<4, 3>},
      {kRow<8, 0>, kRow<8, 1>, kRow<8, 2>, kRow<8, 3>},
      {kRow<16, 0>, kRow<16, 1>, kRow<16, 2>, kRow<16, 3>},
  };
  return t[vi][pol].data();
}

int width_index(int V) { return V == 4 ? 0 : V == 8 ? 1 : V == 16 ? 2 : -1; }

}  // namespace

const void* plain_kernel(int K, int V, int policy) {
  const int vi = width_index(V);
  if (vi < 0 || K < 1 || K > kMaxK || policy < 0 || policy >= kNumPolicies) return nullptr;
  return reinterpret_cast<const void*>(table(vi, policy)[K - 1]);
}

}  // namespace ilp
