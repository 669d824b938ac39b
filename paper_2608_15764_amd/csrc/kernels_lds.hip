// LDS-ring kernels of the path comparison (Section 4.3) and the
// same-workgroup two-stream kernel (Section 4.4).
//
//  lds_async    loads go straight to LDS (global_load_lds_dwordx4, no
//               destination register), the analogue of cp.async;
//  lds_matched  the same ring through registers (global_load_dwordx4, then
//               ds_write_b128 and ds_read_b128), the matched plain kernel;
//  two_stream   one workgroup per CU whose first waves run the plain
//               batched K-load loop over the first half of the buffer and
//               whose last waves run either the LDS-direct ring or the
//               same plain loop over the second; or, split, half of the
//               workgroups run stream A and the other half stream B, so
//               the two streams share no CU.
// Each wave owns `depth` 1 KiB slots of the workgroup's dynamic LDS.
#include <array>
#include <utility>

#include "kernels.hpp"
#include "wave_loops.hpp"

namespace ilp {

extern __shared__ u32x4 lds_ring[];

template <int KIND, int D, int POL>
__global__ __launch_bounds__(1024) void lds_kernel_t(LdsArgs a) {
  const uint64_t t0 = wall_ticks();
  const uint32_t lane = lane_id();
  const uint32_t wv = wave_in_wg();
  const uint32_t wid = blockIdx.x * a.waves + wv;
  const uint32_t n_waves = gridDim.x * a.waves;
  u32x4* ring = lds_ring + wv * (D * kWave);
  uint32_t s = 0, x = 0;
  if constexpr (KIND == SWEEP_KIND_LDS_ASYNC) {
    async_ring_loop<D, POL>(a.buf, a.n_vec, a.Q, a.stride, wid, n_waves, lane,
                            ring, s, x);
  } else {
    matched_ring_loop<D, POL>(a.buf, a.n_vec, a.Q, a.stride, wid, n_waves,
                              lane, ring, s, x);
  }
  const uint64_t t1 = wall_ticks();
  wave_epilogue(s, x, t0, t1, wid, a.rec, a.lane_out);
}

// Stream B of a two-stream launch: the LDS-direct ring or the plain loop.
template <int D, int POL>
__device__ __forceinline__ void stream_b(const TwoStreamArgs& a, uint32_t wid,
                                         uint32_t n_waves, uint32_t wb,
                                         uint32_t lane, uint32_t& s, uint32_t& x) {
  if (a.b_plain) {
    plain_loop16<D, POL>(a.buf_b, a.n_vec_b, a.Q_b, a.stride_b, wid, n_waves,
                         lane, s, x);
  } else {
    u32x4* ring = lds_ring + wb * (D * kWave);
    async_ring_loop<D, POL>(a.buf_b, a.n_vec_b, a.Q_b, a.stride_b, wid, n_waves,
                            lane, ring, s, x);
  }
}

template <int D, int POL>
__global__ __launch_bounds__(1024) void two_stream_t(TwoStreamArgs a) {
  const uint64_t t0 = wall_ticks();
  const uint32_t lane = lane_id();
  const uint32_t wv = wave_in_wg();
  uint32_t s = 0, x = 0;
  if (a.split) {
    // Workgroups 16m .. 16m+7 run stream A and 16m+8 .. 16m+15 stream B
    // (the grid is a multiple of 16).  Workgroups are dealt to the 8 XCDs
    // in turn, so every XCD holds as many workgroups of A as of B; with one
    // workgroup per CU no CU runs both.  Waves beyond the stream's count
    // leave at once and write no record.
    const uint32_t g = blockIdx.x;
    const bool is_a = ((g >> 3) & 1u) == 0;
    const uint32_t idx = (g >> 4) * 8u + (g & 7u);   // among its stream's workgroups
    const uint32_t n_wg = gridDim.x / 2;
    const uint32_t w = is_a ? a.waves_a : a.waves_b;
    if (wv >= w) return;
    const uint32_t wid = idx * w + wv;
    if (is_a) {
      plain_loop16<D, POL>(a.buf_a, a.n_vec_a, a.Q_a, a.stride_a, wid,
                           n_wg * a.waves_a, lane, s, x);
      const uint64_t t1 = wall_ticks();
      wave_epilogue(s, x, t0, t1, wid, a.rec, a.lane_out);
    } else {
      stream_b<D, POL>(a, wid, n_wg * a.waves_b, wv, lane, s, x);
      const uint64_t t1 = wall_ticks();
      wave_epilogue(s, x, t0, t1, n_wg * a.waves_a + wid, a.rec, a.lane_out);
    }
    return;
  }
  if (wv < a.waves_a) {
    const uint32_t wid = blockIdx.x * a.waves_a + wv;
    plain_loop16<D, POL>(a.buf_a, a.n_vec_a, a.Q_a, a.stride_a, wid,
                         gridDim.x * a.waves_a, lane, s, x);
    const uint64_t t1 = wall_ticks();
    wave_epilogue(s, x, t0, t1, wid, a.rec, a.lane_out);
  } else {
    const uint32_t wb = wv - a.waves_a;
    const uint32_t wid = blockIdx.x * a.waves_b + wb;
    stream_b<D, POL>(a, wid, gridDim.x * a.waves_b, wb, lane, s, x);
    const uint64_t t1 = wall_ticks();
    const uint32_t base = gridDim.x * a.waves_a;
    wave_epilogue(s, x, t0, t1, base + wid, a.rec, a.lane_out);
  }
}

namespace {

typedef void (*LdsFn)(LdsArgs);
typedef void (*TwoFn)(TwoStreamArgs);

template <int KIND, int POL, int... Ds>
constexpr std::array<LdsFn, sizeof...(Ds)> lds_row(std::integer_sequence<int, Ds...>) {
  return {&lds_kernel_t<KIND, Ds + 1, POL>...};
}
template <int POL, int... Ds>
constexpr std::array<TwoFn, sizeof...(Ds)> two_row(std::integer_sequence<int, Ds...>) {
  return {&two_stream_t<Ds + 1, POL>...};
}
template <int KIND, int POL>
constexpr auto kLdsRow = lds_row<KIND, POL>(std::make_integer_sequence<int, kMaxK>{});
template <int POL>
constexpr auto kTwoRow = two_row<POL>(std::make_integer_sequence<int, kMaxK>{});

}  // namespace

const void* lds_kernel(int kind, int D, int policy) {
  static const std::array<LdsFn, kMaxK> t[2][kNumPolicies] = {
      {kLdsRow<SWEEP_KIND_LDS_ASYNC, 0>, kLdsRow<SWEEP_KIND_LDS_ASYNC, 1>,
       kLdsRow<SWEEP_KIND_LDS_ASYNC, 2>, kLdsRow<SWEEP_KIND_LDS_ASYNC, 3>},
      {kLdsRow<SWEEP_KIND_LDS_MATCHED, 0>, kLdsRow<SWEEP_KIND_LDS_MATCHED, 1>,
       kLdsRow<SWEEP_KIND_LDS_MATCHED, 2>, kLdsRow<SWEEP_KIND_LDS_MATCHED, 3>},
  };
  if (D < 1 || D > kMaxK || policy < 0 || policy >= kNumPolicies) return nullptr;
  if (kind == SWEEP_KIND_LDS_ASYNC) return reinterpret_cast<const void*>(t[0][policy][D - 1]);
  if (kind == SWEEP_KIND_LDS_MATCHED) return reinterpret_cast<const void*>(t[1][policy][D - 1]);
  return nullptr;
}

const void* two_stream_kernel(int D, int policy) {
  static const std::array<TwoFn, kMaxK> t[kNumPolicies] = {kTwoRow<0>, kTwoRow<1>,
                                                           kTwoRow<2>, kTwoRow<3>};
  if (D < 1 || D > kMaxK || policy < 0 || policy >= kNumPolicies) return nullptr;
  return reinterpret_cast<const void*>(t[policy][D - 1]);
}

}  // namespace ilp
