// Streaming read by a subset of the XCDs: the plain K-load loop (K = 8,
// 16-byte vectors, adjacent segments, dealt round robin) run only by the
// workgroups of chosen XCDs, the others returning at once.  It measures the
// bandwidth one XCD, or a set of them, can draw, which locates the ceiling
// the sweep's plateau meets.
#include "device.hpp"
#include "kernels.hpp"

namespace ilp {

template <int POL>
__global__ __launch_bounds__(kPlainWgThreads) void xcd_subset(XcdArgs a) {
  const uint64_t t0 = wall_ticks();
  // The dispatcher deals workgroups to the 8 XCDs in turn, but the XCD it
  // starts on changes from launch to launch, so workgroup b runs on XCD
  // (b + r) mod 8 for an r fixed within the launch.  Each round of eight
  // workgroups (b >> 3) then puts one on every XCD, and numbering the
  // active ones by (round, rank of the XCD in the mask) is dense whatever r
  // is.  The XCD itself comes from the hardware register.
  const uint32_t b = blockIdx.x;
  const uint32_t x = xcc_id_reg() & 0xFu;
  if (x > 7u || !((a.mask >> x) & 1u)) return;
  const uint32_t rank = __builtin_popcount(a.mask & ((1u << x) - 1u));
  const uint32_t awg = (b >> 3) * a.pop + rank;
  const uint32_t aw = awg * (kPlainWgThreads / kWave) + wave_in_wg();
  const uint32_t lane = lane_id();
  uint32_t s = 0, xr = 0;
  uint64_t p = (uint64_t)aw * (kXcdK * kWave);       // first vector of group aw
  const uint64_t step = a.n_act * (kXcdK * kWave);
#pragma unroll 1
  for (uint64_t i = 0; i < a.groups; ++i) {
    u32x4 v[kXcdK];
#pragma unroll
    for (int j = 0; j < kXcdK; ++j)
      v[j] = load_seg<16, POL>(a.buf + (p + (uint64_t)j * kWave) * 16u, lane);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < kXcdK; ++j) fold(v[j], s, xr);
    p += step;
  }
  const uint64_t t1 = wall_ticks();
  wave_epilogue(s, xr, t0, t1, aw, a.rec, nullptr);
}

// The same loop with a share of the groups per XCD: the XCD comes from the
// hardware register, each round of eight workgroups holds one workgroup of
// every XCD, so (round, wave in workgroup) numbers an XCD's waves densely.
template <int POL>
__global__ __launch_bounds__(kPlainWgThreads) void xcd_split(XcdSplitArgs a) {
  const uint64_t t0 = wall_ticks();
  const uint32_t x = xcc_id_reg() & 0xFu;
  if (x > 7u || !((a.mask >> x) & 1u)) return;
  const uint32_t rank = __builtin_popcount(a.mask & ((1u << x) - 1u));
  const uint32_t lw = (blockIdx.x >> 3) * (kPlainWgThreads / kWave) + wave_in_wg();
  const uint32_t lane = lane_id();
  uint32_t s = 0, xr = 0;
  const uint64_t g1 = a.starts[x + 1];
#pragma unroll 1
  for (uint64_t g = a.starts[x] + lw; g < g1; g += a.per_xcd) {
    const uint8_t* base = a.buf + g * (kXcdK * kWave) * 16u;
    u32x4 v[kXcdK];
#pragma unroll
    for (int j = 0; j < kXcdK; ++j) v[j] = load_seg<16, POL>(base + j * (kWave * 16), lane);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < kXcdK; ++j) fold(v[j], s, xr);
  }
  const uint64_t t1 = wall_ticks();
  wave_epilogue(s, xr, t0, t1, rank * a.per_xcd + lw, a.rec, nullptr);
}

const void* xcd_split_kernel(int policy) {
  switch (policy) {
    case SWEEP_CACHE_DEFAULT: return reinterpret_cast<const void*>(&xcd_split<SWEEP_CACHE_DEFAULT>);
    case SWEEP_CACHE_NT: return reinterpret_cast<const void*>(&xcd_split<SWEEP_CACHE_NT>);
    case SWEEP_CACHE_BYPASS_L1: return reinterpret_cast<const void*>(&xcd_split<SWEEP_CACHE_BYPASS_L1>);
    case SWEEP_CACHE_BYPASS_L1_NT: return reinterpret_cast<const void*>(&xcd_split<SWEEP_CACHE_BYPASS_L1_NT>);
    default: return nullptr;
  }
}

const void* xcd_kernel(int policy) {
  switch (policy) {
    case SWEEP_CACHE_DEFAULT: return reinterpret_cast<const void*>(&xcd_subset<SWEEP_CACHE_DEFAULT>);
    case SWEEP_CACHE_NT: return reinterpret_cast<const void*>(&xcd_subset<SWEEP_CACHE_NT>);
    case SWEEP_CACHE_BYPASS_L1: return reinterpret_cast<const void*>(&xcd_subset<SWEEP_CACHE_BYPASS_L1>);
    case SWEEP_CACHE_BYPASS_L1_NT: return reinterpret_cast<const void*>(&xcd_subset<SWEEP_CACHE_BYPASS_L1_NT>);
    default: return nullptr;
  }
}

}  // namespace ilp
