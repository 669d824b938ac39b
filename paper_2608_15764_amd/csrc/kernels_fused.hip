// Fused batch of plain K-load cells (the batched sweep): the points of one
// tuned configuration run as a single persistent launch over their
// concatenated wave-groups, so a small point costs a few groups of the
// running grid instead of a launch of its own.  The loop is the plain
// kernel's: K independent loads issued before the first is consumed, then
// folded oldest first, nothing from the next group in flight, no stores
// inside the loop.  A wave closes a point's record (DPP reduction, one
// store) when its next group belongs to another point, or at the end.
#include <array>
#include <utility>

#include "device.hpp"
#include "kernels.hpp"

namespace ilp {

// The point list is read at a wave-uniform index; readfirstlane makes the
// fields scalars, so the buffer descriptors built from them stay scalar.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// A point's buffer is addressed from the launch's base pointer (a kernel
// argument, so loads through it stay global loads).
struct PointRegs {
  const uint8_t* buf;
  uint64_t n_vec, g0, end, stride;
};

// The point list is never written while the kernel runs: read it through
// the constant address space, so the loads are scalar and stay out of the
// vector-memory counter the K loads of a group wait on.
typedef const __attribute__((address_space(4))) FusedPoint* ConstPoints;

__device__ __forceinline__ PointRegs point_regs(const uint8_t* base, const FusedPoint* pts,
                                                uint32_t i) {
  const auto& f = reinterpret_cast<ConstPoints>(reinterpret_cast<uintptr_t>(pts))[i];
  PointRegs r;
  r.buf = base + uniform64(f.off);
  r.n_vec = uniform64(f.n_vec);
  r.g0 = uniform64(f.g0);
  r.end = r.g0 + uniform64(f.Q);
  r.stride = uniform64(f.stride);
  return r;
}

template <int K, int V, int POL>
__global__ __launch_bounds__(kPlainWgThreads) void fused_kload(FusedArgs a) {
  const uint32_t lane = lane_id();
  const uint32_t wid = blockIdx.x * (kPlainWgThreads / kWave) + wave_in_wg();
  const uint32_t n_waves = gridDim.x * (kPlainWgThreads / kWave);

  // the wave's current point, cached in scalars (wave-uniform)
  uint32_t pi = 0;
  PointRegs pt = point_regs(a.base, a.pts, 0);
  uint64_t p = 0;               // start vector of the wave's next group
  bool open = false;            // the wave has read a group of point pi
  uint32_t s = 0, x = 0;
  uint64_t t0 = 0;
#pragma unroll 1
  for (uint64_t g = wid; g < a.total_groups; g += n_waves) {
    if (g >= pt.end) {
      if (open) wave_epilogue(s, x, t0, wall_ticks(), pi * n_waves + wid, a.rec, nullptr);
      open = false;
      do {
        ++pi;
        pt = point_regs(a.base, a.pts, pi);
      } while (g >= pt.end);
    }
    if (!open) {
      open = true;
      s = 0;
      x = 0;
      t0 = wall_ticks();
      p = ((g - pt.g0) * (uint64_t)(K * kWave)) % pt.n_vec;
    }
    typename Vec<V>::T v[K];
    uint64_t pj = p;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      v[j] = load_seg<V, POL>(pt.buf + pj * V, lane);
      pj += kWave;
      if (pj >= pt.n_vec) pj -= pt.n_vec;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < K; ++j) fold(v[j], s, x);
    p += pt.stride;
    if (p >= pt.n_vec) p -= pt.n_vec;
  }
  if (open) wave_epilogue(s, x, t0, wall_ticks(), pi * n_waves + wid, a.rec, nullptr);
}

__global__ __launch_bounds__(256) void clear_records(sweep_wave_rec_t* rec, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    u32x4* r = reinterpret_cast<u32x4*>(rec + i);
    r[0] = u32x4{0u, 0u, 0u, 0u};
    r[1] = u32x4{0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u};
  }
}

hipError_t launch_clear_records(sweep_wave_rec_t* rec, uint64_t n, hipStream_t st) {
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(clear_records, dim3((uint32_t)blocks), dim3(256), 0, st, rec, n);
  return hipGetLastError();
}

namespace {

typedef void (*FusedFn)(FusedArgs);

template <int V, int POL, int... Ks>
constexpr std::array<FusedFn, sizeof...(Ks)> row(std::integer_sequence<int, Ks...>) {
  return {&fused_kload<Ks + 1, V, POL>...};
}

template <int V, int POL>
constexpr auto kRow = row<V, POL>(std::make_integer_sequence<int, kMaxK>{});

// [vector width index][policy][K-1]
const FusedFn* table(int vi, int pol) {
  static const std::array<FusedFn, kMaxK> t[3][kNumPolicies] = {
      {kRow<4, 0>, kRow<4, 1>, kRow<4, 2>, kRow<4, 3>},
      {kRow<8, 0>, kRow<8, 1>, kRow<8, 2>, kRow<8, 3>},
      {kRow<16, 0>, kRow<16, 1>, kRow<16, 2>, kRow<16, 3>},
  };
  return t[vi][pol].data();
}

int width_index(int V) { return V == 4 ? 0 : V == 8 ? 1 : V == 16 ? 2 : -1; }

}  // namespace

const void* fused_kernel(int K, int V, int policy) {
  const int vi = width_index(V);
  if (vi < 0 || K < 1 || K > kMaxK || policy < 0 || policy >= kNumPolicies) return nullptr;
  return reinterpret_cast<const void*>(table(vi, policy)[K - 1]);
}

}  // namespace ilp
