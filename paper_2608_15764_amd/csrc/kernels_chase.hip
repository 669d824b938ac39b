// Pointer-chase latency probe (the latency ladder of Section 4.1): one lane
// follows a dependent chain idx <- buf[idx], so exactly one load is in
// flight at a time and no load can be elided.  The mean latency comes from
// the constant-rate wall clock over all timed hops; the per-hop spread from
// shader-clock deltas of the first hops, kept in LDS so that no global store
// sits inside a timed interval.
#include "device.hpp"
#include "kernels.hpp"

namespace ilp {

// Every policy goes through a buffer load over the whole chain, so an index
// outside the chain reads 0 (the hardware range check) instead of faulting.
template <int POL>
__device__ __forceinline__ uint32_t chase_load(const uint32_t* buf, uint32_t n_bytes,
                                               uint32_t idx) {
  constexpr int aux = POL == SWEEP_CACHE_DEFAULT ? 0
                      : POL == SWEEP_CACHE_NT    ? 2
                      : POL == SWEEP_CACHE_BYPASS_L1 ? kAuxSc1 : kAuxSc1Nt;
  __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint32_t*>(buf), 0, (int)n_bytes, kRsrcWord3);
  return __builtin_amdgcn_raw_buffer_load_b32(r, idx * 4u, 0, aux);
}

template <int POL>
__global__ __launch_bounds__(64) void chase(ChaseArgs a) {
  __shared__ uint32_t cyc[kMaxChaseSamples];
  if (threadIdx.x != 0) return;
  uint32_t idx = a.start;
#pragma unroll 1
  for (uint32_t i = 0; i < a.warm; ++i) idx = chase_load<POL>(a.buf, a.n_bytes, idx);
  // the clocks bracket exactly the timed hops: the last warm-up load has
  // landed before they start, the last timed one before they stop
  wait_vmcnt<0>();
  const uint64_t r0 = wall_ticks();
  const uint64_t m0 = __builtin_amdgcn_s_memtime();
#pragma unroll 1
  for (uint32_t i = 0; i < a.n_samples; ++i) {
    const uint64_t c0 = __builtin_amdgcn_s_memtime();
    idx = chase_load<POL>(a.buf, a.n_bytes, idx);
    wait_vmcnt<0>();
    const uint64_t c1 = __builtin_amdgcn_s_memtime();
    cyc[i] = (uint32_t)(c1 - c0);
  }
#pragma unroll 1
  for (uint32_t i = a.n_samples; i < a.steps; ++i)
    idx = chase_load<POL>(a.buf, a.n_bytes, idx);
  wait_vmcnt<0>();
  const uint64_t r1 = wall_ticks();
  const uint64_t m1 = __builtin_amdgcn_s_memtime();
  for (uint32_t i = 0; i < a.n_samples; ++i) a.samples[i] = cyc[i];
  a.out[0] = idx;
  a.out[1] = r0;
  a.out[2] = r1;
  a.out[3] = m0;
  a.out[4] = m1;
}

// Walker b of the grid follows the chain from starts[b]: one dependent load
// in flight per walker, every walker on its own workgroup, so the
// dispatcher places them on the XCDs in turn and each reports its own.
template <int POL>
__global__ __launch_bounds__(64) void chase_walkers(WalkArgs a) {
  if (threadIdx.x != 0) return;
  const uint32_t b = blockIdx.x;
  uint32_t idx = a.starts[b];
#pragma unroll 1
  for (uint32_t i = 0; i < a.warm; ++i) idx = chase_load<POL>(a.buf, a.n_bytes, idx);
  wait_vmcnt<0>();
  const uint64_t r0 = wall_ticks();
#pragma unroll 1
  for (uint32_t i = 0; i < a.steps; ++i) idx = chase_load<POL>(a.buf, a.n_bytes, idx);
  wait_vmcnt<0>();
  const uint64_t r1 = wall_ticks();
  uint64_t* o = a.out + 4u * b;
  o[0] = idx;
  o[1] = r0;
  o[2] = r1;
  o[3] = xcc_id_reg();
}

const void* chase_kernel(int policy) {
  switch (policy) {
    case SWEEP_CACHE_DEFAULT: return reinterpret_cast<const void*>(&chase<SWEEP_CACHE_DEFAULT>);
    case SWEEP_CACHE_NT: return reinterpret_cast<const void*>(&chase<SWEEP_CACHE_NT>);
    case SWEEP_CACHE_BYPASS_L1: return reinterpret_cast<const void*>(&chase<SWEEP_CACHE_BYPASS_L1>);
    case SWEEP_CACHE_BYPASS_L1_NT: return reinterpret_cast<const void*>(&chase<SWEEP_CACHE_BYPASS_L1_NT>);
    default: return nullptr;
  }
}

hipError_t launch_walkers(int policy, hipStream_t st, const WalkArgs& a) {
  const void* fn = nullptr;
  switch (policy) {
    case SWEEP_CACHE_DEFAULT: fn = reinterpret_cast<const void*>(&chase_walkers<SWEEP_CACHE_DEFAULT>); break;
    case SWEEP_CACHE_NT: fn = reinterpret_cast<const void*>(&chase_walkers<SWEEP_CACHE_NT>); break;
    case SWEEP_CACHE_BYPASS_L1: fn = reinterpret_cast<const void*>(&chase_walkers<SWEEP_CACHE_BYPASS_L1>); break;
    case SWEEP_CACHE_BYPASS_L1_NT: fn = reinterpret_cast<const void*>(&chase_walkers<SWEEP_CACHE_BYPASS_L1_NT>); break;
    default: return hipErrorInvalidValue;
  }
  if (a.n_walkers == 0 || a.n_walkers > kMaxWalkers) return hipErrorInvalidValue;
  void* args[] = {const_cast<WalkArgs*>(&a)};
  return hipLaunchKernel(fn, dim3(a.n_walkers), dim3(64), args, 0, st);
}

hipError_t launch_chase(int policy, hipStream_t st, const ChaseArgs& a) {
  const void* fn = chase_kernel(policy);
  if (!fn) return hipErrorInvalidValue;
  void* args[] = {const_cast<ChaseArgs*>(&a)};
  return hipLaunchKernel(fn, dim3(1), dim3(64), args, 0, st);
}

}  // namespace ilp
