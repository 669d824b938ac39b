// Wave-level loops shared by the LDS-ring kernels and the two-stream
// kernel.  A wave owns wave-groups q = wid, wid + n_waves, ... below Q; the
// request for load j of group q is the 64-lane segment starting at vector
// (q*D + j)*64 mod n_vec, exactly the plain map with K = D.
#pragma once

#include <utility>

#include "device.hpp"

namespace ilp {

template <typename F, int... Js>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Js...>) {
  (f(std::integral_constant<int, Js>{}), ...);
}
// f(integral_constant<int, J>) for J = 0 .. N-1, fully unrolled
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ uint64_t wrap_add(uint64_t p, uint64_t d, uint64_t n) {
  p += d;
  return p >= n ? p - n : p;
}

// Number of groups of wave `wid`.
__device__ __forceinline__ uint64_t groups_of(uint64_t wid, uint64_t Q,
                                              uint64_t n_waves) {
  return wid < Q ? (Q - 1 - wid) / n_waves + 1 : 0;
}

// One 16-byte-per-lane LDS-direct request: lane l's bytes land in
// slot[l] (global_load_lds_dwordx4 writes LDS at M0 + 16*lane).  The last
// builtin operand is the cache policy: 0, nt (2), sc1 (16) or sc1 nt (18).
template <int POL>
__device__ __forceinline__ void lds_issue(const uint8_t* seg, u32x4* slot,
                                          uint32_t lane) {
  typedef __attribute__((address_space(3))) void lds_void;
  lds_void* dst = (lds_void*)slot;
  if constexpr (POL == SWEEP_CACHE_DEFAULT) {
    __builtin_amdgcn_global_load_lds(seg + lane * 16, dst, 16, 0, 0);
  } else if constexpr (POL == SWEEP_CACHE_NT) {
    __builtin_amdgcn_global_load_lds(seg + lane * 16, dst, 16, 0, 2);
  } else if constexpr (POL == SWEEP_CACHE_BYPASS_L1) {
    __builtin_amdgcn_global_load_lds(seg + lane * 16, dst, 16, 0, 16);
  } else {
    __builtin_amdgcn_global_load_lds(seg + lane * 16, dst, 16, 0, 18);
  }
}

// Plain batched loop (K loads, then K folds) over one region.
template <int K, int POL>
__device__ __forceinline__ void plain_loop16(const uint8_t* buf, uint64_t n_vec,
                                             uint64_t Q, uint64_t stride,
                                             uint32_t wid, uint32_t n_waves,
                                             uint32_t lane, uint32_t& s,
                                             uint32_t& x) {
  uint64_t p = ((uint64_t)wid * (K * kWave)) % n_vec;
#pragma unroll 1
  for (uint64_t q = wid; q < Q; q += n_waves) {
    u32x4 v[K];
    uint64_t pj = p;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      v[j] = load_seg<16, POL>(buf + pj * 16, lane);
      pj = wrap_add(pj, kWave, n_vec);
    }
    __builtin_amdgcn_sched_barrier(0);   // all K issued before any fold
#pragma unroll
    for (int j = 0; j < K; ++j) fold(v[j], s, x);
    p = wrap_add(p, stride, n_vec);
  }
}

// LDS-direct ring of depth D: D requests in flight, each consumed as soon
// as it lands (s_waitcnt vmcnt(D-1)) and its slot refilled at once.
template <int D, int POL>
__device__ __forceinline__ void async_ring_loop(const uint8_t* buf, uint64_t n_vec,
                                                uint64_t Q, uint64_t stride,
                                                uint32_t wid, uint32_t n_waves,
                                                uint32_t lane, u32x4* ring,
                                                uint32_t& s, uint32_t& x) {
  const uint64_t iters = groups_of(wid, Q, n_waves);
  if (iters == 0) return;
  uint64_t p = ((uint64_t)wid * (D * kWave)) % n_vec;
  {
    uint64_t pj = p;
    static_for<D>([&](auto J) {
      lds_issue<POL>(buf + pj * 16, ring + J * kWave, lane);
      pj = wrap_add(pj, kWave, n_vec);
    });
  }
#pragma unroll 1
  for (uint64_t i = 1; i < iters; ++i) {
    p = wrap_add(p, stride, n_vec);
    uint64_t pj = p;
    static_for<D>([&](auto J) {
      wait_vmcnt<D - 1>();
      const u32x4 v = ring[J * kWave + lane];
      fold(v, s, x);
      wait_lgkmcnt0();      // the slot's read has returned before refill
      lds_issue<POL>(buf + pj * 16, ring + J * kWave, lane);
      pj = wrap_add(pj, kWave, n_vec);
    });
  }
  static_for<D>([&](auto J) {
    wait_vmcnt<D - 1 - J>();
    const u32x4 v = ring[J * kWave + lane];
    fold(v, s, x);
  });
}

// Matched plain ring: the same D requests in flight, loaded into registers,
// then written to the lane's LDS slot and read back before folding.
template <int D, int POL>
__device__ __forceinline__ void matched_ring_loop(const uint8_t* buf, uint64_t n_vec,
                                                  uint64_t Q, uint64_t stride,
                                                  uint32_t wid, uint32_t n_waves,
                                                  uint32_t lane, u32x4* ring,
                                                  uint32_t& s, uint32_t& x) {
  const uint64_t iters = groups_of(wid, Q, n_waves);
  if (iters == 0) return;
  uint64_t p = ((uint64_t)wid * (D * kWave)) % n_vec;
  u32x4 v[D];
  {
    uint64_t pj = p;
    static_for<D>([&](auto J) {
      v[J] = load_seg<16, POL>(buf + pj * 16, lane);
      pj = wrap_add(pj, kWave, n_vec);
    });
  }
  auto through_lds = [&](int j) {
    ring[j * kWave + lane] = v[j];
    compiler_fence();       // no store-to-load forwarding through LDS
    const u32x4 r = ring[j * kWave + lane];
    fold(r, s, x);
    compiler_fence();       // the refill below stays after this fold
  };
#pragma unroll 1
  for (uint64_t i = 1; i < iters; ++i) {
    p = wrap_add(p, stride, n_vec);
    uint64_t pj = p;
    static_for<D>([&](auto J) {
      through_lds(J);
      v[J] = load_seg<16, POL>(buf + pj * 16, lane);
      pj = wrap_add(pj, kWave, n_vec);
    });
  }
  static_for<D>([&](auto J) { through_lds(J); });
}

}  // namespace ilp
