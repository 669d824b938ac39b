// Device-side building blocks shared by the gfx950 sweep kernels.
//
//  - 4/8/16-byte vector loads of one coalesced 64-lane segment under the
//    four cache policies of the C ABI,
//  - the per-lane sinks (wrapping 32-bit sum and XOR of every loaded word,
//    the non-eliminable sink of Section 3, "Instruments"),
//  - DPP wave reductions of the sinks,
//  - the per-wave clock / hardware-id record.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ilpsweep.h"

namespace ilp {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int V> struct Vec;
template <> struct Vec<4>  { typedef uint32_t T; };
template <> struct Vec<8>  { typedef u32x2 T; };
template <> struct Vec<16> { typedef u32x4 T; };

constexpr int kWave = 64;
// Buffer-resource word 3 for gfx9-family raw (untyped) buffer loads:
// DATA_FORMAT = 32-bit, everything else zero.
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kNumPolicies = 4;
// Cache-policy bits of the gfx940-family MUBUF/global encodings as taken by
// the buffer-load builtins' aux operand: sc0 = 1, nt = 2, sc1 = 16.
constexpr int kAuxSc1 = 16;
constexpr int kAuxSc1Nt = 16 | 2;

// --------------------------------------------------------------- identities
__device__ __forceinline__ uint32_t wave_in_wg() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

// Constant-rate device wall clock (s_memrealtime), comparable across CUs
// and XCDs, unlike the per-CU shader cycle counter.
__device__ __forceinline__ uint64_t wall_ticks() {
  return __builtin_amdgcn_s_memrealtime();
}
// hwreg(HW_REG_HW_ID) and hwreg(HW_REG_XCC_ID), full 32 bits.
__device__ __forceinline__ uint32_t hw_id_reg() {
  return __builtin_amdgcn_s_getreg((31 << 11) | 4);
}
__device__ __forceinline__ uint32_t xcc_id_reg() {
  return __builtin_amdgcn_s_getreg((31 << 11) | 20);
}

// ----------------------------------------------------------------- loading
// Load lane `lane`'s V bytes of the 64-lane segment starting at `seg`
// (a wave-uniform pointer).
template <int V, int POL>
__device__ __forceinline__ typename Vec<V>::T load_seg(const uint8_t* seg,
                                                       uint32_t lane) {
  typedef typename Vec<V>::T T;
  if constexpr (POL == SWEEP_CACHE_DEFAULT) {
    return *reinterpret_cast<const T*>(seg + lane * V);
  } else if constexpr (POL == SWEEP_CACHE_NT) {
    return __builtin_nontemporal_load(reinterpret_cast<const T*>(seg + lane * V));
  } else {
    // buffer load over exactly this segment (out-of-range lanes would read 0)
    constexpr int aux = POL == SWEEP_CACHE_BYPASS_L1 ? kAuxSc1 : kAuxSc1Nt;
    __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(seg), 0, kWave * V, kRsrcWord3);
    if constexpr (V == 4) {
      return __builtin_amdgcn_raw_buffer_load_b32(r, lane * V, 0, aux);
    } else if constexpr (V == 8) {
      return __builtin_amdgcn_raw_buffer_load_b64(r, lane * V, 0, aux);
    } else {
      return __builtin_amdgcn_raw_buffer_load_b128(r, lane * V, 0, aux);
    }
  }
}

// ------------------------------------------------------------------- sinks
__device__ __forceinline__ void fold(uint32_t w, uint32_t& s, uint32_t& x) {
  s += w;
  x ^= w;
}
__device__ __forceinline__ void fold(u32x2 w, uint32_t& s, uint32_t& x) {
  fold(w.x, s, x);
  fold(w.y, s, x);
}
__device__ __forceinline__ void fold(u32x4 w, uint32_t& s, uint32_t& x) {
  fold(w.x, s, x);
  fold(w.y, s, x);
  fold(w.z, s, x);
  fold(w.w, s, x);
}

// ------------------------------------------------------- wave reductions
// DPP controls (gfx9): quad_perm [1,0,3,2], quad_perm [2,3,0,1], and
// rotations by 4 and 8 lanes within a 16-lane row.  After the four steps
// every lane of a row holds the row total; the four row totals are then
// combined from lanes 0, 16, 32 and 48.
constexpr int kDppQuadSwap1 = 0xB1;
constexpr int kDppQuadSwap2 = 0x4E;
constexpr int kDppRowRor4 = 0x124;
constexpr int kDppRowRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return __builtin_amdgcn_update_dpp(0u, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  v += dpp<kDppQuadSwap1>(v);
  v += dpp<kDppQuadSwap2>(v);
  v += dpp<kDppRowRor4>(v);
  v += dpp<kDppRowRor8>(v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

__device__ __forceinline__ uint32_t wave_xor_u32(uint32_t v) {
  v ^= dpp<kDppQuadSwap1>(v);
  v ^= dpp<kDppQuadSwap2>(v);
  v ^= dpp<kDppRowRor4>(v);
  v ^= dpp<kDppRowRor8>(v);
  return __builtin_amdgcn_readlane(v, 0) ^ __builtin_amdgcn_readlane(v, 16) ^
         __builtin_amdgcn_readlane(v, 32) ^ __builtin_amdgcn_readlane(v, 48);
}

// ---------------------------------------------------------- wave epilogue
// Reduce the lane sinks, then lane 0 stores the wave record (two 16-byte
// vector stores).  Optionally every lane first stores its own sinks.
__device__ __forceinline__ void wave_epilogue(uint32_t s, uint32_t x,
                                              uint64_t t0, uint64_t t1,
                                              uint32_t wid,
                                              sweep_wave_rec_t* rec,
                                              uint32_t* lane_out) {
  const uint32_t lane = lane_id();
  if (lane_out) {
    u32x2* lo = reinterpret_cast<u32x2*>(lane_out);
    lo[(uint64_t)wid * kWave + lane] = u32x2{s, x};
  }
  const uint32_t ws = wave_sum_u32(s);
  const uint32_t wx = wave_xor_u32(x);
  if (lane == 0) {
    u32x4* r = reinterpret_cast<u32x4*>(rec + wid);
    r[0] = u32x4{ws, wx, hw_id_reg(), xcc_id_reg()};
    r[1] = u32x4{(uint32_t)t0, (uint32_t)(t0 >> 32), (uint32_t)t1,
                 (uint32_t)(t1 >> 32)};
  }
}

// Wait until at most N vector-memory operations of this wave are
// outstanding.  The compiler does not track LDS-DMA writes for later LDS
// reads, so the LDS-direct path places its waits itself; the memory clobber
// keeps the compiler from moving memory accesses across the wait.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit counter");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
__device__ __forceinline__ void wait_lgkmcnt0() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}
__device__ __forceinline__ void compiler_fence() {
  asm volatile("" ::: "memory");
}

}  // namespace ilp
