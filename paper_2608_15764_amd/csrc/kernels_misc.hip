// Buffer fill, per-cell finishing, clock probe and the precision variant's
// streaming FP reduction.
#include "device.hpp"
#include "kernels.hpp"

namespace ilp {

// ------------------------------------------------------------------ fill
// Word i of the buffer is the low half of SplitMix64 output i for state
// `seed`: z = seed + (i+1)*gamma, then the SplitMix64 finaliser
// (Steele, Lea and Flood, 2014).
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint32_t splitmix_word(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * kGamma;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (uint32_t)z;
}

__global__ __launch_bounds__(256) void fill_u32(uint32_t* buf, uint64_t n_words,
                                                uint64_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t n4 = n_words / 4;
  u32x4* b4 = reinterpret_cast<u32x4*>(buf);
  for (uint64_t v = tid; v < n4; v += stride) {
    const uint64_t i = v * 4;
    b4[v] = u32x4{splitmix_word(seed, i), splitmix_word(seed, i + 1),
                  splitmix_word(seed, i + 2), splitmix_word(seed, i + 3)};
  }
  for (uint64_t i = n4 * 4 + tid; i < n_words; i += stride)
    buf[i] = splitmix_word(seed, i);
}

hipError_t launch_fill(uint32_t* buf, uint64_t n_words, uint64_t seed,
                       hipStream_t st) {
  const uint64_t n4 = (n_words + 3) / 4;
  uint64_t blocks = (n4 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(fill_u32, dim3((uint32_t)blocks), dim3(256), 0, st, buf,
                     n_words, seed);
  return hipGetLastError();
}

// ---------------------------------------------------------------- finish
// Workgroup c folds the wave records of cell c, rec[offsets[c] ..
// offsets[c+1]), into the cell's global sinks and its clock window
// [min t0, max t1].
__global__ __launch_bounds__(256) void finish_cells(const sweep_wave_rec_t* rec,
                                                    const uint64_t* offsets,
                                                    CellRes* out) {
  __shared__ uint32_t ss[256], sx[256];
  __shared__ uint64_t smin[256], smax[256];
  const uint64_t lo_i = offsets[blockIdx.x], hi_i = offsets[blockIdx.x + 1];
  uint32_t s = 0, x = 0;
  uint64_t lo = ~0ull, hi = 0;
  for (uint64_t i = lo_i + threadIdx.x; i < hi_i; i += 256) {
    const sweep_wave_rec_t r = rec[i];
    s += r.sum32;
    x ^= r.xor32;
    lo = r.t0 < lo ? r.t0 : lo;
    hi = r.t1 > hi ? r.t1 : hi;
  }
  ss[threadIdx.x] = s;
  sx[threadIdx.x] = x;
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (uint32_t h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      ss[threadIdx.x] += ss[threadIdx.x + h];
      sx[threadIdx.x] ^= sx[threadIdx.x + h];
      if (smin[threadIdx.x + h] < smin[threadIdx.x]) smin[threadIdx.x] = smin[threadIdx.x + h];
      if (smax[threadIdx.x + h] > smax[threadIdx.x]) smax[threadIdx.x] = smax[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    CellRes r;
    r.sum = ss[0];
    r.xr = sx[0];
    r.tmin = smin[0];
    r.tmax = smax[0];
    out[blockIdx.x] = r;
  }
}

hipError_t launch_finish_cells(const sweep_wave_rec_t* rec, const uint64_t* offsets,
                               uint32_t n_cells, CellRes* out, hipStream_t st) {
  hipLaunchKernelGGL(finish_cells, dim3(n_cells), dim3(256), 0, st, rec, offsets, out);
  return hipGetLastError();
}

// ----------------------------------------------------------------- clock
__global__ void read_clock(uint64_t* out) {
  if (threadIdx.x == 0) out[0] = wall_ticks();
}

hipError_t launch_read_clock(uint64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(read_clock, dim3(1), dim3(64), 0, st, out);
  return hipGetLastError();
}

// --------------------------------------------------- precision reduction
// Sum2 (Ogita, Rump and Oishi, 2005) per lane: TwoSum (Knuth) is
// error-free, s' + e = s + x exactly; the errors e are summed plainly in c.
struct Pair {
  float s, c;
};

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void add_term(Pair& p, float x) {
  float s, e;
  two_sum(p.s, x, s, e);
  p.s = s;
  p.c += e;
}

// Merge two pairs: TwoSum of the leading parts, the rest summed plainly.
__device__ __forceinline__ Pair merge(Pair a, Pair b) {
  Pair r;
  float e;
  two_sum(a.s, b.s, r.s, e);
  r.c = (a.c + b.c) + e;
  return r;
}

__device__ __forceinline__ float f32_of(uint32_t w) { return __uint_as_float(w); }

// Decode-and-accumulate of one 16-byte vector.
template <int DT>
__device__ __forceinline__ void acc_vec(Pair& p, u32x4 v);

template <>
__device__ __forceinline__ void acc_vec<SWEEP_F32>(Pair& p, u32x4 v) {
  add_term(p, f32_of(v.x));
  add_term(p, f32_of(v.y));
  add_term(p, f32_of(v.z));
  add_term(p, f32_of(v.w));
}

template <>
__device__ __forceinline__ void acc_vec<SWEEP_BF16>(Pair& p, u32x4 v) {
  // element 2k is the low half of word k (little endian)
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    add_term(p, f32_of(w[k] << 16));
    add_term(p, f32_of(w[k] & 0xFFFF0000u));
  }
}

// Plain FP32 sum of the 16 FP8 values of a vector (exact, see below).
__device__ __forceinline__ float fp8_vec_sum(u32x4 v) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  float t = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w[k], false);  // bytes 0, 1
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w[k], true);   // bytes 2, 3
    t += lo[0];
    t += lo[1];
    t += hi[0];
    t += hi[1];
  }
  return t;
}

template <>
__device__ __forceinline__ void acc_vec<SWEEP_FP8_E4M3>(Pair& p, u32x4 v) {
  add_term(p, fp8_vec_sum(v));
}

// Elements per 16-byte vector and bytes per element.
template <int DT> constexpr int elem_bytes() { return DT == SWEEP_F32 ? 4 : DT == SWEEP_BF16 ? 2 : 1; }

template <int DT>
__device__ __forceinline__ float decode_one(const uint8_t* p) {
  if constexpr (DT == SWEEP_F32) {
    uint32_t w = p[0] | (p[1] << 8) | (p[2] << 16) | ((uint32_t)p[3] << 24);
    return f32_of(w);
  } else if constexpr (DT == SWEEP_BF16) {
    uint32_t w = (p[0] | (p[1] << 8)) << 16;
    return f32_of(w);
  } else {
    return __builtin_amdgcn_cvt_pk_f32_fp8((uint32_t)p[0], false)[0];
  }
}

// NL = loads in flight per lane per iteration (4 or 8); a wave-group is
// NL x 64 lanes x 16 bytes.
template <int DT, int NL>
__global__ __launch_bounds__(256) void reduce_fp(ReduceArgs a) {
  static_assert(NL % 4 == 0, "FP8 groups of four vectors are summed exactly");
  const uint64_t t0 = wall_ticks();
  const uint32_t lane = lane_id();
  const uint32_t wv = wave_in_wg();
  const uint32_t wid = blockIdx.x * 4 + wv;
  const uint32_t n_waves = gridDim.x * 4;
  Pair p{0.0f, 0.0f};

  // full wave-groups; all NL loads are issued before any is consumed
#pragma unroll 1
  for (uint64_t g = wid; g < a.n_groups; g += n_waves) {
    const uint8_t* base = a.payload + g * (NL * kWave * 16);
    u32x4 v[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j)
      v[j] = load_seg<16, SWEEP_CACHE_NT>(base + j * (kWave * 16), lane);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (DT == SWEEP_FP8_E4M3) {
      // 64 e4m3 values are k * 2^-9 with |k| <= 64 * 229376 < 2^24, so
      // their FP32 sum is exact; one TwoSum per 64 values (four vectors)
#pragma unroll
      for (int q = 0; q < NL / 4; ++q) {
        float t = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) t += fp8_vec_sum(v[4 * q + j]);
        add_term(p, t);
      }
    } else {
#pragma unroll
      for (int j = 0; j < NL; ++j) acc_vec<DT>(p, v[j]);
    }
  }
  // remaining whole vectors, one per thread of the grid
  const uint64_t gtid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t first_rem = a.n_groups * (NL * kWave);
  if (first_rem + gtid < a.n_vec) {
    const u32x4 v = *reinterpret_cast<const u32x4*>(a.payload + (first_rem + gtid) * 16);
    acc_vec<DT>(p, v);
  }
  // trailing bytes that do not fill a vector
  if (gtid == 0) {
    for (uint64_t off = a.n_vec * 16; off + elem_bytes<DT>() <= a.n_bytes;
         off += elem_bytes<DT>())
      add_term(p, decode_one<DT>(a.payload + off));
  }

  // wave merge: rotations within 16-lane rows, then the four rows in order
  auto xchg = [](Pair q, auto ctrl) {
    Pair o;
    o.s = __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(q.s), decltype(ctrl)::value, 0xF, 0xF, false));
    o.c = __uint_as_float(__builtin_amdgcn_update_dpp(0u, __float_as_uint(q.c), decltype(ctrl)::value, 0xF, 0xF, false));
    return o;
  };
  p = merge(p, xchg(p, std::integral_constant<int, kDppQuadSwap1>{}));
  p = merge(p, xchg(p, std::integral_constant<int, kDppQuadSwap2>{}));
  p = merge(p, xchg(p, std::integral_constant<int, kDppRowRor4>{}));
  p = merge(p, xchg(p, std::integral_constant<int, kDppRowRor8>{}));
  Pair r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r[k].s = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(p.s), 16 * k));
    r[k].c = __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(p.c), 16 * k));
  }
  const Pair wsum = merge(merge(r[0], r[1]), merge(r[2], r[3]));

  __shared__ Pair wg[4];
  if (lane == 0) wg[wv] = wsum;
  const uint64_t t1 = wall_ticks();
  if (lane == 0) {
    u32x4* rr = reinterpret_cast<u32x4*>(a.rec + wid);
    rr[0] = u32x4{0u, 0u, hw_id_reg(), xcc_id_reg()};
    rr[1] = u32x4{(uint32_t)t0, (uint32_t)(t0 >> 32), (uint32_t)t1, (uint32_t)(t1 >> 32)};
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const Pair b = merge(merge(wg[0], wg[1]), merge(wg[2], wg[3]));
    a.partials[2 * blockIdx.x] = b.s;
    a.partials[2 * blockIdx.x + 1] = b.c;
  }
}

template <int NL>
const void* reduce_of(int dtype) {
  switch (dtype) {
    case SWEEP_F32: return reinterpret_cast<const void*>(&reduce_fp<SWEEP_F32, NL>);
    case SWEEP_BF16: return reinterpret_cast<const void*>(&reduce_fp<SWEEP_BF16, NL>);
    case SWEEP_FP8_E4M3: return reinterpret_cast<const void*>(&reduce_fp<SWEEP_FP8_E4M3, NL>);
    default: return nullptr;
  }
}

const void* reduce_kernel(int dtype, int loads) {
  if (loads == 4) return reduce_of<4>(dtype);
  if (loads == 8) return reduce_of<8>(dtype);
  return nullptr;
}

// Final combine in FP64, in a fixed order: thread t sums partial pairs
// t, t+256, ... and the 256 totals are added up a fixed binary tree.
__global__ __launch_bounds__(256) void reduce_finish(const float* partials,
                                                     uint32_t n, double* out) {
  __shared__ double sd[256];
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < n; i += 256)
    acc += (double)partials[2 * i] + (double)partials[2 * i + 1];
  sd[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) sd[threadIdx.x] += sd[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sd[0];
}

hipError_t launch_reduce_finish(const float* partials, uint32_t n, double* out,
                                hipStream_t st) {
  hipLaunchKernelGGL(reduce_finish, dim3(1), dim3(256), 0, st, partials, n, out);
  return hipGetLastError();
}

}  // namespace ilp
