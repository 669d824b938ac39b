// Kernel argument blocks and host-side launch entry points of the gfx950
// kernels.  Each kernel family lives in its own translation unit and is
// reached from the runtime only through the functions declared here.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ilpsweep.h"

namespace ilp {

constexpr int kMaxK = 16;
constexpr int kPlainWgThreads = 256;   // 4 waves, one per SIMD

// Plain K-load cell.  Round robin (and strided): wave w of n_waves handles
// wave-groups q = w, w + n_waves, ... below Q; blocked: q = w*G .. w*G +
// G - 1.  Load j of group q reads the 64 vectors starting at vector
// (q*gstep + j*jstep) mod n_vec: gstep = K*64, jstep = 64 (adjacent
// segments, (q*K + j)*64), or in the strided layout gstep = 64, jstep =
// Q*64 ((j*Q + q)*64).  `stride` is the vector step between a wave's
// consecutive groups, mod n_vec: n_waves*gstep (round robin, strided) or
// gstep (blocked).
struct PlainArgs {
  const uint8_t* buf;
  uint64_t n_vec;
  uint64_t Q;
  uint64_t stride;
  sweep_wave_rec_t* rec;
  uint32_t* lane_out;
  uint64_t G;          // groups per wave in blocked order
  uint32_t order;      // SWEEP_ORDER_*
  uint64_t gstep;      // start vector of group q: q * gstep (mod n_vec)
  uint64_t jstep;      // from load j to load j + 1 (mod n_vec), below n_vec
};

// Fused batch of plain cells that share K, vector width, cache policy and
// launch shape: one persistent launch over their concatenated wave-groups.
// Point p owns global groups [g0, g0 + Q); wave w of n_waves handles global
// groups w, w + n_waves, ... (round robin over the concatenation), reading
// load j of its point's local group q at vector (q*K + j)*64 mod n_vec.
// `stride` = (n_waves*K*64) mod n_vec is a wave's vector step between two
// of its groups inside one point.  Wave w's record for point p is
// rec[p*n_waves + w]; records of points a wave never reaches are left as
// they are (cleared once, before the first launch, to "empty").
struct FusedPoint {
  uint64_t off;            // the point's buffer: FusedArgs::base + off
  uint64_t n_vec;
  uint64_t Q;
  uint64_t g0;
  uint64_t stride;
};
struct FusedArgs {
  const uint8_t* base;     // the lowest point buffer of the launch
  const FusedPoint* pts;   // device, n_pts entries
  uint64_t total_groups;   // sum of Q over the points
  sweep_wave_rec_t* rec;   // n_pts * n_waves records
};

// LDS-ring cell (async or matched), `waves` waves per workgroup.
struct LdsArgs {
  const uint8_t* buf;
  uint64_t n_vec;
  uint64_t Q;
  uint64_t stride;        // (n_waves*D*64) mod n_vec
  sweep_wave_rec_t* rec;
  uint32_t* lane_out;
  uint32_t waves;         // waves per workgroup
};

// Two co-resident streams: A (plain K = D) on region A, B (LDS-async ring
// of depth D) on region B.  Records of A come first (n_waves_a of them),
// then those of B.
struct TwoStreamArgs {
  const uint8_t* buf_a;
  uint64_t n_vec_a, Q_a, stride_a;
  const uint8_t* buf_b;
  uint64_t n_vec_b, Q_b, stride_b;
  sweep_wave_rec_t* rec;   // n_waves_a + n_waves_b records
  uint32_t* lane_out;      // lanes of A then lanes of B, or null
  uint32_t waves_a, waves_b;  // per workgroup
  uint32_t b_plain;           // 1: stream B runs the plain loop as well
  uint32_t split;             // 1: each workgroup runs one stream only
};

// Precision variant: full wave-groups of 4 or 8 loads x 64 lanes x 16 bytes,
// then the ragged remainder (whole 16-byte vectors, then the last bytes).
struct ReduceArgs {
  const uint8_t* payload;
  uint64_t n_groups;        // full wave-groups (loads x 1 KiB each)
  uint64_t n_vec;           // whole 16-byte vectors
  uint64_t n_bytes;         // payload bytes
  float* partials;          // 2 floats (s, c) per workgroup
  sweep_wave_rec_t* rec;
};

// Pointer chase: buf[idx] holds the next index (32-bit words); `out`
// receives {final index, wall t0, wall t1, shader-clock t0, shader-clock t1}.
constexpr uint32_t kMaxChaseSamples = 4096;
struct ChaseArgs {
  const uint32_t* buf;
  uint32_t n_bytes;        // buffer bytes (< 4 GiB)
  uint32_t start;
  uint32_t warm;           // untimed hops
  uint32_t steps;          // timed hops
  uint32_t n_samples;      // per-hop cycle samples (first hops), <= 4096
  uint32_t* samples;       // device [n_samples] or null if n_samples == 0
  uint64_t* out;           // device [5]
};

// Several dependent-chain walkers at once, one single-lane wave per
// workgroup; walker b starts at starts[b] and writes out[4b .. 4b+3] =
// final index, wall clock at the start and end of its timed hops, XCC_ID.
constexpr uint32_t kMaxWalkers = 64;
struct WalkArgs {
  const uint32_t* buf;
  uint32_t n_bytes;        // buffer bytes (< 4 GiB)
  uint32_t warm;           // untimed hops per walker
  uint32_t steps;          // timed hops per walker
  uint32_t n_walkers;      // 1..kMaxWalkers (= the grid)
  uint32_t starts[kMaxWalkers];
  uint64_t* out;           // device [4 * n_walkers]
};

// Streaming read by the workgroups of chosen XCDs only (sweep_xcd_subset).
// Workgroup b belongs to XCD b mod 8; the active waves, numbered densely,
// read groups of kXcdK adjacent 64-lane segments of 16-byte vectors dealt
// round robin: group i * n_act + w goes to active wave w.
constexpr int kXcdK = 8;
struct XcdArgs {
  const uint8_t* buf;
  uint64_t groups;         // groups per active wave
  uint64_t n_act;          // active waves
  uint32_t mask;           // bit x set: workgroups on XCD x work
  uint32_t pop;            // set bits in mask
  sweep_wave_rec_t* rec;   // device [n_act]
};

// Static split weighted per XCD (sweep_xcd_split): XCD x reads groups
// [starts[x], starts[x+1]) of kXcdK segments, dealt round robin over its own
// waves; waves are numbered (rank of the XCD among those with a share,
// wave within the XCD).
struct XcdSplitArgs {
  const uint8_t* buf;
  uint64_t starts[9];      // group prefix sums per XCD
  uint32_t per_xcd;        // waves per XCD
  uint32_t mask;           // XCDs with a nonzero share
  sweep_wave_rec_t* rec;   // device [popcount(mask) * per_xcd]
};

// Per-cell result reduced on the device from the wave records.
struct CellRes {
  uint64_t sum;   // low 32 bits used
  uint64_t xr;    // low 32 bits used
  uint64_t tmin;
  uint64_t tmax;
};

// ---- static scratch of the allocation-free entry point (static_scratch.hip)
// Layout: per-wave records, then the cell result, then the two record
// offsets the finishing kernel reads.  512 KiB + 256 bytes per device.
constexpr uint64_t kStaticRecords = 16384;
constexpr uint64_t kStaticResOffset = kStaticRecords * sizeof(sweep_wave_rec_t);
constexpr uint64_t kStaticOffsOffset = kStaticResOffset + 64;
constexpr uint64_t kStaticScratchBytes = kStaticResOffset + 256;
// Device address of the calling thread's current device's copy of the
// static scratch (resolved once per device, with that device current).
hipError_t static_scratch(int ordinal, uint8_t** ptr);

// ---- kernel lookup: the host launches these with their one argument
// struct (PlainArgs, LdsArgs, TwoStreamArgs, ReduceArgs); nullptr for an
// unknown combination.
// plain (kernels_plain.hip)
const void* plain_kernel(int K, int V, int policy);
// fused plain batch (kernels_fused.hip)
const void* fused_kernel(int K, int V, int policy);
const void* xcd_kernel(int policy);
const void* xcd_split_kernel(int policy);
// Set `n` records to "empty" (zero sinks, t0 = all ones, t1 = 0), which
// the finishing kernel's min / max ignore.
hipError_t launch_clear_records(sweep_wave_rec_t* rec, uint64_t n, hipStream_t st);

// ---- LDS paths (kernels_lds.hip)
const void* lds_kernel(int kind, int D, int policy);
const void* two_stream_kernel(int D, int policy);

// ---- pointer chase (kernels_chase.hip)
const void* chase_kernel(int policy);
hipError_t launch_chase(int policy, hipStream_t st, const ChaseArgs& a);
hipError_t launch_walkers(int policy, hipStream_t st, const WalkArgs& a);

// ---- fill, finishing, clock, reduction (kernels_misc.hip)
hipError_t launch_fill(uint32_t* buf, uint64_t n_words, uint64_t seed,
                       hipStream_t st);
// One workgroup per cell: cell c owns records [offsets[c], offsets[c+1]).
hipError_t launch_finish_cells(const sweep_wave_rec_t* rec, const uint64_t* offsets,
                               uint32_t n_cells, CellRes* out, hipStream_t st);
hipError_t launch_read_clock(uint64_t* out, hipStream_t st);
// `loads` (4 or 8) 16-byte loads in flight per lane per iteration.
const void* reduce_kernel(int dtype, int loads);
hipError_t launch_reduce_finish(const float* partials, uint32_t n,
                                double* out, hipStream_t st);

}  // namespace ilp
