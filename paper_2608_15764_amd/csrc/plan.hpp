// Host-only planning of a sweep cell: validation, the fixed-work
// decomposition, grid sizing and occupancy padding.  No HIP calls, so it is
// exercised on machines without a GPU through sweep_plan().
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "ilpsweep.h"

namespace ilp {

struct PlanIn {
  size_t bytes = 0;
  int K = 0;               // loads per iteration / ring depth
  int V = 0;               // vector width in bytes
  int kind = SWEEP_KIND_PLAIN;
  int waves_per_cu = 0;    // plain: total per CU; LDS kinds: waves per WG
  uint64_t L = 0;
  int mode = SWEEP_FIXED_WORK;
  uint32_t fixed_iters = 0;
  uint32_t num_cus = 0;
  uint32_t grid_wgs = 0;   // 0 = automatic
  uint32_t lds_per_cu = 0;      // 0 = unknown (no padding computed)
  uint32_t lds_per_wg_max = 0;
  int order = SWEEP_ORDER_ROUND_ROBIN;
};

struct Plan {
  sweep_plan_t pub{};
  uint64_t stride = 0;       // vector step between a wave's groups, mod n_vec
  uint64_t gstep = 0;        // vector step from group q to q + 1 (start vectors)
  uint64_t jstep = 0;        // vector step from load j to j + 1 of a group, mod n_vec
  uint64_t G = 0;            // groups per wave in blocked order
  uint32_t wg_waves = 0;     // waves per workgroup
  uint32_t wgs_per_cu = 0;   // residency the grid asks for
  uint32_t lds_ring_bytes = 0;  // LDS the kernel itself uses per WG
};

// Returns SWEEP_OK or a negative code with *err set.
int plan_cell(const PlanIn& in, Plan* out, std::string* err);

// Fixed-work split of `L` over one region of `n_vec` vectors: wave-groups,
// issued loads and the wrap stride for n_waves waves.
void region_plan(uint64_t n_vec, int K, uint64_t L, uint32_t n_waves,
                 uint64_t* Q, uint64_t* stride);

// LDS padding that lets at most `target` workgroups share a CU: the padded
// size p satisfies target * p <= lds_per_cu < (target + 1) * p, clamped to
// the per-workgroup maximum.  Returns 0 if no padding is possible.
uint32_t pin_padding(uint32_t target, uint32_t base, uint32_t lds_per_cu,
                     uint32_t lds_per_wg_max);

}  // namespace ilp
