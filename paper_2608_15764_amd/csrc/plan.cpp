// Fixed-work control (Section 3, "Fixed-work control") and exact-work
// accounting (Section 4.2, "Exact-work accounting") on the host.
#include "plan.hpp"

#include <algorithm>

namespace ilp {

static int bad(std::string* err, int code, const char* msg) {
  if (err) *err = msg;
  return code;
}

void region_plan(uint64_t n_vec, int K, uint64_t L, uint32_t n_waves,
                 uint64_t* Q, uint64_t* stride) {
  *Q = L / (64ull * (uint64_t)K);
  *stride = n_vec ? ((uint64_t)n_waves * (uint64_t)K * 64ull) % n_vec : 0;
}

uint32_t pin_padding(uint32_t target, uint32_t base, uint32_t lds_per_cu,
                     uint32_t lds_per_wg_max) {
  if (target == 0 || lds_per_cu == 0) return 0;
  // smallest 256-byte multiple above lds_per_cu / (target + 1)
  uint64_t p = (uint64_t)lds_per_cu / (target + 1) + 1;
  p = (p + 255) / 256 * 256;
  p = std::max<uint64_t>(p, base);
  if ((uint64_t)target * p > lds_per_cu) return 0;   // cannot hold target
  p = std::min<uint64_t>(p, lds_per_wg_max);
  return (uint32_t)p;
}

int plan_cell(const PlanIn& in, Plan* out, std::string* err) {
  const bool plain = in.kind == SWEEP_KIND_PLAIN;
  if (!plain && in.kind != SWEEP_KIND_LDS_ASYNC && in.kind != SWEEP_KIND_LDS_MATCHED)
    return bad(err, SWEEP_EINVAL, "unknown kernel kind");
  if (in.K < 1 || in.K > 16) return bad(err, SWEEP_EINVAL, "K (depth) must be in 1..16");
  if (plain) {
    if (in.V != 4 && in.V != 8 && in.V != 16)
      return bad(err, SWEEP_EINVAL, "vec_width must be 4, 8 or 16");
    if (in.waves_per_cu < 4 || in.waves_per_cu > 32 || in.waves_per_cu % 4)
      return bad(err, SWEEP_EINVAL, "waves_per_cu must be a multiple of 4 in 4..32");
  } else {
    if (in.V != 16) return bad(err, SWEEP_EINVAL, "LDS paths use 16-byte requests");
    if (in.waves_per_cu < 1 || in.waves_per_cu > 16)
      return bad(err, SWEEP_EINVAL, "LDS paths take 1..16 waves per CU");
  }
  if (in.bytes == 0) return bad(err, SWEEP_EINVAL, "empty buffer");
  // every 64-lane segment must lie inside the buffer, also after a wrap
  if (in.bytes % (64ull * (uint64_t)in.V))
    return bad(err, SWEEP_EALIGN, "bytes must be a multiple of 64 * vec_width");
  if (in.num_cus == 0 && in.grid_wgs == 0)
    return bad(err, SWEEP_EINVAL, "no CU count to size the grid");
  if (in.mode != SWEEP_FIXED_WORK && in.mode != SWEEP_FIXED_ITERS &&
      in.mode != SWEEP_PER_THREAD_FLOOR)
    return bad(err, SWEEP_EINVAL, "unknown work mode");
  if (in.order != SWEEP_ORDER_ROUND_ROBIN && in.order != SWEEP_ORDER_BLOCKED &&
      in.order != SWEEP_ORDER_STRIDED)
    return bad(err, SWEEP_EINVAL, "unknown work-group order");
  if (!plain && in.order != SWEEP_ORDER_ROUND_ROBIN)
    return bad(err, SWEEP_EINVAL, "the LDS paths deal work-groups round robin only");

  Plan p;
  p.wg_waves = plain ? 4u : (uint32_t)in.waves_per_cu;
  p.wgs_per_cu = plain ? (uint32_t)in.waves_per_cu / 4u : 1u;
  p.lds_ring_bytes = plain ? 0u : (uint32_t)(in.waves_per_cu * in.K * 1024);
  if (in.lds_per_wg_max && p.lds_ring_bytes > in.lds_per_wg_max)
    return bad(err, SWEEP_EOCCUPANCY, "LDS ring exceeds the per-workgroup LDS");

  sweep_plan_t& o = p.pub;
  o.grid_wgs = in.grid_wgs ? in.grid_wgs : in.num_cus * p.wgs_per_cu;
  o.wg_threads = p.wg_waves * 64u;
  o.waves = o.grid_wgs * p.wg_waves;
  o.n_vec = in.bytes / (uint64_t)in.V;
  const uint64_t nw = o.waves;
  const uint64_t threads = nw * 64ull;
  const uint64_t K = (uint64_t)in.K;
  switch (in.mode) {
    case SWEEP_FIXED_WORK:
      if (in.L == 0) return bad(err, SWEEP_EINVAL, "total_logical_loads is 0");
      o.Q = in.L / (64ull * K);
      break;
    case SWEEP_FIXED_ITERS:
      if (in.fixed_iters == 0) return bad(err, SWEEP_EINVAL, "fixed_iters is 0");
      o.Q = nw * (uint64_t)in.fixed_iters;
      break;
    default:  // SWEEP_PER_THREAD_FLOOR
      if (in.L == 0) return bad(err, SWEEP_EINVAL, "total_logical_loads is 0");
      o.Q = nw * (in.L / (threads * K));
      break;
  }
  if (o.Q == 0) return bad(err, SWEEP_EINVAL, "L is smaller than one wave-group per wave");
  o.issued_loads = 64ull * K * o.Q;
  if (o.issued_loads > UINT64_MAX / (uint64_t)in.V)
    return bad(err, SWEEP_EINVAL, "issued bytes do not fit 64 bits");
  o.issued_bytes = o.issued_loads * (uint64_t)in.V;
  p.G = (o.Q + nw - 1) / nw;
  // per-wave iteration counts are reported in 32 bits
  if (p.G > UINT32_MAX)
    return bad(err, SWEEP_EINVAL, "a wave would run more than 2^32 - 1 iterations");
  if (in.order == SWEEP_ORDER_BLOCKED) {
    // wave w handles min(G, max(0, Q - w G)) groups
    const uint64_t last = (nw - 1) * p.G;
    o.iters_min = (uint32_t)(o.Q > last ? std::min<uint64_t>(p.G, o.Q - last) : 0);
    o.iters_max = (uint32_t)p.G;
  } else {
    o.iters_min = (uint32_t)(o.Q / nw);
    o.iters_max = (uint32_t)p.G;
  }
  o.mismatch = in.mode == SWEEP_FIXED_ITERS
                   ? 0.0
                   : (double)(in.L - o.issued_loads) / (double)in.L;
  // contiguous layouts: group q starts at vector q*K*64 and its loads are
  // adjacent segments; strided: group q starts at q*64 and load j is
  // j*Q segments further on
  const bool strided = in.order == SWEEP_ORDER_STRIDED;
  p.gstep = strided ? 64ull : K * 64ull;
  p.jstep = strided ? (o.Q * 64ull) % o.n_vec : 64ull % o.n_vec;
  p.stride = in.order == SWEEP_ORDER_BLOCKED ? p.gstep % o.n_vec
                                             : (nw * p.gstep) % o.n_vec;
  o.lds_pad_bytes = pin_padding(p.wgs_per_cu, p.lds_ring_bytes, in.lds_per_cu,
                                in.lds_per_wg_max);
  *out = p;
  return SWEEP_OK;
}

}  // namespace ilp
