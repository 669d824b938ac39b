// Host-only fuzz driver for the planner: reads cases "bytes K V kind waves L
// mode fixed_iters num_cus grid order" from stdin and prints one line per
// case: "rc Q issued iters_min iters_max grid waves stride G pad".  Built
// with the address and undefined-behaviour sanitizers by the test.
#include <cstdio>
#include <string>

#include "plan.hpp"

int main() {
  unsigned long long bytes, L;
  int K, V, kind, waves, mode, order;
  unsigned fixed, cus, grid;
  while (std::scanf("%llu %d %d %d %d %llu %d %u %u %u %d", &bytes, &K, &V, &kind, &waves,
                    &L, &mode, &fixed, &cus, &grid, &order) == 11) {
    ilp::PlanIn in;
    in.bytes = bytes;
    in.K = K;
    in.V = V;
    in.kind = kind;
    in.waves_per_cu = waves;
    in.L = L;
    in.mode = mode;
    in.fixed_iters = fixed;
    in.num_cus = cus;
    in.grid_wgs = grid;
    in.order = order;
    in.lds_per_cu = 163840;
    in.lds_per_wg_max = 163840;
    ilp::Plan p;
    std::string err;
    const int rc = ilp::plan_cell(in, &p, &err);
    if (rc)
      std::printf("%d\n", rc);
    else
      std::printf("0 %llu %llu %u %u %u %u %llu %llu %u\n", (unsigned long long)p.pub.Q,
                  (unsigned long long)p.pub.issued_loads, p.pub.iters_min, p.pub.iters_max,
                  p.pub.grid_wgs, p.pub.waves, (unsigned long long)p.stride,
                  (unsigned long long)p.G, p.pub.lds_pad_bytes);
  }
  return 0;
}
