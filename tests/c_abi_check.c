/* Plain-C user of the C ABI: no torch, no Python.  Allocates a buffer with
 * the HIP runtime, fills it with the seeded generator, runs one plain-load
 * cell in each address order, the allocation-free entry point, one
 * LDS-direct cell, one graph-batched pair, two replays of a captured graph
 * (the buffer refilled with seed + 1 between them), one fused graph and a
 * split two-stream launch, and prints the global sinks as "name sum xor
 * issued" lines for the calling test to check against the oracle. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "ilpsweep.h"

#define CHECK(x)                                                              \
  do {                                                                        \
    int rc_ = (x);                                                            \
    if (rc_ != SWEEP_OK) {                                                    \
      fprintf(stderr, "%s -> %d (%s: %s)\n", #x, rc_, sweep_strerror(rc_),    \
              sweep_last_error());                                            \
      return 1;                                                               \
    }                                                                         \
  } while (0)

int main(int argc, char** argv) {
  const size_t bytes = (argc > 1) ? (size_t)strtoull(argv[1], 0, 0) : (64u << 20);
  const unsigned long long seed = (argc > 2) ? strtoull(argv[2], 0, 0) : 7ull;
  void* buf = NULL;
  if (hipMalloc(&buf, bytes) != hipSuccess) return 2;
  CHECK(sweep_init(0));
  CHECK(sweep_fill_u32(buf, bytes, seed, NULL));

  sweep_opts_t opt = {0};
  opt.pin_occupancy = 1;
  opt.cache_policy = SWEEP_CACHE_BYPASS_L1_NT;
  sweep_result_t r;
  CHECK(sweep_plain(buf, bytes, 4, 16, 16, bytes / 16, &opt, &r));
  printf("plain %u %u %llu\n", r.sum32, r.xor32, (unsigned long long)r.issued_loads);
  opt.order = SWEEP_ORDER_BLOCKED;
  CHECK(sweep_plain(buf, bytes, 3, 16, 8, bytes / 16, &opt, &r));
  printf("blocked_K3 %u %u %llu\n", r.sum32, r.xor32, (unsigned long long)r.issued_loads);
  opt.order = SWEEP_ORDER_STRIDED;
  CHECK(sweep_plain(buf, bytes, 3, 16, 8, bytes / 16, &opt, &r));
  printf("strided_K3 %u %u %llu\n", r.sum32, r.xor32, (unsigned long long)r.issued_loads);
  opt.order = SWEEP_ORDER_ROUND_ROBIN;
  CHECK(sweep_plain_noalloc(buf, bytes, 4, 16, 16, bytes / 16, &opt, &r));
  printf("noalloc %u %u %llu\n", r.sum32, r.xor32, (unsigned long long)r.issued_loads);
  CHECK(sweep_lds_async(buf, bytes, 8, 16, 4, bytes / 16, &opt, &r));
  printf("lds_async %u %u %llu\n", r.sum32, r.xor32, (unsigned long long)r.issued_loads);

  sweep_cell_t cells[2] = {{0}};
  for (int i = 0; i < 2; ++i) {
    cells[i].kind = SWEEP_KIND_PLAIN;
    cells[i].K = i ? 3 : 2;
    cells[i].vec_width = 16;
    cells[i].waves_per_cu = 32;
    cells[i].cache_policy = SWEEP_CACHE_NT;
    cells[i].mode = SWEEP_FIXED_WORK;
    cells[i].buf = buf;
    cells[i].bytes = bytes;
    cells[i].total_logical_loads = bytes / 16;
  }
  sweep_result_t rs[2];
  double ms = 0;
  CHECK(sweep_batched(cells, 2, &opt, rs, &ms));
  for (int i = 0; i < 2; ++i)
    printf("batched_K%d %u %u %llu\n", cells[i].K, rs[i].sum32, rs[i].xor32,
           (unsigned long long)rs[i].issued_loads);
  sweep_graph_t* g = NULL;
  CHECK(sweep_graph_create(cells, 2, &opt, &g));
  for (int rep = 0; rep < 2; ++rep) {
    if (rep) CHECK(sweep_fill_u32(buf, bytes, seed + 1, NULL));
    CHECK(sweep_graph_launch(g, NULL, rs, &ms));
    for (int i = 0; i < 2; ++i)
      printf("graph_K%d_rep%d %u %u %llu\n", cells[i].K, rep, rs[i].sum32, rs[i].xor32,
             (unsigned long long)rs[i].issued_loads);
  }
  CHECK(sweep_graph_destroy(g));
  /* two cells of one configuration fused into one persistent launch */
  sweep_cell_t fc[2] = {cells[1], cells[1]};
  opt.fuse = 1;
  g = NULL;
  CHECK(sweep_graph_create(fc, 2, &opt, &g));
  CHECK(sweep_graph_launch(g, NULL, rs, &ms));
  for (int i = 0; i < 2; ++i)
    printf("fused_%d %u %u %llu\n", i, rs[i].sum32, rs[i].xor32,
           (unsigned long long)rs[i].issued_loads);
  CHECK(sweep_graph_destroy(g));
  opt.fuse = 0;
  /* the two streams on different CUs, over the buffer's two halves */
  sweep_result_t r2[2];
  CHECK(sweep_two_stream_split(buf, bytes, 4, 8, 8, SWEEP_KIND_PLAIN, bytes / 16, &opt, r2));
  for (int i = 0; i < 2; ++i)
    printf("split_%c %u %u %llu\n", i ? 'b' : 'a', r2[i].sum32, r2[i].xor32,
           (unsigned long long)r2[i].issued_loads);
  CHECK(sweep_shutdown());
  (void)hipFree(buf);
  return 0;
}
