// Host runtime behind the C ABI of include/ilpsweep.h: per-device state and
// scratch, validation through the planner, occupancy checks, launches on
// the caller's stream with hipEvents, per-cell finishing, the back-to-back
// sweep driver, the hipGraph-batched sweep, the autotuner and the clock
// calibration.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "ilpsweep.h"
#include "kernels.hpp"
#include "plan.hpp"

using namespace ilp;

namespace {

thread_local std::string t_err;

int fail(int code, std::string msg) {
  t_err = std::move(msg);
  return code;
}

#define HIP_TRY(x)                                                          \
  do {                                                                      \
    hipError_t e__ = (x);                                                   \
    if (e__ != hipSuccess)                                                  \
      return fail(SWEEP_EHIP, std::string(#x) + ": " + hipGetErrorString(e__)); \
  } while (0)

#define SW_TRY(x)           \
  do {                      \
    int r__ = (x);          \
    if (r__ != SWEEP_OK) return r__; \
  } while (0)

struct Dev {
  int ordinal = -1;
  char arch[64] = {0};
  uint32_t num_cus = 0, lds_per_cu = 0, lds_per_wg_max = 0, l2 = 0;
  uint64_t hbm = 0;
  double nominal_hz = 0, cal_hz = 0;
  int clock_khz = 0, mem_khz = 0, bus_bits = 0;
  sweep_wave_rec_t* rec = nullptr;
  size_t rec_cap = 0;
  CellRes* res = nullptr;
  size_t res_cap = 0;
  CellRes* res_h = nullptr;   // pinned host copy
  size_t res_h_cap = 0;
  float* partials = nullptr;
  size_t partials_cap = 0;
  double* dsum = nullptr;
  double* dsum_h = nullptr;
  uint64_t* clk = nullptr;
  uint64_t* chase_out = nullptr;  // 5 words per chase call
  uint64_t* walk_out = nullptr;   // 4 words per walker
  uint64_t* offs = nullptr;     // per-cell record offsets (device)
  size_t offs_cap = 0;
  uint64_t* offs_h = nullptr;   // pinned staging copy
  size_t offs_h_cap = 0;
  std::vector<hipEvent_t> ev;
  hipStream_t capture = nullptr;
  // kernel attributes and residency limit per (kernel, WG threads, LDS)
  struct Occ {
    hipFuncAttributes fa;
    int max_wgs;
  };
  std::map<std::tuple<const void*, uint32_t, size_t>, Occ> occ;
  bool scratch_ready = false;   // setup_device has run
  double hz() const { return cal_hz > 0 ? cal_hz : nominal_hz; }
};

std::mutex g_mu;
std::map<int, Dev*> g_devs;

template <class T>
int ensure_dev(T*& p, size_t& cap, size_t n) {
  if (n <= cap) return SWEEP_OK;
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
  if (hipMalloc(reinterpret_cast<void**>(&p), std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SWEEP_ENOMEM, "device scratch allocation failed");
  }
  cap = n;
  return SWEEP_OK;
}

template <class T>
int ensure_host(T*& p, size_t& cap, size_t n) {
  if (n <= cap) return SWEEP_OK;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  cap = 0;
  if (hipHostMalloc(reinterpret_cast<void**>(&p), std::max<size_t>(n, 1) * sizeof(T),
                    hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SWEEP_ENOMEM, "pinned host allocation failed");
  }
  cap = n;
  return SWEEP_OK;
}

int ensure_events(Dev& d, size_t n) {
  while (d.ev.size() < n) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    d.ev.push_back(e);
  }
  return SWEEP_OK;
}

// Frees everything a Dev holds, then the Dev (its device is current).
void release_device(Dev* d) {
  if (d->rec) (void)hipFree(d->rec);
  if (d->res) (void)hipFree(d->res);
  if (d->res_h) (void)hipHostFree(d->res_h);
  if (d->partials) (void)hipFree(d->partials);
  if (d->dsum) (void)hipFree(d->dsum);
  if (d->dsum_h) (void)hipHostFree(d->dsum_h);
  if (d->clk) (void)hipFree(d->clk);
  if (d->chase_out) (void)hipFree(d->chase_out);
  if (d->walk_out) (void)hipFree(d->walk_out);
  if (d->offs) (void)hipFree(d->offs);
  if (d->offs_h) (void)hipHostFree(d->offs_h);
  for (auto e : d->ev) (void)hipEventDestroy(e);
  if (d->capture) (void)hipStreamDestroy(d->capture);
  delete d;
}

// Allocates the device's scratch and events; on failure frees what it got.
int setup_device(Dev* d) {
  // scratch for the largest default grid (32 waves per CU)
  SW_TRY(ensure_dev(d->rec, d->rec_cap, (size_t)d->num_cus * 32));
  SW_TRY(ensure_dev(d->res, d->res_cap, 64));
  SW_TRY(ensure_host(d->res_h, d->res_h_cap, 64));
  size_t one = 0, one_h = 0, clk_cap = 0;
  SW_TRY(ensure_dev(d->dsum, one, 1));
  SW_TRY(ensure_host(d->dsum_h, one_h, 1));
  SW_TRY(ensure_dev(d->clk, clk_cap, 1));
  size_t chase_cap = 0;
  SW_TRY(ensure_dev(d->chase_out, chase_cap, 5));
  size_t walk_cap = 0;
  SW_TRY(ensure_dev(d->walk_out, walk_cap, 4 * (size_t)kMaxWalkers));
  SW_TRY(ensure_events(*d, 8));
  d->scratch_ready = true;
  return SWEEP_OK;
}

// The device's state: its properties always; its library-owned scratch and
// events too when `alloc` is set (every entry point but the allocation-free
// one).
int init_device(int ordinal, Dev** out, bool alloc = true) {
  auto it = g_devs.find(ordinal);
  if (it != g_devs.end()) {
    Dev* d = it->second;
    if (alloc && !d->scratch_ready) SW_TRY(setup_device(d));
    *out = d;
    return SWEEP_OK;
  }
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, ordinal));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SWEEP_ENODEV, std::string("library is built for gfx950, device is ") +
                                  prop.gcnArchName);
  int wc_khz = 0;
  HIP_TRY(hipDeviceGetAttribute(&wc_khz, hipDeviceAttributeWallClockRate, ordinal));
  Dev* d = new Dev();
  d->ordinal = ordinal;
  std::strncpy(d->arch, prop.gcnArchName, sizeof(d->arch) - 1);
  d->num_cus = (uint32_t)prop.multiProcessorCount;
  d->lds_per_cu = (uint32_t)prop.maxSharedMemoryPerMultiProcessor;
  d->lds_per_wg_max = (uint32_t)prop.sharedMemPerBlock;
  d->l2 = (uint32_t)prop.l2CacheSize;
  d->hbm = (uint64_t)prop.totalGlobalMem;
  d->clock_khz = prop.clockRate;
  d->mem_khz = prop.memoryClockRate;
  d->bus_bits = prop.memoryBusWidth;
  d->nominal_hz = wc_khz > 0 ? wc_khz * 1000.0 : 1.0e8;
  const int rc = alloc ? setup_device(d) : SWEEP_OK;
  if (rc != SWEEP_OK) {
    release_device(d);
    return rc;
  }
  g_devs[ordinal] = d;
  *out = d;
  return SWEEP_OK;
}

int current_dev(Dev** out, bool alloc = true) {
  int ord = 0;
  HIP_TRY(hipGetDevice(&ord));
  return init_device(ord, out, alloc);
}

// ----------------------------------------------------------- cell prep
struct Prepared {
  sweep_cell_t c{};
  Plan plan{};
  const void* fn = nullptr;
  uint32_t grid = 0, threads = 0;
  size_t lds = 0;
  int max_wgs = 0;
  hipFuncAttributes fa{};
};

// Plans and checks a cell.  With `cache` the kernel's attributes and
// residency limit are kept per device; without, they are queried afresh
// (the allocation-free entry point keeps no state of its own).
int prepare(Dev& d, const sweep_cell_t& c, int pin, Prepared* out, bool cache = true) {
  PlanIn in;
  in.bytes = c.bytes;
  in.K = c.K;
  in.V = c.vec_width;
  in.kind = c.kind;
  in.waves_per_cu = c.waves_per_cu;
  in.L = c.total_logical_loads;
  in.mode = c.mode;
  in.fixed_iters = c.fixed_iters;
  in.num_cus = d.num_cus;
  in.grid_wgs = c.grid_wgs;
  in.lds_per_cu = d.lds_per_cu;
  in.lds_per_wg_max = d.lds_per_wg_max;
  in.order = c.order;
  Prepared p;
  p.c = c;
  std::string err;
  int rc = plan_cell(in, &p.plan, &err);
  if (rc != SWEEP_OK) return fail(rc, err);
  if (c.buf == nullptr) return fail(SWEEP_EINVAL, "buffer pointer is NULL");
  if (reinterpret_cast<uintptr_t>(c.buf) % 16)
    return fail(SWEEP_EALIGN, "buffer must be 16-byte aligned");
  if (c.cache_policy < 0 || c.cache_policy > 3)
    return fail(SWEEP_EINVAL, "unknown cache policy");
  p.fn = c.kind == SWEEP_KIND_PLAIN ? plain_kernel(c.K, c.vec_width, c.cache_policy)
                                    : lds_kernel(c.kind, c.K, c.cache_policy);
  if (!p.fn) return fail(SWEEP_EINVAL, "no kernel for this cell");
  p.grid = p.plan.pub.grid_wgs;
  p.threads = p.plan.pub.wg_threads;
  if (c.kind == SWEEP_KIND_PLAIN && p.threads != (uint32_t)kPlainWgThreads)
    return fail(SWEEP_EINVAL, "plain cells run 256-thread workgroups");
  p.lds = p.plan.lds_ring_bytes;
  if (pin && p.plan.pub.lds_pad_bytes > p.lds) p.lds = p.plan.pub.lds_pad_bytes;
  Dev::Occ o;
  const auto key = std::make_tuple(p.fn, p.threads, p.lds);
  auto it = d.occ.find(key);
  if (it != d.occ.end()) {
    o = it->second;
  } else {
    HIP_TRY(hipFuncGetAttributes(&o.fa, p.fn));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o.max_wgs, p.fn, (int)p.threads,
                                                         p.lds));
    if (cache) d.occ.emplace(key, o);
  }
  p.fa = o.fa;
  const int nb = o.max_wgs;
  p.max_wgs = nb;
  if ((uint32_t)nb < p.plan.wgs_per_cu)
    return fail(SWEEP_EOCCUPANCY,
                "kernel resources allow " + std::to_string(nb) +
                    " workgroups per CU, the cell needs " +
                    std::to_string(p.plan.wgs_per_cu) + " (VGPRs " +
                    std::to_string(p.fa.numRegs) + ", LDS " + std::to_string(p.lds) + ")");
  *out = p;
  return SWEEP_OK;
}

// Launches kernel `fn` whose one parameter is the struct `a`.  With events,
// hipExtLaunchKernel stamps them from the kernel's own dispatch (its start
// and its end), with no marker packets between kernels; without (as under
// graph capture), a plain launch.
template <class Args>
hipError_t launch_timed(const void* fn, uint32_t grid, uint32_t threads, size_t lds,
                        hipStream_t st, const Args& a, hipEvent_t e0, hipEvent_t e1) {
  void* args[] = {const_cast<Args*>(&a)};
  if (e0 || e1)
    return hipExtLaunchKernel(fn, dim3(grid), dim3(threads), args, lds, st, e0, e1, 0);
  return hipLaunchKernel(fn, dim3(grid), dim3(threads), args, lds, st);
}

// Launches the cell's kernel; the wave records go to `rec`, which holds at
// least the cell's waves.
hipError_t enqueue(const Prepared& p, hipStream_t st, sweep_wave_rec_t* rec,
                   uint32_t* lane_out, hipEvent_t e0, hipEvent_t e1) {
  if (p.c.kind == SWEEP_KIND_PLAIN) {
    const PlainArgs a{static_cast<const uint8_t*>(p.c.buf), p.plan.pub.n_vec, p.plan.pub.Q,
                      p.plan.stride, rec, lane_out, p.plan.G, (uint32_t)p.c.order,
                      p.plan.gstep, p.plan.jstep};
    return launch_timed(p.fn, p.grid, p.threads, p.lds, st, a, e0, e1);
  }
  const LdsArgs a{static_cast<const uint8_t*>(p.c.buf), p.plan.pub.n_vec, p.plan.pub.Q,
                  p.plan.stride, rec, lane_out, p.plan.wg_waves};
  return launch_timed(p.fn, p.grid, p.threads, p.lds, st, a, e0, e1);
}

// Copies the record offsets of `n` cells (n + 1 entries) to the device.
int upload_offsets(Dev& d, const std::vector<uint64_t>& offs, hipStream_t st) {
  SW_TRY(ensure_host(d.offs_h, d.offs_h_cap, offs.size()));
  SW_TRY(ensure_dev(d.offs, d.offs_cap, offs.size()));
  std::copy(offs.begin(), offs.end(), d.offs_h);
  HIP_TRY(hipMemcpyAsync(d.offs, d.offs_h, offs.size() * sizeof(uint64_t),
                         hipMemcpyHostToDevice, st));
  return SWEEP_OK;
}

std::vector<uint64_t> record_offsets(const std::vector<Prepared>& ps) {
  std::vector<uint64_t> o(ps.size() + 1, 0);
  for (size_t i = 0; i < ps.size(); ++i) o[i + 1] = o[i] + ps[i].plan.pub.waves;
  return o;
}

void fill_result(const Dev& d, const Prepared& p, const CellRes& r, double ms,
                 sweep_result_t* o) {
  sweep_result_t x;
  std::memset(&x, 0, sizeof(x));
  x.target_loads = p.c.total_logical_loads;
  x.issued_loads = p.plan.pub.issued_loads;
  x.issued_bytes = p.plan.pub.issued_bytes;
  x.mismatch = p.plan.pub.mismatch;
  x.sum32 = (uint32_t)r.sum;
  x.xor32 = (uint32_t)r.xr;
  x.grid_wgs = p.grid;
  x.wg_threads = p.threads;
  x.waves = p.plan.pub.waves;
  x.iters_min = p.plan.pub.iters_min;
  x.iters_max = p.plan.pub.iters_max;
  x.max_wgs_per_cu = (uint32_t)p.max_wgs;
  x.vgprs = (uint32_t)p.fa.numRegs;
  x.sgprs = 0;
  x.lds_bytes = (uint32_t)(p.lds + p.fa.sharedSizeBytes);
  x.scratch_bytes = (uint32_t)p.fa.localSizeBytes;
  x.window_ticks = r.tmax >= r.tmin ? r.tmax - r.tmin : 0;
  x.window_ns = (double)x.window_ticks / d.hz() * 1e9;
  x.event_ms = ms;
  x.gbps = x.window_ns > 0 ? (double)x.issued_bytes / x.window_ns : 0.0;
  *o = x;
}

hipStream_t as_stream(const sweep_opts_t* o) {
  return o ? static_cast<hipStream_t>(o->stream) : nullptr;
}

sweep_cell_t cell_from(int kind, const void* buf, size_t bytes, int K, int V,
                       int waves, uint64_t L, const sweep_opts_t* o) {
  sweep_cell_t c;
  std::memset(&c, 0, sizeof(c));
  c.kind = kind;
  c.K = K;
  c.vec_width = V;
  c.waves_per_cu = waves;
  c.cache_policy = o ? o->cache_policy : SWEEP_CACHE_DEFAULT;
  c.mode = o ? o->mode : SWEEP_FIXED_WORK;
  c.fixed_iters = o ? o->fixed_iters : 0;
  c.grid_wgs = o ? o->grid_wgs : 0;
  c.buf = buf;
  c.bytes = bytes;
  c.total_logical_loads = L;
  c.order = o ? o->order : SWEEP_ORDER_ROUND_ROBIN;
  return c;
}

int pin_of(const sweep_opts_t* o) { return o ? o->pin_occupancy : 1; }

// The caller's per-wave and per-lane output buffers must hold a launch of
// `waves` waves; checked before anything is enqueued.
int check_outputs(const sweep_opts_t* o, uint64_t waves) {
  if (!o) return SWEEP_OK;
  if (o->wave_out && o->wave_out_cap < waves)
    return fail(SWEEP_EINVAL, "wave_out holds " + std::to_string(o->wave_out_cap) +
                                  " records, the launch has " + std::to_string(waves) + " waves");
  if (o->lane_out && o->lane_out_cap < waves * 64ull)
    return fail(SWEEP_EINVAL, "lane_out holds " + std::to_string(o->lane_out_cap) +
                                  " lanes, the launch has " + std::to_string(waves * 64ull));
  return SWEEP_OK;
}

// Runs prepared cells back to back, each writing its own record region,
// then one finishing kernel for all cells; one synchronisation at the end.
int run_prepared(Dev& d, std::vector<Prepared>& ps, hipStream_t st,
                 sweep_wave_rec_t* wave_out, uint32_t* lane_out,
                 sweep_result_t* results) {
  const size_t n = ps.size();
  const std::vector<uint64_t> offs = record_offsets(ps);
  if (!wave_out) SW_TRY(ensure_dev(d.rec, d.rec_cap, offs[n]));
  SW_TRY(ensure_dev(d.res, d.res_cap, n));
  SW_TRY(ensure_host(d.res_h, d.res_h_cap, n));
  SW_TRY(ensure_events(d, 2 * n + 1));
  sweep_wave_rec_t* rec = wave_out ? wave_out : d.rec;
  if (wave_out && n != 1) return fail(SWEEP_EINVAL, "wave_out takes a single cell");
  SW_TRY(upload_offsets(d, offs, st));
  for (size_t i = 0; i < n; ++i)
    HIP_TRY(enqueue(ps[i], st, rec + offs[i], lane_out, d.ev[2 * i], d.ev[2 * i + 1]));
  HIP_TRY(launch_finish_cells(rec, d.offs, (uint32_t)n, d.res, st));
  HIP_TRY(hipMemcpyAsync(d.res_h, d.res, n * sizeof(CellRes), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(d.ev[2 * n], st));
  HIP_TRY(hipEventSynchronize(d.ev[2 * n]));
  for (size_t i = 0; i < n; ++i) {
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, d.ev[2 * i], d.ev[2 * i + 1]));
    fill_result(d, ps[i], d.res_h[i], ms, &results[i]);
  }
  return SWEEP_OK;
}

// The XCD reads share the launch shape of the full-grid plain cell at
// K = kXcdK and 16-byte vectors: validated like it (size, occupancy, LDS
// padding that pins residency), with their own kernel's resources.
int xcd_prepare(Dev& d, const void* buf, size_t bytes, int waves_per_cu,
                const sweep_opts_t* opt, const void* fn, Prepared* out) {
  if (!buf) return fail(SWEEP_EINVAL, "buffer pointer is NULL");
  if (reinterpret_cast<uintptr_t>(buf) % 16)
    return fail(SWEEP_EALIGN, "buffer must be 16-byte aligned");
  PlanIn in;
  in.bytes = bytes;
  in.K = kXcdK;
  in.V = 16;
  in.kind = SWEEP_KIND_PLAIN;
  in.waves_per_cu = waves_per_cu;
  in.L = bytes / 16;
  in.mode = SWEEP_FIXED_WORK;
  in.num_cus = d.num_cus;
  in.lds_per_cu = d.lds_per_cu;
  in.lds_per_wg_max = d.lds_per_wg_max;
  in.order = SWEEP_ORDER_ROUND_ROBIN;
  Prepared p;
  std::string err;
  int rc = plan_cell(in, &p.plan, &err);
  if (rc != SWEEP_OK) return fail(rc, err);
  p.grid = p.plan.pub.grid_wgs;
  if (p.grid % 8) return fail(SWEEP_EINVAL, "the grid is not a whole number of workgroups per XCD");
  p.lds = pin_of(opt) ? p.plan.pub.lds_pad_bytes : 0;
  p.fn = fn;
  p.threads = kPlainWgThreads;
  HIP_TRY(hipFuncGetAttributes(&p.fa, fn));
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&p.max_wgs, fn, kPlainWgThreads, p.lds));
  if ((uint32_t)p.max_wgs < p.plan.wgs_per_cu)
    return fail(SWEEP_EOCCUPANCY, "kernel resources allow " + std::to_string(p.max_wgs) +
                                      " workgroups per CU, the launch needs " +
                                      std::to_string(p.plan.wgs_per_cu));
  p.c = cell_from(SWEEP_KIND_PLAIN, buf, bytes, kXcdK, 16, waves_per_cu, 0, opt);
  *out = p;
  return SWEEP_OK;
}

// Records what an XCD read issues: `groups` groups of kXcdK segments over
// n_act active waves, each handling it_min..it_max of them.
void xcd_account(Prepared* p, uint64_t n_act, uint64_t groups, uint32_t it_min,
                 uint32_t it_max) {
  const uint64_t issued = groups * kXcdK * 64;
  p->c.total_logical_loads = issued;
  p->plan.pub.waves = (uint32_t)n_act;
  p->plan.pub.issued_loads = issued;
  p->plan.pub.issued_bytes = issued * 16;
  p->plan.pub.mismatch = 0.0;
  p->plan.pub.iters_min = it_min;
  p->plan.pub.iters_max = it_max;
}

// One XCD read: records (the caller's or the library's, cleared first),
// the launch with dispatch-stamped events, the finishing kernel, one
// synchronisation, then a check that active wave i wrote its record from
// XCD want[i]: if the dispatcher did not put one workgroup of each round of
// eight on every XCD, the dense numbering does not hold, groups were read
// twice or not at all, and the call fails instead of reporting a rate.
template <class Args>
int xcd_run(Dev& d, const sweep_opts_t* opt, Prepared& p, uint64_t n_act, Args& a,
            const std::vector<uint8_t>& want, sweep_result_t* out) {
  SW_TRY(check_outputs(opt, n_act));
  sweep_wave_rec_t* wave_out = opt ? opt->wave_out : nullptr;
  if (!wave_out) SW_TRY(ensure_dev(d.rec, d.rec_cap, n_act));
  a.rec = wave_out ? wave_out : d.rec;
  SW_TRY(ensure_dev(d.res, d.res_cap, 1));
  SW_TRY(ensure_host(d.res_h, d.res_h_cap, 1));
  SW_TRY(ensure_events(d, 3));
  hipStream_t st = as_stream(opt);
  SW_TRY(upload_offsets(d, std::vector<uint64_t>{0, n_act}, st));
  HIP_TRY(launch_clear_records(a.rec, n_act, st));
  HIP_TRY(launch_timed(p.fn, p.grid, p.threads, p.lds, st, a, d.ev[0], d.ev[1]));
  HIP_TRY(launch_finish_cells(a.rec, d.offs, 1, d.res, st));
  HIP_TRY(hipMemcpyAsync(d.res_h, d.res, sizeof(CellRes), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(d.ev[2], st));
  HIP_TRY(hipEventSynchronize(d.ev[2]));
  std::vector<sweep_wave_rec_t> h(n_act);
  HIP_TRY(hipMemcpy(h.data(), a.rec, n_act * sizeof(sweep_wave_rec_t), hipMemcpyDeviceToHost));
  for (uint64_t i = 0; i < n_act; ++i)
    if (h[i].t0 == 0 || (h[i].xcc_id & 0xFu) != want[i])
      return fail(SWEEP_ENODEV, "active wave " + std::to_string(i) +
                                    (h[i].t0 == 0 ? " wrote no record"
                                                  : " ran on XCD " + std::to_string(h[i].xcc_id & 0xFu) +
                                                        ", not " + std::to_string(want[i])) +
                                    ": workgroups were not dealt one per XCD per round of eight");
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, d.ev[0], d.ev[1]));
  fill_result(d, p, d.res_h[0], ms, out);
  return SWEEP_OK;
}

int single_cell(const sweep_cell_t& c, const sweep_opts_t* opt, sweep_result_t* out) {
  if (!out) return fail(SWEEP_EINVAL, "result pointer is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  std::vector<Prepared> ps(1);
  SW_TRY(prepare(*d, c, pin_of(opt), &ps[0]));
  SW_TRY(check_outputs(opt, ps[0].plan.pub.waves));
  sweep_result_t r;
  SW_TRY(run_prepared(*d, ps, as_stream(opt), opt ? opt->wave_out : nullptr,
                      opt ? opt->lane_out : nullptr, &r));
  *out = r;
  return SWEEP_OK;
}

// Both two-stream placements.  Same workgroup: every workgroup holds
// waves_plain waves of stream A and waves_async of stream B.  Split: half of
// the workgroups hold waves_plain waves of A, the other half waves_async of
// B, in workgroups of the larger count.
int two_stream_impl(const void* buf, size_t bytes, int depth, int waves_plain,
                    int waves_async, int kind_b, uint64_t total_logical_loads,
                    bool split, const sweep_opts_t* opt, sweep_result_t out[2]) {
  if (!out) return fail(SWEEP_EINVAL, "result pointer is NULL");
  if (kind_b != SWEEP_KIND_PLAIN && kind_b != SWEEP_KIND_LDS_ASYNC)
    return fail(SWEEP_EINVAL, "stream B runs plain loads or the LDS-direct ring");
  const bool b_plain = kind_b == SWEEP_KIND_PLAIN;
  if (!buf) return fail(SWEEP_EINVAL, "buffer pointer is NULL");
  if (depth < 1 || depth > 16) return fail(SWEEP_EINVAL, "depth must be in 1..16");
  const int max_w = split ? 16 : 8;
  if (waves_plain < 0 || waves_plain > max_w || waves_async < 0 || waves_async > max_w ||
      waves_plain + waves_async == 0)
    return fail(SWEEP_EINVAL, split ? "stream waves must be in 0..16, not both 0"
                                    : "waves_plain and waves_async must be in 0..8, not both 0");
  if (bytes == 0) return fail(SWEEP_EINVAL, "empty buffer");
  if (bytes % 2048 || reinterpret_cast<uintptr_t>(buf) % 16)
    return fail(SWEEP_EALIGN, "two-stream needs a 16-byte aligned buffer, bytes % 2048 == 0");
  if (total_logical_loads == 0) return fail(SWEEP_EINVAL, "total_logical_loads is 0");
  if (total_logical_loads > UINT64_MAX / 16)
    return fail(SWEEP_EINVAL, "issued bytes do not fit 64 bits");
  const int pol = opt ? opt->cache_policy : SWEEP_CACHE_DEFAULT;
  if (pol < 0 || pol > 3) return fail(SWEEP_EINVAL, "unknown cache policy");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  const uint32_t grid = (opt && opt->grid_wgs) ? opt->grid_wgs : d->num_cus;
  if (split && grid % 16)
    return fail(SWEEP_EINVAL, "the split placement needs a grid that is a multiple of 16");
  // workgroups per stream
  const uint32_t wg_a = split ? grid / 2 : grid, wg_b = wg_a;
  const uint64_t n_vec = bytes / 16, half = n_vec / 2;
  const uint64_t La = total_logical_loads / 2, Lb = total_logical_loads - La;
  TwoStreamArgs a;
  std::memset(&a, 0, sizeof(a));
  a.buf_a = static_cast<const uint8_t*>(buf);
  a.n_vec_a = half;
  a.buf_b = static_cast<const uint8_t*>(buf) + half * 16;
  a.n_vec_b = n_vec - half;
  a.waves_a = (uint32_t)waves_plain;
  a.waves_b = (uint32_t)waves_async;
  a.b_plain = b_plain ? 1u : 0u;
  a.split = split ? 1u : 0u;
  if (waves_plain) region_plan(a.n_vec_a, depth, La, wg_a * a.waves_a, &a.Q_a, &a.stride_a);
  if (waves_async) region_plan(a.n_vec_b, depth, Lb, wg_b * a.waves_b, &a.Q_b, &a.stride_b);
  if ((waves_plain && a.Q_a == 0) || (waves_async && a.Q_b == 0))
    return fail(SWEEP_EINVAL, "L is smaller than one wave-group per stream");
  // per-wave iteration counts are reported in 32 bits
  const uint64_t nwa = (uint64_t)wg_a * a.waves_a, nwb = (uint64_t)wg_b * a.waves_b;
  if ((nwa && (a.Q_a + nwa - 1) / nwa > UINT32_MAX) ||
      (nwb && (a.Q_b + nwb - 1) / nwb > UINT32_MAX))
    return fail(SWEEP_EINVAL, "a wave would run more than 2^32 - 1 iterations");
  const uint32_t threads =
      (uint32_t)(split ? std::max(waves_plain, waves_async) : waves_plain + waves_async) * 64u;
  const uint32_t ring = b_plain ? 0u : (uint32_t)waves_async * (uint32_t)depth * 1024u;
  if (ring > d->lds_per_wg_max) return fail(SWEEP_EOCCUPANCY, "LDS ring exceeds the per-workgroup LDS");
  size_t lds = ring;
  if (pin_of(opt)) lds = std::max<size_t>(lds, pin_padding(1, ring, d->lds_per_cu, d->lds_per_wg_max));
  const void* fn = two_stream_kernel(depth, pol);
  if (!fn) return fail(SWEEP_EINVAL, "no two-stream kernel for this depth and policy");
  hipFuncAttributes fa;
  HIP_TRY(hipFuncGetAttributes(&fa, fn));
  int nb = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)threads, lds));
  if (nb < 1) return fail(SWEEP_EOCCUPANCY, "two-stream workgroup does not fit a CU");
  const uint32_t wa = wg_a * a.waves_a, wb = wg_b * a.waves_b;
  SW_TRY(check_outputs(opt, (uint64_t)wa + wb));
  SW_TRY(ensure_dev(d->rec, d->rec_cap, (size_t)wa + wb));
  SW_TRY(ensure_events(*d, 3));
  sweep_wave_rec_t* rec = (opt && opt->wave_out) ? opt->wave_out : d->rec;
  a.rec = rec;
  a.lane_out = opt ? opt->lane_out : nullptr;
  hipStream_t st = as_stream(opt);
  SW_TRY(upload_offsets(*d, {0ull, (uint64_t)wa, (uint64_t)wa + wb}, st));
  HIP_TRY(launch_timed(fn, grid, threads, lds, st, a, d->ev[0], d->ev[1]));
  HIP_TRY(launch_finish_cells(rec, d->offs, 2, d->res, st));
  HIP_TRY(hipMemcpyAsync(d->res_h, d->res, 2 * sizeof(CellRes), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(d->ev[2], st));
  HIP_TRY(hipEventSynchronize(d->ev[2]));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, d->ev[0], d->ev[1]));
  for (int s = 0; s < 2; ++s) {
    const bool on = s == 0 ? waves_plain > 0 : waves_async > 0;
    Prepared p;
    p.c = cell_from(s == 0 ? SWEEP_KIND_PLAIN : kind_b, buf, bytes,
                    depth, 16, s == 0 ? waves_plain : waves_async,
                    s == 0 ? La : Lb, opt);
    p.grid = grid;
    p.threads = threads;
    p.lds = lds;
    p.max_wgs = nb;
    p.fa = fa;
    const uint64_t Q = s == 0 ? a.Q_a : a.Q_b;
    const uint32_t nw = s == 0 ? wa : wb;
    p.plan.pub.grid_wgs = grid;
    p.plan.pub.wg_threads = threads;
    p.plan.pub.waves = nw;
    p.plan.pub.n_vec = s == 0 ? a.n_vec_a : a.n_vec_b;
    p.plan.pub.Q = Q;
    p.plan.pub.issued_loads = 64ull * (uint64_t)depth * Q;
    p.plan.pub.issued_bytes = p.plan.pub.issued_loads * 16ull;
    p.plan.pub.iters_min = nw ? (uint32_t)(Q / nw) : 0;
    p.plan.pub.iters_max = nw ? (uint32_t)((Q + nw - 1) / nw) : 0;
    const uint64_t Ls = s == 0 ? La : Lb;
    p.plan.pub.mismatch = Ls ? (double)(Ls - p.plan.pub.issued_loads) / (double)Ls : 0.0;
    if (on) {
      fill_result(*d, p, d->res_h[s], ms, &out[s]);
    } else {
      std::memset(&out[s], 0, sizeof(out[s]));
    }
  }
  return SWEEP_OK;
}

}  // namespace

extern "C" {

int sweep_init(int ordinal) {
  std::lock_guard<std::mutex> lk(g_mu);
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (ordinal < 0 || ordinal >= n) return fail(SWEEP_ENODEV, "no such device");
  HIP_TRY(hipSetDevice(ordinal));
  Dev* d = nullptr;
  SW_TRY(init_device(ordinal, &d));
  // the allocation-free entry point's static scratch on this device
  uint8_t* sp = nullptr;
  HIP_TRY(static_scratch(ordinal, &sp));
  return SWEEP_OK;
}

int sweep_shutdown(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : g_devs) {
    Dev* d = kv.second;
    (void)hipSetDevice(d->ordinal);
    (void)hipDeviceSynchronize();
    release_device(d);
  }
  g_devs.clear();
  (void)hipSetDevice(cur);
  return SWEEP_OK;
}

int sweep_device_info(sweep_device_t* out) {
  if (!out) return fail(SWEEP_EINVAL, "NULL output");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  sweep_device_t o;
  std::memset(&o, 0, sizeof(o));
  o.ordinal = d->ordinal;
  std::strncpy(o.arch, d->arch, sizeof(o.arch) - 1);
  o.num_cus = d->num_cus;
  o.lds_per_cu = d->lds_per_cu;
  o.lds_per_wg_max = d->lds_per_wg_max;
  o.l2_bytes = d->l2;
  o.hbm_bytes = d->hbm;
  o.wall_clock_hz = d->nominal_hz;
  o.calibrated_hz = d->cal_hz;
  o.clock_khz = d->clock_khz;
  o.mem_clock_khz = d->mem_khz;
  o.mem_bus_bits = d->bus_bits;
  *out = o;
  return SWEEP_OK;
}

int sweep_calibrate_clock(double seconds, double* hz) {
  if (!hz || !(seconds >= 0.01) || seconds > 60) return fail(SWEEP_EINVAL, "seconds must be in [0.01, 60]");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  using clk = std::chrono::steady_clock;
  auto sample = [&](uint64_t* ticks, double* ns) -> int {
    double best_span = 1e300;
    for (int rep = 0; rep < 5; ++rep) {
      const auto a = clk::now();
      HIP_TRY(launch_read_clock(d->clk, nullptr));
      HIP_TRY(hipStreamSynchronize(nullptr));
      const auto b = clk::now();
      uint64_t t = 0;
      HIP_TRY(hipMemcpy(&t, d->clk, sizeof(t), hipMemcpyDeviceToHost));
      const double span = std::chrono::duration<double, std::nano>(b - a).count();
      if (span < best_span) {
        best_span = span;
        *ticks = t;
        *ns = std::chrono::duration<double, std::nano>(a.time_since_epoch()).count() + span / 2;
      }
    }
    return SWEEP_OK;
  };
  uint64_t t1 = 0, t2 = 0;
  double n1 = 0, n2 = 0;
  SW_TRY(sample(&t1, &n1));
  std::this_thread::sleep_for(std::chrono::duration<double>(seconds));
  SW_TRY(sample(&t2, &n2));
  if (t2 <= t1 || n2 <= n1) return fail(SWEEP_EHIP, "device clock did not advance");
  d->cal_hz = (double)(t2 - t1) / ((n2 - n1) * 1e-9);
  *hz = d->cal_hz;
  return SWEEP_OK;
}

int sweep_plan(size_t bytes, int K, int vec_width, int waves_per_cu,
               uint64_t total_logical_loads, int mode, uint32_t fixed_iters,
               uint32_t num_cus, uint32_t grid_wgs, int order,
               sweep_plan_t* out) {
  if (!out) return fail(SWEEP_EINVAL, "NULL output");
  PlanIn in;
  in.bytes = bytes;
  in.K = K;
  in.V = vec_width;
  in.kind = SWEEP_KIND_PLAIN;
  in.waves_per_cu = waves_per_cu;
  in.L = total_logical_loads;
  in.mode = mode;
  in.fixed_iters = fixed_iters;
  in.num_cus = num_cus;
  in.grid_wgs = grid_wgs;
  in.order = order;
  Plan p;
  std::string err;
  int rc = plan_cell(in, &p, &err);
  if (rc != SWEEP_OK) return fail(rc, err);
  *out = p.pub;
  return SWEEP_OK;
}

int sweep_fill_u32(void* buf, size_t bytes, uint64_t seed, void* stream) {
  if (!buf) return fail(SWEEP_EINVAL, "buffer pointer is NULL");
  if (bytes == 0) return fail(SWEEP_EINVAL, "empty buffer");
  if (bytes % 4 || reinterpret_cast<uintptr_t>(buf) % 16)
    return fail(SWEEP_EALIGN, "fill needs a 16-byte aligned buffer of whole words");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  HIP_TRY(launch_fill(static_cast<uint32_t*>(buf), bytes / 4, seed,
                      static_cast<hipStream_t>(stream)));
  return SWEEP_OK;
}

int sweep_plain(const void* buf, size_t bytes, int K, int vec_width,
                int waves_per_cu, uint64_t total_logical_loads,
                const sweep_opts_t* opt, sweep_result_t* out) {
  return single_cell(cell_from(SWEEP_KIND_PLAIN, buf, bytes, K, vec_width,
                               waves_per_cu, total_logical_loads, opt),
                     opt, out);
}

int sweep_lds_async(const void* buf, size_t bytes, int depth, int vec_width,
                    int waves_per_cu, uint64_t total_logical_loads,
                    const sweep_opts_t* opt, sweep_result_t* out) {
  return single_cell(cell_from(SWEEP_KIND_LDS_ASYNC, buf, bytes, depth,
                               vec_width, waves_per_cu, total_logical_loads, opt),
                     opt, out);
}

int sweep_lds_matched_plain(const void* buf, size_t bytes, int depth,
                            int vec_width, int waves_per_cu,
                            uint64_t total_logical_loads,
                            const sweep_opts_t* opt, sweep_result_t* out) {
  return single_cell(cell_from(SWEEP_KIND_LDS_MATCHED, buf, bytes, depth,
                               vec_width, waves_per_cu, total_logical_loads, opt),
                     opt, out);
}

int sweep_two_stream(const void* buf, size_t bytes, int depth, int waves_plain,
                     int waves_async, uint64_t total_logical_loads,
                     const sweep_opts_t* opt, sweep_result_t out[2]) {
  return sweep_two_stream_kind(buf, bytes, depth, waves_plain, waves_async,
                               SWEEP_KIND_LDS_ASYNC, total_logical_loads, opt, out);
}

int sweep_two_stream_kind(const void* buf, size_t bytes, int depth, int waves_plain,
                          int waves_async, int kind_b, uint64_t total_logical_loads,
                          const sweep_opts_t* opt, sweep_result_t out[2]) {
  return two_stream_impl(buf, bytes, depth, waves_plain, waves_async, kind_b,
                         total_logical_loads, false, opt, out);
}

int sweep_two_stream_split(const void* buf, size_t bytes, int depth, int waves_a,
                           int waves_b, int kind_b, uint64_t total_logical_loads,
                           const sweep_opts_t* opt, sweep_result_t out[2]) {
  return two_stream_impl(buf, bytes, depth, waves_a, waves_b, kind_b,
                         total_logical_loads, true, opt, out);
}

int sweep_run(const sweep_cell_t* cells, int n, const sweep_opts_t* opt,
              sweep_result_t* results) {
  if (!cells || !results || n <= 0) return fail(SWEEP_EINVAL, "empty cell list");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  std::vector<Prepared> ps((size_t)n);
  for (int i = 0; i < n; ++i) SW_TRY(prepare(*d, cells[i], pin_of(opt), &ps[(size_t)i]));
  return run_prepared(*d, ps, as_stream(opt), nullptr, nullptr, results);
}

int sweep_plain_noalloc(const void* buf, size_t bytes, int K, int vec_width,
                        int waves_per_cu, uint64_t total_logical_loads,
                        const sweep_opts_t* opt, sweep_result_t* out) {
  if (!out) return fail(SWEEP_EINVAL, "result pointer is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d, false));
  uint8_t* sp = nullptr;
  HIP_TRY(static_scratch(d->ordinal, &sp));
  Prepared p;
  SW_TRY(prepare(*d, cell_from(SWEEP_KIND_PLAIN, buf, bytes, K, vec_width, waves_per_cu,
                               total_logical_loads, opt),
                 pin_of(opt), &p, false));
  const uint64_t waves = p.plan.pub.waves;
  SW_TRY(check_outputs(opt, waves));
  sweep_wave_rec_t* wave_out = opt ? opt->wave_out : nullptr;
  if (!wave_out && waves > kStaticRecords)
    return fail(SWEEP_EINVAL, "the launch's waves exceed the static scratch (16384 records)");
  sweep_wave_rec_t* rec = wave_out ? wave_out : reinterpret_cast<sweep_wave_rec_t*>(sp);
  CellRes* res = reinterpret_cast<CellRes*>(sp + kStaticResOffset);
  uint64_t* offs = reinterpret_cast<uint64_t*>(sp + kStaticOffsOffset);
  hipStream_t st = as_stream(opt);
  // every value the kernels read is written first in this call: the record
  // offsets here, the records by the sweep kernel, the result by the finish
  const uint64_t offs_h[2] = {0, waves};
  CellRes r;
  HIP_TRY(hipMemcpyAsync(offs, offs_h, sizeof(offs_h), hipMemcpyHostToDevice, st));
  HIP_TRY(enqueue(p, st, rec, opt ? opt->lane_out : nullptr, nullptr, nullptr));
  HIP_TRY(launch_finish_cells(rec, offs, 1, res, st));
  HIP_TRY(hipMemcpyAsync(&r, res, sizeof(r), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  fill_result(*d, p, r, 0.0, out);
  return SWEEP_OK;
}

}  // extern "C"

// A captured sweep with its own scratch (see sweep_graph_create).
struct sweep_graph {
  int ordinal = -1;
  std::vector<Prepared> ps;
  sweep_wave_rec_t* rec = nullptr;
  CellRes* res = nullptr;
  CellRes* res_h = nullptr;
  uint64_t* offs = nullptr;
  FusedPoint* pts = nullptr;    // point lists of the fused launches
  size_t fused_launches = 0;
  std::vector<hipEvent_t> ev;   // start, end, done of a launch
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void free_graph(sweep_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (auto e : g->ev) (void)hipEventDestroy(e);
  if (g->rec) (void)hipFree(g->rec);
  if (g->res) (void)hipFree(g->res);
  if (g->offs) (void)hipFree(g->offs);
  if (g->pts) (void)hipFree(g->pts);
  if (g->res_h) (void)hipHostFree(g->res_h);
  delete g;
}

// A run of consecutive cells launched together: one cell alone, or (with
// opts->fuse) plain fixed-work round-robin cells that share the kernel and
// launch shape, fused into one persistent launch over their groups.
struct LaunchGroup {
  size_t first = 0, count = 1;
  const void* fused = nullptr;   // fused kernel, or null for a lone cell
  size_t pt0 = 0;                // index of its first point in the point list
  const uint8_t* base = nullptr; // lowest point buffer (points are offsets from it)
};

bool fusable(const Prepared& p) {
  return p.c.kind == SWEEP_KIND_PLAIN && p.c.mode == SWEEP_FIXED_WORK &&
         p.c.order == SWEEP_ORDER_ROUND_ROBIN;
}

bool same_launch(const Prepared& a, const Prepared& b) {
  return a.fn == b.fn && a.grid == b.grid && a.threads == b.threads && a.lds == b.lds;
}

// Splits the prepared cells into launch groups and builds the fused point
// lists (g0 = the point's first group in the concatenation).
int plan_groups(const std::vector<Prepared>& ps, bool fuse, std::vector<LaunchGroup>* groups,
                std::vector<FusedPoint>* pts) {
  for (size_t i = 0; i < ps.size();) {
    LaunchGroup lg;
    lg.first = i;
    size_t j = i + 1;
    if (fuse && fusable(ps[i]))
      while (j < ps.size() && fusable(ps[j]) && same_launch(ps[i], ps[j])) ++j;
    lg.count = j - i;
    if (lg.count > 1) {
      const Prepared& p0 = ps[i];
      const void* fn = fused_kernel(p0.c.K, p0.c.vec_width, p0.c.cache_policy);
      int nb = 0;
      if (fn) HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, (int)p0.threads,
                                                                   p0.lds));
      if (fn && (uint32_t)nb >= p0.plan.wgs_per_cu) {
        lg.fused = fn;
        lg.pt0 = pts->size();
        uint64_t g0 = 0;
        const uint64_t nw = p0.plan.pub.waves;
        uintptr_t base = reinterpret_cast<uintptr_t>(p0.c.buf);
        for (size_t k = i; k < j; ++k)
          base = std::min(base, reinterpret_cast<uintptr_t>(ps[k].c.buf));
        lg.base = reinterpret_cast<const uint8_t*>(base);
        for (size_t k = i; k < j; ++k) {
          const Prepared& p = ps[k];
          FusedPoint fp;
          fp.off = reinterpret_cast<uintptr_t>(p.c.buf) - base;
          fp.n_vec = p.plan.pub.n_vec;
          fp.Q = p.plan.pub.Q;
          fp.g0 = g0;
          fp.stride = (nw * (uint64_t)p.c.K * 64ull) % fp.n_vec;
          g0 += fp.Q;
          pts->push_back(fp);
        }
      } else {
        lg.count = 1;     // the fused kernel cannot reach the residency: alone
        j = i + 1;
      }
    }
    groups->push_back(lg);
    i = j;
  }
  return SWEEP_OK;
}

int create_graph(Dev& d, const sweep_cell_t* cells, int n, const sweep_opts_t* opt,
                 sweep_graph** out) {
  sweep_graph* g = new sweep_graph();
  g->ordinal = d.ordinal;
  g->ps.resize((size_t)n);
  int rc = SWEEP_OK;
  for (int i = 0; i < n && rc == SWEEP_OK; ++i)
    rc = prepare(d, cells[i], pin_of(opt), &g->ps[(size_t)i]);
  if (rc != SWEEP_OK) {
    free_graph(g);
    return rc;
  }
  const std::vector<uint64_t> offs = record_offsets(g->ps);
  auto fail_g = [&](int code, const std::string& msg) {
    free_graph(g);
    return fail(code, msg);
  };
  const size_t n_rec = std::max<uint64_t>(offs.back(), 1);
  if (hipMalloc(reinterpret_cast<void**>(&g->rec), n_rec * sizeof(sweep_wave_rec_t)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&g->res), (size_t)n * sizeof(CellRes)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&g->offs), offs.size() * sizeof(uint64_t)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&g->res_h), (size_t)n * sizeof(CellRes), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail_g(SWEEP_ENOMEM, "graph scratch allocation failed");
  }
  if (hipMemcpy(g->offs, offs.data(), offs.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess)
    return fail_g(SWEEP_EHIP, "graph offsets upload failed");
  std::vector<LaunchGroup> groups;
  std::vector<FusedPoint> pts;
  rc = plan_groups(g->ps, opt && opt->fuse, &groups, &pts);
  if (rc != SWEEP_OK) {
    free_graph(g);
    return rc;
  }
  if (!pts.empty()) {
    // fused launches write only the records of points their waves reach:
    // every other record is cleared once, here, and never written again
    if (hipMalloc(reinterpret_cast<void**>(&g->pts), pts.size() * sizeof(FusedPoint)) != hipSuccess) {
      (void)hipGetLastError();
      return fail_g(SWEEP_ENOMEM, "graph point list allocation failed");
    }
    if (hipMemcpy(g->pts, pts.data(), pts.size() * sizeof(FusedPoint), hipMemcpyHostToDevice) != hipSuccess)
      return fail_g(SWEEP_EHIP, "graph point list upload failed");
    if (launch_clear_records(g->rec, n_rec, nullptr) != hipSuccess ||
        hipStreamSynchronize(nullptr) != hipSuccess)
      return fail_g(SWEEP_EHIP, "graph record clear failed");
  }
  g->ev.resize(3, nullptr);
  for (auto& e : g->ev)
    if (hipEventCreate(&e) != hipSuccess) return fail_g(SWEEP_EHIP, "hipEventCreate failed");
  if (!d.capture && hipStreamCreateWithFlags(&d.capture, hipStreamNonBlocking) != hipSuccess)
    return fail_g(SWEEP_EHIP, "capture stream creation failed");
  if (hipStreamBeginCapture(d.capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return fail_g(SWEEP_EHIP, "hipStreamBeginCapture failed");
  hipError_t cap_err = hipSuccess;
  for (size_t k = 0; k < groups.size() && cap_err == hipSuccess; ++k) {
    const LaunchGroup& lg = groups[k];
    const Prepared& p0 = g->ps[lg.first];
    if (!lg.fused) {
      cap_err = enqueue(p0, d.capture, g->rec + offs[lg.first], nullptr, nullptr, nullptr);
      continue;
    }
    FusedArgs a;
    a.base = lg.base;
    a.pts = g->pts + lg.pt0;
    a.total_groups = pts[lg.pt0 + lg.count - 1].g0 + pts[lg.pt0 + lg.count - 1].Q;
    a.rec = g->rec + offs[lg.first];
    cap_err = launch_timed(lg.fused, p0.grid, p0.threads, p0.lds, d.capture, a, nullptr, nullptr);
    ++g->fused_launches;
  }
  if (cap_err == hipSuccess)
    cap_err = launch_finish_cells(g->rec, g->offs, (uint32_t)n, g->res, d.capture);
  hipError_t end_err = hipStreamEndCapture(d.capture, &g->graph);
  if (cap_err != hipSuccess || end_err != hipSuccess)
    return fail_g(SWEEP_EHIP, std::string("graph capture failed: ") +
                                  hipGetErrorString(cap_err != hipSuccess ? cap_err : end_err));
  hipError_t ie = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (ie != hipSuccess)
    return fail_g(SWEEP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  *out = g;
  return SWEEP_OK;
}

int launch_graph(Dev& d, sweep_graph* g, hipStream_t st, sweep_result_t* results,
                 double* graph_ms) {
  const size_t n = g->ps.size();
  hipEvent_t e_start = g->ev[0], e_end = g->ev[1], e_done = g->ev[2];
  HIP_TRY(hipEventRecord(e_start, st));
  HIP_TRY(hipGraphLaunch(g->exec, st));
  HIP_TRY(hipEventRecord(e_end, st));
  HIP_TRY(hipMemcpyAsync(g->res_h, g->res, n * sizeof(CellRes), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(e_done, st));
  HIP_TRY(hipEventSynchronize(e_done));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e_start, e_end));
  if (graph_ms) *graph_ms = ms;
  for (size_t i = 0; i < n; ++i) fill_result(d, g->ps[i], g->res_h[i], 0.0, &results[i]);
  return SWEEP_OK;
}

}  // namespace

extern "C" {

int sweep_graph_create(const sweep_cell_t* cells, int n, const sweep_opts_t* opt,
                       sweep_graph_t** out) {
  if (!cells || !out || n <= 0) return fail(SWEEP_EINVAL, "empty cell list");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  return create_graph(*d, cells, n, opt, out);
}

int sweep_graph_launch(sweep_graph_t* graph, void* stream, sweep_result_t* results,
                       double* graph_ms) {
  if (!graph || !results) return fail(SWEEP_EINVAL, "NULL graph or results");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(init_device(graph->ordinal, &d));
  return launch_graph(*d, graph, static_cast<hipStream_t>(stream), results, graph_ms);
}

int sweep_graph_destroy(sweep_graph_t* graph) {
  if (!graph) return SWEEP_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(graph->ordinal);
  free_graph(graph);
  (void)hipSetDevice(cur);
  return SWEEP_OK;
}

int sweep_batched(const sweep_cell_t* cells, int n, const sweep_opts_t* opt,
                  sweep_result_t* results, double* graph_ms) {
  if (!cells || !results || n <= 0) return fail(SWEEP_EINVAL, "empty cell list");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  sweep_graph* g = nullptr;
  SW_TRY(create_graph(*d, cells, n, opt, &g));
  const int rc = launch_graph(*d, g, as_stream(opt), results, graph_ms);
  free_graph(g);
  return rc;
}

int sweep_autotune(const void* buf, size_t bytes, const int* vec_widths,
                   int n_vec_widths, const int* Ks, int n_Ks,
                   const int* waves_per_cu, int n_waves, int cache_policy,
                   int reps, sweep_cell_t* best, double* best_gbps) {
  if (!vec_widths || !Ks || !waves_per_cu || n_vec_widths <= 0 || n_Ks <= 0 ||
      n_waves <= 0 || reps < 1 || !best || !best_gbps)
    return fail(SWEEP_EINVAL, "empty candidate set or reps < 1");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  double top = -1.0;
  sweep_cell_t top_cell;
  std::memset(&top_cell, 0, sizeof(top_cell));
  int last_err = SWEEP_OK;
  for (int vi = 0; vi < n_vec_widths; ++vi)
    for (int ki = 0; ki < n_Ks; ++ki)
      for (int wi = 0; wi < n_waves; ++wi) {
        sweep_cell_t c;
        std::memset(&c, 0, sizeof(c));
        c.kind = SWEEP_KIND_PLAIN;
        c.K = Ks[ki];
        c.vec_width = vec_widths[vi];
        c.waves_per_cu = waves_per_cu[wi];
        c.cache_policy = cache_policy;
        c.mode = SWEEP_FIXED_WORK;
        c.buf = buf;
        c.bytes = bytes;
        c.total_logical_loads = vec_widths[vi] > 0 ? bytes / (size_t)vec_widths[vi] : 0;
        Prepared p;
        int rc = prepare(*d, c, 1, &p);
        if (rc == SWEEP_EOCCUPANCY || (rc == SWEEP_EINVAL && c.total_logical_loads > 0 &&
                                       c.total_logical_loads < 64ull * (uint64_t)c.K)) {
          last_err = rc;
          continue;
        }
        if (rc != SWEEP_OK) return rc;
        std::vector<Prepared> ps((size_t)reps + 1, p);
        std::vector<sweep_result_t> rs((size_t)reps + 1);
        SW_TRY(run_prepared(*d, ps, nullptr, nullptr, nullptr, rs.data()));
        std::vector<double> g;
        for (int r = 1; r <= reps; ++r) g.push_back(rs[(size_t)r].gbps);
        std::sort(g.begin(), g.end());
        const double med = g.size() % 2 ? g[g.size() / 2]
                                        : 0.5 * (g[g.size() / 2 - 1] + g[g.size() / 2]);
        if (med > top) {
          top = med;
          top_cell = c;
        }
      }
  if (top < 0) return fail(last_err ? last_err : SWEEP_EINVAL, "no candidate could run");
  *best = top_cell;
  *best_gbps = top;
  return SWEEP_OK;
}

int sweep_reduce_fp(const void* payload, size_t n_elems, int dtype,
                    int waves_per_cu, const sweep_opts_t* opt, double* sum,
                    sweep_result_t* out) {
  if (!sum) return fail(SWEEP_EINVAL, "sum pointer is NULL");
  if (dtype != SWEEP_F32 && dtype != SWEEP_BF16 && dtype != SWEEP_FP8_E4M3)
    return fail(SWEEP_EINVAL, "unknown dtype");
  if (waves_per_cu < 4 || waves_per_cu > 32 || waves_per_cu % 4)
    return fail(SWEEP_EINVAL, "waves_per_cu must be a multiple of 4 in 4..32");
  if (n_elems && !payload) return fail(SWEEP_EINVAL, "payload pointer is NULL");
  if (reinterpret_cast<uintptr_t>(payload) % 16)
    return fail(SWEEP_EALIGN, "payload must be 16-byte aligned");
  const size_t esz = dtype == SWEEP_F32 ? 4 : dtype == SWEEP_BF16 ? 2 : 1;
  if (n_elems > SIZE_MAX / esz) return fail(SWEEP_EINVAL, "payload bytes do not fit 64 bits");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  const uint32_t grid = (opt && opt->grid_wgs) ? opt->grid_wgs
                                               : d->num_cus * (uint32_t)waves_per_cu / 4u;
  ReduceArgs a;
  a.payload = static_cast<const uint8_t*>(payload);
  a.n_bytes = (uint64_t)n_elems * esz;
  a.n_vec = a.n_bytes / 16;
  // Loads in flight per lane: 8 at one wave per SIMD, 4 above, so that at
  // least 8 MiB is in flight at every occupancy of the default grid.
  const int loads = waves_per_cu == 4 ? 8 : 4;
  a.n_groups = a.n_vec / (64u * (uint64_t)loads);
  if (a.n_vec - a.n_groups * 64u * (uint64_t)loads > (uint64_t)grid * 256)
    return fail(SWEEP_EINVAL, "grid too small for the ragged remainder");
  const void* fn = reduce_kernel(dtype, loads);
  if (!fn) return fail(SWEEP_EINVAL, "no reduction kernel for this dtype");
  hipFuncAttributes fa;
  HIP_TRY(hipFuncGetAttributes(&fa, fn));
  int nb = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, 0));
  SW_TRY(ensure_dev(d->rec, d->rec_cap, (size_t)grid * 4));
  SW_TRY(ensure_dev(d->partials, d->partials_cap, (size_t)grid * 2));
  SW_TRY(ensure_events(*d, 3));
  a.partials = d->partials;
  a.rec = d->rec;
  hipStream_t st = as_stream(opt);
  SW_TRY(upload_offsets(*d, {0ull, (uint64_t)grid * 4}, st));
  HIP_TRY(launch_timed(fn, grid, 256u, 0, st, a, d->ev[0], d->ev[1]));
  HIP_TRY(launch_reduce_finish(d->partials, grid, d->dsum, st));
  HIP_TRY(launch_finish_cells(d->rec, d->offs, 1, d->res, st));
  HIP_TRY(hipMemcpyAsync(d->dsum_h, d->dsum, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(d->res_h, d->res, sizeof(CellRes), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipEventRecord(d->ev[2], st));
  HIP_TRY(hipEventSynchronize(d->ev[2]));
  *sum = *d->dsum_h;
  if (out) {
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, d->ev[0], d->ev[1]));
    Prepared p;
    p.c.total_logical_loads = a.n_vec;
    p.grid = grid;
    p.threads = 256;
    p.max_wgs = nb;
    p.fa = fa;
    p.plan.pub.waves = grid * 4;
    p.plan.pub.issued_loads = a.n_vec;
    p.plan.pub.issued_bytes = a.n_bytes;
    CellRes r = d->res_h[0];
    r.sum = 0;
    r.xr = 0;
    fill_result(*d, p, r, ms, out);
  }
  return SWEEP_OK;
}

int sweep_chase(const void* chain, size_t bytes, uint32_t start,
                uint32_t warm_hops, uint32_t hops, int cache_policy,
                uint32_t* samples, uint32_t n_samples, void* stream,
                sweep_chase_t* out) {
  if (!out || !chain) return fail(SWEEP_EINVAL, "NULL argument");
  if (bytes == 0 || bytes >= (1ull << 32)) return fail(SWEEP_EINVAL, "chain must be below 4 GiB");
  if (bytes % 4 || reinterpret_cast<uintptr_t>(chain) % 16)
    return fail(SWEEP_EALIGN, "chain must be 16-byte aligned and whole words");
  if (start >= bytes / 4) return fail(SWEEP_EINVAL, "start index outside the chain");
  if (cache_policy < 0 || cache_policy > 3) return fail(SWEEP_EINVAL, "unknown cache policy");
  if (hops == 0) return fail(SWEEP_EINVAL, "no timed hops");
  if (n_samples > kMaxChaseSamples || n_samples > hops || (n_samples && !samples))
    return fail(SWEEP_EINVAL, "n_samples must be <= 4096 and <= hops, with a buffer");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  uint64_t* dout = d->chase_out;
  ChaseArgs a{static_cast<const uint32_t*>(chain), (uint32_t)bytes, start, warm_hops,
              hops, n_samples, samples, dout};
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t h[5] = {0, 0, 0, 0, 0};
  hipError_t e = launch_chase(cache_policy, st, a);
  if (e == hipSuccess) e = hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(SWEEP_EHIP, std::string("chase: ") + hipGetErrorString(e));
  sweep_chase_t o;
  std::memset(&o, 0, sizeof(o));
  o.final_index = (uint32_t)h[0];
  o.hops = hops;
  o.wall_ticks = h[2] - h[1];
  const double secs = (double)o.wall_ticks / d->hz();
  o.ns_per_hop = secs * 1e9 / hops;
  o.shader_clock_hz = secs > 0 ? (double)(h[4] - h[3]) / secs : 0.0;
  *out = o;
  return SWEEP_OK;
}

int sweep_xcd_subset(const void* buf, size_t bytes, int waves_per_cu, uint32_t xcd_mask,
                     const sweep_opts_t* opt, sweep_result_t* out) {
  if (!out) return fail(SWEEP_EINVAL, "result pointer is NULL");
  if (xcd_mask == 0 || xcd_mask > 0xFFu) return fail(SWEEP_EINVAL, "xcd_mask must be 1..255");
  const void* fn = xcd_kernel(opt ? opt->cache_policy : SWEEP_CACHE_DEFAULT);
  if (!fn) return fail(SWEEP_EINVAL, "unknown cache policy");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  Prepared p;
  SW_TRY(xcd_prepare(*d, buf, bytes, waves_per_cu, opt, fn, &p));
  const uint32_t pop = (uint32_t)__builtin_popcount(xcd_mask);
  const uint64_t n_act = (uint64_t)(p.grid / 8) * pop * (kPlainWgThreads / 64);
  const uint64_t groups = (bytes / 16) / (n_act * kXcdK * 64);
  if (groups == 0) return fail(SWEEP_EINVAL, "buffer smaller than one group per active wave");
  xcd_account(&p, n_act, n_act * groups, (uint32_t)groups, (uint32_t)groups);
  XcdArgs a{static_cast<const uint8_t*>(buf), groups, n_act, xcd_mask, pop, nullptr};
  // active wave w belongs to workgroup w / 4, the (w / 4) mod pop-th active
  // XCD of its round
  std::vector<uint8_t> bits, want(n_act);
  for (uint8_t x = 0; x < 8; ++x)
    if ((xcd_mask >> x) & 1u) bits.push_back(x);
  for (uint64_t w = 0; w < n_act; ++w) want[w] = bits[(w / 4) % pop];
  return xcd_run(*d, opt, p, n_act, a, want, out);
}

int sweep_xcd_split(const void* buf, size_t bytes, int waves_per_cu, const double* weights,
                    const sweep_opts_t* opt, sweep_result_t* out) {
  if (!out || !weights) return fail(SWEEP_EINVAL, "NULL argument");
  double sum = 0;
  for (int x = 0; x < 8; ++x) {
    if (!(weights[x] >= 0.0) || weights[x] > 1e300)
      return fail(SWEEP_EINVAL, "weights must be finite and non-negative");
    sum += weights[x];
  }
  if (!(sum > 0.0)) return fail(SWEEP_EINVAL, "no XCD has a weight");
  const void* fn = xcd_split_kernel(opt ? opt->cache_policy : SWEEP_CACHE_DEFAULT);
  if (!fn) return fail(SWEEP_EINVAL, "unknown cache policy");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  Prepared p;
  SW_TRY(xcd_prepare(*d, buf, bytes, waves_per_cu, opt, fn, &p));
  const uint32_t per_xcd = p.grid / 8 * (kPlainWgThreads / 64);
  const uint64_t total = (bytes / 16) / (kXcdK * 64);
  XcdSplitArgs a{};
  a.buf = static_cast<const uint8_t*>(buf);
  a.per_xcd = per_xcd;
  uint64_t acc = 0;
  uint32_t it_min = ~0u, it_max = 0;
  for (int x = 0; x < 8; ++x) {
    a.starts[x] = acc;
    const uint64_t share = (uint64_t)((double)total * (weights[x] / sum));
    acc += share;
    if (share) {
      a.mask |= 1u << x;
      it_min = std::min<uint32_t>(it_min, (uint32_t)(share / per_xcd));
      it_max = std::max<uint32_t>(it_max, (uint32_t)((share + per_xcd - 1) / per_xcd));
    }
  }
  a.starts[8] = acc;
  if (a.mask == 0) return fail(SWEEP_EINVAL, "every share rounds to zero groups");
  const uint64_t n_act = (uint64_t)__builtin_popcount(a.mask) * per_xcd;
  xcd_account(&p, n_act, acc, it_min, it_max);
  std::vector<uint8_t> bits, want(n_act);
  for (uint8_t x = 0; x < 8; ++x)
    if ((a.mask >> x) & 1u) bits.push_back(x);
  for (uint64_t w = 0; w < n_act; ++w) want[w] = bits[w / per_xcd];
  return xcd_run(*d, opt, p, n_act, a, want, out);
}

int sweep_chase_walkers(const void* chain, size_t bytes, const uint32_t* starts,
                        int n_walkers, uint32_t warm_hops, uint32_t hops, int cache_policy,
                        void* stream, sweep_walker_t* out) {
  if (!out || !chain || !starts) return fail(SWEEP_EINVAL, "NULL argument");
  if (n_walkers < 1 || n_walkers > (int)kMaxWalkers)
    return fail(SWEEP_EINVAL, "n_walkers must be 1..64");
  if (bytes == 0 || bytes >= (1ull << 32)) return fail(SWEEP_EINVAL, "chain must be below 4 GiB");
  if (bytes % 4 || reinterpret_cast<uintptr_t>(chain) % 16)
    return fail(SWEEP_EALIGN, "chain must be 16-byte aligned and whole words");
  for (int i = 0; i < n_walkers; ++i)
    if (starts[i] >= bytes / 4) return fail(SWEEP_EINVAL, "start index outside the chain");
  if (cache_policy < 0 || cache_policy > 3) return fail(SWEEP_EINVAL, "unknown cache policy");
  if (hops == 0) return fail(SWEEP_EINVAL, "no timed hops");
  std::lock_guard<std::mutex> lk(g_mu);
  Dev* d = nullptr;
  SW_TRY(current_dev(&d));
  WalkArgs a{};
  a.buf = static_cast<const uint32_t*>(chain);
  a.n_bytes = (uint32_t)bytes;
  a.warm = warm_hops;
  a.steps = hops;
  a.n_walkers = (uint32_t)n_walkers;
  std::copy(starts, starts + n_walkers, a.starts);
  a.out = d->walk_out;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t h[4 * kMaxWalkers];
  hipError_t e = launch_walkers(cache_policy, st, a);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h, d->walk_out, 4 * sizeof(uint64_t) * (size_t)n_walkers,
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(SWEEP_EHIP, std::string("walkers: ") + hipGetErrorString(e));
  for (int i = 0; i < n_walkers; ++i) {
    const uint64_t* w = h + 4 * i;
    sweep_walker_t o;
    std::memset(&o, 0, sizeof(o));
    o.final_index = (uint32_t)w[0];
    o.xcc_id = (uint32_t)(w[3] & 0xF);
    o.hops = hops;
    o.wall_ticks = w[2] >= w[1] ? w[2] - w[1] : 0;
    o.ns_per_hop = (double)o.wall_ticks / d->hz() * 1e9 / hops;
    out[i] = o;
  }
  return SWEEP_OK;
}

const char* sweep_strerror(int code) {
  switch (code) {
    case SWEEP_OK: return "success";
    case SWEEP_EINVAL: return "invalid argument";
    case SWEEP_EALIGN: return "alignment or size granularity violated";
    case SWEEP_EOCCUPANCY: return "requested occupancy not achievable";
    case SWEEP_EHIP: return "HIP runtime error";
    case SWEEP_ENOMEM: return "scratch allocation failed";
    case SWEEP_ENODEV: return "no usable gfx950 device";
    default: return "unknown error";
  }
}

const char* sweep_last_error(void) { return t_err.c_str(); }

const char* sweep_version(void) { return "ilpsweep 0.1.0 (gfx950)"; }

}  // extern "C"
