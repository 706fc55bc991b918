// swarm_run_noalloc: the dummy-mode run of swarm_run for callers that cannot allocate device
// memory.  The per-run scratch that swarm_run allocates (work items and their counter, the
// tally tiles, partial sums, totals and the tally output) lives here in one file-scope device
// array instead; the records go to memory the caller passes in.  The kernels are the ones
// swarm_run launches, with the same arguments, so the records and tallies are the same bits.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "swarm_api_internal.hpp"

using namespace swarm_impl;

namespace {

constexpr int64_t kMaxElectrons = int64_t(1) << 22;
constexpr int64_t kMaxItems = 16384;
constexpr int64_t kMaxTiles = (kMaxElectrons + kTallyTile - 1) / kTallyTile;
constexpr int kMaxDevices = 64;

constexpr size_t al256(size_t n) { return (n + 255) & ~static_cast<size_t>(255); }
// layout of the scratch array (byte offsets)
constexpr size_t kOffItems = 0;
constexpr size_t kOffCounter = al256(kOffItems + kMaxItems * sizeof(WorkItem));
constexpr size_t kOffTiles = kOffCounter + 256;
constexpr size_t kOffBase = al256(kOffTiles + kMaxTiles * sizeof(TallyTile));
constexpr size_t kOffNrec = kOffBase + 256;
constexpr size_t kOffPart1 = kOffNrec + 256;
constexpr size_t kOffPart2 = al256(kOffPart1 + kMaxTiles * kTally1 * sizeof(double));
constexpr size_t kOffTot = al256(kOffPart2 + kMaxTiles * kTally2 * sizeof(double));
constexpr size_t kOffOut = al256(kOffTot + (kTally1 + kTally2) * sizeof(double));
constexpr size_t kScratchBytes = al256(kOffOut + sizeof(swarm_tallies_t));
static_assert(kScratchBytes <= (size_t(2) << 20), "scratch stays within 2 MiB");

}  // namespace

// Every GPU the library runs on holds one copy of this array until the process ends.  Host
// code never uses its name as an address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu[kMaxDevices];         // one call at a time per device (they share the array)
void* g_scratch[kMaxDevices] = {};    // device address of `scratch` on each device

// Work items of one instance (electron ranges of `chunk`), the tally tiles of its records,
// and the counters both start from: what swarm_run builds on the host and copies over.
__global__ void k_noalloc_plan(WorkItem* __restrict__ items, int32_t n_items, int64_t n_e, int64_t chunk,
                               int32_t* __restrict__ item_ctr, TallyTile* __restrict__ tiles, int32_t n_tiles,
                               int32_t* __restrict__ base, int64_t* __restrict__ nrec) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_items) {
    WorkItem w;
    w.inst = 0;
    w.pad = 0;
    w.first = i * chunk;
    w.count = n_e - w.first < chunk ? n_e - w.first : chunk;
    items[i] = w;
  }
  if (i < n_tiles) {
    TallyTile t;
    t.inst = 0;
    t.tile = static_cast<int32_t>(i);
    t.first = i * kTallyTile;
    t.count = n_e - t.first < kTallyTile ? n_e - t.first : static_cast<int64_t>(kTallyTile);
    tiles[i] = t;
  }
  if (i == 0) {
    *item_ctr = 0;
    *base = 0;
    *nrec = n_e;
  }
}

// The device address of `scratch` on the current device, looked up once per device.
swarm_status scratch_address(int dev, char** out) {
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch[dev] = p;
  }
  *out = static_cast<char*>(g_scratch[dev]);
  return SWARM_OK;
}

}  // namespace

extern "C" {

swarm_status swarm_run_noalloc(swarm_t h, int64_t n_electrons, int64_t n_collisions, uint64_t seed,
                               swarm_record* records) {
  if (!h || !records) return fail(SWARM_ERR_INVALID_ARG, "NULL argument");
  if (h->in_flight) return fail(SWARM_ERR_STATE, "a run started by swarm_run_async is in flight: call swarm_wait first");
  if (h->desc.secondaries != SWARM_DUMMY) return fail(SWARM_ERR_INVALID_ARG, "swarm_run_noalloc runs dummy-secondaries swarms");
  if (h->n_trace > 0) return fail(SWARM_ERR_INVALID_ARG, "swarm_run_noalloc does not trace (swarm_set_trace(h, NULL, 0, 0))");
  if (n_electrons < 1 || n_electrons > kMaxElectrons)
    return fail(SWARM_ERR_INVALID_ARG, "n_electrons must be in [1, %lld] for swarm_run_noalloc",
                static_cast<long long>(kMaxElectrons));
  if (n_collisions < 1 || n_collisions > 0xffffffffLL)
    return fail(SWARM_ERR_INVALID_ARG, "n_collisions must be in [1, 2^32-1]");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(SWARM_ERR_DEVICE, "device %d beyond the library's table", dev);
  std::lock_guard<std::mutex> lk(g_mu[dev]);
  char* base = nullptr;
  swarm_status st = scratch_address(dev, &base);
  if (st != SWARM_OK) return st;
  WorkItem* d_items = reinterpret_cast<WorkItem*>(base + kOffItems);
  int32_t* d_ctr = reinterpret_cast<int32_t*>(base + kOffCounter);
  TallyTile* d_tiles = reinterpret_cast<TallyTile*>(base + kOffTiles);
  int32_t* d_base = reinterpret_cast<int32_t*>(base + kOffBase);
  int64_t* d_nrec = reinterpret_cast<int64_t*>(base + kOffNrec);
  double* d_part1 = reinterpret_cast<double*>(base + kOffPart1);
  double* d_part2 = reinterpret_cast<double*>(base + kOffPart2);
  double* d_tot = reinterpret_cast<double*>(base + kOffTot);
  swarm_tallies_t* d_out = reinterpret_cast<swarm_tallies_t*>(base + kOffOut);

  h->have_run = false;
  hipStream_t s = h->stream;
  InstanceDesc& d = h->desc;
  d.n_electrons = n_electrons;
  d.n_collisions = static_cast<uint32_t>(n_collisions);
  d.quantum = 0;
  d.seed = seed;
  d.capacity = n_electrons;
  d.records = records;
  d.saved = nullptr;
  d.children = nullptr;
  d.trace_ids = nullptr;
  d.n_trace = 0;
  d.trace_out = nullptr;
  d.trace_count = nullptr;
  // the launch shape of swarm_run (a schedule only: records do not depend on it)
  const swarm_launch_opts& o = h->opts;
  const LdsLayout ll = lds_layout(d.precision, d.G, d.nc, o.service_waves, o.table_layout);
  if (static_cast<int64_t>(ll.bytes) > device_info().lds_per_block)
    return fail(SWARM_ERR_INVALID_ARG, "the tables need %zu bytes of LDS per work-group", ll.bytes);
  const int ext = d.thermal_targets || d.relativistic ? 2 : d.trial_strategy != SWARM_TRIAL_CONSTANT ? 1 : 0;
  const int per_cu = swarm_kernel_max_blocks_per_cu(d.precision, h->has_b, false, false, ext, o.service_waves,
                                                    o.block_size, ll.bytes);
  const int64_t slots = static_cast<int64_t>(device_info().n_cu) * per_cu;
  auto round_up = [&](int64_t n) { return (n + o.block_size - 1) / o.block_size * o.block_size; };
  int64_t chunk = round_up((n_electrons + 4 * slots - 1) / (4 * slots));
  chunk = std::max<int64_t>(o.block_size, std::min<int64_t>(chunk, o.chunk));
  chunk = std::max(chunk, round_up((n_electrons + kMaxItems - 1) / kMaxItems));   // at most kMaxItems items
  const int64_t n_items = (n_electrons + chunk - 1) / chunk;
  const int64_t n_tiles = (n_electrons + kTallyTile - 1) / kTallyTile;
  if (n_items > kMaxItems || n_tiles > kMaxTiles) return fail(SWARM_ERR_INVALID_ARG, "work does not fit the scratch");
  const int64_t plan_n = std::max(n_items, n_tiles);
  hipLaunchKernelGGL(k_noalloc_plan, dim3(static_cast<unsigned>((plan_n + 255) / 256)), dim3(256), 0, s, d_items,
                     static_cast<int32_t>(n_items), n_electrons, chunk, d_ctr, d_tiles, static_cast<int32_t>(n_tiles),
                     d_base, d_nrec);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "plan launch");
  if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(d.ctr), 0ull, sizeof(RunCounters) / sizeof(uint64_t), s)) != hipSuccess)
    return hip_fail(e, "counters");
  if ((e = hipMemcpyAsync(h->d_desc, &h->desc, sizeof(InstanceDesc), hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(e, "descriptor");
  if ((e = hipEventRecord(h->ev[0], s)) != hipSuccess) return hip_fail(e, "event");
  const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(n_items, slots)));
  if ((e = launch_swarm_dummy(h->d_desc, d_items, static_cast<int32_t>(n_items), d_ctr, d.precision, h->has_b, false,
                              ext, o.service_waves, o.block_size, grid, o.pending_trigger, ll.bytes, ll.ch_off,
                              ll.pool_off, ll.cum_off, s)) != hipSuccess)
    return hip_fail(e, "swarm kernel launch");
  if ((e = hipEventRecord(h->ev[1], s)) != hipSuccess) return hip_fail(e, "event");
  if ((e = launch_tallies(h->d_desc, d_tiles, static_cast<int32_t>(n_tiles), d_base, d_nrec, 1, d_part1, d_part2,
                          d_tot, d_out, s)) != hipSuccess)
    return hip_fail(e, "tally launch");
  if ((e = hipEventRecord(h->ev[2], s)) != hipSuccess) return hip_fail(e, "event");
  if ((e = hipMemcpyAsync(&h->tallies, d_out, sizeof(swarm_tallies_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "swarm run");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, h->ev[0], h->ev[1]);
  h->kernel_ms = ms;
  (void)hipEventElapsedTime(&ms, h->ev[0], h->ev[2]);
  h->total_ms = ms;
  h->n_records = n_electrons;
  h->noalloc_records = true;
  h->traced = false;
  h->n_launches = 1;
  h->n_parked = 0;
  h->have_run = true;
  return SWARM_OK;
}

}  // extern "C"
