// Host-side objects behind the opaque handles of swarm.h.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "swarm_internal.hpp"

namespace swarm_impl {

struct DeviceInfo {
  int device;
  int n_cu;
  int64_t lds_per_block;
};
DeviceInfo& device_info();

// Device memory owned by the caller (for example a torch tensor), handed to a swarm or a
// server to take all its device allocations from: first-fit sub-allocation of the region in
// 256-byte aligned blocks; a freed block merges with its free neighbours.  Thread-safe.
class Arena {
 public:
  Arena(void* base, size_t bytes);
  void* alloc(size_t n);       // nullptr when no free block is large enough
  void release(void* p);       // p from alloc(); nullptr is ignored
  size_t capacity() const { return bytes_; }
  size_t in_use() const;

 private:
  char* base_;
  size_t bytes_;
  mutable std::mutex mu_;
  std::map<size_t, size_t> free_;   // offset -> size of every free block
  std::map<size_t, size_t> used_;   // offset -> size of every allocated block
  size_t in_use_ = 0;
};

// Device allocation that grows on demand: hipMalloc, or a block of `arena` when set.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Arena* arena = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  void reset();
  hipError_t ensure(size_t n);
};

// Tiles, partial sums and outputs of the tally reductions of a set of instances.
struct TallyPlan {
  DevBuf d_tiles, d_base, d_nrec, d_part1, d_part2, d_tot, d_out;
  std::vector<TallyTile> h_tiles;
  std::vector<int32_t> h_base;
  std::vector<int64_t> h_nrec;
  int32_t n_inst = 0, n_tiles = 0;
  hipError_t prepare(const std::vector<int64_t>& nrec, hipStream_t s);
  hipError_t launch(const InstanceDesc* d_descs, hipStream_t s);
  void bind(Arena* a) {
    for (DevBuf* b : {&d_tiles, &d_base, &d_nrec, &d_part1, &d_part2, &d_tot, &d_out}) b->arena = a;
  }
};

// Device bytes of the tally buffers for one instance of n records (with block rounding).
size_t tally_bytes(int64_t n_records);

swarm_status fail(swarm_status st, const char* fmt, ...);
swarm_status hip_fail(hipError_t e, const char* what);
// Dynamic LDS of a swarm launch: rate pairs, channel descriptors, candidate pool.
struct LdsLayout {
  size_t bytes;
  int ch_off, pool_off;
  int cum_off;     // running sums staged at this offset, or -1 (read from global memory)
};
LdsLayout lds_layout(int precision, int G, int nc, int service_waves, int table_layout);
// Work items of `chunk` electrons (fewer towards the end of the launch), instance by instance:
// the heaviest collision budget first, or the largest `rank` first where one is given (the
// expected device work per electron); instances of equal rank in the caller's order.
void make_items(const std::vector<int64_t>& n_e, const std::vector<int64_t>& n_c, int64_t chunk,
                std::vector<WorkItem>& items, int64_t slots, int64_t block,
                const std::vector<double>* rank = nullptr);
swarm_launch_opts resolve_opts(const swarm_launch_opts* o, int precision);
// Builds a swarm handle (validation, tables); with `mem` every device allocation of the
// handle comes from that caller-owned region.
swarm_status create_swarm(const swarm_component* comps, int32_t n_comps, const swarm_params* params,
                          Arena* mem, swarm_t* out);
// Device bytes that create_swarm allocates for these inputs (tables, descriptor, counters).
size_t create_bytes(const swarm_component* comps, int32_t n_comps, const swarm_params* params);

}  // namespace swarm_impl

struct swarm {
  // caller-owned device memory (declared first: released last, after every buffer below)
  std::unique_ptr<swarm_impl::Arena> own_mem;
  swarm_impl::Arena* mem = nullptr;
  swarm_params params{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool has_b = false;
  std::vector<int32_t> kinds;
  swarm_impl::InstanceDesc desc{};          // host copy (device constants read back after build)
  swarm_impl::InstanceDesc* d_desc = nullptr;
  swarm_impl::DevBuf arena;                 // raw inputs, tables, descriptor, counters
  swarm_impl::DevBuf records, children, items;
  swarm_impl::DevBuf parked;                 // real mode: electrons parked between launches (two buffers)
  std::vector<swarm_impl::WorkItem> h_items;
  swarm_impl::DevBuf trace_ids, trace_out, trace_count;
  int32_t n_trace = 0, max_events = 0;
  bool traced = false;
  swarm_impl::TallyPlan tally;
  swarm_tallies_t tallies{};
  int64_t n_records = 0;
  bool have_run = false;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  double kernel_ms = 0.0, total_ms = 0.0;
  int64_t n_launches = 0, n_parked = 0;     // the last run's simulation launches, parked electrons
  swarm_launch_opts opts{};
  // a run started by swarm_run_async: 1 enqueued on the stream (dummy mode), 2 running on
  // `worker` (real mode, whose generations need the host between launches)
  int in_flight = 0;
  std::thread worker;
  swarm_status async_status = SWARM_OK;
  std::string async_error;
  swarm_status run_status = SWARM_OK;   // status to report once the enqueued run is waited for
  std::string run_error;
  bool noalloc_records = false;         // the last run wrote records to caller memory

  void bind_arena(swarm_impl::Arena* a) {
    mem = a;
    for (swarm_impl::DevBuf* b : {&arena, &records, &children, &items, &parked, &trace_ids, &trace_out, &trace_count})
      b->arena = a;
    tally.bind(a);
  }
};
