// Host-side objects behind the opaque handles of swarm.h.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "swarm_internal.hpp"

namespace swarm_impl {

struct DeviceInfo {
  int device;
  int n_cu;
  int64_t lds_per_block;
};
DeviceInfo& device_info();

// Owned device allocation that grows on demand.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
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
};

swarm_status fail(swarm_status st, const char* fmt, ...);
swarm_status hip_fail(hipError_t e, const char* what);
// Dynamic LDS of a swarm launch: rate pairs, channel descriptors, candidate pool.
struct LdsLayout {
  size_t bytes;
  int ch_off, pool_off;
  int cum_off;     // running sums staged at this offset, or -1 (read from global memory)
};
LdsLayout lds_layout(int precision, int G, int nc, int service_waves, int table_layout);
void make_items(const std::vector<int64_t>& n_e, const std::vector<int64_t>& n_c, int64_t chunk,
                std::vector<WorkItem>& items, int64_t slots, int64_t block);
swarm_launch_opts resolve_opts(const swarm_launch_opts* o, int precision);

}  // namespace swarm_impl

struct swarm {
  swarm_params params{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool has_b = false;
  std::vector<int32_t> kinds;
  swarm_impl::InstanceDesc desc{};          // host copy (device constants read back after build)
  swarm_impl::InstanceDesc* d_desc = nullptr;
  swarm_impl::DevBuf arena;                 // raw inputs, tables, descriptor, counters
  swarm_impl::DevBuf records, children, items;
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
  swarm_launch_opts opts{};
};
