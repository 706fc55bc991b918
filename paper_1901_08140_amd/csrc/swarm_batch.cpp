// Batched runs: many swarm instances in one persistent launch, optionally captured in a
// hipGraph, and the launch-shape autotuner.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "swarm_api_internal.hpp"

using namespace swarm_impl;

struct swarm_batch {
  std::vector<swarm*> hs;
  std::vector<swarm_job> jobs;
  int precision = 0;
  bool magnetic = false;
  int extended = 0;   // kernel level: 1 some instance uses an adaptive trial frequency,
                      // 2 some instance has moving targets or the relativistic mover
  hipStream_t stream = nullptr;
  DevBuf descs, items;
  std::vector<InstanceDesc> h_descs;
  std::vector<WorkItem> h_items;
  TallyPlan tally;
  swarm_launch_opts opts{};
  int grid = 1;
  size_t lds = 0;
  int ch_off = 0, pool_off = 0, cum_off = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<swarm_tallies_t> h_out;
  bool launched = false, done = false;
  double device_ms = 0.0;
  std::vector<int64_t> ne, nc;   // electrons and collision budget per instance
  int64_t slots = 0;             // resident work-groups of the launch shape
  bool reordered = false;        // items ordered by the measured work (after the first launch)

  ~swarm_batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

int32_t* item_counter(swarm_batch* b) {
  return reinterpret_cast<int32_t*>(static_cast<char*>(b->items.p) + b->h_items.size() * sizeof(WorkItem));
}

// The device work of one batch launch: reset the work counter, run the persistent swarm
// kernel over all work items, reduce the tallies of every instance.
hipError_t enqueue(swarm_batch* b) {
  hipError_t e;
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(item_counter(b)), 0u, 1, b->stream)) != hipSuccess) return e;
  if ((e = launch_swarm_dummy(static_cast<const InstanceDesc*>(b->descs.p), static_cast<const WorkItem*>(b->items.p),
                              static_cast<int32_t>(b->h_items.size()), item_counter(b), b->precision, b->magnetic,
                              false, b->extended, b->opts.service_waves, b->opts.block_size, b->grid,
                              b->opts.pending_trigger, b->lds, b->ch_off, b->pool_off, b->cum_off, b->stream)) != hipSuccess)
    return e;
  return b->tally.launch(static_cast<const InstanceDesc*>(b->descs.p), b->stream);
}

// Capture the launch in a hipGraph (replacing an earlier capture).
hipError_t capture(swarm_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t e2 = enqueue(b);
  e = hipStreamEndCapture(b->stream, &b->graph);
  if (e2 != hipSuccess) return e2;
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
}

// Upload the work items and size the grid to them.
hipError_t upload_items(swarm_batch* b, int per_cu) {
  hipError_t e = b->items.ensure(b->h_items.size() * sizeof(WorkItem) + 256);
  if (e != hipSuccess) return e;
  if ((e = hipMemcpyAsync(b->items.p, b->h_items.data(), b->h_items.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                          b->stream)) != hipSuccess)
    return e;
  b->grid = std::max(1, std::min<int>(static_cast<int>(b->h_items.size()), device_info().n_cu * per_cu));
  return hipSuccess;
}

// After the first launch, the items are ordered by each instance's measured device work per
// electron, collision budget x (trials per real collision + 3, the collision pass counted as
// about three trials), longest first.  The order matters as much as the item size (the argon
// sweep listed with its fast instances first took 1071 ms instead of 873 ms), and the caller's
// order need not be the right one.  Item sizes stay those of the collision budgets (items
// sized by the measured cost made the step slower).  Results do not depend on the order.
hipError_t reorder(swarm_batch* b) {
  std::vector<double> rank(b->hs.size());
  for (size_t i = 0; i < rank.size(); ++i) {
    const double reals = static_cast<double>(b->h_out[i].n_real);
    const double trials = reals + static_cast<double>(b->h_out[i].n_null) + static_cast<double>(b->h_out[i].n_forbidden);
    rank[i] = static_cast<double>(b->nc[i]) * (reals > 0 ? trials / reals + 3.0 : 4.0);
  }
  std::vector<WorkItem> items;
  make_items(b->ne, b->nc, b->opts.chunk, items, b->slots, b->opts.block_size, &rank);
  const bool same = items.size() == b->h_items.size() &&
                    std::equal(items.begin(), items.end(), b->h_items.begin(), [](const WorkItem& x, const WorkItem& y) {
                      return x.inst == y.inst && x.first == y.first && x.count == y.count;
                    });
  if (same) return hipSuccess;
  b->h_items.swap(items);
  const int per_cu = static_cast<int>(b->slots / std::max(1, device_info().n_cu));
  hipError_t e = upload_items(b, per_cu);
  if (e == hipSuccess && b->exec) e = capture(b);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  return e;
}

}  // namespace

extern "C" {

swarm_status swarm_batch_create(swarm_t* handles, const swarm_job* jobs, int32_t n, const swarm_launch_opts* opts,
                                swarm_batch_t* out) {
  if (!out) return fail(SWARM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!handles || !jobs || n <= 0) return fail(SWARM_ERR_INVALID_ARG, "empty batch");
  auto b = std::make_unique<swarm_batch>();
  b->precision = handles[0] ? handles[0]->desc.precision : 0;
  int G = 0, n_ch = 0;
  for (int i = 0; i < n; ++i) {
    swarm* h = handles[i];
    if (!h) return fail(SWARM_ERR_INVALID_ARG, "handle %d is NULL", i);
    if (h->desc.precision != b->precision) return fail(SWARM_ERR_INVALID_ARG, "batch mixes precisions");
    if (h->desc.secondaries != SWARM_DUMMY)
      return fail(SWARM_ERR_INVALID_ARG, "batched launches take dummy-secondaries instances only (handle %d)", i);
    if (jobs[i].n_electrons < 1) return fail(SWARM_ERR_INVALID_ARG, "job %d: n_electrons must be >= 1", i);
    if (jobs[i].n_collisions < 1 || jobs[i].n_collisions > 0xffffffffLL)
      return fail(SWARM_ERR_INVALID_ARG, "job %d: n_collisions must be in [1, 2^32-1]", i);
    for (int j = 0; j < i; ++j)
      if (handles[j] == h) return fail(SWARM_ERR_INVALID_ARG, "handle %d appears twice", i);
    b->magnetic |= h->has_b;
    b->extended = std::max(b->extended, h->desc.thermal_targets || h->desc.relativistic ? 2
                                        : h->desc.trial_strategy != SWARM_TRIAL_CONSTANT ? 1 : 0);
    G = std::max(G, h->desc.G);
    n_ch = std::max(n_ch, h->desc.nc);
    b->hs.push_back(h);
    b->jobs.push_back(jobs[i]);
  }
  b->opts = resolve_opts(opts, b->precision);
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  if ((e = hipEventCreate(&b->ev0)) != hipSuccess || (e = hipEventCreate(&b->ev1)) != hipSuccess)
    return hip_fail(e, "hipEventCreate");
  // per-instance results live in the handles
  std::vector<int64_t> ne, nc;
  for (int i = 0; i < n; ++i) {
    swarm* h = b->hs[i];
    if ((e = h->records.ensure(static_cast<size_t>(jobs[i].n_electrons) * sizeof(swarm_record))) != hipSuccess)
      return hip_fail(e, "allocating records");
    InstanceDesc d = h->desc;
    d.n_electrons = jobs[i].n_electrons;
    d.n_collisions = static_cast<uint32_t>(jobs[i].n_collisions);
    d.quantum = 0;
    d.seed = jobs[i].seed;
    d.capacity = jobs[i].n_electrons;
    d.records = static_cast<swarm_record*>(h->records.p);
    d.saved = nullptr;
    d.children = nullptr;
    d.trace_ids = nullptr;
    d.n_trace = 0;
    d.max_events = 0;
    d.trace_out = nullptr;
    d.trace_count = nullptr;
    b->h_descs.push_back(d);
    ne.push_back(jobs[i].n_electrons);
    nc.push_back(jobs[i].n_collisions);
  }
  const LdsLayout ll = lds_layout(b->precision, G, n_ch, b->opts.service_waves, b->opts.table_layout);
  if (static_cast<int64_t>(ll.bytes) > device_info().lds_per_block)
    return fail(SWARM_ERR_INVALID_ARG, "the tables need %zu bytes of LDS per work-group, the device has %lld",
                ll.bytes, static_cast<long long>(device_info().lds_per_block));
  b->lds = ll.bytes;
  b->ch_off = ll.ch_off;
  b->pool_off = ll.pool_off;
  b->cum_off = ll.cum_off;
  const int per_cu = swarm_kernel_max_blocks_per_cu(b->precision, b->magnetic, false, false, b->extended,
                                                    b->opts.service_waves, b->opts.block_size, b->lds);
  b->slots = static_cast<int64_t>(device_info().n_cu) * per_cu;
  b->ne = ne;
  b->nc = nc;
  make_items(ne, nc, b->opts.chunk, b->h_items, b->slots, b->opts.block_size);
  if ((e = b->descs.ensure(n * sizeof(InstanceDesc))) != hipSuccess) return hip_fail(e, "descriptors");
  if ((e = hipMemcpyAsync(b->descs.p, b->h_descs.data(), n * sizeof(InstanceDesc), hipMemcpyHostToDevice, b->stream)) != hipSuccess ||
      (e = upload_items(b.get(), per_cu)) != hipSuccess)
    return hip_fail(e, "uploading batch");
  if ((e = b->tally.prepare(ne, b->stream)) != hipSuccess) return hip_fail(e, "tally plan");
  if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return hip_fail(e, "uploading batch");
  if (b->opts.use_graph && (e = capture(b.get())) != hipSuccess) return hip_fail(e, "graph capture");
  b->h_out.resize(n);
  *out = b.release();
  return SWARM_OK;
}

swarm_status swarm_batch_launch(swarm_batch_t b) {
  if (!b) return fail(SWARM_ERR_INVALID_ARG, "batch is NULL");
  hipError_t e;
  if ((e = hipEventRecord(b->ev0, b->stream)) != hipSuccess) return hip_fail(e, "event");
  if (b->exec) e = hipGraphLaunch(b->exec, b->stream);
  else e = enqueue(b);
  if (e != hipSuccess) return hip_fail(e, "batch launch");
  if ((e = hipEventRecord(b->ev1, b->stream)) != hipSuccess) return hip_fail(e, "event");
  if ((e = hipMemcpyAsync(b->h_out.data(), b->tally.d_out.p, b->h_out.size() * sizeof(swarm_tallies_t),
                          hipMemcpyDeviceToHost, b->stream)) != hipSuccess)
    return hip_fail(e, "tallies");
  b->launched = true;
  b->done = false;
  return SWARM_OK;
}

swarm_status swarm_batch_wait(swarm_batch_t b, double* device_ms) {
  if (!b) return fail(SWARM_ERR_INVALID_ARG, "batch is NULL");
  if (!b->launched) return fail(SWARM_ERR_STATE, "batch not launched");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "batch");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, b->ev0, b->ev1);
  b->device_ms = ms;
  if (device_ms) *device_ms = ms;
  for (size_t i = 0; i < b->hs.size(); ++i) {
    swarm* h = b->hs[i];
    h->desc.n_electrons = b->h_descs[i].n_electrons;
    h->desc.n_collisions = b->h_descs[i].n_collisions;
    h->desc.seed = b->h_descs[i].seed;
    h->desc.records = b->h_descs[i].records;
    h->tallies = b->h_out[i];
    h->n_records = b->jobs[i].n_electrons;
    h->have_run = true;
    h->traced = false;
    h->kernel_ms = ms;
    h->total_ms = ms;
    h->n_launches = 1;
    h->n_parked = 0;
  }
  b->done = true;
  if (!b->reordered) {
    b->reordered = true;
    if ((e = reorder(b)) != hipSuccess) return hip_fail(e, "reordering the batch");
  }
  return SWARM_OK;
}

swarm_status swarm_batch_tallies(swarm_batch_t b, int32_t i, swarm_tallies_t* out) {
  if (!b || !out) return fail(SWARM_ERR_INVALID_ARG, "NULL argument");
  if (!b->done) return fail(SWARM_ERR_STATE, "batch has not completed");
  if (i < 0 || i >= static_cast<int32_t>(b->h_out.size())) return fail(SWARM_ERR_INVALID_ARG, "bad instance index");
  *out = b->h_out[i];
  return SWARM_OK;
}

void swarm_batch_destroy(swarm_batch_t b) { delete b; }

swarm_status swarm_batch_run(swarm_t* handles, const swarm_job* jobs, int32_t n, const swarm_launch_opts* opts) {
  swarm_batch_t b = nullptr;
  swarm_status st = swarm_batch_create(handles, jobs, n, opts, &b);
  if (st != SWARM_OK) return st;
  b->reordered = true;   // one launch: no later launch to order
  st = swarm_batch_launch(b);
  if (st == SWARM_OK) st = swarm_batch_wait(b, nullptr);
  swarm_batch_destroy(b);
  return st;
}

// Coordinate search over the result-invariant launch options on a probe copy of the batch
// (same instances and electron counts, budgets cut to probe_collisions): block size, then
// the pending-lane trigger, then the work-item size, then the LDS table layout.  Each
// candidate takes the faster of two launches (one launch varies by a few percent), after
// one untimed launch of the default shape.
swarm_status swarm_autotune(swarm_t* handles, const swarm_job* jobs, int32_t n, int64_t probe_collisions,
                            swarm_launch_opts* best) {
  if (!best || !handles || !jobs || n <= 0) return fail(SWARM_ERR_INVALID_ARG, "NULL argument");
  if (probe_collisions < 1) return fail(SWARM_ERR_INVALID_ARG, "probe_collisions must be >= 1");
  std::vector<swarm_job> probe(jobs, jobs + n);
  for (auto& j : probe) j.n_collisions = std::min<int64_t>(j.n_collisions, probe_collisions);
  auto time_it = [&](const swarm_launch_opts& o, double* ms) -> swarm_status {
    swarm_batch_t b = nullptr;
    swarm_status st = swarm_batch_create(handles, probe.data(), n, &o, &b);
    if (st != SWARM_OK) return st;
    *ms = 1e300;
    for (int rep = 0; rep < 2 && st == SWARM_OK; ++rep) {
      double t1 = 0.0;
      st = swarm_batch_launch(b);
      if (st == SWARM_OK) st = swarm_batch_wait(b, &t1);
      if (st == SWARM_OK) *ms = std::min(*ms, t1);
    }
    swarm_batch_destroy(b);
    return st;
  };
  swarm_launch_opts cur = resolve_opts(nullptr, handles[0] ? handles[0]->desc.precision : 0);
  cur.use_graph = 0;
  double t = 0.0;
  swarm_status st = time_it(cur, &t);   // warm-up
  if (st != SWARM_OK) return st;
  double best_t = 1e300;
  const int per_lane = cur.chunk / cur.block_size;   // the precision's default
  for (int bs : {128, 256, 512}) {
    swarm_launch_opts o = cur;
    o.block_size = bs;
    o.chunk = bs * per_lane;
    if ((st = time_it(o, &t)) != SWARM_OK) return st;
    if (t < best_t) { best_t = t; cur = o; }
  }
  const swarm_launch_opts base1 = cur;
  for (int trig : {16, 24, 32, 40, 48}) {
    swarm_launch_opts o = base1;
    o.pending_trigger = trig;
    if ((st = time_it(o, &t)) != SWARM_OK) return st;
    if (t < best_t) { best_t = t; cur = o; }
  }
  const swarm_launch_opts base2 = cur;
  for (int mult : {2, 3, 4, 8}) {
    swarm_launch_opts o = base2;
    o.chunk = base2.block_size * mult;
    if ((st = time_it(o, &t)) != SWARM_OK) return st;
    if (t < best_t) { best_t = t; cur = o; }
  }
  // LDS table layout: running sums in LDS too (taken only where they fit; see lds_layout)
  {
    swarm_launch_opts o = cur;
    o.table_layout = 1;
    if ((st = time_it(o, &t)) != SWARM_OK) return st;
    if (t < best_t) { best_t = t; cur = o; }
  }
  *best = cur;
  return SWARM_OK;
}

}  // extern "C"
