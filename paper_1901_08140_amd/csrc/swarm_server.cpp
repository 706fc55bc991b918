// Serving: continuous batching of swarm requests on one GPU.
//
// A scheduler thread owns the device work.  Requests wait in FIFO order until the device
// memory they need (tables, per-electron state and records) fits the HBM budget; admitted
// requests keep that memory until they finish.  All admitted, unfinished requests advance
// together in epochs: one persistent launch in which every unfinished electron makes up to
// `quantum` more real collisions and stops at a real-collision boundary, saving its state.
// Requests admitted while an epoch runs (their tables are built on a second stream) join
// the next epoch.  Finished requests get their tallies reduced on the device and their
// memory is released.  Since electrons stop only at real-collision boundaries and the
// random streams are keyed by (seed, electron, counter), a request's results are the same
// bits whatever it was batched with and however the epochs fell.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "swarm_api_internal.hpp"

using namespace swarm_impl;

namespace {

struct ChannelCopy {
  int32_t kind;
  double thr;
  std::vector<double> e, s;
};
struct ComponentCopy {
  double mass, frac;
  std::vector<ChannelCopy> ch;
  int32_t scattering = SWARM_SCATTER_ISOTROPIC;
  double mt_over_el = 1.0;
};

struct Request {
  int64_t ticket = 0;
  std::vector<ComponentCopy> comps;
  swarm_params params{};
  int64_t n_e = 0, n_c = 0;
  uint64_t seed = 0;
  swarm_record* records_out = nullptr;   // host memory for the records, if the caller asked
  int64_t need = 0;                        // device bytes it holds while admitted
  // scheduler state
  swarm* h = nullptr;
  DevBuf saved;
  int slot = -1;
  int64_t bytes = 0;
  int64_t epochs = 0;
  int64_t done_coll = 0;    // collisions per electron made so far (the epochs' quanta, capped)
  int64_t quantum = 0;      // this epoch's collisions per electron
  double cost = 0.0;        // device work per real collision in trial blocks, measured (0: no epoch yet)
  uint64_t blocks_seen = 0; // trial blocks its electrons had drawn at its last measurement
  int64_t coll_seen = 0;    // and its collisions per electron then
  double submit_s = 0, admit_s = 0, done_s = 0;
  swarm_status status = SWARM_PENDING;
  swarm_tallies_t tallies{};
};

}  // namespace

struct swarm_server {
  std::unique_ptr<Arena> mem;   // caller-owned device memory, if any (released last)
  swarm_server_params p{};
  std::chrono::steady_clock::time_point t0;
  hipStream_t compute = nullptr, setup = nullptr;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<std::shared_ptr<Request>> pending;
  std::vector<std::shared_ptr<Request>> active;
  std::map<int64_t, std::shared_ptr<Request>> all;
  int64_t next_ticket = 1;
  int64_t n_unfinished = 0;
  int64_t used_bytes = 0;
  int64_t budget = 0;           // admission limit: the HBM budget, or the arena if smaller
  bool stop = false;
  std::thread th;
  // device state of the epochs
  DevBuf ctrs, descs, items;
  DevBuf mdescs, mparts;    // the requests measured after an epoch and their block sums
  std::vector<int> free_slots;
  int max_slots = 0;
  TallyPlan tally;
  double rate = 0.0;   // measured real collisions per second (quantum before any cost is known)
  double block_rate = 0.0;  // measured device work per second, in trial blocks (adaptive quanta)
  int64_t epoch = 0;   // epochs started so far (failure injection counts them)
  int64_t n_epochs = 0;     // epochs completed
  int64_t work_done = 0;    // real collisions made by all requests so far
  int64_t n_ok = 0, n_failed = 0;
  int64_t fail_epoch = 0;   // tests: epoch number that reports a device failure (0 = none)

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// Estimate of the device memory of a request whose inputs failed validation (it is
// refused at admission): tables plus records and resumable state of every electron.
int64_t request_bytes(const Request& r) {
  int64_t nc = 0, pts = 0;
  for (const auto& c : r.comps) {
    nc += static_cast<int64_t>(c.ch.size());
    for (const auto& ch : c.ch) pts += static_cast<int64_t>(ch.e.size());
  }
  const int P = r.params.grid_points_per_octave ? r.params.grid_points_per_octave : 64;
  int emin = r.params.grid_min_exp2, emax = r.params.grid_max_exp2;
  if (emin == 0 && emax == 0) { emin = -14; emax = 12; }
  const int64_t G = static_cast<int64_t>(emax - emin) * P + 1;
  // (the binned strategy adds a bin of every table entry and at most 785 bins of 16 bytes)
  const int64_t bins = r.params.trial_strategy == SWARM_TRIAL_BINNED ? 4 * (G + 1) + 16 * 1024 : 0;
  const int64_t tables = 16 * pts + G * (8 + 16 + 8) + G * nc * (8 + 16 + 8) + nc * 128 + 8192 + bins;
  return tables + r.n_e * static_cast<int64_t>(sizeof(swarm_record) + sizeof(SavedState));
}

swarm_status admit(swarm_server* s, const std::shared_ptr<Request>& r) {
  std::vector<std::vector<swarm_channel>> chs(r->comps.size());
  std::vector<swarm_component> comps(r->comps.size());
  for (size_t k = 0; k < r->comps.size(); ++k) {
    for (auto& c : r->comps[k].ch)
      chs[k].push_back({c.kind, c.thr, static_cast<int32_t>(c.e.size()), c.e.data(), c.s.data()});
    comps[k] = {r->comps[k].mass, r->comps[k].frac, static_cast<int32_t>(chs[k].size()), chs[k].data(),
                r->comps[k].scattering, r->comps[k].mt_over_el};
  }
  swarm_params p = r->params;
  p.precision = s->p.precision;
  p.secondaries = SWARM_DUMMY;
  p.stream = s->setup;
  swarm_t h = nullptr;
  swarm_status st = create_swarm(comps.data(), static_cast<int32_t>(comps.size()), &p, s->mem.get(), &h);
  if (st != SWARM_OK) return st;
  r->h = h;
  r->saved.arena = s->mem.get();
  hipError_t e;
  if ((e = h->records.ensure(static_cast<size_t>(r->n_e) * sizeof(swarm_record))) != hipSuccess ||
      (e = r->saved.ensure(static_cast<size_t>(r->n_e) * sizeof(SavedState))) != hipSuccess)
    return hip_fail(e, "request memory");
  // saved.started = 0 for every electron: clear the whole state array
  if ((e = launch_fill_u64(static_cast<uint64_t*>(r->saved.p), 0ull,
                           static_cast<int64_t>(r->n_e) * sizeof(SavedState) / 8, s->setup)) != hipSuccess)
    return hip_fail(e, "clearing state");
  RunCounters* c = static_cast<RunCounters*>(s->ctrs.p) + r->slot;
  if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(c), 0ull, sizeof(RunCounters) / 8, s->setup)) != hipSuccess)
    return hip_fail(e, "clearing counters");
  if ((e = hipStreamSynchronize(s->setup)) != hipSuccess) return hip_fail(e, "request setup");
  InstanceDesc& d = h->desc;
  d.n_electrons = r->n_e;
  d.n_collisions = static_cast<uint32_t>(r->n_c);
  d.seed = r->seed;
  d.capacity = r->n_e;
  d.records = static_cast<swarm_record*>(h->records.p);
  d.saved = static_cast<SavedState*>(r->saved.p);
  d.children = nullptr;
  d.ctr = c;
  d.trace_ids = nullptr;
  d.n_trace = 0;
  d.trace_out = nullptr;
  d.trace_count = nullptr;
  return SWARM_OK;
}

void finish(swarm_server* s, const std::shared_ptr<Request>& r, swarm_status st) {
  std::lock_guard<std::mutex> lk(s->mu);
  r->status = st;
  r->done_s = s->now();
  if (st == SWARM_OK) ++s->n_ok;
  else ++s->n_failed;
  if (r->h) {
    swarm_destroy(r->h);
    r->h = nullptr;
  }
  r->saved.reset();
  if (r->slot >= 0) s->free_slots.push_back(r->slot);
  r->slot = -1;
  s->used_bytes -= r->bytes;
  r->bytes = 0;
  r->comps.clear();
  --s->n_unfinished;
  s->cv_done.notify_all();
}

// Admit queued requests in arrival order while they fit the budget and a slot is free.
void admit_pending(swarm_server* s) {
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->pending.empty() || s->free_slots.empty()) return;
      const int64_t need = s->pending.front()->need;
      if (s->used_bytes + need > s->budget && !s->active.empty()) return;
      r = s->pending.front();
      s->pending.pop_front();
      r->slot = s->free_slots.back();
      s->free_slots.pop_back();
      r->bytes = need;
      s->used_bytes += need;
      r->admit_s = s->now();
    }
    const swarm_status st = admit(s, r);
    if (st == SWARM_ERR_OUT_OF_MEMORY && s->mem) {
      // The caller's region is fragmented (or the budget overstates it): give the memory
      // back and retry once an admitted request has finished and released its blocks.
      std::lock_guard<std::mutex> lk(s->mu);
      if (!s->active.empty()) {
        if (r->h) swarm_destroy(r->h);
        r->h = nullptr;
        r->saved.reset();
        s->free_slots.push_back(r->slot);
        r->slot = -1;
        s->used_bytes -= r->bytes;
        r->bytes = 0;
        s->pending.push_front(r);
        return;
      }
    }
    if (st != SWARM_OK) {
      finish(s, r, st);
      continue;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->active.push_back(r);
  }
}

// Shortest remaining work first: the admitted requests with the least device work left
// (electron-collisions left times the measured work per collision), until the epoch holds
// about kEpochElectronsPerCu electrons per compute unit (enough to fill the device).  Two
// more always run: the earliest admitted request, so that no request waits forever behind a
// stream of small ones, and the one with the most work per electron left, the longest chain
// of sequential work, so that it does not end up running alone on an underfilled device.
// Results do not depend on the schedule; only which requests finish first does.
constexpr int64_t kEpochElectronsPerCu = 10240;

// Serving accounting, one work-group of 256 per (part, request): the trial blocks drawn so far
// by the electrons of request blockIdx.y (the block index in the resumable state of an
// electron that has run and not finished, the record's count of one that has finished), as
// kEpochBlocksParts partial sums that the host adds up.  Differences between measurements
// give a request's blocks per real collision, from which its quantum is sized.
constexpr int kEpochBlocksParts = 32;

__global__ void __launch_bounds__(256) k_epoch_blocks(const InstanceDesc* __restrict__ descs,
                                                      unsigned long long* __restrict__ out) {
  __shared__ unsigned long long s_part[4];
  const InstanceDesc& d = descs[blockIdx.y];
  unsigned long long acc = 0ull;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < d.n_electrons;
       e += static_cast<int64_t>(gridDim.x) * 256) {
    const uint32_t st = d.saved[e].started;
    acc += st == 1u ? d.saved[e].block : st == 2u ? d.records[e].blocks : 0ull;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    out[static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x] = s_part[0] + s_part[1] + s_part[2] + s_part[3];
}

hipError_t launch_epoch_blocks(const InstanceDesc* descs, int n, unsigned long long* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_epoch_blocks, dim3(kEpochBlocksParts, static_cast<unsigned>(n)), dim3(256), 0, s, descs, out);
  return hipGetLastError();
}

// Device work of a real collision in units of trial blocks: a collision pass serves about
// two thirds of a wave and runs about 1.5 times the instructions of a trial block.
constexpr double kCollisionBlocks = 1.5;

std::vector<std::shared_ptr<Request>> pick_shortest_first(const std::vector<std::shared_ptr<Request>>& active) {
  const int64_t target = kEpochElectronsPerCu * device_info().n_cu;
  // remaining device work: electron-collisions left times the measured work per collision
  // (the mean over the measured requests for one without a measurement)
  double mean = 0.0;
  int n_mean = 0;
  for (auto& r : active)
    if (r->cost > 0) { mean += r->cost; ++n_mean; }
  mean = n_mean > 0 ? mean / n_mean : 1.0;
  auto left = [mean](const std::shared_ptr<Request>& r) {
    return static_cast<double>(r->n_e * (r->n_c - r->done_coll)) * (r->cost > 0 ? r->cost : mean);
  };
  auto chain = [mean](const std::shared_ptr<Request>& r) {
    return static_cast<double>(r->n_c - r->done_coll) * (r->cost > 0 ? r->cost : mean);
  };
  std::vector<std::shared_ptr<Request>> out{active.front()};
  const auto longest = std::max_element(active.begin(), active.end(),
      [&](const std::shared_ptr<Request>& a, const std::shared_ptr<Request>& b) { return chain(a) < chain(b); });
  if (*longest != active.front()) out.push_back(*longest);
  int64_t electrons = 0;
  for (auto& r : out) electrons += r->n_e;
  std::vector<std::shared_ptr<Request>> rest;
  for (auto& r : active)
    if (std::find(out.begin(), out.end(), r) == out.end()) rest.push_back(r);
  std::stable_sort(rest.begin(), rest.end(),
                   [&](const std::shared_ptr<Request>& a, const std::shared_ptr<Request>& b) { return left(a) < left(b); });
  for (auto& r : rest) {
    if (electrons >= target) break;
    out.push_back(r);
    electrons += r->n_e;
  }
  return out;
}

void scheduler(swarm_server* s) {
  std::vector<InstanceDesc> descs;
  std::vector<WorkItem> items;
  hipEvent_t ev0, ev1;
  (void)hipEventCreate(&ev0);
  (void)hipEventCreate(&ev1);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->active.empty(); });
      if (s->stop) break;
    }
    admit_pending(s);
    std::vector<std::shared_ptr<Request>> act;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      act = s->active;
    }
    if (act.empty()) continue;
    if (s->p.schedule == SWARM_SCHEDULE_SHORTEST_FIRST && act.size() > 1) act = pick_shortest_first(act);
    // epoch quanta: fixed, or sized so that an epoch lasts about 100 ms (with one quantum for
    // every request, a stream of random-mixture requests at 50 req/s over 40 s served 1.22e10
    // real/s with 50 ms epochs, 1.30e10 with 100 ms, 1.32e10 with 200 ms; p50 1.27-1.31 s for
    // all three).  Once trial
    // blocks per real collision have been measured, every electron of the epoch gets about the
    // same number of trial blocks: a request whose gas makes many null trials per real
    // collision gets fewer real collisions, so that its electrons do not keep the device
    // running for the others' tail.  A request without a measurement yet is given the largest
    // cost measured, which bounds the tail its first epoch can make.
    int64_t electrons = 0;
    double worst = 0.0;
    for (auto& r : act) { electrons += r->n_e; worst = std::max(worst, r->cost); }
    const int64_t q_fixed = s->p.quantum_collisions;
    const double blocks_per_electron = s->block_rate > 0 && worst > 0
        ? 0.1 * s->block_rate / static_cast<double>(std::max<int64_t>(1, electrons)) : 0.0;
    const int64_t q_rate = s->rate > 0 ? static_cast<int64_t>(0.1 * s->rate / std::max<int64_t>(1, electrons)) : 1000;
    for (auto& r : act) {
      int64_t q;
      if (q_fixed > 0) q = q_fixed;
      else if (blocks_per_electron > 0) q = static_cast<int64_t>(blocks_per_electron / (r->cost > 0 ? r->cost : worst));
      else q = q_rate;
      if (q_fixed <= 0) q = std::max<int64_t>(64, q);
      r->quantum = std::max<int64_t>(1, std::min<int64_t>(q, r->n_c - r->done_coll));   // no electron needs more
    }
    descs.clear();
    std::vector<int64_t> ne, nc;
    int G = 0, n_ch = 0;
    bool magnetic = false;
    int extended = 0;
    for (auto& r : act) {
      InstanceDesc d = r->h->desc;
      d.quantum = static_cast<uint32_t>(std::min<int64_t>(r->quantum, 0xffffffffLL));
      descs.push_back(d);
      ne.push_back(r->n_e);
      // the items' order and sizes follow the expected device work per electron (longest
      // first), not the collision count: with per-request quanta the requests with the
      // fewest collisions per epoch are the slowest ones
      const double c_r = r->cost > 0 ? r->cost : worst > 0 ? worst : 1.0;
      nc.push_back(std::max<int64_t>(1, std::llround(16.0 * c_r * static_cast<double>(r->quantum))));
      G = std::max(G, d.G);
      n_ch = std::max(n_ch, d.nc);
      magnetic |= r->h->has_b;
      extended = std::max(extended, d.thermal_targets || d.relativistic ? 2 : d.trial_strategy != SWARM_TRIAL_CONSTANT ? 1 : 0);
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);   // swarm_server_poll reads the count
      for (auto& r : act) r->epochs += 1;
    }
    const swarm_launch_opts o = resolve_opts(&s->p.opts, s->p.precision);
    const LdsLayout ll = lds_layout(s->p.precision, G, n_ch, o.service_waves, o.table_layout);
    const size_t lds = ll.bytes;
    const int per_cu = swarm_kernel_max_blocks_per_cu(s->p.precision, magnetic, false, false, extended,
                                                      o.service_waves, o.block_size, lds);
    make_items(ne, nc, o.chunk, items, static_cast<int64_t>(device_info().n_cu) * per_cu, o.block_size);
    hipError_t e;
    bool ok = (e = s->descs.ensure(descs.size() * sizeof(InstanceDesc))) == hipSuccess &&
              (e = s->items.ensure(items.size() * sizeof(WorkItem) + 256)) == hipSuccess;
    int32_t* item_ctr = ok ? reinterpret_cast<int32_t*>(static_cast<char*>(s->items.p) + items.size() * sizeof(WorkItem)) : nullptr;
    if (ok) ok = (e = hipMemcpyAsync(s->descs.p, descs.data(), descs.size() * sizeof(InstanceDesc), hipMemcpyHostToDevice, s->compute)) == hipSuccess &&
                 (e = hipMemcpyAsync(s->items.p, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, s->compute)) == hipSuccess &&
                 (e = launch_fill_u32(reinterpret_cast<uint32_t*>(item_ctr), 0u, 1, s->compute)) == hipSuccess &&
                 (e = hipEventRecord(ev0, s->compute)) == hipSuccess;
    if (ok && ++s->epoch == s->fail_epoch) {
      // failure injection (tests of the error path): nothing is launched
      ok = false;
      e = hipErrorLaunchFailure;
    }
    if (ok) {
      const int grid = std::max(1, std::min<int>(static_cast<int>(items.size()), device_info().n_cu * per_cu));
      ok = (e = launch_swarm_dummy(static_cast<const InstanceDesc*>(s->descs.p), static_cast<const WorkItem*>(s->items.p),
                                   static_cast<int32_t>(items.size()), item_ctr, s->p.precision, magnetic, false, extended,
                                   o.service_waves, o.block_size, grid, o.pending_trigger, lds, ll.ch_off,
                                   ll.pool_off, ll.cum_off, s->compute)) == hipSuccess &&
           (e = hipEventRecord(ev1, s->compute)) == hipSuccess;
    }
    // while the epoch runs, prepare the requests that arrived meanwhile
    if (ok) admit_pending(s);
    // Requests measured after this epoch: on their epochs 1, 2, 4, 8, ... (their cost settles
    // as their electrons relax from the initial energy), by one reduction over their state.
    std::vector<size_t> meas;
    for (size_t i = 0; i < act.size(); ++i)
      if ((act[i]->epochs & (act[i]->epochs - 1)) == 0) meas.push_back(i);
    std::vector<unsigned long long> parts(meas.size() * kEpochBlocksParts);
    if (ok && !meas.empty()) {
      std::vector<InstanceDesc> md;
      for (size_t i : meas) md.push_back(descs[i]);
      ok = (e = s->mdescs.ensure(md.size() * sizeof(InstanceDesc))) == hipSuccess &&
           (e = s->mparts.ensure(parts.size() * sizeof(unsigned long long))) == hipSuccess &&
           (e = hipMemcpyAsync(s->mdescs.p, md.data(), md.size() * sizeof(InstanceDesc), hipMemcpyHostToDevice, s->compute)) == hipSuccess &&
           (e = launch_epoch_blocks(static_cast<const InstanceDesc*>(s->mdescs.p), static_cast<int>(md.size()),
                                    static_cast<unsigned long long*>(s->mparts.p), s->compute)) == hipSuccess &&
           (e = hipMemcpyAsync(parts.data(), s->mparts.p, parts.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s->compute)) == hipSuccess;
    }
    std::vector<RunCounters> hc(s->max_slots);
    if (ok) ok = (e = hipMemcpyAsync(hc.data(), s->ctrs.p, s->max_slots * sizeof(RunCounters), hipMemcpyDeviceToHost, s->compute)) == hipSuccess &&
                 (e = hipStreamSynchronize(s->compute)) == hipSuccess;
    if (!ok) {
      // The device state of every admitted request is suspect: all of them fail, including
      // those the schedule left out of this epoch and those admitted while it ran.
      (void)hip_fail(e, "serving epoch");
      std::vector<std::shared_ptr<Request>> failed;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        failed.swap(s->active);
      }
      for (auto& r : failed) finish(s, r, SWARM_ERR_DEVICE);
      continue;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev0, ev1);
    // finished requests: tallies on the device, then release
    std::vector<std::shared_ptr<Request>> fin;
    std::vector<int64_t> fin_n;
    std::vector<InstanceDesc> fin_desc;
    int64_t work = 0;
    for (size_t i = 0; i < act.size(); ++i) {
      const int64_t done_now = static_cast<int64_t>(hc[act[i]->slot].n_done);
      work += act[i]->quantum * act[i]->n_e;
      if (done_now >= act[i]->n_e) {
        fin.push_back(act[i]);
        fin_n.push_back(act[i]->n_e);
        fin_desc.push_back(descs[i]);
      }
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (auto& r : act) {
        // every unfinished electron of the request made exactly the epoch's quantum (or the
        // rest of its budget): the progress is exact at epoch boundaries
        const int64_t nd = std::min<int64_t>(r->n_c, r->done_coll + r->quantum);
        s->work_done += r->n_e * (nd - r->done_coll);
        r->done_coll = nd;
      }
      ++s->n_epochs;
      // the measured requests' cost: blocks drawn per real collision since their last
      // measurement, plus the collision's own work
      for (size_t j = 0; j < meas.size(); ++j) {
        Request& r = *act[meas[j]];
        unsigned long long total = 0;
        for (int k = 0; k < kEpochBlocksParts; ++k) total += parts[j * kEpochBlocksParts + k];
        const double db = static_cast<double>(total - r.blocks_seen);
        const double made = static_cast<double>(r.n_e) * static_cast<double>(r.done_coll - r.coll_seen);
        if (made > 0 && total > r.blocks_seen) r.cost = db / made + kCollisionBlocks;
        r.blocks_seen = total;
        r.coll_seen = r.done_coll;
      }
    }
    if (ms > 0) {
      const double r_now = static_cast<double>(work) / (ms * 1e-3);
      s->rate = s->rate > 0 ? 0.5 * s->rate + 0.5 * r_now : r_now;
      // device work of the epoch in trial blocks, from the requests' costs as now measured
      double units = 0.0, worst_now = 0.0;
      for (auto& r : act) worst_now = std::max(worst_now, r->cost);
      for (auto& r : act)
        units += static_cast<double>(r->quantum) * static_cast<double>(r->n_e) * (r->cost > 0 ? r->cost : worst_now);
      const double b_now = units / (ms * 1e-3);
      if (b_now > 0) s->block_rate = s->block_rate > 0 ? 0.5 * s->block_rate + 0.5 * b_now : b_now;
    }
    if (!fin.empty()) {
      DevBuf fd;
      fd.arena = s->mem.get();
      ok = (e = fd.ensure(fin_desc.size() * sizeof(InstanceDesc))) == hipSuccess &&
           (e = hipMemcpyAsync(fd.p, fin_desc.data(), fin_desc.size() * sizeof(InstanceDesc), hipMemcpyHostToDevice, s->compute)) == hipSuccess &&
           (e = s->tally.prepare(fin_n, s->compute)) == hipSuccess &&
           (e = s->tally.launch(static_cast<const InstanceDesc*>(fd.p), s->compute)) == hipSuccess;
      std::vector<swarm_tallies_t> out(fin.size());
      if (ok) ok = (e = hipMemcpyAsync(out.data(), s->tally.d_out.p, out.size() * sizeof(swarm_tallies_t), hipMemcpyDeviceToHost, s->compute)) == hipSuccess &&
                   (e = hipStreamSynchronize(s->compute)) == hipSuccess;
      for (auto& r : fin)
        if (ok && r->records_out)
          ok = (e = hipMemcpyAsync(r->records_out, r->h->records.p, static_cast<size_t>(r->n_e) * sizeof(swarm_record),
                                   hipMemcpyDeviceToHost, s->compute)) == hipSuccess &&
               (e = hipStreamSynchronize(s->compute)) == hipSuccess;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& r : fin) s->active.erase(std::find(s->active.begin(), s->active.end(), r));
      }
      for (size_t i = 0; i < fin.size(); ++i) {
        if (ok) fin[i]->tallies = out[i];
        else (void)hip_fail(e, "serving tallies");
        finish(s, fin[i], ok ? SWARM_OK : SWARM_ERR_DEVICE);
      }
    }
  }
  // Stopped (swarm_server_destroy): the running epoch has ended; every request not yet
  // finished is cancelled and releases its memory.
  std::vector<std::shared_ptr<Request>> left;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    left.swap(s->active);
    left.insert(left.end(), s->pending.begin(), s->pending.end());
    s->pending.clear();
  }
  for (auto& r : left) finish(s, r, SWARM_ERR_STATE);
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
}

}  // namespace

namespace {

swarm_status server_create(const swarm_server_params* p, void* arena, int64_t arena_bytes, swarm_server_t* out) {
  if (!p || !out) return fail(SWARM_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (p->hbm_budget_bytes <= 0) return fail(SWARM_ERR_INVALID_ARG, "hbm budget must be > 0");
  if (p->precision != SWARM_FP64 && p->precision != SWARM_FP32_MIXED) return fail(SWARM_ERR_INVALID_ARG, "bad precision");
  if (p->quantum_collisions < 0) return fail(SWARM_ERR_INVALID_ARG, "quantum must be >= 0");
  if (p->schedule != SWARM_SCHEDULE_ALL && p->schedule != SWARM_SCHEDULE_SHORTEST_FIRST)
    return fail(SWARM_ERR_INVALID_ARG, "schedule must be SWARM_SCHEDULE_ALL or SWARM_SCHEDULE_SHORTEST_FIRST");
  auto s = std::make_unique<swarm_server>();
  s->p = *p;
  s->budget = p->hbm_budget_bytes;
  if (arena) {
    s->mem = std::make_unique<Arena>(arena, static_cast<size_t>(arena_bytes));
    s->budget = std::min<int64_t>(s->budget, static_cast<int64_t>(s->mem->capacity()));
    for (DevBuf* b : {&s->ctrs, &s->descs, &s->items, &s->mdescs, &s->mparts}) b->arena = s->mem.get();
    s->tally.bind(s->mem.get());
  }
  s->t0 = std::chrono::steady_clock::now();
  if (const char* f = std::getenv("SWARM_SERVER_FAIL_EPOCH")) s->fail_epoch = std::atoll(f);
  s->max_slots = p->max_active > 0 ? p->max_active : 1024;
  hipError_t e;
  if (p->stream) s->compute = static_cast<hipStream_t>(p->stream);
  else if ((e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
  if ((e = hipStreamCreateWithFlags(&s->setup, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
  if ((e = s->ctrs.ensure(s->max_slots * sizeof(RunCounters))) != hipSuccess) return hip_fail(e, "counters");
  for (int i = s->max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  swarm_server* raw = s.get();
  s->th = std::thread([raw] { scheduler(raw); });
  *out = s.release();
  return SWARM_OK;
}

}  // namespace

extern "C" {

swarm_status swarm_server_create(const swarm_server_params* p, swarm_server_t* out) {
  return server_create(p, nullptr, 0, out);
}

swarm_status swarm_server_create_in_arena(const swarm_server_params* p, void* arena, int64_t arena_bytes,
                                          swarm_server_t* out) {
  if (!arena || arena_bytes <= 0) return fail(SWARM_ERR_INVALID_ARG, "arena must be a device pointer with bytes > 0");
  return server_create(p, arena, arena_bytes, out);
}

swarm_status swarm_server_submit(swarm_server_t s, const swarm_component* comps, int32_t n_comps,
                                 const swarm_params* params, int64_t n_electrons, int64_t n_collisions,
                                 uint64_t seed, int64_t* ticket) {
  return swarm_server_submit_records(s, comps, n_comps, params, n_electrons, n_collisions, seed, nullptr, ticket);
}

swarm_status swarm_server_submit_records(swarm_server_t s, const swarm_component* comps, int32_t n_comps,
                                         const swarm_params* params, int64_t n_electrons, int64_t n_collisions,
                                         uint64_t seed, swarm_record* records_out, int64_t* ticket) {
  if (!s || !comps || !params || !ticket) return fail(SWARM_ERR_INVALID_ARG, "NULL argument");
  if (params->secondaries != SWARM_DUMMY) return fail(SWARM_ERR_INVALID_ARG, "serving takes dummy-secondaries requests");
  if (n_electrons < 1) return fail(SWARM_ERR_INVALID_ARG, "n_electrons must be >= 1");
  if (n_collisions < 1 || n_collisions > 0xffffffffLL) return fail(SWARM_ERR_INVALID_ARG, "bad n_collisions");
  auto r = std::make_shared<Request>();
  for (int k = 0; k < n_comps; ++k) {
    ComponentCopy c;
    c.mass = comps[k].mass_amu;
    c.frac = comps[k].fraction;
    c.scattering = comps[k].scattering;
    c.mt_over_el = comps[k].mt_over_el;
    for (int j = 0; j < comps[k].n_channels && comps[k].channels; ++j) {
      const swarm_channel& q = comps[k].channels[j];
      ChannelCopy ch;
      ch.kind = q.kind;
      ch.thr = q.threshold_eV;
      if (q.n_points > 0 && q.energy_eV && q.sigma_m2) {
        ch.e.assign(q.energy_eV, q.energy_eV + q.n_points);
        ch.s.assign(q.sigma_m2, q.sigma_m2 + q.n_points);
      }
      c.ch.push_back(std::move(ch));
    }
    r->comps.push_back(std::move(c));
  }
  r->params = *params;
  r->params.stream = nullptr;
  r->n_e = n_electrons;
  r->n_c = n_collisions;
  r->seed = seed;
  r->records_out = records_out;
  {
    // device memory while admitted: the tables exactly as swarm_create allocates them, then
    // records and resumable state (256-byte blocks)
    swarm_params p = *params;
    p.precision = s->p.precision;
    p.secondaries = SWARM_DUMMY;
    const int64_t tables = static_cast<int64_t>(create_bytes(comps, n_comps, &p));
    r->need = (tables > 0 ? tables + 256 : request_bytes(*r)) +
              ((r->n_e * static_cast<int64_t>(sizeof(swarm_record)) + 255) & ~int64_t(255)) +
              ((r->n_e * static_cast<int64_t>(sizeof(SavedState)) + 255) & ~int64_t(255));
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->submit_s = s->now();
    s->pending.push_back(r);
    s->all[r->ticket] = r;
    ++s->n_unfinished;
    *ticket = r->ticket;
  }
  s->cv.notify_all();
  return SWARM_OK;
}

swarm_status swarm_server_poll(swarm_server_t s, int64_t ticket, swarm_tallies_t* out, swarm_request_info* info) {
  if (!s) return fail(SWARM_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return fail(SWARM_ERR_INVALID_ARG, "unknown ticket %lld", static_cast<long long>(ticket));
  const Request& r = *it->second;
  if (info) {
    info->submit_s = r.submit_s;
    info->admit_s = r.admit_s;
    info->done_s = r.done_s;
    info->n_real = r.status == SWARM_OK ? r.tallies.n_real : 0;
    info->epochs = r.epochs;
    info->bytes = r.bytes;
    info->progress = r.n_e * r.done_coll;
    info->blocks_per_real = r.cost > 0 ? r.cost - kCollisionBlocks : 0.0;
  }
  if (r.status == SWARM_PENDING) return SWARM_PENDING;
  if (r.status != SWARM_OK) return fail(r.status, "request %lld failed", static_cast<long long>(ticket));
  if (out) *out = r.tallies;
  return SWARM_OK;
}

swarm_status swarm_server_drain(swarm_server_t s) {
  if (!s) return fail(SWARM_ERR_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->n_unfinished == 0; });
  return SWARM_OK;
}

double swarm_server_now(swarm_server_t s) { return s ? s->now() : 0.0; }

swarm_status swarm_server_stats(swarm_server_t s, swarm_server_stats_t* out) {
  if (!s || !out) return fail(SWARM_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  swarm_server_stats_t t{};
  t.time_s = s->now();
  t.n_submitted = s->next_ticket - 1;
  t.n_pending = static_cast<int64_t>(s->pending.size());
  t.n_active = static_cast<int64_t>(s->active.size());
  t.n_finished = s->n_ok;
  t.n_failed = s->n_failed;
  t.bytes_in_use = s->used_bytes;
  t.work_done = s->work_done;
  for (const auto& r : s->pending) t.work_left += r->n_e * r->n_c;
  for (const auto& r : s->active) t.work_left += r->n_e * (r->n_c - r->done_coll);
  t.epochs = s->n_epochs;
  *out = t;
  return SWARM_OK;
}

void swarm_server_destroy(swarm_server_t s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  for (auto& kv : s->all) {
    if (kv.second->h) swarm_destroy(kv.second->h);
    kv.second->h = nullptr;
  }
  if (s->setup) (void)hipStreamDestroy(s->setup);
  if (!s->p.stream && s->compute) (void)hipStreamDestroy(s->compute);
  delete s;
}

}  // extern "C"
