// Host runtime of libswarm: argument validation, device memory, kernel launches, hipGraph
// capture of batched launches, the launch-shape autotuner and the C ABI of swarm.h.
// No method arithmetic happens here: tables, physics constants, the simulation and the
// tallies are all computed by the kernels in swarm_kernels.hip.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "swarm_api_internal.hpp"
#include "unit_log.hpp"

using namespace swarm_impl;

namespace swarm_impl {

thread_local std::string g_last_error;

swarm_status fail(swarm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

swarm_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? SWARM_ERR_OUT_OF_MEMORY : SWARM_ERR_DEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

DeviceInfo& device_info() {
  static DeviceInfo info = [] {
    DeviceInfo d{};
    if (hipGetDevice(&d.device) != hipSuccess) d.device = 0;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, d.device) == hipSuccess) {
      d.n_cu = p.multiProcessorCount;
      d.lds_per_block = static_cast<int64_t>(p.sharedMemPerBlock);
    } else {
      d.n_cu = 256;
      d.lds_per_block = 65536;
    }
    return d;
  }();
  return info;
}

// Dynamic LDS of the swarm kernels: the total-rate pairs of the G grid nodes plus one
// padding entry in front, then (16-byte aligned) the nc channel descriptors, then with table
// layout 1 the (G+1) x nc running-sum pairs (if everything fits the work-group's LDS), then with
// the pooled schedule the candidate pool (64 slots per service wave).
LdsLayout lds_layout(int precision, int G, int nc, int service_waves, int table_layout) {
  auto al = [](size_t n) { return (n + 15) & ~static_cast<size_t>(15); };
  const size_t pair = precision == SWARM_FP32_MIXED ? sizeof(float2) : sizeof(double2);
  const size_t pool = service_waves > 0 ? static_cast<size_t>(64 * service_waves) * swarm_pool_slot_bytes(precision) : 0;
  LdsLayout l;
  l.ch_off = static_cast<int>(al(static_cast<size_t>(G + 1) * pair));
  const size_t after_ch = al(static_cast<size_t>(l.ch_off) + static_cast<size_t>(nc) * sizeof(ChannelDev));
  l.cum_off = -1;
  l.pool_off = static_cast<int>(after_ch);
  if (table_layout == 1) {
    const size_t with_cum = al(after_ch + (static_cast<size_t>(G + 1) * static_cast<size_t>(nc) + 8) * pair);
    if (static_cast<int64_t>(with_cum + pool) <= device_info().lds_per_block) {
      l.cum_off = static_cast<int>(after_ch);
      l.pool_off = static_cast<int>(with_cum);
    }
  }
  l.bytes = static_cast<size_t>(l.pool_off) + pool;
  return l;
}

constexpr size_t kArenaAlign = 256;

Arena::Arena(void* base, size_t bytes) {
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  const uintptr_t a = (b + kArenaAlign - 1) & ~static_cast<uintptr_t>(kArenaAlign - 1);
  const size_t lost = static_cast<size_t>(a - b);
  base_ = reinterpret_cast<char*>(a);
  bytes_ = bytes > lost ? ((bytes - lost) & ~(kArenaAlign - 1)) : 0;
  if (bytes_ > 0) free_[0] = bytes_;
}

void* Arena::alloc(size_t n) {
  const size_t want = std::max(kArenaAlign, (n + kArenaAlign - 1) & ~(kArenaAlign - 1));
  std::lock_guard<std::mutex> lk(mu_);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < want) continue;
    const size_t off = it->first, size = it->second;
    free_.erase(it);
    if (size > want) free_[off + want] = size - want;
    used_[off] = want;
    in_use_ += want;
    return base_ + off;
  }
  return nullptr;
}

void Arena::release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  auto u = used_.find(static_cast<size_t>(static_cast<char*>(p) - base_));
  if (u == used_.end()) return;
  size_t off = u->first, size = u->second;
  used_.erase(u);
  in_use_ -= size;
  auto next = free_.lower_bound(off);
  if (next != free_.end() && off + size == next->first) {   // merge with the block after
    size += next->second;
    next = free_.erase(next);
  }
  if (next != free_.begin()) {                               // and with the block before
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += size;
      return;
    }
  }
  free_[off] = size;
}

size_t Arena::in_use() const {
  std::lock_guard<std::mutex> lk(mu_);
  return in_use_;
}

DevBuf::~DevBuf() { reset(); }
void DevBuf::reset() {
  if (p) {
    if (arena) arena->release(p);
    else (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
}
hipError_t DevBuf::ensure(size_t n) {
  if (n <= bytes && p) return hipSuccess;
  reset();
  if (n == 0) return hipSuccess;
  if (arena) {
    p = arena->alloc(n);
    if (!p) return hipErrorOutOfMemory;
  } else {
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
  }
  bytes = n;
  return hipSuccess;
}

size_t tally_bytes(int64_t n_records) {
  auto blk = [](size_t n) { return std::max(kArenaAlign, (n + kArenaAlign - 1) & ~(kArenaAlign - 1)); };
  const size_t tiles = static_cast<size_t>(std::max<int64_t>(1, (n_records + kTallyTile - 1) / kTallyTile));
  return blk(tiles * sizeof(TallyTile)) + blk(sizeof(int32_t)) + blk(sizeof(int64_t)) +
         blk(tiles * kTally1 * sizeof(double)) + blk(tiles * kTally2 * sizeof(double)) +
         blk((kTally1 + kTally2) * sizeof(double)) + blk(sizeof(swarm_tallies_t));
}

}  // namespace swarm_impl

namespace {

// Bins of the binned trial frequency (BinnedTrialFrequency, section "Trial frequency
// strategies"): b per decade of energy, bin k = [10^(k/b), 10^((k+1)/b)) eV, counted from the
// bin of the lowest grid node.  A grid cell belongs to the bin of its lower node.  The table
// is indexed like the padded rate table of the kernels: entry 0 (below the grid) belongs to
// node 0, entry g + 1 to node g (its cell, or for the top node the energies above it).
// Bins are numbered from 0 to the top node's bin; on a coarse grid some hold no node (their
// nu' is 0 and only the range maximum after a fail visits them).  Entries first[k] ..
// first[k+1] - 1 are those of bin k (an empty range for an empty bin); first[n_bins] = G + 1.
// Node energies are exact (a power of two times 1 + i/P); 1, 10, 100 and 1000 eV are nodes,
// and log10 returns their exact logarithms, so those nodes open their bins.
void decade_bins(int P, int emin, int G, int b, std::vector<int32_t>& entry_bin, std::vector<int32_t>& first) {
  auto bin = [&](int g) {
    const double e = std::ldexp(1.0 + static_cast<double>(g % P) / P, emin + g / P);
    return static_cast<int32_t>(std::floor(std::log10(e) * b));
  };
  const int32_t k0 = bin(0);
  entry_bin.assign(G + 1, 0);
  for (int i = 1; i <= G; ++i) entry_bin[i] = bin(i - 1) - k0;
  const int nb = entry_bin[G] + 1;
  first.assign(nb + 1, G + 1);
  for (int i = G; i >= 0; --i) first[entry_bin[i]] = i;
  for (int k = nb - 1; k >= 0; --k) first[k] = std::min(first[k], first[k + 1]);
}

swarm_status busy() {
  return fail(SWARM_ERR_STATE, "a run started by swarm_run_async is in flight: call swarm_wait first");
}

swarm_status validate(const swarm_component* comps, int32_t n_comps, const swarm_params* p) {
  if (!comps || n_comps <= 0) return fail(SWARM_ERR_INVALID_ARG, "need at least one component");
  if (!p) return fail(SWARM_ERR_INVALID_ARG, "params is NULL");
  if (!(p->N_per_m3 > 0.0) || !std::isfinite(p->N_per_m3)) return fail(SWARM_ERR_INVALID_ARG, "N must be > 0");
  if (!(p->E_V_per_m >= 0.0) || !std::isfinite(p->E_V_per_m)) return fail(SWARM_ERR_INVALID_ARG, "E must be >= 0");
  if (!(p->B_T >= 0.0) || !std::isfinite(p->B_T)) return fail(SWARM_ERR_INVALID_ARG, "B must be >= 0");
  if (!std::isfinite(p->B_angle_rad)) return fail(SWARM_ERR_INVALID_ARG, "B angle must be finite");
  if (!(p->init_energy_eV >= 0.0) || !std::isfinite(p->init_energy_eV))
    return fail(SWARM_ERR_INVALID_ARG, "initial energy must be >= 0");
  if (p->precision != SWARM_FP64 && p->precision != SWARM_FP32_MIXED)
    return fail(SWARM_ERR_INVALID_ARG, "unknown precision %d", p->precision);
  if (p->secondaries != SWARM_DUMMY && p->secondaries != SWARM_REAL)
    return fail(SWARM_ERR_INVALID_ARG, "unknown secondaries mode %d", p->secondaries);
  if (!(p->user_majorant >= 0.0) || !std::isfinite(p->user_majorant))
    return fail(SWARM_ERR_INVALID_ARG, "user majorant must be >= 0");
  if (p->capacity < 0) return fail(SWARM_ERR_INVALID_ARG, "capacity must be >= 0");
  if (p->trial_strategy != SWARM_TRIAL_CONSTANT && p->trial_strategy != SWARM_TRIAL_VARIABLE &&
      p->trial_strategy != SWARM_TRIAL_BINNED)
    return fail(SWARM_ERR_INVALID_ARG, "unknown trial strategy %d", p->trial_strategy);
  if (p->trial_strategy == SWARM_TRIAL_VARIABLE) {
    if (!(p->trial_zeta >= 0.0) || !std::isfinite(p->trial_zeta))
      return fail(SWARM_ERR_INVALID_ARG, "trial zeta must be finite and > 0 (0 = default)");
  }
  if (p->trial_strategy != SWARM_TRIAL_CONSTANT && (p->trial_grace < 0 || p->trial_grace > 0x7fffffffLL))
    return fail(SWARM_ERR_INVALID_ARG, "trial grace must be in [1, 2^31 - 1] (0 = default)");
  if (p->trial_strategy == SWARM_TRIAL_BINNED && (p->trial_bins < 0 || p->trial_bins > 100))
    return fail(SWARM_ERR_INVALID_ARG, "trial bins per decade must be in [1, 100] (0 = default)");
  if (p->thermal_targets != 0 && p->thermal_targets != 1)
    return fail(SWARM_ERR_INVALID_ARG, "thermal_targets must be 0 or 1");
  if (p->thermal_targets && (!(p->T_K >= 0.0) || !std::isfinite(p->T_K)))
    return fail(SWARM_ERR_INVALID_ARG, "moving targets need a gas temperature T_K >= 0");
  if (p->relativistic != 0 && p->relativistic != 1) return fail(SWARM_ERR_INVALID_ARG, "relativistic must be 0 or 1");
  if (p->relativistic && p->thermal_targets)
    return fail(SWARM_ERR_INVALID_ARG, "the relativistic mover does not take moving targets");
  if (p->relativistic && p->precision != SWARM_FP64)
    return fail(SWARM_ERR_INVALID_ARG, "the relativistic mover runs in SWARM_FP64");
  const int P = p->grid_points_per_octave ? p->grid_points_per_octave : 64;
  if (P <= 0 || P > 1024 || (P & (P - 1)) != 0)
    return fail(SWARM_ERR_INVALID_ARG, "grid points per octave must be a power of two <= 1024");
  int emin = p->grid_min_exp2, emax = p->grid_max_exp2;
  if (emin == 0 && emax == 0) { emin = -14; emax = 12; }
  if (emax <= emin || emin < -60 || emax > 60) return fail(SWARM_ERR_INVALID_ARG, "bad grid exponent range");
  double fsum = 0.0;
  int nc = 0;
  for (int k = 0; k < n_comps; ++k) {
    const swarm_component& c = comps[k];
    if (!(c.mass_amu > 0.0) || !std::isfinite(c.mass_amu))
      return fail(SWARM_ERR_INVALID_ARG, "component %d: mass must be > 0", k);
    if (!(c.fraction >= 0.0) || !std::isfinite(c.fraction))
      return fail(SWARM_ERR_INVALID_ARG, "component %d: fraction must be >= 0", k);
    if (c.n_channels <= 0 || !c.channels) return fail(SWARM_ERR_INVALID_ARG, "component %d: no channels", k);
    if (c.scattering < SWARM_SCATTER_ISOTROPIC || c.scattering > SWARM_SCATTER_CONSTANT_XI)
      return fail(SWARM_ERR_INVALID_ARG, "component %d: unknown scattering %d", k, c.scattering);
    if (c.scattering == SWARM_SCATTER_CONSTANT_XI && !(c.mt_over_el > 0.0 && c.mt_over_el <= 1.0))
      return fail(SWARM_ERR_INVALID_ARG, "component %d: sigma_mt/sigma_el must be in (0, 1]", k);
    fsum += c.fraction;
    for (int j = 0; j < c.n_channels; ++j) {
      const swarm_channel& q = c.channels[j];
      if (q.kind < 0 || q.kind > 3) return fail(SWARM_ERR_INVALID_ARG, "component %d channel %d: bad kind", k, j);
      if (!(q.threshold_eV >= 0.0) || !std::isfinite(q.threshold_eV))
        return fail(SWARM_ERR_INVALID_ARG, "component %d channel %d: threshold must be >= 0", k, j);
      if (q.n_points < 2 || !q.energy_eV || !q.sigma_m2)
        return fail(SWARM_ERR_INVALID_ARG, "component %d channel %d: need >= 2 points", k, j);
      for (int i = 0; i < q.n_points; ++i) {
        if (!(q.energy_eV[i] > 0.0) || !std::isfinite(q.energy_eV[i]))
          return fail(SWARM_ERR_INVALID_ARG, "component %d channel %d: energies must be > 0 and finite", k, j);
        if (!(q.sigma_m2[i] >= 0.0) || !std::isfinite(q.sigma_m2[i]))
          return fail(SWARM_ERR_INVALID_ARG, "component %d channel %d: cross-sections must be >= 0 and finite", k, j);
        if (i > 0 && !(q.energy_eV[i] > q.energy_eV[i - 1]))
          return fail(SWARM_ERR_INVALID_ARG, "component %d channel %d: energies must increase strictly", k, j);
      }
      ++nc;
    }
  }
  if (std::fabs(fsum - 1.0) > 1e-9) return fail(SWARM_ERR_INVALID_ARG, "fractions sum to %.12g, not 1", fsum);
  if (nc > 4096) return fail(SWARM_ERR_INVALID_ARG, "too many channels (%d > 4096)", nc);
  return SWARM_OK;
}

hipError_t sync_desc_to_device(swarm* h) {
  return hipMemcpyAsync(h->d_desc, &h->desc, sizeof(InstanceDesc), hipMemcpyHostToDevice, h->stream);
}

// Tally tiles of a set of instances with known record counts.
void make_tiles(const std::vector<int64_t>& nrec, std::vector<TallyTile>& tiles, std::vector<int32_t>& base) {
  tiles.clear();
  base.assign(nrec.size(), 0);
  int32_t b = 0;
  for (size_t i = 0; i < nrec.size(); ++i) {
    base[i] = b;
    const int64_t nt = (nrec[i] + kTallyTile - 1) / kTallyTile;
    for (int64_t t = 0; t < nt; ++t) {
      TallyTile tt;
      tt.inst = static_cast<int32_t>(i);
      tt.tile = static_cast<int32_t>(t);
      tt.first = t * kTallyTile;
      tt.count = std::min<int64_t>(kTallyTile, nrec[i] - tt.first);
      tiles.push_back(tt);
    }
    b += static_cast<int32_t>(nt);
  }
}

}  // namespace

namespace swarm_impl {

hipError_t TallyPlan::prepare(const std::vector<int64_t>& nrec, hipStream_t s) {
  std::vector<TallyTile> tiles;
  std::vector<int32_t> base;
  make_tiles(nrec, tiles, base);
  n_inst = static_cast<int32_t>(nrec.size());
  n_tiles = static_cast<int32_t>(tiles.size());
  hipError_t e;
  if ((e = d_tiles.ensure(std::max<size_t>(1, tiles.size()) * sizeof(TallyTile))) != hipSuccess) return e;
  if ((e = d_base.ensure(base.size() * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = d_nrec.ensure(nrec.size() * sizeof(int64_t))) != hipSuccess) return e;
  if ((e = d_part1.ensure(std::max<size_t>(1, tiles.size()) * kTally1 * sizeof(double))) != hipSuccess) return e;
  if ((e = d_part2.ensure(std::max<size_t>(1, tiles.size()) * kTally2 * sizeof(double))) != hipSuccess) return e;
  if ((e = d_tot.ensure(nrec.size() * (kTally1 + kTally2) * sizeof(double))) != hipSuccess) return e;
  if ((e = d_out.ensure(nrec.size() * sizeof(swarm_tallies_t))) != hipSuccess) return e;
  h_tiles = tiles;
  h_base = base;
  h_nrec = nrec;
  if (!tiles.empty() && (e = hipMemcpyAsync(d_tiles.p, h_tiles.data(), tiles.size() * sizeof(TallyTile),
                                            hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_base.p, h_base.data(), base.size() * sizeof(int32_t), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(d_nrec.p, h_nrec.data(), nrec.size() * sizeof(int64_t), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t TallyPlan::launch(const InstanceDesc* d_descs, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  return launch_tallies(d_descs, static_cast<const TallyTile*>(d_tiles.p), n_tiles,
                        static_cast<const int32_t*>(d_base.p), static_cast<const int64_t*>(d_nrec.p), n_inst,
                        static_cast<double*>(d_part1.p), static_cast<double*>(d_part2.p),
                        static_cast<double*>(d_tot.p), static_cast<swarm_tallies_t*>(d_out.p), s);
}

// Work items: instances with the largest collision budgets first (or the largest `rank`, the
// expected device work per electron, where the caller measured it), so that the long items
// start early and the persistent grid drains evenly.  An item holds up to `chunk` electrons;
// when `slots` (resident work-groups) is given, an instance's items are cut smaller, down to
// one electron per lane (`block`), so that no item holds much more than 1/slots of the
// launch's work (electrons x collisions) and a small launch still spreads over the whole GPU.
void make_items(const std::vector<int64_t>& n_e, const std::vector<int64_t>& n_c, int64_t chunk,
                std::vector<WorkItem>& items, int64_t slots, int64_t block, const std::vector<double>* rank) {
  items.clear();
  std::vector<int> order(n_e.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
  if (rank) std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return (*rank)[a] > (*rank)[b]; });
  else std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n_c[a] > n_c[b]; });
  double total = 0.0;
  for (size_t i = 0; i < n_e.size(); ++i) total += static_cast<double>(n_e[i]) * static_cast<double>(n_c[i]);
  // Guided sizes: the last part of the work (about one item of two electrons per lane for
  // every resident work-group) is cut into small items, so the launch ends on a fine tail,
  // while the items before it keep `chunk` electrons (fewer item boundaries, at each of which
  // a work-group waits for its slowest lane).  On the argon sweep (32 x 1e5 x 2e4, items of
  // eight electrons per lane) this gave 835 ms per FP32 step against 893 ms without the
  // small tail, and FP64 2413 ms against 2450 ms.
  double n_all = 0.0;
  for (size_t i = 0; i < n_e.size(); ++i) n_all += static_cast<double>(n_e[i]);
  const int64_t small = block > 0 ? 2 * block : chunk;
  const double tail = (slots > 0 && block > 0 && n_all > 0.0)
                          ? std::min(0.5 * total, static_cast<double>(slots) * static_cast<double>(small) * total / n_all)
                          : 0.0;
  double left = total;
  for (int i : order) {
    int64_t ch = chunk;
    if (slots > 0 && block > 0 && n_c[i] > 0) {
      const double want = total / static_cast<double>(slots) / static_cast<double>(n_c[i]);
      const int64_t w = (static_cast<int64_t>(std::min(want, 1e15)) + block - 1) / block * block;
      ch = std::max(block, std::min(chunk, w));
    }
    for (int64_t f = 0; f < n_e[i];) {
      const int64_t c = left <= tail ? std::min(ch, small) : ch;
      WorkItem w;
      w.inst = i;
      w.pad = 0;
      w.first = f;
      w.count = std::min<int64_t>(c, n_e[i] - f);
      items.push_back(w);
      f += w.count;
      left -= static_cast<double>(w.count) * static_cast<double>(n_c[i]);
    }
  }
}

// Default launch shape (the autotuner's pick on MI355X for the argon-like sweep, probed with
// a fifth of the collision budget): work-groups of 256, items of 4 electrons per lane in FP32
// and 8 in FP64.  Against 128 lanes and 3 per lane the FP32 step went 833 -> 789 ms, and FP64
// with 8 per lane 2409 -> 2131 ms (32 x 1e5 x 2e4).
int default_block(int) { return 256; }

swarm_launch_opts resolve_opts(const swarm_launch_opts* o, int precision) {
  swarm_launch_opts r{};
  r.block_size = (o && o->block_size) ? o->block_size : default_block(precision);
  // electrons per lane and work item: FP32 4, FP64 8 (measured on the argon sweep, the
  // 256-instance batch and serving: small items balance uneven work; the slower FP64 lanes
  // lose more to the wait for the slowest lane at every item boundary)
  r.chunk = (o && o->chunk) ? o->chunk : r.block_size * (precision == SWARM_FP64 ? 8 : 4);
  r.pending_trigger = (o && o->pending_trigger) ? o->pending_trigger : 32;
  r.use_graph = o ? o->use_graph : 0;
  r.block_size = std::max(64, std::min(1024, (r.block_size / 64) * 64));
  r.chunk = std::max(r.block_size, (r.chunk / r.block_size) * r.block_size);
  r.pending_trigger = std::max(1, std::min(64, r.pending_trigger));
  r.service_waves = o ? std::max(0, std::min(r.block_size / 64 - 1, o->service_waves)) : 0;
  r.table_layout = (o && o->table_layout == 1) ? 1 : 0;
  r.park_lanes = (o && o->park_lanes) ? std::max(-1, std::min(64, o->park_lanes)) : kParkLanes;
  return r;
}

}  // namespace swarm_impl

// =======================================================================================
// Single-instance API
// =======================================================================================
namespace swarm_impl {

// Validation, table build and constants of a new handle.  With bytes_only set, only the
// device bytes the handle's tables need are computed (nothing is allocated or launched).
static swarm_status build_swarm(swarm* h, const swarm_component* comps, int32_t n_comps,
                                const swarm_params* params, size_t* bytes_only) {
  swarm_status st = validate(comps, n_comps, params);
  if (st != SWARM_OK) return st;
  h->params = *params;
  // Flatten the raw tables (argument marshalling only).
  std::vector<double> e_all, s_all, thr, mass, frac, ratio;
  std::vector<int32_t> off, npt, kind, comp, scat;
  for (int k = 0; k < n_comps; ++k) {
    mass.push_back(comps[k].mass_amu);
    frac.push_back(comps[k].fraction);
    scat.push_back(comps[k].scattering);
    ratio.push_back(comps[k].scattering == SWARM_SCATTER_CONSTANT_XI ? comps[k].mt_over_el : 1.0);
    for (int j = 0; j < comps[k].n_channels; ++j) {
      const swarm_channel& q = comps[k].channels[j];
      off.push_back(static_cast<int32_t>(e_all.size()));
      npt.push_back(q.n_points);
      kind.push_back(q.kind);
      comp.push_back(k);
      thr.push_back(q.threshold_eV);
      e_all.insert(e_all.end(), q.energy_eV, q.energy_eV + q.n_points);
      s_all.insert(s_all.end(), q.sigma_m2, q.sigma_m2 + q.n_points);
      h->kinds.push_back(q.kind);
    }
  }
  const int nc = static_cast<int>(off.size());
  const int P = params->grid_points_per_octave ? params->grid_points_per_octave : 64;
  int emin = params->grid_min_exp2, emax = params->grid_max_exp2;
  if (emin == 0 && emax == 0) { emin = -14; emax = 12; }
  int p_log2 = 0;
  while ((1 << p_log2) < P) ++p_log2;
  const int G = (emax - emin) * P + 1;
  InstanceDesc& d = h->desc;
  std::memset(&d, 0, sizeof(d));
  d.G = G; d.nc = nc; d.p_log2 = p_log2; d.emin = emin; d.emax = emax; d.n_raw_channels = nc;
  d.precision = params->precision; d.secondaries = params->secondaries;
  d.E = params->E_V_per_m; d.B = params->B_T; d.B_angle = params->B_angle_rad; d.N = params->N_per_m3;
  d.eps0 = params->init_energy_eV; d.user_majorant = params->user_majorant;
  d.T_K = params->T_K; d.thermal_targets = params->thermal_targets; d.relativistic = params->relativistic;
  d.trial_strategy = params->trial_strategy;
  d.trial_zeta = params->trial_zeta > 0.0 ? params->trial_zeta : 0.25;
  d.trial_grace = static_cast<uint32_t>(params->trial_grace > 0 ? params->trial_grace : 5000);
  d.trial_bins = params->trial_bins > 0 ? params->trial_bins : 10;
  std::vector<int32_t> entry_bin, bin_first;
  if (params->trial_strategy == SWARM_TRIAL_BINNED) decade_bins(P, emin, G, d.trial_bins, entry_bin, bin_first);
  d.n_bins = entry_bin.empty() ? 0 : static_cast<int32_t>(bin_first.size()) - 1;
  h->has_b = params->B_T > 0.0;
  // one arena for the raw inputs and the tables
  auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
  const size_t b_e = al(e_all.size() * 8), b_s = b_e, b_i = al(nc * 4), b_cd = al(nc * 8), b_k = al(n_comps * 8);
  const size_t b_nodes = al(static_cast<size_t>(G) * 8);
  const size_t b_cm = al(static_cast<size_t>(G) * nc * 8);
  const size_t b_nu64 = al(static_cast<size_t>(G) * 16), b_nu32 = al(static_cast<size_t>(G) * 8);
  // running sums, node major, padded with a row in front (below the grid), with spare pairs
  // after the last row (the channel search reads a whole row of up to 8 pairs at once)
  const size_t b_c64 = al((static_cast<size_t>(G + 1) * nc + 8) * 16), b_c32 = al((static_cast<size_t>(G + 1) * nc + 8) * 8);
  const size_t b_ch = al(nc * sizeof(ChannelDev)), b_th = al(nc * sizeof(ThermalChannel));
  const size_t b_eb = al(entry_bin.size() * 4), b_bf = al(bin_first.size() * 4);
  const size_t b_bn = al(static_cast<size_t>(d.n_bins) * 8), b_bn32 = al(static_cast<size_t>(d.n_bins) * 4);
  std::vector<double> logtab(kUnitLogStride * kUnitLogEntries);
  unit_log_table(logtab.data());
  const size_t b_lt = al(logtab.size() * 8);
  const size_t total = b_e + b_s + 4 * b_i + b_cd + 4 * b_k + b_nodes + b_cm + b_nu64 + b_nu32 + b_c64 + b_c32 + b_ch +
                       b_th + b_eb + b_bf + b_bn + b_bn32 + b_lt + al(sizeof(InstanceDesc)) + al(sizeof(RunCounters));
  if (bytes_only) {
    *bytes_only = total;
    return SWARM_OK;
  }
  if (params->stream) {
    h->stream = static_cast<hipStream_t>(params->stream);
    h->own_stream = false;
  } else {
    hipError_t es = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (es != hipSuccess) return hip_fail(es, "hipStreamCreate");
    h->own_stream = true;
  }
  hipError_t e = h->arena.ensure(total);
  if (e != hipSuccess) return hip_fail(e, "allocating instance tables");
  char* base = static_cast<char*>(h->arena.p);
  size_t o = 0;
  auto take = [&](size_t n) { char* r = base + o; o += n; return r; };
  double* d_e = reinterpret_cast<double*>(take(b_e));
  double* d_s = reinterpret_cast<double*>(take(b_s));
  int32_t* d_off = reinterpret_cast<int32_t*>(take(b_i));
  int32_t* d_n = reinterpret_cast<int32_t*>(take(b_i));
  int32_t* d_kind = reinterpret_cast<int32_t*>(take(b_i));
  int32_t* d_comp = reinterpret_cast<int32_t*>(take(b_i));
  double* d_thr = reinterpret_cast<double*>(take(b_cd));
  double* d_mass = reinterpret_cast<double*>(take(b_k));
  double* d_frac = reinterpret_cast<double*>(take(b_k));
  int32_t* d_scat = reinterpret_cast<int32_t*>(take(b_k));
  double* d_ratio = reinterpret_cast<double*>(take(b_k));
  d.nodes = reinterpret_cast<double*>(take(b_nodes));
  d.cum_cm = reinterpret_cast<double*>(take(b_cm));
  d.nu64 = reinterpret_cast<double2*>(take(b_nu64));
  d.nu32 = reinterpret_cast<float2*>(take(b_nu32));
  d.cum64 = reinterpret_cast<double2*>(take(b_c64));
  d.cum32 = reinterpret_cast<float2*>(take(b_c32));
  d.chan = reinterpret_cast<ChannelDev*>(take(b_ch));
  d.chan_th = reinterpret_cast<ThermalChannel*>(take(b_th));
  int32_t* d_entry_bin = reinterpret_cast<int32_t*>(take(b_eb));
  int32_t* d_bin_first = reinterpret_cast<int32_t*>(take(b_bf));
  d.bin_of = d_entry_bin;
  d.bin_first = d_bin_first;
  d.bin_nup64 = reinterpret_cast<double*>(take(b_bn));
  d.bin_nup32 = reinterpret_cast<float*>(take(b_bn32));
  double* d_logtab = reinterpret_cast<double*>(take(b_lt));
  d.logtab = d_logtab;
  h->d_desc = reinterpret_cast<InstanceDesc*>(take(al(sizeof(InstanceDesc))));
  d.ctr = reinterpret_cast<RunCounters*>(take(al(sizeof(RunCounters))));
  d.raw_e = d_e; d.raw_s = d_s; d.raw_off = d_off; d.raw_n = d_n; d.raw_kind = d_kind;
  d.raw_comp = d_comp; d.raw_thr = d_thr; d.comp_mass_amu = d_mass; d.comp_frac = d_frac;
  d.comp_scat = d_scat; d.comp_ratio = d_ratio;
  hipStream_t s = h->stream;
#define CP(dst, v) if ((e = hipMemcpyAsync(dst, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e, "copying tables");
  CP(d_e, e_all) CP(d_s, s_all) CP(d_off, off) CP(d_n, npt) CP(d_kind, kind) CP(d_comp, comp)
  CP(d_thr, thr) CP(d_mass, mass) CP(d_frac, frac) CP(d_scat, scat) CP(d_ratio, ratio)
  if (!entry_bin.empty()) { CP(d_entry_bin, entry_bin) CP(d_bin_first, bin_first) }
  CP(d_logtab, logtab)
#undef CP
  if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(d.ctr), 0, sizeof(RunCounters) / 8, s)) != hipSuccess)
    return hip_fail(e, "clearing counters");
  if ((e = sync_desc_to_device(h)) != hipSuccess) return hip_fail(e, "copying descriptor");
  if ((e = launch_build(h->d_desc, d, s)) != hipSuccess) return hip_fail(e, "table build launch");
  if ((e = hipMemcpyAsync(&h->desc, h->d_desc, sizeof(InstanceDesc), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_fail(e, "reading descriptor");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "table build");
  if (h->desc.built_ok == -1)
    return fail(SWARM_ERR_INVALID_ARG, "the total collision frequency vanishes on part of the energy grid");
  if (h->desc.built_ok == -2)
    return fail(SWARM_ERR_INVALID_ARG, "user trial frequency %.6g is below the maximum collision frequency %.6g",
                params->user_majorant, h->desc.numax);
  if (h->desc.built_ok != 1) return fail(SWARM_ERR_DEVICE, "table build did not complete");
  for (int i = 0; i < 3; ++i)
    if ((e = hipEventCreate(&h->ev[i])) != hipSuccess) return hip_fail(e, "hipEventCreate");
  // Single runs default to work-groups of 128: a run of one swarm often holds fewer electrons
  // than the GPU has lanes, and the smaller groups spread it over more CUs (32 single FP64
  // runs of the argon sweep, 1e5 electrons each: 1.21e10 real/s with 128, 1.07e10 with 256).
  swarm_launch_opts single{};
  single.block_size = 128;
  h->opts = resolve_opts(&single, params->precision);
  return SWARM_OK;
}

swarm_status create_swarm(const swarm_component* comps, int32_t n_comps, const swarm_params* params,
                          Arena* mem, swarm_t* out) {
  if (!out) return fail(SWARM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  auto h = std::make_unique<swarm>();
  if (mem) h->bind_arena(mem);
  const swarm_status st = build_swarm(h.get(), comps, n_comps, params, nullptr);
  if (st != SWARM_OK) {
    const std::string msg = g_last_error;
    swarm_destroy(h.release());
    g_last_error = msg;
    return st;
  }
  *out = h.release();
  return SWARM_OK;
}

size_t create_bytes(const swarm_component* comps, int32_t n_comps, const swarm_params* params) {
  swarm h;
  size_t bytes = 0;
  if (build_swarm(&h, comps, n_comps, params, &bytes) != SWARM_OK) return 0;
  return bytes;
}

}  // namespace swarm_impl

extern "C" {

const char* swarm_strerror(swarm_status s) {
  switch (s) {
    case SWARM_OK: return "ok";
    case SWARM_ERR_INVALID_ARG: return "invalid argument";
    case SWARM_ERR_OUT_OF_MEMORY: return "out of memory";
    case SWARM_ERR_CAPACITY: return "capacity exceeded";
    case SWARM_ERR_DEVICE: return "device error";
    case SWARM_ERR_STATE: return "invalid state";
    case SWARM_PENDING: return "pending";
  }
  return "unknown status";
}

const char* swarm_last_error(void) { return g_last_error.c_str(); }

swarm_status swarm_create(const swarm_component* comps, int32_t n_comps, const swarm_params* params,
                          swarm_t* out) {
  return create_swarm(comps, n_comps, params, nullptr, out);
}

swarm_status swarm_create_in_arena(const swarm_component* comps, int32_t n_comps, const swarm_params* params,
                                   void* arena, int64_t arena_bytes, swarm_t* out) {
  if (!out) return fail(SWARM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!arena || arena_bytes <= 0) return fail(SWARM_ERR_INVALID_ARG, "arena must be a device pointer with bytes > 0");
  auto mem = std::make_unique<Arena>(arena, static_cast<size_t>(arena_bytes));
  swarm_t h = nullptr;
  const swarm_status st = create_swarm(comps, n_comps, params, mem.get(), &h);
  if (st != SWARM_OK) return st;
  h->own_mem = std::move(mem);
  *out = h;
  return SWARM_OK;
}

swarm_status swarm_arena_bytes(const swarm_component* comps, int32_t n_comps, const swarm_params* params,
                               int64_t n_electrons, int64_t* bytes) {
  if (!bytes) return fail(SWARM_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = 0;
  if (n_electrons < 1) return fail(SWARM_ERR_INVALID_ARG, "n_electrons must be >= 1");
  const size_t tables = create_bytes(comps, n_comps, params);
  if (tables == 0) return SWARM_ERR_INVALID_ARG;     // validation failed; the message is set
  auto blk = [](size_t n) { return (n + 2 * 256 - 1) & ~static_cast<size_t>(255); };   // block + alignment
  const bool real = params->secondaries == SWARM_REAL;
  const int64_t capacity = real ? (params->capacity ? params->capacity : 64 * n_electrons) : n_electrons;
  size_t run = blk(static_cast<size_t>(capacity) * sizeof(swarm_record)) + tally_bytes(capacity);
  if (real && capacity > n_electrons) run += blk(static_cast<size_t>(capacity - n_electrons) * sizeof(ChildState));
  // real mode: the two buffers of parked electrons, for the most lanes a device can hold
  if (real) run += blk(2 * static_cast<size_t>(parked_capacity(static_cast<int64_t>(device_info().n_cu) * 2048, 64)) * sizeof(ParkedState));
  // dummy-mode work items: at most one per 64 electrons (the smallest work-group), plus the counter
  if (!real) run += blk(static_cast<size_t>((n_electrons + 63) / 64) * sizeof(WorkItem) + 256);
  *bytes = static_cast<int64_t>(blk(tables) + run);
  return SWARM_OK;
}

void swarm_destroy(swarm_t h) {
  if (!h) return;
  if (h->worker.joinable()) h->worker.join();
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (int i = 0; i < 3; ++i)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

swarm_status swarm_set_trace(swarm_t h, const uint64_t* ids, int32_t n_ids, int32_t max_events) {
  if (!h) return fail(SWARM_ERR_INVALID_ARG, "handle is NULL");
  if (h->in_flight) return busy();
  if (n_ids < 0 || n_ids > kMaxTraceIds) return fail(SWARM_ERR_INVALID_ARG, "n_ids must be in [0, %d]", kMaxTraceIds);
  if (n_ids > 0 && (!ids || max_events <= 0 || max_events > 4096))
    return fail(SWARM_ERR_INVALID_ARG, "max_events must be in [1, 4096]");
  h->n_trace = n_ids;
  h->max_events = n_ids ? max_events : 0;
  if (n_ids == 0) return SWARM_OK;
  hipError_t e;
  if ((e = h->trace_ids.ensure(n_ids * sizeof(uint64_t))) != hipSuccess) return hip_fail(e, "trace ids");
  if ((e = h->trace_out.ensure(static_cast<size_t>(n_ids) * max_events * sizeof(swarm_event))) != hipSuccess)
    return hip_fail(e, "trace buffer");
  if ((e = h->trace_count.ensure(n_ids * sizeof(int32_t))) != hipSuccess) return hip_fail(e, "trace counts");
  if ((e = hipMemcpyAsync(h->trace_ids.p, ids, n_ids * sizeof(uint64_t), hipMemcpyHostToDevice, h->stream)) != hipSuccess)
    return hip_fail(e, "trace ids");
  if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_fail(e, "trace ids");
  return SWARM_OK;
}

swarm_status swarm_set_launch_opts(swarm_t h, const swarm_launch_opts* opts) {
  if (!h) return fail(SWARM_ERR_INVALID_ARG, "NULL handle");
  if (h->in_flight) return busy();
  h->opts = resolve_opts(opts, h->desc.precision);
  return SWARM_OK;
}

}  // extern "C"

namespace {

// A run up to the point where everything is on the stream: records, counters, the swarm
// kernel (dummy mode: one launch; real mode: the generations, which need the host between
// launches and therefore wait for each), then the tally reductions.  Nothing waits for the
// dummy-mode work, so swarm_run_async returns while it runs.  A capacity overflow is kept
// in run_status: its tallies are still reduced.
swarm_status run_start(swarm_t h, int64_t n_electrons, int64_t n_collisions, uint64_t seed) {
  if (n_electrons < 1) return fail(SWARM_ERR_INVALID_ARG, "n_electrons must be >= 1");
  if (n_collisions < 1 || n_collisions > 0xffffffffLL)
    return fail(SWARM_ERR_INVALID_ARG, "n_collisions must be in [1, 2^32-1]");
  h->run_status = SWARM_OK;
  h->run_error.clear();
  h->noalloc_records = false;
  const bool real = h->desc.secondaries == SWARM_REAL;
  int64_t capacity = n_electrons;
  if (real) {
    capacity = h->params.capacity ? h->params.capacity : 64 * n_electrons;
    if (capacity < n_electrons) return fail(SWARM_ERR_INVALID_ARG, "capacity below n_electrons");
  }
  hipStream_t s = h->stream;
  hipError_t e;
  h->have_run = false;
  if ((e = h->records.ensure(static_cast<size_t>(capacity) * sizeof(swarm_record))) != hipSuccess)
    return hip_fail(e, "allocating records");
  InstanceDesc& d = h->desc;
  d.n_electrons = n_electrons;
  d.n_collisions = static_cast<uint32_t>(n_collisions);
  d.quantum = 0;
  d.seed = seed;
  d.capacity = capacity;
  d.records = static_cast<swarm_record*>(h->records.p);
  d.saved = nullptr;
  d.children = nullptr;
  const int64_t child_cap = capacity - n_electrons;
  if (real && child_cap > 0) {
    if ((e = h->children.ensure(static_cast<size_t>(child_cap) * sizeof(ChildState))) != hipSuccess)
      return hip_fail(e, "allocating secondary queue");
    d.children = static_cast<ChildState*>(h->children.p);
  }
  if (real && (e = launch_mark_empty(d.records, capacity, s)) != hipSuccess) return hip_fail(e, "clearing records");
  const bool trace = h->n_trace > 0;
  d.trace_ids = trace ? static_cast<const uint64_t*>(h->trace_ids.p) : nullptr;
  d.n_trace = h->n_trace;
  d.max_events = h->max_events;
  d.trace_out = trace ? static_cast<swarm_event*>(h->trace_out.p) : nullptr;
  d.trace_count = trace ? static_cast<int32_t*>(h->trace_count.p) : nullptr;
  if (trace && (e = launch_fill_u32(reinterpret_cast<uint32_t*>(d.trace_count), 0u, h->n_trace, s)) != hipSuccess)
    return hip_fail(e, "clearing trace counts");
  // counters: all zero
  if ((e = launch_fill_u64(reinterpret_cast<uint64_t*>(d.ctr), 0ull, sizeof(RunCounters) / sizeof(uint64_t), s)) != hipSuccess)
    return hip_fail(e, "counters");
  if ((e = sync_desc_to_device(h)) != hipSuccess) return hip_fail(e, "descriptor");
  const swarm_launch_opts& o = h->opts;
  const int svc = trace || real ? 0 : o.service_waves;
  const LdsLayout ll = lds_layout(d.precision, d.G, d.nc, svc, o.table_layout);
  if (static_cast<int64_t>(ll.bytes) > device_info().lds_per_block)
    return fail(SWARM_ERR_INVALID_ARG, "the tables need %zu bytes of LDS per work-group, the device has %lld",
                ll.bytes, static_cast<long long>(device_info().lds_per_block));
  const size_t lds = ll.bytes;
  const int ch_off = ll.ch_off;
  DeviceInfo& dev = device_info();
  const int ext = d.thermal_targets || d.relativistic ? 2 : d.trial_strategy != SWARM_TRIAL_CONSTANT ? 1 : 0;
  const int per_cu = swarm_kernel_max_blocks_per_cu(d.precision, h->has_b, trace, real, ext, svc, o.block_size, lds);
  if ((e = hipEventRecord(h->ev[0], s)) != hipSuccess) return hip_fail(e, "event");
  if (!real) {
    // enough work items to give every resident work-group several of them
    const int64_t slots = static_cast<int64_t>(dev.n_cu) * per_cu;
    int64_t chunk = (n_electrons + 4 * slots - 1) / (4 * slots);
    chunk = ((chunk + o.block_size - 1) / o.block_size) * o.block_size;
    chunk = std::max<int64_t>(o.block_size, std::min<int64_t>(chunk, o.chunk));
    std::vector<WorkItem> items;
    make_items({n_electrons}, {n_collisions}, chunk, items, 0, 0);
    if ((e = h->items.ensure(items.size() * sizeof(WorkItem) + 256)) != hipSuccess) return hip_fail(e, "work items");
    h->h_items = items;
    int32_t* d_ctr = reinterpret_cast<int32_t*>(static_cast<char*>(h->items.p) + items.size() * sizeof(WorkItem));
    if ((e = hipMemcpyAsync(h->items.p, h->h_items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, s)) != hipSuccess)
      return hip_fail(e, "work items");
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(d_ctr), 0u, 1, s)) != hipSuccess) return hip_fail(e, "item counter");
    const int grid = std::max(1, std::min<int>(static_cast<int>(items.size()), dev.n_cu * per_cu));
    if ((e = launch_swarm_dummy(h->d_desc, static_cast<const WorkItem*>(h->items.p), static_cast<int32_t>(items.size()),
                                d_ctr, d.precision, h->has_b, trace, ext, svc, o.block_size, grid, o.pending_trigger, lds, ch_off,
                                ll.pool_off, ll.cum_off, s)) != hipSuccess)
      return hip_fail(e, "swarm kernel launch");
    h->n_launches = 1;
    h->n_parked = 0;
  }
  RunCounters hc{};
  if (real) {
    // One launch per generation: the primaries, then the secondaries each generation
    // appended to the queue (slots [first, first + count)), until a generation creates none.
    // Every generation starts at least one collision later in its lineage budget than the
    // one before, so there are at most n_collisions + 1.  After an overflow the next launch
    // records the queued secondaries unstarted (flag 8) and creates none.  A launch that has
    // created secondaries for at least an eighth of the device's lanes lets its last few
    // running electrons park, and the next launch resumes them first (1e6 primaries of the
    // argon:CO2 mixture at 1 T: FP32 399 -> 372 ms, FP64 1004 -> 966 ms; waves of at most 16
    // running lanes parking after half a device of secondaries: 379 and 988 ms; 48 lanes after
    // a sixteenth: 384 and 960 ms).
    const int64_t lanes = static_cast<int64_t>(dev.n_cu) * per_cu * o.block_size;
    const int park_lanes = std::max(0, o.park_lanes);   // -1: never
    const int64_t park_cap = parked_capacity(lanes, park_lanes);
    if ((e = h->parked.ensure(2 * static_cast<size_t>(park_cap) * sizeof(ParkedState))) != hipSuccess)
      return hip_fail(e, "allocating parked electrons");
    ParkedState* park_in = static_cast<ParkedState*>(h->parked.p);
    ParkedState* park_out = park_in + park_cap;
    int64_t first = -1, count = n_electrons, queued = 0, n_parked = 0;
    h->n_launches = 0;
    h->n_parked = 0;
    for (;;) {
      if ((e = launch_fill_u64(&d.ctr->gen_next, 0ull, 1, s)) != hipSuccess) return hip_fail(e, "generation counter");
      if ((e = launch_fill_u64(&d.ctr->parked, 0ull, 1, s)) != hipSuccess) return hip_fail(e, "park counter");
      const int64_t want = (n_parked + count + o.block_size - 1) / o.block_size;
      const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want * 4, static_cast<int64_t>(dev.n_cu) * per_cu)));
      const int64_t park_min = hc.dropped != 0 || park_lanes == 0 ? 0 : std::max<int64_t>(1, lanes / 8);
      if ((e = launch_swarm_real(h->d_desc, d.precision, h->has_b, trace, ext, o.block_size, grid, o.pending_trigger, lds,
                                 ch_off, ll.cum_off, first, count, hc.dropped != 0 ? 1 : 0, park_in, n_parked, park_out,
                                 park_min, park_lanes, queued, s)) != hipSuccess)
        return hip_fail(e, "swarm kernel launch");
      h->n_launches += 1;
      if ((e = hipMemcpyAsync(&hc, d.ctr, sizeof(hc), hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "counters");
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "swarm kernel");
      const int64_t tail = std::min<int64_t>(static_cast<int64_t>(hc.child_tail), child_cap);
      if (tail == queued && hc.parked == 0) break;   // no secondary created, none parked
      first = queued;
      count = tail - queued;
      queued = tail;
      n_parked = std::min<int64_t>(static_cast<int64_t>(hc.parked),
                                   parked_capacity(static_cast<int64_t>(grid) * o.block_size, park_lanes));
      h->n_parked += n_parked;
      std::swap(park_in, park_out);
    }
  }
  if ((e = hipEventRecord(h->ev[1], s)) != hipSuccess) return hip_fail(e, "event");
  if (real) {
    if ((e = hipMemcpyAsync(&hc, d.ctr, sizeof(hc), hipMemcpyDeviceToHost, s)) != hipSuccess) return hip_fail(e, "counters");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "swarm kernel");
  }
  h->n_records = n_electrons + (real ? std::min<int64_t>(static_cast<int64_t>(hc.child_tail), child_cap) : 0);
  if ((e = h->tally.prepare({h->n_records}, s)) != hipSuccess) return hip_fail(e, "tally plan");
  if ((e = h->tally.launch(h->d_desc, s)) != hipSuccess) return hip_fail(e, "tally launch");
  if ((e = hipEventRecord(h->ev[2], s)) != hipSuccess) return hip_fail(e, "event");
  h->traced = trace;
  if (hc.dropped) {
    h->run_status = fail(SWARM_ERR_CAPACITY, "%llu secondaries did not fit the capacity of %lld electrons",
                         static_cast<unsigned long long>(hc.dropped), static_cast<long long>(capacity));
    h->run_error = g_last_error;
  }
  return SWARM_OK;
}

// Wait for the enqueued run, read its tallies and timings back.
swarm_status run_finish(swarm_t h) {
  hipError_t e;
  if ((e = hipEventSynchronize(h->ev[2])) != hipSuccess) return hip_fail(e, "swarm run");
  if ((e = hipMemcpyAsync(&h->tallies, h->tally.d_out.p, sizeof(swarm_tallies_t), hipMemcpyDeviceToHost,
                          h->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(h->stream)) != hipSuccess)
    return hip_fail(e, "tallies");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, h->ev[0], h->ev[1]);
  h->kernel_ms = ms;
  (void)hipEventElapsedTime(&ms, h->ev[0], h->ev[2]);
  h->total_ms = ms;
  h->have_run = true;
  if (h->run_status != SWARM_OK) g_last_error = h->run_error;
  return h->run_status;
}

}  // namespace

extern "C" {

swarm_status swarm_run(swarm_t h, int64_t n_electrons, int64_t n_collisions, uint64_t seed) {
  if (!h) return fail(SWARM_ERR_INVALID_ARG, "handle is NULL");
  if (h->in_flight) return busy();
  const swarm_status st = run_start(h, n_electrons, n_collisions, seed);
  if (st != SWARM_OK) return st;
  return run_finish(h);
}

swarm_status swarm_run_async(swarm_t h, int64_t n_electrons, int64_t n_collisions, uint64_t seed) {
  if (!h) return fail(SWARM_ERR_INVALID_ARG, "handle is NULL");
  if (h->in_flight) return busy();
  h->have_run = false;
  if (h->desc.secondaries == SWARM_REAL) {
    // the generations need the host between launches: they run on a worker thread
    if (n_electrons < 1 || n_collisions < 1 || n_collisions > 0xffffffffLL)
      return fail(SWARM_ERR_INVALID_ARG, "n_electrons must be >= 1 and n_collisions in [1, 2^32-1]");
    h->in_flight = 2;
    h->worker = std::thread([h, n_electrons, n_collisions, seed] {
      swarm_status st = run_start(h, n_electrons, n_collisions, seed);
      if (st == SWARM_OK) st = run_finish(h);
      h->async_status = st;
      h->async_error = st != SWARM_OK ? g_last_error : std::string();
    });
    return SWARM_OK;
  }
  const swarm_status st = run_start(h, n_electrons, n_collisions, seed);
  if (st != SWARM_OK) return st;
  h->in_flight = 1;
  return SWARM_OK;
}

swarm_status swarm_wait(swarm_t h) {
  if (!h) return fail(SWARM_ERR_INVALID_ARG, "handle is NULL");
  if (h->in_flight == 0) return fail(SWARM_ERR_STATE, "no run in flight");
  if (h->in_flight == 2) {
    h->worker.join();
    h->in_flight = 0;
    if (h->async_status != SWARM_OK) g_last_error = h->async_error;
    return h->async_status;
  }
  h->in_flight = 0;
  return run_finish(h);
}

swarm_status swarm_tallies(swarm_t h, swarm_tallies_t* out) {
  if (!h || !out) return fail(SWARM_ERR_INVALID_ARG, "NULL argument");
  if (h->in_flight) return busy();
  if (!h->have_run) return fail(SWARM_ERR_STATE, "no completed run");
  *out = h->tallies;
  return SWARM_OK;
}

swarm_status swarm_records(swarm_t h, swarm_record* out, int64_t max_records, int64_t* n_out) {
  if (!h || !n_out) return fail(SWARM_ERR_INVALID_ARG, "NULL argument");
  if (h->in_flight) return busy();
  if (h->noalloc_records) return fail(SWARM_ERR_STATE, "the last run wrote its records to caller memory");
  if (!h->have_run) return fail(SWARM_ERR_STATE, "no completed run");
  // Slots of secondaries that a run stopped early never simulated are empty (id all ones)
  // and are left out: *n_out counts the electrons that have a record.
  std::vector<swarm_record> all(static_cast<size_t>(h->n_records));
  if (h->n_records > 0) {
    hipError_t e = hipMemcpyAsync(all.data(), h->desc.records, all.size() * sizeof(swarm_record),
                                  hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "copying records");
  }
  int64_t n = 0;
  for (const swarm_record& r : all) {
    if (r.id == ~0ull) continue;
    if (out && n < max_records) out[n] = r;
    ++n;
  }
  *n_out = n;
  return SWARM_OK;
}

swarm_status swarm_trace_events(swarm_t h, swarm_event* out, int32_t* counts) {
  if (!h || !out || !counts) return fail(SWARM_ERR_INVALID_ARG, "NULL argument");
  if (h->in_flight) return busy();
  if (!h->have_run || !h->traced) return fail(SWARM_ERR_STATE, "no traced run");
  hipError_t e = hipMemcpyAsync(out, h->trace_out.p, static_cast<size_t>(h->n_trace) * h->max_events * sizeof(swarm_event),
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(counts, h->trace_count.p, h->n_trace * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "copying trace");
  return SWARM_OK;
}

swarm_status swarm_tables(swarm_t h, int32_t* grid_size, int32_t* n_channels, double* nodes, double* cum,
                          double* majorant) {
  if (!h) return fail(SWARM_ERR_INVALID_ARG, "handle is NULL");
  if (grid_size) *grid_size = h->desc.G;
  if (n_channels) *n_channels = h->desc.nc;
  if (majorant) *majorant = h->desc.majorant;
  hipError_t e = hipSuccess;
  if (nodes) e = hipMemcpyAsync(nodes, h->desc.nodes, h->desc.G * sizeof(double), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && cum)
    e = hipMemcpyAsync(cum, h->desc.cum_cm, static_cast<size_t>(h->desc.G) * h->desc.nc * sizeof(double),
                       hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "copying tables");
  return SWARM_OK;
}

swarm_status swarm_last_timing(swarm_t h, double* kernel_ms, double* total_ms) {
  if (!h) return fail(SWARM_ERR_INVALID_ARG, "handle is NULL");
  if (h->in_flight) return busy();
  if (!h->have_run) return fail(SWARM_ERR_STATE, "no completed run");
  if (kernel_ms) *kernel_ms = h->kernel_ms;
  if (total_ms) *total_ms = h->total_ms;
  return SWARM_OK;
}

swarm_status swarm_last_launches(swarm_t h, int64_t* launches, int64_t* parked) {
  if (!h) return fail(SWARM_ERR_INVALID_ARG, "handle is NULL");
  if (h->in_flight) return busy();
  if (!h->have_run) return fail(SWARM_ERR_STATE, "no completed run");
  if (launches) *launches = h->n_launches;
  if (parked) *parked = h->n_parked;
  return SWARM_OK;
}

}  // extern "C"
