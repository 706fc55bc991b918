// Internal structures shared by the host runtime (swarm_api.cpp) and the device code
// (swarm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/swarm.h"

namespace swarm_impl {

constexpr int kMaxTraceIds = 256;
constexpr int kTallyTile = 2048;          // records per tally work-group (fixed: determinism)
constexpr int kTallyThreads = 256;
constexpr int kTally1 = 26;               // pass-1 accumulators
constexpr int kTally2 = 32;               // pass-2 accumulators
constexpr uint32_t kMaxBlocks = 0x7fffffffu;   // per-electron cap on trial blocks

// Lane states of the swarm kernels.
// ACTIVE: drawing trials; READY: holds a real-collision candidate (served with the wave's
// other READY lanes, which draw their scattering words then); IDLE: needs an electron; WAIT:
// pooled schedule, has its candidate in the work-group pool; CAND: pooled schedule, holds a
// candidate not yet in the pool; STOPPED: must store its record or state; DONE: no more work.
enum : int { ST_ACTIVE = 0, ST_IDLE = 2, ST_WAIT = 3, ST_DONE = 4, ST_STOPPED = 5, ST_READY = 6,
             ST_CAND = 7 };

// Per-channel constants built on the device from the raw inputs.
struct ChannelDev {
  int32_t kind;
  int32_t comp;
  double thr;      // threshold (eV)
  double onset;    // thr * (m+M)/M: lowest energy at which the inelastic process is allowed
  double c_ela;    // 2 m M / (m+M)^2
  double c_M;      // M / (m+M)
  double c_mM;     // (m+M) / M
  float thr_f, c_ela_f, c_M_f, c_mM_f;
  int32_t scat;    // swarm_scattering of its component
  float xi_f;
  double xi;       // SWARM_SCATTER_CONSTANT_XI: the anisotropy parameter
};

// Per-channel constants of moving targets, kept out of ChannelDev (which the kernels copy
// from LDS into registers) and read from global memory only at such collisions.
struct ThermalChannel {
  double mass;     // target mass M (kg)
  double sigma;    // sqrt(k T / M), spread of each target velocity component
  double loss;     // 2 eps_k M / ((m + M) m): the threshold in |V1 - Vcm|^2
  double cM;       // M / (m + M): V1 - Vcm = (M / (m + M)) (V1 - V2)
};

// Saved electron state at a real-collision boundary (serving epochs resume from it).
struct SavedState {
  double r[3], t;
  double v[3];
  double sum_eps, sum_epsp;
  uint64_t id;
  uint32_t block, k, k_start, G, D, n_forb, n_over, n_first;
  uint32_t started, pad;
  double nup;                 // trial frequency in use (variable strategy)
  uint32_t grace, n_fail;     // trials left before its next update; fails so far
};

// Real-secondaries runs: an electron a launch parked at a real-collision boundary (its
// resumable state and its record slot), to be resumed by the next launch together with the
// secondaries the launch created.
struct ParkedState {
  SavedState s;
  int64_t rec;
};

// A wave parks only when at most park_lanes of its 64 lanes still run (by default
// kParkLanes), and at most once per launch, so a launch of `threads` threads writes at most
// parked_capacity(threads, park_lanes) states.
constexpr int kParkLanes = 32;
constexpr int64_t parked_capacity(int64_t threads, int park_lanes) { return threads / 64 * park_lanes + 64; }

// Secondary electron in the real-secondaries queue, written by the generation that
// created it and run by the next one.
struct ChildState {
  double r[3], t;
  double v[3];
  uint64_t id;
  uint32_t k, pad;
  double eps_birth;           // energy it was created with (eV), for its first trial frequency
};

// Device counters of one instance's run.  The counters that real-mode waves update
// concurrently sit on 128-byte lines of their own, so their atomics do not queue behind
// each other.
struct RunCounters {
  uint64_t gen_next;      // real mode: electrons of the running generation taken so far
  uint64_t pad0[15];
  uint64_t child_tail;    // real mode: reserved secondary slots
  uint64_t pad1[15];
  uint64_t dropped;       // secondaries that did not fit the capacity
  uint64_t n_done;        // dummy mode: electrons that reached their final collision or stopped
  uint64_t parked;        // real mode: electrons the running launch parked for the next one
  uint64_t pad2[13];
};

// One swarm instance as seen by the kernels.  Fields in the first group are written by
// the host (pointers, sizes, run parameters); the physics constants in the second group
// are computed by the build kernels from the raw inputs.
struct InstanceDesc {
  // ---- host-written ----------------------------------------------------------------
  int32_t G, nc, p_log2, emin, emax;
  int32_t n_raw_channels;
  int32_t precision, secondaries;
  double E, B, B_angle, N, eps0, user_majorant;
  double T_K;                 // gas temperature (moving targets)
  int32_t thermal_targets;    // 1: moving targets
  int32_t relativistic;       // 1: relativistic mover (FP64, B = 0)
  int32_t trial_strategy;     // swarm_trial_strategy
  uint32_t trial_grace;       // variable and binned: trials between updates of nu'
  double trial_zeta;          // variable: nu' = (1 + zeta) nu(eps)
  int32_t trial_bins;         // binned: bins per decade
  int32_t n_bins;             // binned: number of bins (0 for the other strategies)
  const int32_t* bin_of;      // binned: bin of every entry of the padded rate table (G + 1)
  const int32_t* bin_first;   // binned: first table entry of every bin (n_bins + 1)
  const double* logtab;       // FP64 flight times: the logarithm table (unit_log.hpp)
  const double* raw_e;        // concatenated raw energies
  const double* raw_s;        // concatenated raw cross-sections
  const int32_t* raw_off;     // per channel: first point
  const int32_t* raw_n;       // per channel: number of points
  const int32_t* raw_kind;
  const int32_t* raw_comp;
  const double* raw_thr;
  const double* comp_mass_amu;
  const double* comp_frac;
  const int32_t* comp_scat;   // swarm_scattering per component
  const double* comp_ratio;   // sigma_mt / sigma_el per component
  double* nodes;              // G node energies (eV)
  double* cum_cm;             // nc x G running sums, channel major (FP64)
  double2* nu64;              // G pairs (F, F[g+1]-F[g]) of the total rate
  float2* nu32;
  double2* cum64;             // (G+1) x nc pairs, node major (row 0: below the grid), + 8 spare
  float2* cum32;
  ChannelDev* chan;
  ThermalChannel* chan_th;    // moving targets: per-channel constants (nc)
  double* bin_nup64;          // binned: nu' of every bin (built on the device)
  float* bin_nup32;
  // run parameters
  int64_t n_electrons;
  uint32_t n_collisions;
  uint32_t quantum;           // real collisions per electron per launch (0 = no limit)
  uint64_t seed;
  int64_t capacity;           // real mode: records available
  swarm_record* records;      // per-electron results
  SavedState* saved;          // resumable runs (serving); NULL otherwise
  ChildState* children;       // real mode queue
  RunCounters* ctr;
  // tracing
  const uint64_t* trace_ids;
  int32_t n_trace, max_events;
  swarm_event* trace_out;
  int32_t* trace_count;
  // ---- device-written (build kernels) ------------------------------------------------
  double majorant, inv_majorant;
  double c_eps;               // m / (2 e): eps (eV) = c_eps |v|^2
  double c_speed;             // sqrt(2 e / m): |v| = c_speed sqrt(eps)
  double speed0;
  double az;                  // -e E / m (acceleration along z)
  double omega;               // e B / m
  double bx, bz;              // unit vector of B
  double vDy;                 // E x B / B^2 = (0, E sin(th) / B, 0)
  double apar;                // a . b
  double numax;
  float majorant_f, cT_f;     // cT_f = ln2 / nu' (flight time from log2)
  float c_eps_f, c_speed_f, speed0_f, az_f, omega_rev_f, bx_f, bz_f, vDy_f, apar_f;
  float sceps_f, aze_f, apare_f, nup24_f, Pf_f, twoPf_f;   // FP32 energy-unit constants
  double Pf_d, twoPf_d;
  double rel_kEc, rel_kBx, rel_kBz;       // relativistic mover in E and B: generator and
  double rel_l1, rel_l2, rel_p1, rel_p2, rel_K;   // field invariants
  int32_t built_ok;           // 1 after a successful build, -1 if a node has zero rate
  int32_t pad_;
};

struct WorkItem {
  int32_t inst;
  int32_t pad;
  int64_t first;       // first electron index of the item
  int64_t count;       // electrons in the item
};

struct TallyTile {
  int32_t inst;
  int32_t tile;        // tile index within the instance
  int64_t first;
  int64_t count;
};

// Launchers implemented in swarm_kernels.hip.
hipError_t launch_build(InstanceDesc* d_desc, const InstanceDesc& h_desc, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_mark_empty(swarm_record* r, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);
// service_waves > 0 (and no trace): the pooled schedule, pool at LDS offset pool_off.
hipError_t launch_swarm_dummy(const InstanceDesc* d_desc, const WorkItem* d_items, int32_t n_items,
                              int32_t* d_item_counter, int precision, bool has_b, bool trace,
                              int ext, int service_waves, int block_size, int grid, int pending_trigger,
                              size_t lds_bytes, int ch_off, int pool_off, int cum_off, hipStream_t s);
size_t swarm_pool_slot_bytes(int precision);
// One real-secondaries launch: the n_park_in electrons in park_in (parked by the launch
// before), then `count` electrons from `first` (the primaries if first < 0, else queued
// secondaries).  Once every electron is claimed, a wave left with few running lanes parks
// them in park_out (at their next real-collision boundary) and ends, provided this launch has
// created at least park_min secondaries (the queue started at tail0): the next launch runs
// them together; park_lanes is the most running lanes a parking wave may have.  park_min <= 0
// parks nothing.
hipError_t launch_swarm_real(const InstanceDesc* d_desc, int precision, bool has_b, bool trace,
                             int ext, int block_size, int grid, int pending_trigger, size_t lds_bytes,
                             int ch_off, int cum_off, int64_t first, int64_t count, int flush,
                             const ParkedState* park_in, int64_t n_park_in, ParkedState* park_out,
                             int64_t park_min, int park_lanes, int64_t tail0, hipStream_t s);
hipError_t launch_tallies(const InstanceDesc* d_desc, const TallyTile* d_tiles, int32_t n_tiles,
                          const int32_t* d_tile_base, const int64_t* d_nrec, int32_t n_inst,
                          double* d_part1, double* d_part2, double* d_tot1,
                          swarm_tallies_t* d_out, hipStream_t s);
int swarm_kernel_max_blocks_per_cu(int precision, bool has_b, bool trace, bool real, int ext,
                                   int service_waves, int block_size,
                                   size_t lds_bytes);

}  // namespace swarm_impl
