/*
 * swarm.h -- C ABI of the MI355X (gfx950) electron-swarm library (libswarm.so).
 *
 * The library runs the Monte-Carlo swarm method of "Betaboltz: a Monte-Carlo simulation
 * tool for gas scattering processes" (Renda, Ciubotaru, Banu; arXiv 1901.08140) on the GPU:
 * electrons fly freely in static uniform E and B fields (section "Theoretical framework",
 * classical equations of motion), collide after flight times drawn against a constant
 * trial frequency nu' >= nu (eq. random_time, null-collision technique), are tested for a
 * real or null collision (eq. null_fraction) with the collision frequency of eq. frequency,
 * scatter isotropically with the energy transfer of eqs. delta_energy_ela/delta_energy_ine,
 * ionise and attach, and are reduced into the swarm attributes of section "Determination
 * of swarm attributes" (drift velocity, mean energies, diffusion, Townsend coefficients).
 *
 * Conventions shared by every entry point
 *  - Units: SI, except energies in eV and masses in unified atomic mass units.
 *  - Frame (section "Determination of swarm attributes"): z along E, B in the xz plane at
 *    angle B_angle_rad from E.  Electrons drift towards -z; scalar drift velocity and
 *    Townsend coefficients are reported along -z (positive numbers), vectors in the frame.
 *  - Every function returns swarm_status (0 = SWARM_OK, < 0 = error) unless stated; no
 *    C++ exception crosses the ABI.  swarm_strerror() names a status; swarm_last_error()
 *    gives a human-readable message for the calling thread's last failure.
 *  - Input arrays are read during the call and copied; the library keeps no caller
 *    pointer.  A handle owns its device memory and frees it in swarm_destroy().
 *  - A handle is not thread-safe; distinct handles may be used from distinct threads.
 *  - Work is issued on params.stream (a hipStream_t, e.g. torch's current stream) or, if
 *    it is NULL, on a stream the handle creates.  Entry points that return results to the
 *    host synchronise that stream before returning.
 */
#ifndef SWARM_H_
#define SWARM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SWARM_OK = 0,
  SWARM_ERR_INVALID_ARG = -1,   /* an argument failed validation (message says which)  */
  SWARM_ERR_OUT_OF_MEMORY = -2, /* device or host allocation failed                     */
  SWARM_ERR_CAPACITY = -3,      /* real-secondaries growth exceeded params.capacity     */
  SWARM_ERR_DEVICE = -4,        /* a HIP call failed (message holds the HIP error)      */
  SWARM_ERR_STATE = -5,         /* e.g. tallies requested before any run               */
  SWARM_PENDING = 1             /* swarm_server_poll: the request has not finished yet */
} swarm_status;

/* Collision process classes (section "Theoretical framework"). */
typedef enum { SWARM_ELASTIC = 0, SWARM_EXCITATION = 1, SWARM_IONIZATION = 2,
               SWARM_ATTACHMENT = 3 } swarm_kind;

/* Arithmetic of the per-electron loop.  SWARM_FP64: everything in binary64.
 * SWARM_FP32_MIXED: flight-time sampling, table interpolation, motion and scattering in
 * binary32; positions, times, energy sums and the energy-versus-threshold comparison near
 * the inelastic onset in binary64.  Both use the same random streams. */
typedef enum { SWARM_FP64 = 0, SWARM_FP32_MIXED = 1 } swarm_precision;

/* Ionisation/attachment handling (section "Determination of swarm attributes"):
 * DUMMY counts ionisations/attachments without creating or removing electrons (an
 * attached electron restarts at rest, an ionising one keeps half the remaining energy);
 * REAL appends the ejected electron as a new swarm member and removes attached ones. */
typedef enum { SWARM_DUMMY = 0, SWARM_REAL = 1 } swarm_secondaries;

/* Trial frequency nu' of the null-collision loop (section "Trial frequency strategies").
 * CONSTANT: one nu' for the whole run, the table maximum (LazyTrialFrequency) or the
 * user's fixed value (FixedTrialFrequency); the method is exact.  VARIABLE: the paper's
 * VariableTrialFrequency, per electron nu' = (1 + zeta) nu(eps) at its current energy,
 * capped at the constant value; renewed after every `trial_grace` trials (from the energy
 * after the trial that used up the count: the trial's energy after a null or forbidden
 * pick, the energy after the collision after a real one) and after every fail.  A fail is
 * a trial at which nu(eps) > nu': the electron returns to the state right after its last
 * real collision, takes nu' = (1 + zeta) nu(eps) from the rate that failed, restarts the
 * grace count, and the fail ends its random-number block like a real collision.  The first
 * nu' of an electron comes from the energy it was created with.  BINNED: the paper's
 * BinnedTrialFrequency.  Each decade of energy (1-10 eV, 10-100 eV, ...) is cut into
 * `trial_bins` bins evenly in log(eps): bin k = [10^(k/b), 10^((k+1)/b)) eV.  A cell of the
 * rate grid belongs to the bin of its lower node, and a bin's nu' is the largest rate on its
 * cells raised by 2^-20 (capped at the constant value).  Renewals as for VARIABLE take the
 * nu' of the current energy's bin.  A fail returns the electron to its last real collision
 * with the largest nu' of the bins from that collision's energy to the failing energy; a
 * second fail before the next real collision or renewal, where the paper throws, sets
 * record flag 16 and continues with the constant nu'.  Both adaptive strategies trade
 * exactness for fewer null trials: returning to the last real collision after a fail
 * favours flights that did not gain energy. */
typedef enum { SWARM_TRIAL_CONSTANT = 0, SWARM_TRIAL_VARIABLE = 1,
               SWARM_TRIAL_BINNED = 2 } swarm_trial_strategy;

/* One cross-section table: n_points >= 2 strictly increasing energies (> 0, eV) and
 * cross-sections (>= 0, finite, m^2).  Extended outside the points as in section
 * "Extension of the cross-section tables" (elastic: constant to the left; inelastic:
 * zero below threshold_eV; right: power law through the last two points). */
typedef struct {
  int32_t kind;            /* swarm_kind */
  double threshold_eV;     /* >= 0; energy lost in excitation/ionisation */
  int32_t n_points;
  const double* energy_eV;
  const double* sigma_m2;
} swarm_channel;

/* Scattering angle of the electron in a real collision (section "Theoretical framework").
 * ISOTROPIC: direction uniform on the sphere.  SCREENED_COULOMB (atoms, eq. collision_angle):
 * cos(theta) = 1 - 2R / (1 + 8 e (1 - R)), e the energy before the collision in Hartree
 * units.  CONSTANT_XI (molecules, eq. collision_angle_xi): cos(theta) = 1 - 2R(1 - xi) /
 * (1 + xi (1 - 2R)), xi solving sigma_mt/sigma_el = (1 - xi)/(2 xi^2) ((1 + xi)
 * ln((1 + xi)/(1 - xi)) - 2 xi) for a ratio given per component (the tables carry only
 * sigma_mt).  The azimuth about the incoming direction is 2 pi R'; R, R' are the scattering
 * block's first two uniforms.  A zero incoming velocity scatters isotropically. */
typedef enum { SWARM_SCATTER_ISOTROPIC = 0, SWARM_SCATTER_SCREENED_COULOMB = 1,
               SWARM_SCATTER_CONSTANT_XI = 2 } swarm_scattering;

/* One gas component: target mass, number fraction of the density (fractions of all
 * components sum to 1 within 1e-9) and its channels.  Channel order (components in
 * order, then channels in order) fixes the collision-process order used in selection. */
typedef struct {
  double mass_amu;         /* > 0 */
  double fraction;         /* >= 0 */
  int32_t n_channels;      /* >= 1 */
  const swarm_channel* channels;
  int32_t scattering;      /* swarm_scattering of its collisions */
  double mt_over_el;       /* SWARM_SCATTER_CONSTANT_XI: sigma_mt / sigma_el in (0, 1] */
} swarm_component;

typedef struct {
  double E_V_per_m;        /* >= 0, along +z */
  double B_T;              /* >= 0 */
  double B_angle_rad;      /* angle of B from E, B in the xz plane */
  double N_per_m3;         /* gas number density, > 0 */
  double T_K;              /* gas temperature (K, >= 0): the targets' Maxwell-Boltzmann
                              temperature with thermal_targets, else bookkeeping only */
  double init_energy_eV;   /* energy of the primaries, isotropic directions; >= 0 */
  int32_t precision;       /* swarm_precision */
  int32_t secondaries;     /* swarm_secondaries */
  int32_t grid_points_per_octave;  /* power of two <= 1024; 0 = default 64 */
  int32_t grid_min_exp2;   /* rate grid covers [2^min, 2^max] eV; both 0 = default -14, 12 */
  int32_t grid_max_exp2;
  double user_majorant;    /* 0: nu' = (1+2^-20) max nu on the grid (the paper's
                              LazyTrialFrequency); > 0: a fixed nu' (FixedTrialFrequency),
                              refused with SWARM_ERR_INVALID_ARG if below that maximum */
  int64_t capacity;        /* REAL mode: maximum number of electrons (primaries plus
                              secondaries) of one run; 0 = 64 x n_electrons */
  void* stream;            /* hipStream_t or NULL */
  int32_t trial_strategy;  /* swarm_trial_strategy */
  double trial_zeta;       /* VARIABLE: the overhead zeta > 0; 0 = default 0.25 */
  int64_t trial_grace;     /* VARIABLE, BINNED: trials between renewals, 1 .. 2^31 - 1;
                              0 = 5000 */
  int32_t trial_bins;      /* BINNED: bins per decade of energy, 1 .. 100; 0 = 10 */
  int32_t thermal_targets; /* 0: targets at rest (eqs. delta_energy_ela / delta_energy_ine);
                              1: moving targets (section "Effect of gas temperature").  At a
                              real collision the target velocity is drawn from the
                              Maxwell-Boltzmann distribution at T_K (three normals of spread
                              sqrt(kT/M), Box-Muller on its own random stream) and the
                              electron's velocity becomes Vcm + sqrt(|V1 - Vcm|^2 - 2 eps_k M /
                              ((m + M) m)) u, u its new direction in the centre-of-momentum
                              frame (isotropic, or theta about V1 - Vcm for the anisotropic
                              models).  A process below its threshold in that frame is
                              forbidden (counted in n_forbidden).  Rates and the null test keep
                              the laboratory energy. */
  int32_t relativistic;    /* 0: classical motion (UniformFieldClassic); 1: relativistic
                              motion in the uniform E and B (the paper's
                              UniformFieldRelativisticChin): lanes hold the proper velocity
                              u = gamma v, moved exactly (closed forms for B = 0; with B, the
                              exponential of the field generator in proper time, whose
                              duration is solved from the laboratory flight time); the rates
                              of eq. (frequency) take the true speed |u|/gamma, and the
                              energy-transfer equations are unchanged.  Needs SWARM_FP64 and
                              thermal_targets = 0 (else SWARM_ERR_INVALID_ARG). */
} swarm_params;

/* Per-electron result record (one per electron that existed in the run), as stored on
 * the device.  r and t are measured from the primary's start (t = 0 at the origin). */
typedef struct {
  uint64_t id;             /* primaries: index; secondaries: 2^63 | hash of (parent, k) */
  uint32_t flags;          /* 1 finished (made all its real collisions), 2 attached,
                              4 stopped at the per-electron trial-block cap (2^31 - 1),
                              8 stopped because the run exceeded its capacity,
                              16 a retry of the binned trial frequency failed again
                              (the electron went on with the constant nu') */
  uint32_t k_start;        /* real collisions inherited from the lineage at birth */
  uint32_t k_end;          /* real-collision count when the electron stopped */
  uint32_t G, D;           /* ionisations and attachments made by this electron */
  uint32_t n_forbidden;    /* channel picks below the inelastic onset (treated as null) */
  uint32_t n_over;         /* real collisions above the top of the rate grid */
  uint32_t n_fail;         /* fails of the variable or binned trial frequency */
  uint64_t n_null;         /* null trials */
  uint64_t blocks;         /* random-number blocks used (two candidate trials each) */
  double r[3], t;
  double sum_eps, sum_epsp; /* sums of the energies before / after its real collisions */
} swarm_record;

/* One traced event (real collision or forbidden channel pick) of a traced electron. */
typedef struct {
  uint64_t id;
  int32_t type;            /* 1 real, 2 forbidden, 3 fail (channel -1) */
  int32_t channel;
  uint32_t k, block, sub, pad;   /* real index before the event, trial block, 0/1 in block */
  double eps, epsp, t, r[3];     /* energy before/after (eV), time and position after */
} swarm_event;

typedef struct { double value, stat_sigma, spread; } swarm_stat;

/* Swarm tallies (section "Determination of swarm attributes").  Over the finished set F:
 *   W = (1/N) sum z_n/t_n (vector W*, scalar along -z);  d_n = x_n - t_n W_z z^ (paper
 *   form) or x_n - t_n W* (vector form);  D = (1/N) sum |d|^2/t, D_L = (1/N) sum
 *   (d.z)^2/(2t), D_T = (1/N) sum |d_perp|^2/(4t);  sigma = (1/N) sum 2|d| (and the L, T
 *   parts);  alpha = (1/N) sum G_n/z_n, eta = (1/N) sum D_n/z_n (z along -z).
 * Over all electrons: mean energies before/after real collisions; counts; efficiency =
 * real/(real + null + forbidden + fail).  spread = sample standard deviation of the per-electron
 * quantity (the paper's printed +-), stat_sigma = spread/sqrt(N). */
typedef struct {
  swarm_stat W, Wx, Wy, Wz, mean_energy, mean_energy_after;
  swarm_stat D, DL, DT, sigma, sigmaL, sigmaT;
  swarm_stat D_vec, DL_vec, DT_vec, sigma_vec, sigmaL_vec, sigmaT_vec;
  swarm_stat alpha, eta;
  double alpha_rate, eta_rate;   /* sum G / sum z and sum D / sum z over F */
  double efficiency, majorant;
  int64_t n_real, n_null, n_forbidden, n_fail, n_over;
  int64_t n_electrons, n_finished, n_attached, n_stuck, n_created;
  int64_t n_ionizations, n_attachments, n_dropped;
  int64_t n_retry_failed;  /* electrons whose binned-strategy retry failed again (flag 16) */
  int32_t exact;           /* 1: constant trial frequency, the method is exact; 0: the variable
                              or binned trial frequency ran: its return to the last real
                              collision after a fail favours flights that gained no energy, so
                              the tallies carry a bias besides their statistical error */
  int32_t trial_strategy;  /* swarm_trial_strategy of the run */
} swarm_tallies_t;

typedef struct swarm* swarm_t;

/* Build a swarm instance: validates the inputs, copies the tables to the device and
 * builds (in kernels) the octave-grid rate tables nu_c(eps_g) = n_k sigma_c(eps_g)
 * sqrt(2 eps_g / m) (eq. frequency), their running sums over channels, the trial
 * frequency and the field constants.  *out is set only on SWARM_OK. */
swarm_status swarm_create(const swarm_component* comps, int32_t n_comps,
                          const swarm_params* params, swarm_t* out);

/* Simulate n_electrons primaries (ids 0..n-1) at the origin, each until it has made
 * n_collisions real collisions (the paper's I; section "Determination of swarm
 * attributes"), with the given seed.  Synchronous.  In REAL mode secondaries inherit the
 * parent's count and run in generations: the primaries, then the secondaries each
 * generation created, one kernel launch per generation.  If REAL growth exceeds the capacity the run stops early and returns
 * SWARM_ERR_CAPACITY: the secondaries that did not fit are counted (n_dropped), electrons
 * still running are recorded with flag 8 at their last real collision, those not yet
 * started with flag 8 as they were created, and the tallies cover the finished ones.
 * Previous results of the handle are replaced. */
swarm_status swarm_run(swarm_t h, int64_t n_electrons, int64_t n_collisions, uint64_t seed);

/* The run of swarm_run, started without waiting for it.  DUMMY mode enqueues all its device
 * work on the handle's stream (work items, the swarm kernel, the tally reductions) and
 * returns; REAL mode runs its generations on a worker thread the handle owns, since each
 * generation's launch depends on the counters of the one before.  Errors found before the
 * work starts (arguments, allocation) are returned here; the run's own status (e.g.
 * SWARM_ERR_CAPACITY) comes from swarm_wait.  Until swarm_wait returns, every other call on
 * the handle except swarm_destroy (which waits) returns SWARM_ERR_STATE, and the stream
 * carries the run: work the caller adds to it afterwards runs after the run's.  The
 * handle's records and device memory are in use until then; distinct handles on distinct
 * streams overlap on the device. */
swarm_status swarm_run_async(swarm_t h, int64_t n_electrons, int64_t n_collisions, uint64_t seed);

/* Wait for the run started by swarm_run_async; returns its status, as swarm_run would have.
 * Afterwards swarm_tallies, swarm_records and swarm_last_timing give its results.
 * SWARM_ERR_STATE if no run is in flight. */
swarm_status swarm_wait(swarm_t h);

/* swarm_create with every device allocation of the handle (tables, records, secondary
 * queue, work items, tally buffers, trace buffers) taken from one region the caller owns:
 * `arena` is a device pointer to arena_bytes bytes (e.g. a torch tensor's data_ptr) that
 * must stay valid until swarm_destroy.  The library sub-allocates it (first fit, 256-byte
 * blocks) and never frees it.  A run that does not fit returns SWARM_ERR_OUT_OF_MEMORY;
 * swarm_arena_bytes gives a size that holds the tables and runs of up to n_electrons. */
swarm_status swarm_create_in_arena(const swarm_component* comps, int32_t n_comps,
                                   const swarm_params* params, void* arena, int64_t arena_bytes,
                                   swarm_t* out);

/* Device bytes a handle of these inputs needs for its tables plus one run of n_electrons
 * primaries (REAL mode: params.capacity electrons, 0 = 64 n_electrons) without tracing.
 * Validates the inputs like swarm_create; allocates nothing. */
swarm_status swarm_arena_bytes(const swarm_component* comps, int32_t n_comps, const swarm_params* params,
                               int64_t n_electrons, int64_t* bytes);

/* Tallies of the last run (computed by deterministic fixed-order device reductions). */
swarm_status swarm_tallies(swarm_t h, swarm_tallies_t* out);

/* Copy up to max_records records of the last run to host memory `out` (primaries in id
 * order first, then secondaries in creation order); *n_out = number of records run. */
swarm_status swarm_records(swarm_t h, swarm_record* out, int64_t max_records, int64_t* n_out);

/* Select electrons to trace in the following runs (n_ids <= 256, max_events per
 * electron <= 4096); n_ids = 0 switches tracing off.  Tracing uses a separate kernel
 * build; results are otherwise identical. */
swarm_status swarm_set_trace(swarm_t h, const uint64_t* ids, int32_t n_ids, int32_t max_events);

/* Copy the events of the last traced run: out holds n_ids x max_events slots (slot
 * i*max_events + j = event j of ids[i]); counts[i] = number of events of ids[i]. */
swarm_status swarm_trace_events(swarm_t h, swarm_event* out, int32_t* counts);

/* Copy the device-built tables: nodes (G energies, eV), cum (n_channels x G, channel
 * major, FP64 running sums of channel rates), majorant (nu', 1/s).  Any may be NULL. */
swarm_status swarm_tables(swarm_t h, int32_t* grid_size, int32_t* n_channels, double* nodes,
                          double* cum, double* majorant);

/* Device time in milliseconds of the last run's simulation kernel (every generation's
 * launch in REAL mode; HIP events on the launch stream) and of its whole device section
 * (simulation plus tallies). */
swarm_status swarm_last_timing(swarm_t h, double* kernel_ms, double* total_ms);

/* Launches of the last run's simulation kernel (one in DUMMY mode; in REAL mode one per
 * generation, and more where the stragglers of a launch were parked for the next one, see
 * swarm_launch_opts.park_lanes) and the electrons parked between them in all.  Either pointer
 * may be NULL.  SWARM_ERR_STATE before the first completed run. */
swarm_status swarm_last_launches(swarm_t h, int64_t* launches, int64_t* parked);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops that must not call hipMalloc, harnesses that forbid it): the DUMMY-mode run of
 * swarm_run with no allocation.  The caller passes `records`, device memory for n_electrons
 * swarm_record entries, which receive the records of ids 0..n-1 in id order (as swarm_run
 * keeps them).  The run's scratch (work items, their counter, tally partial sums and
 * output) is a library array of 1.4 MB in device memory, one per GPU, held until the
 * process ends; n_electrons is limited to 4194304 (2^22) and larger runs are refused with
 * SWARM_ERR_INVALID_ARG, as are REAL mode and tracing.  Every call on a GPU shares that
 * GPU's array and leaves its contents behind (each call rebuilds what it reads); calls that
 * overlapped on one GPU would race on it, so the library runs them one at a time (a call
 * holds a per-device lock until its results are back).  Synchronous: on return
 * swarm_tallies gives the tallies (the same bits as swarm_run's); swarm_records refuses
 * (SWARM_ERR_STATE), the records being in the caller's memory. */
swarm_status swarm_run_noalloc(swarm_t h, int64_t n_electrons, int64_t n_collisions, uint64_t seed,
                               swarm_record* records);

void swarm_destroy(swarm_t h);             /* NULL-safe */
const char* swarm_strerror(swarm_status s);
const char* swarm_last_error(void);        /* thread-local message of the last failure */

/* ---- Batched runs: many uneven instances in one persistent launch ------------------ */

typedef struct {
  int64_t n_electrons;
  int64_t n_collisions;
  uint64_t seed;
} swarm_job;

/* Launch-shape options.  They only change how work is scheduled on the GPU, never the
 * per-electron arithmetic or random streams, so results are bit-identical for any
 * choice.  Zero fields mean "autotune" (swarm_autotune) or the built-in default. */
typedef struct {
  int32_t block_size;      /* 64..1024, multiple of 64 */
  int32_t chunk;           /* electrons per work item (multiple of block_size) */
  int32_t pending_trigger; /* lanes waiting on a real collision before the wave serves them (1..64) */
  int32_t use_graph;       /* capture the launch in a hipGraph and replay it */
  int32_t service_waves;   /* 0: every wave serves its own candidates; n >= 1: pooled schedule,
                              n waves of each work-group serve the candidates of the others at
                              full width (n < block_size/64; traced runs use the per-wave one) */
  int32_t table_layout;    /* LDS tables of a work-group: 0 the total-rate pairs and channel
                              descriptors (running sums read through L2); 1 also the running
                              sums of every channel, when they fit the work-group's LDS
                              (otherwise 0) */
  int32_t park_lanes;      /* real secondaries: once all electrons of a launch are claimed, a
                              wave with at most this many running lanes parks them (each at its
                              next real collision) for the next launch, if the launch has
                              created secondaries for an eighth of the device; 0: 32, -1: never,
                              at most 64 */
} swarm_launch_opts;

/* Launch shape of the handle's own runs (swarm_run); zero fields take the defaults.  Like
 * every launch option it changes the schedule only, never the results. */
swarm_status swarm_set_launch_opts(swarm_t h, const swarm_launch_opts* opts);

typedef struct swarm_batch* swarm_batch_t;

/* A batch of instances (all DUMMY mode, all the same precision) with one job each.  The
 * batch keeps the per-instance results on the device; swarm_batch_launch runs every job
 * in one persistent kernel (work items of `chunk` electrons, instance tables staged in
 * LDS), followed by the tally kernels, captured in a hipGraph when use_graph != 0.  The
 * first launch hands out the instances' items heaviest collision budget first, then in the
 * order given; swarm_batch_wait of the first launch orders them again by each instance's
 * measured work per electron (trials per real collision), longest first, for the launches
 * after it.  The order changes no result. */
swarm_status swarm_batch_create(swarm_t* handles, const swarm_job* jobs, int32_t n,
                                const swarm_launch_opts* opts, swarm_batch_t* out);
swarm_status swarm_batch_launch(swarm_batch_t b);                  /* asynchronous */
swarm_status swarm_batch_wait(swarm_batch_t b, double* device_ms); /* synchronise */
/* Tallies of instance i of the last launch (also stored in handle i). */
swarm_status swarm_batch_tallies(swarm_batch_t b, int32_t i, swarm_tallies_t* out);
void swarm_batch_destroy(swarm_batch_t b);

/* Convenience: create, launch, wait and destroy a batch; afterwards swarm_tallies and
 * swarm_records of each handle return its instance's results. */
swarm_status swarm_batch_run(swarm_t* handles, const swarm_job* jobs, int32_t n,
                             const swarm_launch_opts* opts);

/* Autotuner: times the result-invariant launch options (block size, pending trigger, electrons
 * per work item, LDS table layout) on a shortened copy of the batch
 * (same instances, budgets cut to probe_collisions) and writes the fastest to *best. */
swarm_status swarm_autotune(swarm_t* handles, const swarm_job* jobs, int32_t n,
                            int64_t probe_collisions, swarm_launch_opts* best);

/* ---- Serving: continuous batching of arriving swarm requests ------------------------ */

/* Which admitted requests an epoch advances. */
typedef enum {
  SWARM_SCHEDULE_ALL = 0,             /* every admitted request in every epoch */
  SWARM_SCHEDULE_SHORTEST_FIRST = 1   /* the least remaining device work (electrons x
                                         collisions left x the measured work per collision)
                                         first, until the epoch holds about 10240 electrons per
                                         compute unit, plus always the earliest admitted request
                                         and the one with the most work per electron left:
                                         lower median latency under overload, at some throughput */
} swarm_schedule;

typedef struct {
  int64_t hbm_budget_bytes;   /* admission limit on device memory held by requests */
  int32_t precision;          /* swarm_precision of every request */
  int64_t quantum_collisions; /* real collisions per electron per scheduling epoch; 0 = per
                                 request, sized so that an epoch lasts about 100 ms and every
                                 electron does about the same device work in it */
  int32_t max_active;         /* instances per epoch (0 = 1024) */
  swarm_launch_opts opts;
  void* stream;               /* hipStream_t or NULL */
  int32_t schedule;           /* swarm_schedule (0 = every admitted request in every epoch) */
} swarm_server_params;

typedef struct {
  double submit_s, admit_s, done_s;   /* seconds on the server's monotonic clock */
  int64_t n_real;                     /* real collisions of the request */
  int64_t epochs;                     /* scheduling epochs the request took part in */
  int64_t bytes;                      /* device memory charged against the budget */
  int64_t progress;                   /* real collisions made so far (all its electrons; exact
                                         at epoch boundaries) */
  double blocks_per_real;             /* trial blocks per real collision, as the server last
                                         measured them to size the request's quantum (after
                                         its epochs 1, 2, 4, 8, ...; 0 before the first) */
} swarm_request_info;

/* A snapshot of the server (swarm_server_stats). */
typedef struct {
  double time_s;                      /* server clock */
  int64_t n_submitted, n_pending, n_active, n_finished, n_failed;   /* requests */
  int64_t bytes_in_use;               /* device memory charged by admitted requests */
  int64_t work_left;                  /* real collisions the unfinished requests still need */
  int64_t work_done;                  /* real collisions made by all requests so far */
  int64_t epochs;                     /* epochs completed */
} swarm_server_stats_t;

typedef struct swarm_server* swarm_server_t;

/* Tests of the error path only: when the environment variable SWARM_SERVER_FAIL_EPOCH is k
 * >= 1 at swarm_server_create, the server's k-th epoch reports a device failure without
 * launching anything, which fails every admitted request with SWARM_ERR_DEVICE. */
/* A server owns a scheduler thread.  Requests are admitted while the device memory they
 * need fits the budget; admitted requests keep their tables and electron state resident
 * and advance together: each epoch is one persistent launch over the admitted requests the
 * schedule picks, in which every unfinished electron makes up to its request's quantum of
 * real collisions (quantum_collisions, or with 0 a per-request quantum: fewer collisions
 * for a request whose gas draws more null trials per real collision).
 * Requests that arrive while an epoch runs join the next one.  Because electrons stop at
 * real-collision boundaries and the random streams are counter based, a request's
 * result does not depend on what it was batched with. */
swarm_status swarm_server_create(const swarm_server_params* p, swarm_server_t* out);
/* A server whose device memory (every request's tables, electron state and records, and
 * the epochs' buffers) comes from one region the caller owns (a device pointer to
 * arena_bytes bytes, valid until swarm_server_destroy returns).  The admission limit is the
 * smaller of hbm_budget_bytes and the region; a request that fits the budget but not the
 * region's free blocks waits until an admitted request finishes. */
swarm_status swarm_server_create_in_arena(const swarm_server_params* p, void* arena, int64_t arena_bytes,
                                          swarm_server_t* out);
/* Queue a request (inputs copied); *ticket identifies it.  DUMMY mode only. */
swarm_status swarm_server_submit(swarm_server_t s, const swarm_component* comps, int32_t n_comps,
                                 const swarm_params* params, int64_t n_electrons,
                                 int64_t n_collisions, uint64_t seed, int64_t* ticket);
/* swarm_server_submit that also returns the request's per-electron records: records_out is
 * host memory for n_electrons swarm_record entries (ids 0..n-1 in id order), written before
 * the request is reported finished; the caller keeps it valid until then. */
swarm_status swarm_server_submit_records(swarm_server_t s, const swarm_component* comps, int32_t n_comps,
                                         const swarm_params* params, int64_t n_electrons,
                                         int64_t n_collisions, uint64_t seed, swarm_record* records_out,
                                         int64_t* ticket);
/* SWARM_OK with the tallies once finished, SWARM_PENDING before; info may be NULL. */
swarm_status swarm_server_poll(swarm_server_t s, int64_t ticket, swarm_tallies_t* out,
                               swarm_request_info* info);
/* Block until every submitted request has finished. */
swarm_status swarm_server_drain(swarm_server_t s);
/* Queue and progress counters (e.g. the backlog against time under overload). */
swarm_status swarm_server_stats(swarm_server_t s, swarm_server_stats_t* out);
/* Seconds on the server clock (the clock of swarm_request_info). */
double swarm_server_now(swarm_server_t s);
/* Stop the server: the running epoch ends, every request that has not finished is
 * cancelled (it would poll SWARM_ERR_STATE) and its memory released, the scheduler thread
 * is joined.  Call swarm_server_drain first to wait for the results instead. */
void swarm_server_destroy(swarm_server_t s);

#ifdef __cplusplus
}
#endif

#endif  /* SWARM_H_ */
