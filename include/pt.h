/*
 * pt.h -- C ABI of the MI355X (gfx950) parallel-tempering Metropolis library.
 *
 * Method: Metropolis-Hastings (paper Sec. 2.1, acceptance Eq. 1) sampling the
 * Boltzmann distribution (Eq. 2) of a lattice spin model (Ising energy, Eq. 3),
 * with Parallel Tempering (Sec. 2.1): R replicas at their own inverse
 * temperatures that, between intervals of sweeps, try to exchange states with
 * a neighbouring temperature, pairs alternating between (0,1),(2,3),... and
 * (1,2),(3,4),... (Sec. 3), accepted with the logistic probability of Sec. 3.
 * As in the paper's GPU design (Sec. 3), all simulation state stays in device
 * memory between calls.
 *
 * Decomposition: sites are updated in checkerboard order (colour 0, then
 * colour 1, per sweep); each flip draws one 32-bit word of a Philox4x32-10
 * stream keyed by (seed, stream_id) and counted by (site group, sweep, slot,
 * colour); acceptance is an integer compare against thresholds precomputed on
 * the host in FP64; a replica exchange permutes the temperature slots of the
 * walkers (no lattice is copied).  Results are a pure function of the
 * configuration and the sequence of calls: they do not depend on the plan
 * (tiling, sweeps per launch, block size), and they equal those of a
 * sequential implementation that swaps states literally.
 *
 * Conventions
 *   - Sites: 2D i = y*L + x; 3D i = (z*L + y)*L + x; periodic boundaries.
 *     Colour of a site = (x + y [+ z]) mod 2.
 *   - Energy: 2D  E = -J sum_<ij> s_i s_j - h sum_i s_i  (each bond once);
 *             EA  E = -sum_<ij> J_ij s_i s_j, J_ij = +-1 per bond.
 *     Integer energy E_int = -sum_<ij> J_b s_i s_j (J_b = 1 in 2D), so that
 *     E = J*E_int - h*M; series and observables report E_int and M = sum s_i.
 *   - "Slot" k is the temperature index (beta[k]); "walker" w is a replica
 *     state.  walker_at[k] is the walker held by slot k; walker w starts at
 *     slot w.
 *
 * Threading: one context must not be used from two host threads at once;
 * distinct contexts may run concurrently on distinct streams.  pt_create and
 * pt_observables synchronise the context's stream; the other calls only queue
 * work on it.
 *
 * Errors: every pt_status function returns PT_OK (0) or a negative code and
 * never throws.  Configuration errors are detected synchronously (PT_EINVAL).
 * A failed HIP call (launch or copy) returns PT_EDEVICE; after PT_EDEVICE the
 * context is poisoned and every later call returns PT_ESTATE.  A persistent
 * launch whose pairwise exchange wait exceeds its bound stops early and is
 * reported as PT_EDEVICE by the next pt_observables.  pt_last_error()
 * returns a thread-local message describing the last failure of this thread.
 */
#ifndef PT_H
#define PT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PT_ABI_VERSION 1u
#define PT_ALL_SLOTS 0xFFFFFFFFu
#define PT_MAX_SWEEPS_PER_LAUNCH 16u

typedef enum {
  PT_OK = 0,
  PT_EINVAL = -1,      /* invalid argument or configuration */
  PT_ENOMEM = -2,      /* workspace too small or host allocation failed */
  PT_EDEVICE = -3,     /* a HIP runtime call failed */
  PT_ESTATE = -4,      /* context poisoned by an earlier device error */
  PT_EUNSUPPORTED = -5 /* valid for the method, not implemented by this library */
} pt_status;

typedef enum { PT_ISING2D = 0, PT_EA3D = 1 } pt_model;

typedef struct {
  uint32_t abi_version;     /* must be PT_ABI_VERSION */
  uint32_t model;           /* pt_model */
  uint32_t L;               /* linear size, even (the checkerboard needs two colours on the
                               periodic lattice): 2D 4 .. 16384, every plan for powers of two
                               >= 8, the whole-replica tiled plan for other sides (up to the
                               side whose replica fits one workgroup's LDS, about 560);
                               EA: a power of two, 8 .. 64 (PT_EUNSUPPORTED otherwise) */
  uint32_t R;               /* replicas = temperature slots, 1 .. 4096 */
  const double *beta;       /* host [R], finite, >= 0, slot order; copied at create */
  double J;                 /* 2D coupling (ignored for EA) */
  double h;                 /* 2D field (finite); ignored for EA */
  uint32_t seed;            /* Philox key word 0 (spins, flips, swaps) */
  uint32_t stream_id;       /* Philox key word 1 (0, or an instance id) */
  uint32_t coupling_seed;   /* Philox key word 0 of the EA couplings */
  const int8_t *init_spins; /* NULL (draw from Philox) or host [R][N] +-1, walker order */
  const int8_t *couplings;  /* NULL (draw from Philox) or host EA [3][N] +-1, bond (i, i+e_d) */
  uint32_t record_every;    /* record E_int, M per slot every n sweeps (0 = never) */
  uint32_t max_records;     /* capacity of the record series */
} pt_config;

/* Launch plan: how the work is decomposed.  Any valid plan gives bit-identical
 * results.  Zero fields mean "choose automatically".
 *   FUSED       one workgroup holds every walker in LDS; whole schedules run in
 *               one launch (small systems).
 *   TILED       a workgroup per (tile of planes, walker); halo tiles, up to
 *               PT_MAX_SWEEPS_PER_LAUNCH sweeps per launch; with halo tiles an
 *               exchange step runs in the epilogue of the launch's last
 *               workgroup, with whole replicas as a launch of its own.
 *   PERSISTENT  one co-resident workgroup per walker keeps its lattice in LDS
 *               for a whole pt_run call; exchange steps are decided pairwise
 *               between neighbouring slots without a global barrier.  With
 *               tile_planes = L/P each walker runs as P co-resident
 *               workgroups of L/P planes (3D z-planes, 2D rows) that trade
 *               boundary planes and energy shares once per sweep (P R
 *               workgroups, one per compute unit): 3D 16 <= L <= 32 with P = 2,
 *               2D 64 <= L <= 1024 with P = 2, 4 or 8 and at least 8 rows per
 *               part; tile_planes = 0 or L means one workgroup per walker.
 *   LANES       the paper's GPU decomposition (Sec. 3: one replica per thread):
 *               each lane holds one walker's whole lattice in registers and
 *               updates it site after site; one workgroup runs every walker and
 *               the exchange steps.  2D, L = 8 or 16, R <= 1024 only; never
 *               chosen automatically (a reference point for the other plans).
 *   WAVE        small 2D lattices: each walker in the registers of L^2/8 lanes
 *               of one wavefront, eight sites per lane, neighbours read across
 *               lanes, so a sweep needs no barrier; one workgroup runs every
 *               walker and the exchange steps.  2D, L = 8 or 16, R L^2/8 <=
 *               1024; block_threads follows R. */
typedef enum {
  PT_PLAN_AUTO = 0,
  PT_PLAN_FUSED = 1,
  PT_PLAN_TILED = 2,
  PT_PLAN_PERSISTENT = 3,
  PT_PLAN_LANES = 4,
  PT_PLAN_WAVE = 5
} pt_plan_mode;
typedef struct {
  uint32_t mode;              /* pt_plan_mode */
  uint32_t tile_planes;       /* TILED: rows (2D) or z-planes (3D) per workgroup tile;
                                 PERSISTENT: L, or L/P for P workgroups per walker */
  uint32_t sweeps_per_launch; /* TILED: 1 .. PT_MAX_SWEEPS_PER_LAUNCH */
  uint32_t block_threads;     /* 64 .. 1024, multiple of 64 */
} pt_plan;

typedef struct pt_ctx pt_ctx; /* opaque host-side context */

/* Caller-owned host buffers filled by pt_observables; NULL pointers are skipped. */
typedef struct {
  int32_t *E_series;     /* [n_records][R] E_int per slot, oldest first */
  int32_t *M_series;     /* [n_records][R] M per slot */
  int32_t *E_slot;       /* [R] current E_int per slot */
  int32_t *M_slot;       /* [R] current M per slot */
  uint64_t *swap_att;    /* [R][R] attempted swaps; only |i-j| = 1 non-zero, symmetric */
  uint64_t *swap_acc;    /* [R][R] accepted swaps; same layout */
  uint32_t *walker_at;   /* [R] walker held by each slot */
  int8_t *spins;         /* +-1: [N] for slot spins_slot, or [R][N] in slot order if PT_ALL_SLOTS */
  uint32_t spins_slot;   /* slot to copy, or PT_ALL_SLOTS */
  uint64_t sweeps_done;    /* out */
  uint64_t exchanges_done; /* out */
  uint32_t n_records;      /* out */
} pt_obs;

/* Device workspace needed for cfg, in bytes (0 and pt_last_error set if cfg is
 * invalid).  The workspace holds every piece of simulation state: two
 * bit-packed spin buffers [R][N/32] (uint32, bit set = down), bit-packed EA bond
 * planes [3][N/32], flip thresholds [R][16] (uint32), swap tables (uint64),
 * walker/slot maps, per-walker E_int and M, per-sweep accumulators, the record
 * series, swap counters, exchange mailboxes, and (only when cfg uploads spins or
 * couplings) a staging area of one byte per uploaded value. */
size_t pt_workspace_bytes(const pt_config *cfg);

/* Initialisation phase (Sec. 3): validate cfg, build the FP64 -> integer flip
 * and swap threshold tables on the host, lay the state out in d_workspace
 * (device memory owned by the caller, >= pt_workspace_bytes(cfg), 256-byte
 * aligned, left untouched after pt_destroy), draw or upload initial spins and
 * couplings, and compute the initial E_int and M (the "first iteration").
 * hip_stream is a hipStream_t (NULL = the null stream); all later work of the
 * context is ordered on it.  On success *out receives the context.
 * Errors: PT_EINVAL (cfg, alignment), PT_ENOMEM (ws_bytes too small), PT_EDEVICE. */
pt_status pt_create(const pt_config *cfg, void *hip_stream, void *d_workspace, size_t ws_bytes,
                    pt_ctx **out);

/* For callers that cannot allocate device memory for the library (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * pt_create, except that the context's sweep scratch -- the per-sweep energy
 * tallies, the pairwise exchange mailboxes and the split plan's boundary posts
 * -- lives in a fixed device array inside the library (PT_STATIC_SCRATCH_BYTES,
 * one copy per GPU and process, held until the process ends) instead of in
 * the caller's memory.  d_state (caller-owned, 256-byte aligned) then holds
 * only the simulation state (lattices, tables, maps, energies, record series,
 * counters): *state_bytes gives its size.  With d_state == NULL nothing is
 * created and *state_bytes receives the bytes needed (never more than
 * pt_workspace_bytes(cfg)).  Neither this call nor any later call on the
 * context allocates device memory; the array's address is looked up once per
 * GPU, on the first call made with that GPU current.
 * Every context created this way on one GPU shares that GPU's array, and the
 * array keeps what the last call left: each pt_sweep / pt_run on such a
 * context first clears the part it uses (a fill kernel on the context's
 * stream), so calls on such contexts that overlap in time -- on different
 * streams or threads -- race and give wrong results; serialise them.  All
 * other calls behave as for a pt_create context, with the same results bit
 * for bit.
 * Errors: as pt_create; PT_ENOMEM if the configuration needs more scratch than
 * the array holds (R, and for the split plan's posts L, too large), or if
 * *state_bytes is below the size needed; PT_EINVAL if state_bytes is NULL. */
#define PT_STATIC_SCRATCH_BYTES (4u << 20)
pt_status pt_create_static(const pt_config *cfg, void *hip_stream, void *d_state,
                           size_t *state_bytes, pt_ctx **out);

/* Override the launch plan (validated; PT_EINVAL if impossible for this size). */
pt_status pt_set_plan(pt_ctx *ctx, const pt_plan *plan);
/* Read the plan in use. */
pt_status pt_get_plan(const pt_ctx *ctx, pt_plan *plan);

/* Bound of the persistent plans' waits for a partner's post: the number of
 * polls (each followed by a short sleep) after which a launch gives up and
 * every workgroup of it leaves its loop; pt_observables then returns
 * PT_EDEVICE.  Default 2^24 polls, orders of magnitude above any legitimate
 * wait.  0 gives up at the first wait, which lets a test exercise that path
 * deterministically.  Applies to launches queued afterwards. */
pt_status pt_set_wait_limit(pt_ctx *ctx, uint32_t polls);

/* Execution phase, MH part (Sec. 2.1, Eq. 1): n_sweeps checkerboard sweeps
 * s, s+1, ..., s+n-1 of every walker at its current slot's beta, recording
 * E_int and M after every sweep with (s'+1) % record_every == 0.  Asynchronous.
 * PT_EINVAL if the records would exceed max_records. */
pt_status pt_sweep(pt_ctx *ctx, uint32_t n_sweeps);

/* Execution phase, PT part (Sec. 3): one exchange step e with pair parity e mod 2:
 * for every slot k = e mod 2, e mod 2 + 2, ... with k+1 < R, the walkers a, b at
 * slots k, k+1 swap slots with probability e^x/(1+e^x), x = (beta_k - beta_k+1)
 * (E_a - E_b).  With a field (2D, h != 0) x splits into x1 = dBeta J dE_int and
 * y = -dBeta h dM, and the swap needs the logistic test on x1 and a Metropolis
 * test min(1, e^y), realised as one test per set binary digit of |dM|/2 (the
 * paper's experiments have no field).  Then e += 1.  Asynchronous. */
pt_status pt_exchange(pt_ctx *ctx);

/* The paper's interval schedule (Sec. 3, Fig. 2): n_sweeps sweeps, and after
 * every sweep s with exchange_every > 0 and (s+1) % exchange_every == 0 one
 * exchange step.  Equivalent to the corresponding sequence of pt_sweep and
 * pt_exchange calls (same results, bit for bit), with fewer launches. */
pt_status pt_run(pt_ctx *ctx, uint32_t n_sweeps, uint32_t exchange_every);

/* Synchronise the context's stream and copy the requested observables into
 * caller-owned host buffers (layouts in pt_obs).  The only device-to-host
 * transfer of the library: the paper keeps all data on the device during the
 * run (Sec. 3) and takes the stored chains of the MH iterations as the result
 * (Sec. 2.1); here the chains are the per-slot E_int and M records (indexed by
 * temperature slot, the paper's replica), plus the swap counts and, on
 * request, the final lattices. */
pt_status pt_observables(pt_ctx *ctx, pt_obs *obs);

/* Host-side view of the threshold tables built at create (for tests and tools):
 * flip thresholds [R][16] (accept a flip of class c in slot k iff r <= T[k][c];
 * class c = 8*b + u with b = 1 for a down spin and u = number of unsatisfied
 * bonds of the site), and for each pair k (0 .. R-2) the half-width D[k] of its
 * swap table.  Buffers may be NULL. */
pt_status pt_flip_thresholds(const pt_ctx *ctx, uint32_t *out_R_by_16);
/* Swap threshold of pair k for energy difference E_a - E_b = 4*d: the number of
 * accepted 32-bit draws (accept iff r < T), 0 .. 2^32, for every d a lattice of
 * this size can reach (|d| <= z N / 4, z = 2 dim); larger |d| return the value at
 * the edge of the table. */
pt_status pt_swap_threshold(const pt_ctx *ctx, uint32_t k, int64_t d, uint64_t *out_T);

/* Free the host context (never the caller's workspace or stream): the end of the
 * execution phase (Sec. 3); the device-resident state stays in the caller's
 * memory until the caller frees it.  NULL is a no-op. */
void pt_destroy(pt_ctx *ctx);

/* ---- batched form: many independent instances advanced together ------------
 * n instances, each a full pt_config (give each its own stream_id so that their
 * random streams differ), share one workspace and advance in lockstep cycles:
 * every cycle runs up to K sweeps of every active instance (K = a divisor of the
 * exchange interval), then the exchange step of the instances whose interval
 * ends, then a device-side counter update -- so the whole cycle is a fixed
 * sequence of launches, captured once in a HIP graph and replayed.  The first
 * cycles of a run time candidate decompositions (walkers per workgroup, block
 * size) per lattice-size group, then candidate cycle lengths K, and keep the
 * fastest (the analogue of the paper's block-size study, Sec. 4.2); choices
 * never change results, so every instance is bit-identical to running it
 * alone. */
typedef struct pt_batch pt_batch;

/* Workspace for the batch (the instances' workspaces plus the batch's tables). */
size_t pt_batch_workspace_bytes(const pt_config *cfgs, uint32_t n);
/* Create n instances (initialisation phase of each) in d_workspace (caller-owned,
 * 256-byte aligned).  hip_stream orders the batch's work against the caller's. */
pt_status pt_batch_create(const pt_config *cfgs, uint32_t n, void *hip_stream, void *d_workspace,
                          size_t ws_bytes, pt_batch **out);
/* Advance every instance by n_sweeps sweeps with an exchange step after every
 * exchange_every-th sweep (0 = none).  Asynchronous on the caller's stream. */
pt_status pt_batch_run(pt_batch *b, uint32_t n_sweeps, uint32_t exchange_every);
/* Observables of instance i (synchronises). */
pt_status pt_batch_observables(pt_batch *b, uint32_t i, pt_obs *obs);
/* Decomposition chosen for lattice-size group g (0 .. groups-1): walkers per
 * workgroup, block size, and the sweeps per cycle of the last run (0 before
 * any); returns PT_EINVAL past the last group.  Output pointers may be NULL.
 * The choices come from the online tuner, which keeps them in a text file
 * keyed by device, model, lattice side and replica count (rounded up to a
 * power of two) -- and, for the sweeps per cycle, the batch's mix of lattice
 * sizes and its exchange interval -- so that later processes start tuned:
 * $PTMI_TUNE_CACHE, else $XDG_CACHE_HOME/ptmi/batch_tuning.txt or
 * ~/.cache/ptmi/batch_tuning.txt (PTMI_TUNE_CACHE set but empty: no file). */
pt_status pt_batch_group_plan(const pt_batch *b, uint32_t g, uint32_t *L, uint32_t *walkers_per_wg,
                              uint32_t *block_threads, uint32_t *sweeps_per_cycle);
void pt_batch_destroy(pt_batch *b);

/* ---- served form: a request loop over jobs that arrive at any time ----------
 * A server owns one device arena (the caller's memory) and admits submitted
 * jobs in arrival order while their footprint (pt_workspace_bytes) fits the
 * free arena, the resident-job limit and the resident-walker limit.  An admitted
 * job's lattices, tables, random-stream position and counters stay on the
 * device until it finishes.  Jobs whose replicas fit one workgroup's LDS
 * (2D L <= 512, EA L <= 32) join a batched lane: a stream whose cycles run
 * up to cycle_sweeps sweeps of every resident job in one launch per lattice-size
 * group, then their exchange steps (the batched form's kernels, membership
 * changing between cycles as jobs arrive and finish).  Every job in a lane
 * advances by the same sweeps per cycle, so a lane's cycle is paced by its
 * largest lattices; class_sites splits the batched jobs by size into lanes of
 * their own, so that small jobs are not paced by large ones.  Larger 2D lattices join
 * a tiled lane: a stream whose cycles run up to tiled_sweeps sweeps of every
 * resident job's tiles in one launch per lattice size, each job's last
 * workgroup folding its energies, records and exchange step; all lanes run
 * concurrently.  A job's results depend only on its own
 * pt_config (seed, stream_id, ...) and schedule, never on what else is
 * resident: they are bit-identical to running it alone with
 * pt_run(ctx, n_sweeps, exchange_every).  When a job finishes its observables
 * are copied to host memory and its arena slice is freed at once.
 * All work runs on streams the server creates (default priority, non-blocking).
 * One server must not be used from two threads at once. */
typedef struct pt_server pt_server;

#define PT_SERVER_CLASSES 3

typedef struct {
  uint32_t max_jobs;       /* resident jobs at once, 1 .. 65536 */
  uint32_t max_walkers;    /* per lane: resident replicas (batched lanes) or replica tiles (tiled lanes) */
  uint32_t tiled_lanes;    /* streams for jobs too large for the batched lanes, 1 .. 8 */
  uint32_t depth;          /* steps in flight per lane, 1 .. 8 */
  uint32_t cycle_sweeps;   /* batched lanes: at most this many sweeps per cycle, 1 .. 16 */
  uint32_t tiled_sweeps;   /* tiled lanes: at most this many sweeps per cycle, 1 .. PT_MAX_SWEEPS_PER_LAUNCH */
  uint32_t class_sites[PT_SERVER_CLASSES]; /* size classes of the batched lanes: ascending
                              sites-per-replica bounds, unused entries 0 (all 0: one batched
                              lane); a batched job runs on the lane of the first class
                              whose bound it does not exceed, lane 0 if none */
} pt_server_opts;

#define PT_JOB_KEEP_SPINS 1u /* keep the final lattices of all slots with the results */

typedef struct {
  uint64_t job_id;
  double arrival;          /* seconds on the server clock (as submitted) */
  double admitted;         /* when its initialisation was queued */
  double finished;         /* when the host saw its last step complete */
  uint64_t attempts;       /* R * L^dim * n_sweeps */
  uint32_t lane;           /* 0 batched (above every class), 1 .. tiled_lanes tiled,
                              tiled_lanes + 1 + k batched class k */
  uint32_t pad;
} pt_job_info;

typedef struct {
  uint64_t submitted, pending, resident, finished;
  uint64_t arena_bytes, arena_used, arena_peak;
  uint64_t walkers_resident;
  uint64_t batched_cycles, tiled_steps;
  uint64_t attempts_finished;
} pt_server_stats;

/* Device bytes the server keeps for its own tables ahead of the job arena. */
size_t pt_server_overhead_bytes(const pt_server_opts *opts);
/* Create a server on d_workspace (caller-owned, 256-byte aligned); the arena
 * for jobs is ws_bytes - pt_server_overhead_bytes(opts).  Uses the current HIP
 * device.  PT_ENOMEM if the workspace cannot hold the tables. */
pt_status pt_server_create(const pt_server_opts *opts, void *d_workspace, size_t ws_bytes,
                           pt_server **out);
/* Queue a job: cfg (copied; no init_spins or couplings uploads; record_every
 * needs max_records >= n_sweeps / record_every), n_sweeps in [1, 2^32 - 1]
 * sweeps with an exchange step after every exchange_every-th (0 = none), flags
 * (PT_JOB_KEEP_SPINS), arrival time on the server clock (negative = now).
 * PT_EINVAL for an invalid job, PT_ENOMEM if it could never fit the arena or
 * a lane, PT_EUNSUPPORTED if no tile of its lattice fits one workgroup. */
pt_status pt_server_submit(pt_server *sv, const pt_config *cfg, uint64_t n_sweeps,
                           uint32_t exchange_every, uint32_t flags, double arrival,
                           uint64_t *job_id);
/* One turn of the request loop: retire jobs whose last step has completed
 * (results to host, memory freed), admit queued jobs that now fit, and keep
 * `depth` steps in flight on every lane that has work.  If nothing completed,
 * waits up to wait_us microseconds for a step to complete.  *n_finished (may be
 * NULL) = jobs retired by this call. */
pt_status pt_server_step(pt_server *sv, uint32_t wait_us, uint32_t *n_finished);
/* Pop up to cap finished jobs (in completion order) into out; *n = count. */
pt_status pt_server_done(pt_server *sv, pt_job_info *out, uint32_t cap, uint32_t *n);
/* Results of a finished job, as pt_observables would give them (spins only with
 * PT_JOB_KEEP_SPINS).  PT_ESTATE if the job has not finished. */
pt_status pt_server_result(const pt_server *sv, uint64_t job_id, pt_obs *obs);
/* Drop a finished job's host-side results. */
pt_status pt_server_release(pt_server *sv, uint64_t job_id);
pt_status pt_server_stats_get(const pt_server *sv, pt_server_stats *out);
/* Seconds since the server was created (monotonic host clock). */
double pt_server_clock(const pt_server *sv);
/* Wait for all queued device work, then free the host state (never the workspace). */
void pt_server_destroy(pt_server *sv);

/* Thread-local message of the last failure on this thread ("" if none). */
const char *pt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PT_H */
