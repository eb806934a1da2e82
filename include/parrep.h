/*
 * parrep.h -- C ABI of libparrep: parallel replica dynamics (ParRep) for
 * bistable continuous-time Markov chain reaction networks on AMD MI355X.
 *
 * Method: Wang & Plechac, "Parallel replica dynamics method for bistable
 * stochastic reaction networks: simulation and sensitivity analysis"
 * (arXiv 1705.06807).  One solve runs Algorithm 1 (Sec. II A): serial
 * decorrelation, Fleming-Viot dephasing of R replicas, and the parallel step
 * whose first exit is credited by the ParRep-CTMC rule, cycling until the
 * ParRep clock reaches the horizon T.  Along the way it accumulates the
 * time-weighted stationary histogram (the ergodic average of Sec. I A) and
 * the path-space Fisher information and relative entropy rate integrands
 * (Sec. III, Appendix A) over the window [t_burn, T].
 *
 * All compute runs in HIP kernels for gfx950.  Conventions shared by every
 * entry point:
 *   - Pointers named "device" are HIP device pointers owned by the caller;
 *     pointers named "host" are read during the call only.
 *   - Calls that take a stream enqueue work on it and return without
 *     waiting; outputs are valid after the stream has been synchronised.
 *   - Functions return PARREP_OK or a negative parrep_status;
 *     parrep_last_error() gives a message for the calling thread.  No C++
 *     exception crosses this interface.
 *   - Random numbers: Philox4x32-10 with key (seed, instance_id) and counter
 *     (step, replica, cycle, phase tag << 28 | step >> 32); one block per SSA
 *     event.  Two solves with equal inputs give equal integer results.
 */
#ifndef PARREP_H
#define PARREP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PARREP_MAX_SPECIES 4
#define PARREP_MAX_REACTIONS 8
#define PARREP_MAX_FACTORS 2
#define PARREP_MAX_PARAMS 8
#define PARREP_MAX_REPLICAS 65536
#define PARREP_NCOUNTERS 12
#define PARREP_CYCLE_REC 12
#define PARREP_NSTATS 80

typedef enum {
    PARREP_OK = 0,
    PARREP_EINVAL = -1,       /* an argument is out of range or inconsistent   */
    PARREP_ENOMEM = -2,       /* device or host allocation failed               */
    PARREP_EDEVICE = -3,      /* a HIP call failed                              */
    PARREP_EUNSUPPORTED = -4, /* valid input the library does not handle       */
    PARREP_EBUSY = -5,        /* result not ready yet (server poll)             */
    PARREP_ECANCELLED = -6,   /* request was cancelled                          */
    PARREP_EOVERFLOW = -7     /* a run's spill table overflowed (see counters) */
} parrep_status;

/* Propensity factor kinds.  A reaction's propensity (Sec. I A) is
 *   lambda_j(x) = k_j * phi_1(x) * phi_2(x) * ...   (state factors, left to right)
 *   k_j = c[rate_param] * kappa * c[p_1] * ...     (PARREP_PARAM factors, left to right;
 *                                                   c[rate_param] omitted when < 0)
 * PARREP_FALLING:     phi = x_s (x_s-1) ... (x_s-order+1)     (mass action)
 * PARREP_HILL_REP:    phi = 1 / (1 + (x_s / K)^c[hill_param])  (repression)
 * PARREP_HILL_SWITCH: phi = c[hill_param] + (c[param2] - c[hill_param]) * q / (1 + q),
 *                     q = (x_s / c[param3])^order, order in 1..8
 *                     (the DNA switching rates F, G of Eq. (10), Sec. IV B)
 * PARREP_PARAM:       a parameter c[hill_param] that multiplies the rate constant
 *                     (e.g. gamma * b of Table IV)                                  */
enum { PARREP_FALLING = 0, PARREP_HILL_REP = 1, PARREP_HILL_SWITCH = 2, PARREP_PARAM = 3 };

/* Threshold units for decorrelation and dephasing: PARREP_STEPS counts
 * transitions (the paper's n_c, n_p); PARREP_TIME uses simulated time. */
enum { PARREP_STEPS = 0, PARREP_TIME = 1 };

/* counters[] slots of a result */
enum {
    PARREP_CNT_EV_DECORR = 0,        /* decorrelation events (all credited)        */
    PARREP_CNT_EV_DEPHASE = 1,       /* dephasing events                           */
    PARREP_CNT_EV_PAR_CREDITED = 2,  /* parallel-step events credited              */
    PARREP_CNT_EV_PAR_DISCARDED = 3, /* drawn in a last round but not credited     */
    PARREP_CNT_CYCLES = 4,           /* parallel steps that ended with an exit     */
    PARREP_CNT_S3_ROUNDS = 5,
    PARREP_CNT_S2_ROUNDS = 6,
    PARREP_CNT_STATUS = 7,           /* a PARREP_RUN_* value                       */
    PARREP_CNT_FV_RESTARTS = 8,
    PARREP_CNT_END_PHASE = 9,        /* 1 horizon in decorrelation, 3 in parallel step, 9 stopped */
    PARREP_CNT_N_CYCLE_LOG = 10,     /* cycle records produced (may exceed the capacity) */
    PARREP_CNT_SPILL_OVERFLOW = 11   /* credited events outside the histogram box whose state
                                        found no spill slot (their time is in the outside
                                        totals but not in FIM/RER/Y); 0 in normal runs */
};

/* counters[PARREP_CNT_STATUS] of a result.  Solves run asynchronously, so a
 * run that cannot complete its outputs reports it here (and a served request
 * through parrep_server_poll's status), not through the return value. */
enum {
    PARREP_RUN_OK = 0,             /* the clock reached the horizon                   */
    PARREP_RUN_BUDGET = 1,         /* the event budget stopped the run first           */
    PARREP_RUN_ABORTED = 2,        /* an instance spread over several workgroups gave up
                                      waiting at a grid barrier (outputs incomplete)  */
    PARREP_RUN_SPILL_OVERFLOW = 3  /* the horizon was reached, but time at states
                                      outside the histogram box found no spill slot:
                                      FIM, RER and Y miss it (PARREP_CNT_SPILL_OVERFLOW
                                      counts those credits)                           */
};

/* stats[] layout of a result (PARREP_NSTATS doubles) */
enum {
    PARREP_ST_T = 0,            /* ParRep clock at the end (= T unless stopped)            */
    PARREP_ST_OUTSIDE = 1,      /* time outside the histogram box, over [0, T]             */
    PARREP_ST_OUTSIDE_W = 2,    /* the same over [t_burn, T]                               */
    PARREP_ST_FIM = 3,          /* n_params x n_params, row-major: (1/(T-t_burn)) int FIM  */
    PARREP_ST_RER = 67,         /* n_params: (1/(T-t_burn)) int RER integrand, c_k*(1+eps_k) */
    PARREP_ST_Y = 75            /* n_species: int_{t_burn}^T x_i ds                          */
};

typedef struct parrep_ctx parrep_ctx;
typedef struct parrep_net parrep_net;
typedef struct parrep_plan parrep_plan;
typedef struct parrep_server parrep_server;

typedef struct {
    int32_t kind;        /* PARREP_FALLING, _HILL_REP, _HILL_SWITCH or _PARAM       */
    int32_t species;     /* species index the factor reads (not PARAM)             */
    int32_t order;       /* FALLING: order 0..8; HILL_SWITCH: exponent 1..8         */
    int32_t hill_param;  /* HILL_REP: exponent; HILL_SWITCH: value at x_s = 0;
                            PARAM: the parameter (indices into c)                   */
    int32_t param2;      /* HILL_SWITCH: index of the value as x_s -> infinity      */
    int32_t param3;      /* HILL_SWITCH: index of the scale (c[param3] > 0)         */
    double K;            /* HILL_REP: scale (> 0)                                    */
} parrep_factor;

typedef struct {
    int32_t rate_param;  /* index into c, or -1 for a fixed rate kappa              */
    int32_t n_factors;   /* 0..PARREP_MAX_FACTORS                                   */
    double kappa;        /* >= 0                                                     */
    int32_t stoich[PARREP_MAX_SPECIES];  /* net change eta_j: produced - consumed   */
    parrep_factor factor[PARREP_MAX_FACTORS];
} parrep_reaction;

/* The problem statement of one solve (Sec. II A, Alg. 1; Sec. IV for T and
 * the burn-in).  Unused array tails are ignored. */
typedef struct {
    double c[PARREP_MAX_PARAMS];         /* rate vector c (finite, >= 0)                 */
    double rer_eps[PARREP_MAX_PARAMS];   /* relative perturbation per parameter for RER  */
    int32_t use_rer;                     /* 0: RER outputs are zero                      */
    int32_t x0[PARREP_MAX_SPECIES];      /* initial population                           */
    int32_t region_w[PARREP_MAX_SPECIES];/* metastable sets: set 1 = {w.x >= theta},    */
    int64_t region_theta;                /*                   set 0 = {w.x <  theta}     */
    int32_t R;                           /* replicas, 1..PARREP_MAX_REPLICAS             */
    int32_t decorr_mode;                 /* PARREP_STEPS (n_c) or PARREP_TIME (t_c)      */
    double decorr;
    int32_t dephase_mode;                /* PARREP_STEPS (n_p) or PARREP_TIME (t_p)      */
    double dephase;
    double T;                            /* horizon, 0 < T < 2^51                        */
    double t_burn;                       /* window start for FIM/RER/Y, 0 <= t_burn < T  */
    int32_t hist_lo[PARREP_MAX_SPECIES]; /* histogram box, inclusive, unit bins,         */
    int32_t hist_hi[PARREP_MAX_SPECIES]; /* row-major with species 0 slowest             */
    uint32_t seed;                       /* Philox key word 0                            */
    uint32_t instance_id;                /* Philox key word 1                            */
    int64_t max_events;                  /* event budget, <= 0: 2^50                     */
} parrep_problem;

/* Caller-owned device buffers that receive one solve's outputs. */
typedef struct {
    double* hist;         /* device, nbins: time per state over [0, T]          (required) */
    double* hist_window;  /* device, nbins: time per state over [t_burn, T]     (required) */
    double* stats;        /* device, PARREP_NSTATS doubles (see PARREP_ST_*)     (required) */
    int32_t* x_final;     /* device, PARREP_MAX_SPECIES: state whose holding interval holds T */
    int64_t* counters;    /* device, PARREP_NCOUNTERS                            (required) */
    int64_t* cycle_log;   /* device, cycle_log_cap * PARREP_CYCLE_REC, or NULL: per cycle
                             {cycle, S1 events, S2 rounds, S3 rounds, K (0: no exit),
                              end phase, state after the cycle[4], 0, 0}               */
    int32_t cycle_log_cap;
    int32_t reserved;
    int64_t* phase_clock; /* device, 4 int64 or NULL: wall-clock ticks the workgroup spent in
                             decorrelation, dephasing, the parallel step, and in total
                             (ticks of the device's constant wall clock, see
                             parrep_wall_clock_hz)                                       */
} parrep_result;

/* Launch shape for the batched solve: replicas per lane and waves per
 * workgroup (0 = let the library choose from the replica count), and two
 * optional hipEvent_t handles (NULL = none) recorded on the stream right
 * before and right after the instance kernel, so a caller can time it.
 *
 * A single-instance batch can instead spread its one instance over the
 * workgroups of a cooperative launch (4 waves each, replicas_per_lane 1 or
 * 4): the replicas are split into contiguous ranges that run their rounds
 * independently and meet only at the end of chunks of rounds, where they
 * agree on the first exit, the dephasing stop and the horizon, and replay
 * the chunk up to that point (outputs equal the one-workgroup solve's:
 * integers exactly, floats up to summation order).  workgroups: 0 = the
 * library's choice (spread when R >= 8192 and no shape is forced, over
 * ceil(R / (256 replicas_per_lane)) workgroups), 1 = one workgroup, n > 1 =
 * spread over n (at least ceil(R / (256 replicas_per_lane)); no more than
 * can be resident at once, else EDEVICE).  Each wait at a chunk's meeting
 * point is bounded by barrier_wait_us (0 = 2 s); a run that gives up ends
 * with status PARREP_RUN_ABORTED. */
typedef struct {
    int32_t replicas_per_lane;  /* 1, 4 or 16; or 64 with 16 waves (R > 16384)       */
    int32_t waves;              /* 1, 4 or 16 (64-lane wavefronts per workgroup)      */
    void* event_before;         /* hipEvent_t or NULL                                 */
    void* event_after;          /* hipEvent_t or NULL                                 */
    int32_t workgroups;         /* single-instance batches, see above                 */
    int32_t chunk_rounds[2];    /* spread runs: dephasing and parallel-step chunk
                                   lengths in rounds (0 = 512 and 64; the second <= 64) */
    int32_t barrier_wait_us;    /* spread runs: longest wait at a meeting point       */
    int32_t histogram_staging;  /* parallel-step credits (<= 2 species, <= 4 reactions,
                                   <= 4 replicas per lane, <= 4 waves; other shapes
                                   credit directly):
                                   0 = library choice (the autotuned setting, else off),
                                   -1 = one HBM atomic per credit, 1 = credits at states
                                   in a 1024-bin tile of the box (placed per parallel
                                   step on the replicas' mean) go to LDS and are flushed
                                   with one atomic per visited bin; either setting fixes
                                   the shape as replicas_per_lane and waves do          */
    int32_t flush_period;       /* staged: also flush every this many rounds (0 = only
                                   at the step's end and at the burn-in time)          */
    int32_t persistent;         /* 0 = one workgroup per instance (the default); 1 = the
                                   persistent form: as many workgroups as the device
                                   holds at once, each taking the group's instances
                                   (longest first) from a counter until all are run;
                                   not with staging or spread instances               */
} parrep_launch;

/* Create a context on a HIP device: it owns the scratch arena and the
 * compiled kernels.  EDEVICE if the device cannot be used. */
int parrep_ctx_create(int device, parrep_ctx** out);
void parrep_ctx_destroy(parrep_ctx* ctx);

/* Frequency in Hz of the wall clock that phase_clock counts (0 on error). */
double parrep_wall_clock_hz(parrep_ctx* ctx);

/* Thread-local message for the last failing call of this thread. */
const char* parrep_last_error(void);

/* Define a reaction network (Sec. I A): n_species <= 4, n_reactions <= 8,
 * n_params <= 8, reactions rx[n_reactions] read during the call (host).
 * EINVAL when an index is out of range, an order exceeds 8 (or a switch
 * exponent is outside 1..8), K <= 0, kappa is negative or not finite, or a
 * stoichiometric coefficient is outside [-128, 127].  Solves need integral
 * Hill exponents in [0, 64] (EUNSUPPORTED otherwise) and positive switch
 * scales c[param3] (EINVAL). */
int parrep_net_create(parrep_ctx* ctx, int32_t n_species, int32_t n_reactions, int32_t n_params,
                      const parrep_reaction* rx, parrep_net** out);
void parrep_net_destroy(parrep_net* net);

/* Number of histogram bins the problem asks for (host arithmetic only);
 * negative on invalid boxes. */
int64_t parrep_problem_nbins(const parrep_net* net, const parrep_problem* prob);

/* One ParRep solve (Alg. 1 from x0 until the clock reaches T), enqueued on
 * stream (a hipStream_t; NULL = the null stream).  prob is host memory read
 * during the call; res holds caller-owned device buffers.  EINVAL on
 * inconsistent input (validated before anything is enqueued). */
int parrep_solve(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                 const parrep_result* res, void* stream);

/* Many independent solves in one launch: count >= 1 instances, nets[i] and
 * probs[i] (host arrays), res[i] (host array of device-buffer descriptors).
 * Each instance's outputs equal its parrep_solve outputs for any launch
 * shape (integers exactly; floats up to summation order).  launch may be
 * NULL; without a forced shape each instance gets: in a batch of no more
 * instances than the device has CUs and 64 < R <= 256, one replica per lane
 * over 4 waves; else the autotuned shape of its replica-count bucket; else
 * the default for R (replicas per lane x waves: R <= 64 1x1, <= 256 4x1,
 * <= 1024 4x4, <= 4096 4x16, <= 16384 16x16, else 64x16). */
int parrep_solve_batch(parrep_ctx* ctx, int32_t count, const parrep_net* const* nets,
                       const parrep_problem* probs, const parrep_result* res,
                       const parrep_launch* launch, void* stream);

/* Bytes of the fixed device array that holds parrep_solve_noalloc's scratch. */
#define PARREP_NOALLOC_SCRATCH_BYTES (2u << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as parrep_solve (equal outputs: integers exactly, floats up to
 * summation order), but it calls no hipMalloc, hipFree or other allocating
 * routine: the instance's descriptor and scratch (propensity table,
 * outside-box accumulators, spill table, exchange and scan buffers) go to a
 * fixed array of PARREP_NOALLOC_SCRATCH_BYTES in device memory that each GPU
 * the library runs on holds until the process ends.  The descriptor is
 * written by a kernel (no host copy), and the scratch is cleared by the
 * solve's own kernels.  EINVAL when the problem's scratch exceeds the array
 * (it grows with R and with the histogram box's largest coordinate: about
 * 48 bytes per replica plus 64 bytes per table state; R = 65536 does not
 * fit).  Every call on one GPU uses that GPU's one array, which keeps the
 * last call's contents: calls whose work can overlap on the device (other
 * streams, other threads, other contexts on the same GPU) race and give
 * wrong results; order them on one stream. */
int parrep_solve_noalloc(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                         const parrep_result* res, void* stream);

/* ---- Batched form: plans ------------------------------------------------
 * A plan is a batch of instances prepared once: descriptors and scratch in
 * device memory the plan owns, the instances grouped by launch shape (the
 * autotuned one where parrep_autotune has run for that replica-count
 * bucket, else the library default), each group ordered longest first, and
 * setup / zero / the group launches (side by side) / finalize captured into
 * one hipGraph.  Outputs go to the res[i] buffers given at creation.
 * launch may be NULL; its shape fields force one launch shape as in
 * parrep_solve_batch (its events are not used: see parrep_plan_run).
 * Problems as in parrep_solve_batch; EINVAL on invalid input, EDEVICE if a
 * HIP call fails (nothing is left allocated then). */
int parrep_plan_create(parrep_ctx* ctx, int32_t count, const parrep_net* const* nets,
                       const parrep_problem* probs, const parrep_result* res,
                       const parrep_launch* launch, parrep_plan** out);

/* Replace instance `index`'s problem (host, read during the call) for the
 * following launches: the copy is enqueued on stream, so updates and
 * launches on one stream apply in order.  Rate vector, seed, instance id,
 * initial state, thresholds, horizon and budget may change; the histogram
 * box and the table length (from hist_hi and x0) must not, and R may not
 * exceed the planned replica count (EINVAL). */
int parrep_plan_update(parrep_plan* plan, int32_t index, const parrep_problem* prob,
                       void* stream);

/* Replay the plan's graph on stream (outputs are rewritten each time). */
int parrep_plan_launch(parrep_plan* plan, void* stream);

/* The same work as a replay, enqueued on stream as individual kernel
 * launches (the plan's resident descriptors and scratch, no graph), with two
 * optional hipEvent_t (NULL = none) recorded on stream right before and right
 * after the instance kernels: the form in which those kernels can be timed
 * with events. */
int parrep_plan_run(parrep_plan* plan, void* event_before, void* event_after, void* stream);

/* Waits for the plan's last launch or update, then frees it. */
void parrep_plan_destroy(parrep_plan* plan);

/* Launch-shape autotuner: times `instances` copies of prob (instance ids
 * prob->instance_id + i, each cut to trial_events events) for every compiled
 * shape that holds prob->R replicas (up to 16x), and for the narrow kernels
 * every histogram staging setting (off, flushed at the step's end, flushed
 * every 64 rounds), keeps the fastest for R's bucket (the next power of two
 * >= max(R, 64)), this species count and reaction class, and returns it in
 * *chosen.  scratch: device buffers that all trial instances overwrite
 * (their values are meaningless), except the histograms: the library
 * allocates one pair per trial instance (up to 64 GiB in all, freed before it
 * returns; beyond that the trials share scratch's), so that the trials'
 * credits do not contend as no real batch's do.  Blocking. */
int parrep_autotune(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                    int32_t instances, int64_t trial_events, const parrep_result* scratch,
                    parrep_launch* chosen);

/* ---- Served form ----------------------------------------------------------
 * A request asks for a ParRep estimate of one problem to a relative standard
 * error: independent runs (instance ids prob.instance_id + k) pooled until
 * the error of the pooled FIM diagonal and window integrals is at most
 * rse_target (<= 0: exactly max_runs runs), max_runs runs are done, or
 * event_budget events were spent (<= 0: no budget), with at least min_runs
 * runs.  The server's worker thread admits requests in arrival order while
 * device memory stays within the budget, and launches whatever runs are
 * ready as one batch on a free server stream, so requests that arrive while
 * others run overlap with them on the device.  Each run equals a plain
 * solve of its problem. */
typedef struct {
    double rse_target;
    int32_t min_runs;      /* >= 1 (the error needs two)                          */
    int32_t max_runs;      /* >= min_runs                                         */
    int64_t event_budget;
} parrep_request;

typedef struct {
    int32_t runs;          /* runs pooled                                         */
    int32_t status;        /* PARREP_OK or the error that stopped the request     */
    double rse;            /* achieved relative standard error (NaN below 2 runs) */
    int64_t events;        /* algorithmic events over all runs                    */
    double latency_s;      /* submit to the last run's completion                 */
    double iaf[PARREP_MAX_SPECIES]; /* integrated autocorrelation of x_i over the
                              window, from the spread of the runs' window integrals:
                              sum_k (Y_k - mean)^2 / ((T - t_burn)(runs - 1))       */
} parrep_request_info;

/* mem_budget: device bytes the server may hold for admitted requests and
 * their in-flight runs (0: half of the free device memory); n_streams in
 * [1, 16] batches may be in flight at once.  The server owns a worker
 * thread; all server calls are thread-safe. */
int parrep_server_create(parrep_ctx* ctx, size_t mem_budget, int32_t n_streams,
                         parrep_server** out);

/* Queue a request (prob and rq are copied; net must outlive the request).
 * ENOMEM if one run alone exceeds the memory budget. */
int parrep_server_submit(parrep_server* server, const parrep_net* net,
                         const parrep_problem* prob, const parrep_request* rq,
                         uint64_t* ticket);

/* EBUSY while the request runs (wait = 0), else blocks until it is done.
 * Then writes the pooled outputs to res (host or device buffers; may be
 * NULL): hist and hist_window summed over runs; stats with the clock and
 * the outside-box times summed and FIM, RER and window integrals averaged;
 * counters summed (status: the largest); x_final of the last run.  info
 * (may be NULL) describes the request.  The ticket is released (EINVAL if
 * unknown); ECANCELLED for a cancelled request. */
int parrep_server_poll(parrep_server* server, uint64_t ticket, const parrep_result* res,
                       parrep_request_info* info, int32_t wait);

/* Stop a request: runs in flight finish and are discarded. */
int parrep_server_cancel(parrep_server* server, uint64_t ticket);

/* Cancels what is still queued or running, waits for the device, frees all. */
void parrep_server_destroy(parrep_server* server);

/* Test hook: Philox4x32-10 blocks.  ctr_key (device, n x 6 uint32:
 * counter words 0-3 then key words 0-1) -> out (device, n x 4 uint32). */
int parrep_philox(parrep_ctx* ctx, int64_t n, const uint32_t* ctr_key, uint32_t* out,
                  void* stream);

/* Test hook: one SSA event (Sec. I A; the "generate tau and J" step of Alg. 1)
 * per row: states (device, n x PARREP_MAX_SPECIES int32), blocks (device,
 * n x 4 uint32 Philox words) -> a0 (device, n), tau (device, n; +inf when
 * absorbing), J (device, n; -1 when absorbing). */
int parrep_events(parrep_ctx* ctx, const parrep_net* net, const double* c_host, int64_t n,
                  const int32_t* states, const uint32_t* blocks, double* a0, double* tau,
                  int32_t* J, void* stream);

/* Test hook: the dephasing step alone (Sec. II A, Alg. 1) from state xt
 * (host, n_species), in the set of xt, with prob's replica count, dephasing
 * threshold and key, at cycle index `cycle`.  Y_out (device, R x
 * PARREP_MAX_SPECIES int32) receives the replica states; rounds_out (device,
 * one int64) the number of rounds. */
int parrep_dephase_only(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                        const int32_t* xt, uint32_t cycle, int32_t* Y_out, int64_t* rounds_out,
                        void* stream);

/* Test hook: the parallel step alone (Sec. II A, Alg. 1) from replica states
 * init (device, R x PARREP_MAX_SPECIES int32, all in the set of replica 0),
 * without a horizon, for at most max_rounds rounds (< 0: no limit).
 * out_i64 (device, 2): {N*, K} ({-1, 0} if the round limit came first);
 * exit_state (device, PARREP_MAX_SPECIES); credited (device, 1 double):
 * the credited time sum_{keys <= R(N*-1)+K} tau. */
int parrep_parallel_only(parrep_ctx* ctx, const parrep_net* net, const parrep_problem* prob,
                         const int32_t* init, uint32_t cycle, int64_t max_rounds,
                         int64_t* out_i64, int32_t* exit_state, double* credited, void* stream);

#ifdef __cplusplus
}
#endif
#endif
