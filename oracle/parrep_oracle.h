/*
 * parrep_oracle.h -- CPU oracle for parallel replica dynamics (ParRep) on
 * continuous-time Markov chain reaction networks.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the GPU library neither includes this
 * header nor links this code, and this code includes nothing of the GPU
 * library's.
 *
 * Everything here follows Wang & Plechac, "Parallel replica dynamics method
 * for bistable stochastic reaction networks" (arXiv 1705.06807):
 *   - the network model and propensities: Sec. I A, eq. (Q);
 *   - the Gillespie step "generate tau and J": Sec. I, Alg. 1;
 *   - decorrelation / dephasing (Fleming-Viot) / parallel step: Sec. II A, Alg. 1;
 *   - ergodic averages, FIM and relative entropy rate: Sec. III, Appendix A.
 */
#ifndef PARREP_ORACLE_H
#define PARREP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_SPECIES 4
#define OR_MAX_REACTIONS 8
#define OR_MAX_FACTORS 2
#define OR_MAX_PARAMS 8
#define OR_NCOUNTERS 12
#define OR_CYCLE_REC 12

enum { OR_FALLING = 0, OR_HILL_REP = 1, OR_HILL_SWITCH = 2, OR_PARAM = 3 };
enum { OR_STEPS = 0, OR_TIME = 1 };
enum { OR_TAG_DECORR = 1, OR_TAG_DEPHASE = 2, OR_TAG_FV = 3, OR_TAG_PARALLEL = 4 };

/* counters[] slots */
enum {
    OR_C_EV_DECORR = 0,      /* S1 events (all credited)                       */
    OR_C_EV_DEPHASE = 1,     /* S2 events                                       */
    OR_C_EV_PAR_CREDITED = 2,/* S3 events credited (key <= key*)                */
    OR_C_EV_PAR_DISCARDED = 3,/* S3 events drawn in a last round but not credited */
    OR_C_CYCLES = 4,         /* parallel steps that ended with an exit           */
    OR_C_S3_ROUNDS = 5,
    OR_C_S2_ROUNDS = 6,
    OR_C_STATUS = 7,         /* 0 horizon reached, 1 event budget exhausted      */
    OR_C_FV_RESTARTS = 8,
    OR_C_END_PHASE = 9,      /* 1: horizon met in S1, 3: in S3, 9: budget        */
    OR_C_N_CYCLE_LOG = 10    /* records written to cycle_log (may exceed cap)    */
};

typedef struct {
    int32_t kind;        /* OR_FALLING, OR_HILL_REP, OR_HILL_SWITCH or OR_PARAM */
    int32_t species;
    int32_t order;       /* falling factorial order; switch exponent */
    int32_t hill_param;  /* Hill exponent; switch value at 0; the PARAM parameter */
    int32_t param2;      /* switch value at infinity */
    int32_t param3;      /* switch scale */
    double K;            /* Hill scale */
} or_factor;

typedef struct {
    int32_t rate_param;  /* index into c, or -1 for a fixed rate kappa */
    int32_t n_factors;
    double kappa;
    int32_t stoich[OR_MAX_SPECIES];   /* net change: produced - consumed */
    or_factor f[OR_MAX_FACTORS];
} or_reaction;

typedef struct {
    int32_t n_species, n_reactions, n_params, reserved;
    or_reaction rx[OR_MAX_REACTIONS];
} or_net;

typedef struct {
    double c[OR_MAX_PARAMS];
    double rer_eps[OR_MAX_PARAMS];
    int32_t use_rer;
    int32_t x0[OR_MAX_SPECIES];
    int32_t region_w[OR_MAX_SPECIES];
    int64_t region_theta;
    int32_t R;
    int32_t decorr_mode;
    double decorr;
    int32_t dephase_mode;
    double dephase;
    double T, t_burn;
    int32_t hist_lo[OR_MAX_SPECIES], hist_hi[OR_MAX_SPECIES];
    uint32_t seed, instance_id;
    int64_t max_events;
} or_problem;

typedef struct {
    double* hist;        /* nbins: time per state over [0, T]           */
    double* hist_w;      /* nbins: time per state over [t_burn, T]      */
    double outside, outside_w;
    double T_s;
    double fim[OR_MAX_PARAMS * OR_MAX_PARAMS];  /* window average */
    double rer[OR_MAX_PARAMS];                  /* window average */
    double y[OR_MAX_SPECIES];                   /* window integrals of x_i */
    int32_t x_final[OR_MAX_SPECIES];
    int64_t counters[OR_NCOUNTERS];
    int64_t* cycle_log;  /* cycle_log_cap records of OR_CYCLE_REC int64, may be NULL */
    int32_t cycle_log_cap;
} or_result;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_uniforms(const uint32_t blk[4], double out[2]);
int or_event(const or_net* net, const double* c, const int32_t* x, const uint32_t blk[4],
             double* lam, double* a0, double* tau, int32_t* J);
void or_fim_rer(const or_net* net, const double* c, const double* rer_eps, int32_t use_rer,
                const int32_t* x, double* fim, double* rer);
int or_run(const or_net* net, const or_problem* pb, or_result* res);
int or_dephase(const or_net* net, const or_problem* pb, const int32_t* xt, uint32_t cycle,
               int32_t* Y_out, int64_t* rounds_out);
int or_parallel(const or_net* net, const or_problem* pb, const int32_t* init, uint32_t cycle,
                int64_t max_rounds, int64_t* nstar_K, int32_t* exit_state, double* credited);
/* Multi-run estimators of Sec. III over n >= 2 independent runs of one
 * problem: fim (n x np*np), rer (n x np) and y (n x ns, window integrals)
 * per run, window = T - t_burn.  Outputs: means of fim, rer and y; the 95 %
 * half-width 1.96 sd / sqrt(n) of each FIM diagonal entry; iaf[i] =
 * sum_r (y_i^r - mean)^2 / (window (n - 1)); bound[i*np + k] =
 * sqrt(iaf[i] fim_mean[k,k]). */
void or_estimate(int n, int np, int ns, const double* fim, const double* rer, const double* y,
                 double window, double* fim_mean, double* fim_hw, double* rer_mean,
                 double* y_mean, double* iaf, double* bound);

#ifdef __cplusplus
}
#endif
#endif
