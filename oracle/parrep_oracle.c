/*
 * parrep_oracle.c -- CPU oracle for ParRep on CTMC reaction networks.
 *
 * TEST INFRASTRUCTURE ONLY (see parrep_oracle.h).  Plain C, single thread,
 * no blocking or reordering: Algorithm 1 of Wang & Plechac (arXiv 1705.06807,
 * Sec. II A) executed step by step, with the numerical conventions below that
 * the paper leaves open.  Build with -ffp-contract=off so that no product is
 * fused into an addition.
 *
 * Conventions (readings of the paper where it is silent):
 *  - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with
 *    key = (seed, instance) and counter = (step, replica, cycle,
 *    tag<<28 | step>>32).  One block per SSA event: words 0-1 give
 *    u_open in (0,1], words 2-3 give u_sel in [0,1).
 *  - SSA event (Gillespie): tau = -log(u_open)/a0; J = first j with
 *    u_sel*a0 < S_j, S_j the left-to-right partial sums of the propensities.
 *    a0 = 0 is absorbing: tau = +inf and no jump.
 *  - Clock: the ParRep clock T_s is an exact 64.64 fixed-point sum of the
 *    credited holding times (each truncated to 2^-64; +inf and values of
 *    2^52 or more saturate at 2^52), so the horizon T and the burn-in time
 *    t_b are crossed at one well-defined event whatever the summation order.
 *  - Decorrelation counts either transitions (paper, n_c) or continuous
 *    credited time in the current set; leaving the set makes the new set
 *    current and resets the count.
 *  - Dephasing runs synchronous embedded-chain rounds; an exited replica
 *    restarts from the post-round state of a survivor picked uniformly
 *    (index floor(word0 * |S| / 2^32) of the survivors in ascending order);
 *    with no survivor all restart from the decorrelated state.  In time mode
 *    it stops after the first round with min_r t^r >= t_p.
 *  - Parallel step: exit is tested on post-jump states; the pre-jump states
 *    of replicas 1..K are credited in replica order; the state after the
 *    cycle is the post-jump state of replica K.
 */
#include "parrep_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11: Philox-4x32 with 10 rounds).   */
/* ------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;  /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;  /* Weyl key increments */
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_uniforms(const uint32_t b[4], double out[2])
{
    uint64_t w01 = (uint64_t)b[0] | ((uint64_t)b[1] << 32);
    uint64_t w23 = (uint64_t)b[2] | ((uint64_t)b[3] << 32);
    out[0] = (double)((w01 >> 11) + 1) * 0x1.0p-53;  /* (0, 1] */
    out[1] = (double)(w23 >> 11) * 0x1.0p-53;        /* [0, 1) */
}

/* ------------------------------------------------------------------ */
/* Propensities (Sec. I A; Tables I and IV give the model forms).      */
/* ------------------------------------------------------------------ */
static int is_small_int(double h)
{
    return h >= 0.0 && h <= 64.0 && h == floor(h);
}

/* y^h: repeated multiplication for integral h (q = y, then q*y, ...), pow otherwise. */
static double hill_power(double y, double h)
{
    if (is_small_int(h)) {
        int n = (int)h;
        if (n == 0) return 1.0;
        double q = y;
        for (int i = 1; i < n; ++i) q = q * y;
        return q;
    }
    return pow(y, h);
}

static double factor_value(const or_factor* f, const int32_t* x, const double* c)
{
    int64_t xs = x[f->species];
    if (f->kind == OR_FALLING) {
        int64_t p = 1;
        for (int i = 0; i < f->order; ++i) {
            int64_t t = xs - i;
            if (t <= 0) return 0.0;
            p *= t;
        }
        return (double)p;
    }
    if (f->kind == OR_HILL_SWITCH) {
        /* c_lo + (c_hi - c_lo) q/(1+q), q = (x/c_K)^n: Eq. (10) of Sec. IV B */
        double y = (double)xs / c[f->param3];
        double q = hill_power(y, (double)f->order);
        double s = q / (1.0 + q);
        return c[f->hill_param] + (c[f->param2] - c[f->hill_param]) * s;
    }
    /* OR_HILL_REP: 1 / (1 + (x/K)^h) */
    double y = (double)xs / f->K;
    double q = hill_power(y, c[f->hill_param]);
    return 1.0 / (1.0 + q);
}

/* lambda = (c_rate kappa) * (PARAM factors) * (state factors), each group
 * left to right. */
static double propensity(const or_reaction* r, const int32_t* x, const double* c)
{
    double lam = (r->rate_param >= 0) ? c[r->rate_param] * r->kappa : r->kappa;
    for (int k = 0; k < r->n_factors; ++k)
        if (r->f[k].kind == OR_PARAM) lam = lam * c[r->f[k].hill_param];
    for (int k = 0; k < r->n_factors; ++k)
        if (r->f[k].kind != OR_PARAM) lam = lam * factor_value(&r->f[k], x, c);
    return lam;
}

/* One Gillespie event at state x from one Philox block.  Returns 1 when the
 * state is absorbing (a0 == 0): tau = +inf and *J = -1. */
int or_event(const or_net* net, const double* c, const int32_t* x, const uint32_t blk[4],
             double* lam, double* a0_out, double* tau, int32_t* J)
{
    double u[2];
    or_uniforms(blk, u);
    double S[OR_MAX_REACTIONS];
    double s = 0.0;
    int m = net->n_reactions;
    for (int j = 0; j < m; ++j) {
        double l = propensity(&net->rx[j], x, c);
        if (lam) lam[j] = l;
        s = s + l;
        S[j] = s;
    }
    double a0 = s;
    if (a0_out) *a0_out = a0;
    if (!(a0 > 0.0)) {
        *tau = INFINITY;
        *J = -1;
        return 1;
    }
    *tau = (-log(u[0])) / a0;
    double t = u[1] * a0;
    int pick = -1;
    for (int j = 0; j < m; ++j) {
        if (t < S[j]) { pick = j; break; }
    }
    if (pick < 0) {  /* cannot happen for finite a0 > 0; keep the last positive channel */
        for (int j = m - 1; j >= 0; --j) {
            double l = propensity(&net->rx[j], x, c);
            if (l > 0.0) { pick = j; break; }
        }
    }
    *J = pick;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Path-space FIM and relative entropy rate integrands (Sec. III and   */
/* Appendix A): FIM(x) = sum_j lam_j grad log lam_j grad log lam_j^T,  */
/* RER_k(x) = sum_j [lam_j log(lam_j/lam'_j) - lam_j + lam'_j] with    */
/* c'_k = c_k (1 + eps_k).                                             */
/* ------------------------------------------------------------------ */
static void grad_log_lambda(const or_reaction* r, const int32_t* x, const double* c, int np,
                            double* g)
{
    for (int p = 0; p < np; ++p) g[p] = 0.0;
    if (r->rate_param >= 0) g[r->rate_param] += 1.0 / c[r->rate_param];
    for (int k = 0; k < r->n_factors; ++k) {
        const or_factor* f = &r->f[k];
        if (f->kind == OR_PARAM) {
            g[f->hill_param] += 1.0 / c[f->hill_param];
        } else if (f->kind == OR_HILL_SWITCH) {
            /* phi = lo + (hi - lo) s, s = q/(1+q): d phi/d lo = 1 - s,
             * d phi/d hi = s, d phi/d K = -(hi - lo) n s (1 - s) / K */
            double phi = factor_value(f, x, c);
            if (!(phi > 0.0)) continue;
            double y = (double)x[f->species] / c[f->param3];
            double q = hill_power(y, (double)f->order);
            double s = q / (1.0 + q);
            double lo = c[f->hill_param], hi = c[f->param2], K = c[f->param3];
            g[f->hill_param] += (1.0 - s) / phi;
            g[f->param2] += s / phi;
            g[f->param3] += -(hi - lo) * f->order * s * (1.0 - s) / (K * phi);
        } else if (f->kind == OR_HILL_REP) {
            double y = (double)x[f->species] / f->K;
            if (!(y > 0.0)) continue;             /* q ln y -> 0 as y -> 0 */
            double q = hill_power(y, c[f->hill_param]);
            g[f->hill_param] += -q * log(y) / (1.0 + q);
        }
    }
}

void or_fim_rer(const or_net* net, const double* c, const double* rer_eps, int32_t use_rer,
                const int32_t* x, double* fim, double* rer)
{
    int np = net->n_params, m = net->n_reactions;
    for (int a = 0; a < np * np; ++a) fim[a] = 0.0;
    for (int a = 0; a < np; ++a) rer[a] = 0.0;
    double g[OR_MAX_PARAMS];
    for (int j = 0; j < m; ++j) {
        const or_reaction* r = &net->rx[j];
        double lam = propensity(r, x, c);
        if (!(lam > 0.0)) continue;
        grad_log_lambda(r, x, c, np, g);
        for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) fim[a * np + b] += lam * g[a] * g[b];
    }
    if (!use_rer) return;
    double cp[OR_MAX_PARAMS];
    for (int k = 0; k < np; ++k) {
        for (int p = 0; p < np; ++p) cp[p] = c[p];
        cp[k] = c[k] * (1.0 + rer_eps[k]);
        double h = 0.0;
        for (int j = 0; j < m; ++j) {
            double lam = propensity(&net->rx[j], x, c);
            double lp = propensity(&net->rx[j], x, cp);
            if (lam > 0.0) h += lam * log(lam / lp) - lam + lp;
            else h += lp;
        }
        rer[k] = h;
    }
}

/* ------------------------------------------------------------------ */
/* Exact 64.64 fixed-point clock.                                      */
/* ------------------------------------------------------------------ */
static u128 to_fx(double d)
{
    if (!(d < 0x1.0p52)) return (u128)1 << 116;   /* +inf and values >= 2^52 saturate */
    if (!(d > 0.0)) return 0;
    double ip = floor(d);
    double a = (d - ip) * 0x1.0p32;
    double ahi = floor(a);
    double b = (a - ahi) * 0x1.0p32;
    double blo = floor(b);
    return ((u128)(uint64_t)ip << 64) | ((u128)(uint64_t)ahi << 32) | (u128)(uint64_t)blo;
}

static double fx_to_double(u128 v)
{
    return (double)(uint64_t)(v >> 64) + ldexp((double)(uint64_t)v, -64);
}

/* Neumaier compensated sum for the scalar accumulators. */
typedef struct { double s, c; } ksum;
static void kadd(ksum* k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static double kval(const ksum* k) { return k->s + k->c; }

/* ------------------------------------------------------------------ */
/* Run state                                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    const or_net* net;
    const or_problem* pb;
    or_result* res;     /* may be NULL for the step-only entry points */
    uint32_t key[2];
    u128 C, Tq, tbq;
    int n, np;
    int64_t stride[OR_MAX_SPECIES];
    int64_t nb[OR_MAX_SPECIES];
    ksum fim[OR_MAX_PARAMS * OR_MAX_PARAMS], rer[OR_MAX_PARAMS], y[OR_MAX_SPECIES];
    int64_t ev_total, max_events;
    int32_t xend[OR_MAX_SPECIES];
} run_t;

static void draw(const run_t* s, uint64_t step, uint32_t rep, uint32_t cycle, uint32_t tag,
                 uint32_t out[4])
{
    uint32_t ctr[4];
    ctr[0] = (uint32_t)step;
    ctr[1] = rep;
    ctr[2] = cycle;
    ctr[3] = (tag << 28) | ((uint32_t)(step >> 32) & 0x0FFFFFFFu);
    or_philox4x32_10(ctr, s->key, out);
}

static int region_of(const run_t* s, const int32_t* x)
{
    int64_t d = 0;
    for (int i = 0; i < s->n; ++i) d += (int64_t)s->pb->region_w[i] * (int64_t)x[i];
    return d >= s->pb->region_theta ? 1 : 0;
}

static void apply_jump(const run_t* s, int32_t* x, int J)
{
    if (J < 0) return;
    for (int i = 0; i < s->n; ++i) x[i] += s->net->rx[J].stoich[i];
}

static int64_t hist_index(const run_t* s, const int32_t* x)
{
    int64_t idx = 0;
    for (int i = 0; i < s->n; ++i) {
        int64_t o = (int64_t)x[i] - s->pb->hist_lo[i];
        if (o < 0 || o >= s->nb[i]) return -1;
        idx += o * s->stride[i];
    }
    return idx;
}

/* Credit the holding time tau spent at x (Alg. 1: T_s += tau, I_s += f(x) tau),
 * truncated at the horizon T.  Returns 1 when the horizon has been reached. */
static int credit(run_t* s, const int32_t* x, double tau)
{
    u128 tq = to_fx(tau);
    u128 E = s->C + tq;
    int hit = 0;
    double full = tau;
    if (E >= s->Tq) {
        hit = 1;
        E = s->Tq;
        full = fx_to_double(E - s->C);
    }
    double w;
    if (E <= s->tbq) w = 0.0;
    else if (s->C >= s->tbq) w = full;
    else w = fx_to_double(E - s->tbq);
    if (s->res) {
        int64_t idx = hist_index(s, x);
        if (idx >= 0) {
            s->res->hist[idx] += full;
            s->res->hist_w[idx] += w;
        } else {
            s->res->outside += full;
            s->res->outside_w += w;
        }
        if (w > 0.0) {
            double fim[OR_MAX_PARAMS * OR_MAX_PARAMS], rer[OR_MAX_PARAMS];
            or_fim_rer(s->net, s->pb->c, s->pb->rer_eps, s->pb->use_rer, x, fim, rer);
            for (int a = 0; a < s->np * s->np; ++a) kadd(&s->fim[a], w * fim[a]);
            for (int a = 0; a < s->np; ++a) kadd(&s->rer[a], w * rer[a]);
            for (int i = 0; i < s->n; ++i) kadd(&s->y[i], w * (double)x[i]);
        }
    }
    s->C = E;
    if (hit) memcpy(s->xend, x, sizeof(int32_t) * (size_t)s->n);
    return hit;
}

static int init_run(run_t* s, const or_net* net, const or_problem* pb, or_result* res)
{
    memset(s, 0, sizeof(*s));
    s->net = net;
    s->pb = pb;
    s->res = res;
    s->n = net->n_species;
    s->np = net->n_params;
    if (s->n < 1 || s->n > OR_MAX_SPECIES || net->n_reactions < 1 ||
        net->n_reactions > OR_MAX_REACTIONS || s->np < 0 || s->np > OR_MAX_PARAMS || pb->R < 1)
        return -1;
    s->key[0] = pb->seed;
    s->key[1] = pb->instance_id;
    s->Tq = to_fx(pb->T);
    s->tbq = to_fx(pb->t_burn);
    s->max_events = pb->max_events > 0 ? pb->max_events : INT64_MAX;
    int64_t st = 1;
    for (int i = s->n - 1; i >= 0; --i) {
        s->nb[i] = (int64_t)pb->hist_hi[i] - pb->hist_lo[i] + 1;
        if (s->nb[i] < 1) return -1;
        s->stride[i] = st;
        st *= s->nb[i];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* S2: dephasing with Fleming-Viot restarts (Sec. II A, Alg. 1).       */
/* Replicas start at xt; W is the set of xt.  On return Y holds R      */
/* states.  Returns the number of rounds, or -1 if the budget ran out. */
/* ------------------------------------------------------------------ */
static int64_t dephase(run_t* s, int W, const int32_t* xt, uint32_t cycle, int32_t* Y)
{
    const or_problem* pb = s->pb;
    int n = s->n, R = pb->R;
    int32_t* Yp = (int32_t*)malloc(sizeof(int32_t) * (size_t)R * (size_t)n);
    double* t = (double*)calloc((size_t)R, sizeof(double));
    int32_t* surv = (int32_t*)malloc(sizeof(int32_t) * (size_t)R);
    for (int r = 0; r < R; ++r) memcpy(&Y[r * n], xt, sizeof(int32_t) * (size_t)n);
    int64_t n_p = (int64_t)pb->dephase;
    int64_t round = 0;
    for (;;) {
        if (pb->dephase_mode == OR_STEPS) {
            if (round >= n_p) break;
        } else {
            double tmin = INFINITY;
            for (int r = 0; r < R; ++r) if (t[r] < tmin) tmin = t[r];
            if (tmin >= pb->dephase) break;
        }
        if (s->ev_total + R > s->max_events) { round = -1; break; }
        s->ev_total += R;
        if (s->res) s->res->counters[OR_C_EV_DEPHASE] += R;
        int ns = 0;
        for (int r = 0; r < R; ++r) {
            uint32_t blk[4];
            double tau;
            int32_t J;
            draw(s, (uint64_t)round, (uint32_t)r, cycle, OR_TAG_DEPHASE, blk);
            or_event(s->net, pb->c, &Y[r * n], blk, NULL, NULL, &tau, &J);
            memcpy(&Yp[r * n], &Y[r * n], sizeof(int32_t) * (size_t)n);
            apply_jump(s, &Yp[r * n], J);
            t[r] = t[r] + tau;
            if (region_of(s, &Yp[r * n]) == W) surv[ns++] = r;
        }
        int64_t restarts = 0;
        for (int r = 0; r < R; ++r) {
            if (region_of(s, &Yp[r * n]) == W) continue;
            ++restarts;
            if (ns > 0) {
                uint32_t blk[4];
                draw(s, (uint64_t)round, (uint32_t)r, cycle, OR_TAG_FV, blk);
                uint32_t pick = (uint32_t)(((uint64_t)blk[0] * (uint64_t)ns) >> 32);
                memcpy(&Y[r * n], &Yp[surv[pick] * n], sizeof(int32_t) * (size_t)n);
            } else {
                memcpy(&Y[r * n], xt, sizeof(int32_t) * (size_t)n);
            }
        }
        for (int k = 0; k < ns; ++k) {
            int r = surv[k];
            memcpy(&Y[r * n], &Yp[r * n], sizeof(int32_t) * (size_t)n);
        }
        if (s->res) s->res->counters[OR_C_FV_RESTARTS] += restarts;
        ++round;
    }
    free(Yp);
    free(t);
    free(surv);
    return round;
}

/* ------------------------------------------------------------------ */
/* S3: parallel step (Sec. II A, Alg. 1).  Replicas start at Y (in W). */
/* Returns 1 on exit (xt <- post-jump state of replica K), 0 when the  */
/* horizon was reached, -1 when the budget or max_rounds ran out.      */
/* ------------------------------------------------------------------ */
static int parallel(run_t* s, int W, int32_t* Z, uint32_t cycle, int64_t max_rounds,
                    int64_t* rounds_out, int32_t* K_out, int32_t* xt)
{
    const or_problem* pb = s->pb;
    int n = s->n, R = pb->R;
    int32_t* Zp = (int32_t*)malloc(sizeof(int32_t) * (size_t)R * (size_t)n);
    double* tau = (double*)malloc(sizeof(double) * (size_t)R);
    int rc = -1;
    int64_t round = 0;
    for (;;) {
        if (max_rounds >= 0 && round >= max_rounds) { rc = -1; break; }
        if (s->ev_total + R > s->max_events) { rc = -1; break; }
        s->ev_total += R;
        int first_exit = -1;  /* 0-based index of the first replica outside W */
        for (int r = 0; r < R; ++r) {
            uint32_t blk[4];
            int32_t J;
            draw(s, (uint64_t)round, (uint32_t)r, cycle, OR_TAG_PARALLEL, blk);
            or_event(s->net, pb->c, &Z[r * n], blk, NULL, NULL, &tau[r], &J);
            memcpy(&Zp[r * n], &Z[r * n], sizeof(int32_t) * (size_t)n);
            apply_jump(s, &Zp[r * n], J);
            if (first_exit < 0 && region_of(s, &Zp[r * n]) != W) first_exit = r;
        }
        int exited = first_exit >= 0;
        int K = exited ? first_exit + 1 : R;  /* Alg. 1: K = R when no replica left W */
        ++round;
        int hit = 0, credited = 0;
        for (int r = 0; r < K; ++r) {
            ++credited;
            if (credit(s, &Z[r * n], tau[r])) { hit = 1; break; }
        }
        if (s->res) {
            s->res->counters[OR_C_EV_PAR_CREDITED] += credited;
            if (hit || exited) s->res->counters[OR_C_EV_PAR_DISCARDED] += R - credited;
        }
        if (hit) { rc = 0; *K_out = 0; break; }
        if (exited) {
            memcpy(xt, &Zp[(K - 1) * n], sizeof(int32_t) * (size_t)n);
            *K_out = K;
            rc = 1;
            break;
        }
        memcpy(Z, Zp, sizeof(int32_t) * (size_t)R * (size_t)n);
    }
    *rounds_out = round;
    free(Zp);
    free(tau);
    return rc;
}

static void log_cycle(run_t* s, int64_t cycle, int64_t s1, int64_t s2, int64_t s3, int64_t K,
                      int64_t phase, const int32_t* x)
{
    or_result* res = s->res;
    int64_t i = res->counters[OR_C_N_CYCLE_LOG]++;
    if (!res->cycle_log || i >= res->cycle_log_cap) return;
    int64_t* rec = &res->cycle_log[i * OR_CYCLE_REC];
    memset(rec, 0, sizeof(int64_t) * OR_CYCLE_REC);
    rec[0] = cycle; rec[1] = s1; rec[2] = s2; rec[3] = s3; rec[4] = K; rec[5] = phase;
    for (int k = 0; k < s->n; ++k) rec[6 + k] = x[k];
}

/* ------------------------------------------------------------------ */
/* Full ParRep run: the cycle S1 -> S2 -> S3 -> S1 until T_s = T.      */
/* ------------------------------------------------------------------ */
int or_run(const or_net* net, const or_problem* pb, or_result* res)
{
    run_t s;
    if (init_run(&s, net, pb, res) != 0) return -1;
    if (!(pb->T > 0.0) || !(pb->T < 0x1.0p51) || !(pb->t_burn >= 0.0) || !(pb->t_burn < pb->T))
        return -1;
    int n = s.n, R = pb->R;
    memset(res->counters, 0, sizeof(res->counters));
    res->outside = res->outside_w = 0.0;
    int64_t nbins = s.stride[0] * s.nb[0];
    for (int64_t i = 0; i < nbins; ++i) res->hist[i] = res->hist_w[i] = 0.0;

    int32_t X[OR_MAX_SPECIES];
    memcpy(X, pb->x0, sizeof(int32_t) * (size_t)n);
    int W = region_of(&s, X);
    uint32_t cycle = 0;
    int32_t* Y = (int32_t*)malloc(sizeof(int32_t) * (size_t)R * (size_t)n);
    int end_phase = 0;
    int64_t n_c = (int64_t)pb->decorr;

    for (;;) {
        /* S1: decorrelation (serial SSA, every event credited). */
        int64_t Nc = 0, k = 0;
        double e = 0.0;
        int stop = 0;
        for (;;) {
            if (pb->decorr_mode == OR_STEPS ? (Nc >= n_c) : (e >= pb->decorr)) break;
            if (s.ev_total + 1 > s.max_events) { stop = 9; break; }
            uint32_t blk[4];
            double tau;
            int32_t J;
            draw(&s, (uint64_t)k, 0u, cycle, OR_TAG_DECORR, blk);
            or_event(net, pb->c, X, blk, NULL, NULL, &tau, &J);
            ++k;
            ++s.ev_total;
            res->counters[OR_C_EV_DECORR] += 1;
            if (credit(&s, X, tau)) { stop = 1; break; }
            apply_jump(&s, X, J);
            if (region_of(&s, X) == W) {
                Nc += 1;
                e = e + tau;
            } else {
                W = region_of(&s, X);
                Nc = 0;
                e = 0.0;
            }
        }
        if (stop) {
            end_phase = stop;
            if (stop == 9) memcpy(s.xend, X, sizeof(int32_t) * (size_t)n);
            log_cycle(&s, cycle, k, 0, 0, 0, stop, s.xend);
            break;
        }
        /* S2: dephasing. */
        int64_t rounds2 = dephase(&s, W, X, cycle, Y);
        if (rounds2 < 0) {
            end_phase = 9;
            memcpy(s.xend, X, sizeof(int32_t) * (size_t)n);
            log_cycle(&s, cycle, k, 0, 0, 0, 9, s.xend);
            break;
        }
        res->counters[OR_C_S2_ROUNDS] += rounds2;
        /* S3: parallel step. */
        int64_t rounds3 = 0;
        int32_t K = 0;
        int rc = parallel(&s, W, Y, cycle, -1, &rounds3, &K, X);
        res->counters[OR_C_S3_ROUNDS] += rounds3;
        if (rc == 1) {
            res->counters[OR_C_CYCLES] += 1;
            log_cycle(&s, cycle, k, rounds2, rounds3, K, 3, X);
            W = region_of(&s, X);
            ++cycle;
            continue;
        }
        end_phase = rc == 0 ? 3 : 9;
        if (rc != 0) memcpy(s.xend, X, sizeof(int32_t) * (size_t)n);
        log_cycle(&s, cycle, k, rounds2, rounds3, 0, end_phase, s.xend);
        break;
    }
    free(Y);

    res->counters[OR_C_STATUS] = end_phase == 9 ? 1 : 0;
    res->counters[OR_C_END_PHASE] = end_phase;
    res->T_s = fx_to_double(s.C);
    double win = pb->T - pb->t_burn;
    for (int a = 0; a < OR_MAX_PARAMS * OR_MAX_PARAMS; ++a)
        res->fim[a] = a < s.np * s.np ? kval(&s.fim[a]) / win : 0.0;
    for (int a = 0; a < OR_MAX_PARAMS; ++a) res->rer[a] = a < s.np ? kval(&s.rer[a]) / win : 0.0;
    for (int i = 0; i < OR_MAX_SPECIES; ++i) res->y[i] = i < n ? kval(&s.y[i]) : 0.0;
    memset(res->x_final, 0, sizeof(res->x_final));
    memcpy(res->x_final, s.xend, sizeof(int32_t) * (size_t)n);
    return 0;
}

/* Dephasing alone from state xt (W = set of xt): replica states after the
 * step.  Lets tests compare the Fleming-Viot ensemble with the exact law of
 * the embedded chain conditioned on survival. */
int or_dephase(const or_net* net, const or_problem* pb, const int32_t* xt, uint32_t cycle,
               int32_t* Y_out, int64_t* rounds_out)
{
    run_t s;
    if (init_run(&s, net, pb, NULL) != 0) return -1;
    int W = region_of(&s, xt);
    *rounds_out = dephase(&s, W, xt, cycle, Y_out);
    return *rounds_out < 0 ? -1 : 0;
}

/* Parallel step alone from given replica states (all in the set of
 * init[0]) with no horizon: reports N* and K (nstar_K[0..1]), the exit
 * state and the credited time.  Lets tests inject exact quasi-stationary
 * samples and check the exit law (Sec. II A, properties 1 and 2). */
int or_parallel(const or_net* net, const or_problem* pb, const int32_t* init, uint32_t cycle,
                int64_t max_rounds, int64_t* nstar_K, int32_t* exit_state, double* credited)
{
    run_t s;
    if (init_run(&s, net, pb, NULL) != 0) return -1;
    s.Tq = (u128)1 << 127;
    s.tbq = s.Tq;
    int n = s.n, R = pb->R;
    int W = region_of(&s, init);
    int32_t* Z = (int32_t*)malloc(sizeof(int32_t) * (size_t)R * (size_t)n);
    memcpy(Z, init, sizeof(int32_t) * (size_t)R * (size_t)n);
    int64_t rounds = 0;
    int32_t K = 0;
    int rc = parallel(&s, W, Z, cycle, max_rounds, &rounds, &K, exit_state);
    free(Z);
    nstar_K[0] = rounds;
    nstar_K[1] = K;
    *credited = fx_to_double(s.C);
    return rc == 1 ? 0 : -1;
}

/* ------------------------------------------------------------------ */
/* Multi-run estimators (Sec. III): sample means over the runs, the    */
/* 95 % half-width of the mean FIM diagonal, the IAF of f = x_i from   */
/* the spread of the window integrals, and the stationary sensitivity  */
/* bounds sqrt(IAF_f v^T FIM v) with v = e_k.  Plain two-pass sums in  */
/* run order.                                                          */
/* ------------------------------------------------------------------ */
static void mean_and_sq(int n, const double* v, int stride, int e, double* mean, double* sq)
{
    double s = 0.0;
    for (int r = 0; r < n; ++r) s += v[(size_t)r * stride + e];
    double m = s / (double)n;
    double q = 0.0;
    for (int r = 0; r < n; ++r) {
        double d = v[(size_t)r * stride + e] - m;
        q += d * d;
    }
    *mean = m;
    *sq = q;
}

void or_estimate(int n, int np, int ns, const double* fim, const double* rer, const double* y,
                 double window, double* fim_mean, double* fim_hw, double* rer_mean,
                 double* y_mean, double* iaf, double* bound)
{
    double q;
    for (int e = 0; e < np * np; ++e) {
        mean_and_sq(n, fim, np * np, e, &fim_mean[e], &q);
        if (e % (np + 1) == 0)
            fim_hw[e / (np + 1)] = 1.96 * (sqrt(q / (double)(n - 1)) / sqrt((double)n));
    }
    for (int k = 0; k < np; ++k) mean_and_sq(n, rer, np, k, &rer_mean[k], &q);
    for (int i = 0; i < ns; ++i) {
        mean_and_sq(n, y, ns, i, &y_mean[i], &q);
        iaf[i] = q / (window * (double)(n - 1));
    }
    for (int i = 0; i < ns; ++i)
        for (int k = 0; k < np; ++k) bound[i * np + k] = sqrt(iaf[i] * fim_mean[k * np + k]);
}

