/* parrep_estimate.h -- multi-run estimators of ParRep results on the device.
 *
 * Sec. III of Wang & Plechac (arXiv 1705.06807) turns N independent runs of
 * one problem (same network, rate vector and window [t_burn, T]) into the
 * mean pathwise FIM with its confidence interval, the integrated
 * autocorrelation function (IAF) of observables from the spread of their
 * window integrals, and the stationary sensitivity bounds
 * |S_{f,v}| <= sqrt(IAF_f v^T FIM v), here with v = e_k.  This call computes
 * them on the device from the results' stats buffers, without copying the
 * runs to the host. */
#ifndef PARREP_ESTIMATE_H
#define PARREP_ESTIMATE_H

#include "parrep.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Layout of the estimates buffer (PARREP_EST_LEN doubles). */
enum {
    PARREP_EST_FIM = 0,     /* n_params x n_params, row-major: mean over runs of the FIM  */
    PARREP_EST_FIM_HW = 64, /* n_params: 1.96 sd / sqrt(n) of each FIM diagonal entry      */
    PARREP_EST_RER = 72,    /* n_params: mean relative entropy rate                        */
    PARREP_EST_Y = 80,      /* n_species: mean window integral of x_i                      */
    PARREP_EST_IAF = 84,    /* n_species: sum_r (Y_i^r - mean)^2 / (window (n - 1))         */
    PARREP_EST_BOUND = 88,  /* n_species x n_params: sqrt(IAF_i FIM_kk), f = x_i, v = e_k   */
    PARREP_EST_LEN = 120
};

/* Estimates over n_runs >= 2 runs.  stats_ptrs: host array of n_runs device
 * pointers, each to one result's stats (PARREP_NSTATS doubles, as written by
 * a solve; read on the stream).  n_params and n_species: the network's.
 * window = T - t_burn (> 0, finite).  out: device, PARREP_EST_LEN doubles;
 * entries beyond n_params / n_species are zero.  Means and squared
 * deviations are two-pass sums in run order.  Enqueued on stream (a
 * hipStream_t, NULL = default); EINVAL for bad arguments, EDEVICE on a HIP
 * error. */
int parrep_estimate(parrep_ctx* ctx, int32_t n_runs, const double* const* stats_ptrs,
                    int32_t n_params, int32_t n_species, double window, double* out,
                    void* stream);

#ifdef __cplusplus
}
#endif
#endif
