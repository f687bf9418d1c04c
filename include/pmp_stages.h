/*
 * pmp_stages.h -- stage-level entry points of libpmp, used by the parity
 * tests to compare each step of the hot path with the CPU oracle.
 *
 * pmp_run_device_debug runs exactly the pipeline of pmp_run_device (same
 * kernels, same launch configuration) and additionally copies internal arrays
 * out to caller-owned buffers.  Every pointer in pmp_debug may be NULL.
 * "cells" below is sum over the lengths of n - m + 1, laid out length by
 * length (lengths ascending), start i ascending within a length.
 */
#ifndef PMP_STAGES_H
#define PMP_STAGES_H

#include "pmp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint32_t size;          /* sizeof(pmp_debug) */
    int32_t  K;             /* out: spectral width used (Sec. 3.2 calibration) */
    /* host arrays with one entry per length */
    int32_t *lengths;       /* out: window lengths                              */
    int32_t *depth;         /* out: directory depth d (Sec. 3.4, Prop. 4); 0
                               at the lengths between anchors, which have no
                               directory                                       */
    int64_t *indexed;       /* out: non-constant windows of the length          */
    /* device arrays */
    double  *mu;            /* [cells] window mean (two-pass, Sec. 3.2)         */
    double  *sigma;         /* [cells] population standard deviation; 0 marks a
                               constant window                                 */
    double  *profile_pass;  /* [cells] one-pass upper profile, snapped; +inf
                               where no pair was evaluated (Sec. 2, 3.4)        */
    double  *profile_final; /* [cells] profile after the certificate            */
    void    *features;      /* [cells][32] F_{i,m} (Sec. 3.2): 30 reals
                               (re, im of bins 1..15, zero-padded), then the
                               error bound e_i and ||F||; FP64 for
                               PMP_PREC_FP64, FP32 otherwise; zero for constant
                               windows                                          */
    uint64_t *keys;         /* [cells] key word: bits 0..B-1 the SimHash
                               signature (paper bit 1 = bit B-1), bits 24..63
                               the Hamming-1 probe bit order, 5 bits each;
                               all ones for constant windows and at the
                               lengths between anchors (only anchor lengths
                               are indexed, Sec. 3.3)                          */
    uint32_t *perm;         /* [indexed windows of the anchor lengths] bucket
                               order: slot -> cell                             */
    uint32_t *bucket_start; /* [sum 2^depth + 1] first slot of every bucket     */
    /* in: 0 = off.  A value in (0, 1) starts the certificate's threshold
       loop at that fraction of the one-pass threshold T.  The result stays
       exact (the loop raises T to the k-th selected value until the greedy
       prefix lies within it, Sec. 3.6), so this forces the rounds after the
       first, which real data reaches only rarely.  Other values: EINVAL. */
    double   t_start_scale;
    /* in: 0 = off.  A positive value caps the threshold join's buffer of
       kept pairs (between its tiles and its exact stage) at that many pairs,
       so that the tiles verify the pairs past the cap themselves, as they do
       when a round keeps more pairs than the buffer holds.  The result is
       the same.  Negative values: EINVAL. */
    int64_t  join_pair_cap;
} pmp_debug;

int pmp_run_device_debug(const double *d_series, int64_t n, int32_t m_min,
                         int32_t m_max, int32_t k, int32_t exclusion,
                         int32_t budget, const pmp_options *opt,
                         void *d_workspace, size_t ws_bytes, void *stream,
                         pmp_motif *out, int32_t *n_out, pmp_stats *stats,
                         pmp_debug *dbg);

/* The Gaussian projection g_{m,l}[c] the library draws for seed `seed`
 * (Sec. 3.4: seeded Gaussian vectors, independent per length): Box-Muller on
 * the SplitMix64 counter stream, counter ((m*64 + l)*64 + c)*2 + {0,1}. */
double pmp_projection(uint64_t seed, int32_t m, int32_t l, int32_t c);

/* Spectral width the calibration of Sec. 3.2 picks for a host series. */
int pmp_calibrate_width(const double *series, int64_t n, int32_t m_min,
                        int32_t m_max, int32_t m_step, int32_t budget,
                        int32_t gamma, int32_t bits, int32_t *K);

#ifdef __cplusplus
}
#endif
#endif /* PMP_STAGES_H */
