/*
 * pmp.h -- exact z-normalized pan-matrix-profile motif search on MI355X.
 *
 * C ABI of libpmp (HIP, gfx950).  Every entry point returns 0 on success or a
 * negative PMP_E* code; no C++ exception crosses this boundary, and
 * pmp_last_error() returns a thread-local text for the last failure.
 *
 * The problem (paper Sec. 2, "Background and Problem"): for a series
 * T = (t_0 .. t_{n-1}) and every window length m of an interval, the matrix
 * profile row P_m[i] = min over valid j (|i-j| >= exclusion) of the
 * z-normalized Euclidean distance d_m(i,j); the top-k pan-motifs are the cells
 * sorted by distance, skipping any cell within m/2 of an already accepted cell
 * of the same length.  Constant windows (sigma = 0) are ignored.
 *
 * The library runs the paper's one-pass method (Sec. 3: normalized spectral
 * features, SimHash keys in occupancy-controlled buckets, Parseval-bound
 * pruning, exact verification) to get a sound upper profile, then certifies
 * the top-k with an exact threshold join whose completeness follows from the
 * Parseval bound (Lemma 2), so the reported motifs equal the brute-force
 * definition:
 *   - ties between cells are ordered by (distance, m, i);
 *   - "within m/2" is inclusive (2|i - i'| <= m);
 *   - distances below 1e-6 are reported as exactly 0 (Sec. 3.6), before ties;
 *   - j is the smallest minimizer;
 *   - a window is constant iff its m samples compare equal.
 */
#ifndef PMP_H
#define PMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PMP_OK          0
#define PMP_EINVAL     -1   /* bad argument or non-finite sample            */
#define PMP_ENOMEM     -2   /* device or host allocation failed / too small */
#define PMP_EDEVICE    -3   /* HIP runtime error                            */
#define PMP_EBUSY      -4   /* request still running (pmp_poll)             */
#define PMP_ENOTFOUND  -5   /* unknown request id                           */
#define PMP_EINTERNAL  -6   /* internal consistency check failed            */

/* One reported pan-motif: cell (m, i) and its nearest neighbour j, at the
 * exact z-normalized distance dist (FP64).  32 bytes. */
typedef struct {
    int64_t i;
    int64_t j;
    int32_t m;
    int32_t flags;      /* reserved, 0 */
    double  dist;
} pmp_motif;

/* Precision of the spectral sketch and the cached features (Sec. 3.2, where
 * features are cached in single precision).  Moments, exact distances and
 * the certificate's verification are FP64 in every form, and every stored
 * feature vector carries a derived bound e_i on its error, which the
 * Parseval prune subtracts, so it stays a true lower bound. */
enum {
    PMP_PREC_FP64 = 0,  /* plain form: FP64 sliding DFT, FP64 features       */
    PMP_PREC_FP32 = 1,  /* windows x DFT basis on the matrix cores, both
                           split exactly into three bf16 parts (six products,
                           FP32 accumulation): FP32-grade features           */
    PMP_PREC_BF16 = 2   /* BF16 keys + FP32 bound: the features, the bound and
                           the join as in PMP_PREC_FP32; the SimHash
                           projection of the keys in plain bf16 (one product
                           instead of three).  Keys only steer candidates
                           (Sec. 3.4, Prop. 2), so plain bf16 costs no
                           validity; features computed from plain-bf16 inputs
                           would make the bound's margin 2^8 times wider.   */
};

typedef struct {
    uint32_t size;            /* sizeof(pmp_options)                          */
    int32_t  m_step;          /* lengths m_min, m_min+m_step, ..., <= m_max   */
    int32_t  precision;       /* PMP_PREC_*                                   */
    int32_t  spectral_width;  /* K in [2,16]; 0 = calibrate (Sec. 3.2)        */
    uint64_t seed;            /* seed of the Gaussian projections (Sec. 3.4)  */
    int32_t  certify;         /* 1: exact top-k (default); 0: top-k of the
                                 one-pass upper profile, no certificate       */
    int32_t  signature_bits;  /* B in [1,24], default 24 (Sec. 4)             */
    int32_t  gamma;           /* R = gamma * budget, default 8 (Sec. 3.4)     */
    int32_t  probe_ref_depth; /* d0, default 12 (Sec. 3.4)                    */
    int32_t  probe_cap;       /* cap on Hamming-1 probes, default 8           */
    /* Anchor lengths and emit-time completion (Sec. 3.3, Sec. 3.6,
     * Algorithm 2).  They change only how fast the certificate's threshold
     * is reached, never the result. */
    int32_t  anchor_stride;   /* s: the one pass probes every s-th length of
                                 the list and the last; the lengths between
                                 are re-cut from their neighbours' partners;
                                 default 16 (the paper's maximum-performance
                                 stride is 6; on this GPU the step keeps
                                 getting faster past it), 1 = every length    */
    int32_t  sieve_width;     /* w of the hot-class sieve over buckets of more
                                 than R entries, default 0 = off (the paper
                                 uses 8; here it costs time and lowers none
                                 of the cells the certificate needs)          */
    int32_t  complete_rounds; /* P_max rounds of local completion around the
                                 top-k cells, default 8; 0 = off (also off
                                 when anchor_stride is 1)                     */
    int32_t  complete_dm;     /* Delta_m of the completion box, in window
                                 length, default 6                            */
    int32_t  complete_dp;     /* Delta_p of the completion box, in samples,
                                 default 4                                    */
    int32_t  reserved;
} pmp_options;

/* Fill *opt with the paper's defaults (Sec. 4 constants). */
void pmp_default_options(pmp_options *opt);

/* Per-call counters and phase times (all optional reading). */
typedef struct {
    uint32_t size;              /* sizeof(pmp_stats)                          */
    int32_t  K;                 /* spectral width used                        */
    int32_t  lengths;           /* number of window lengths                   */
    int32_t  certify_rounds;    /* threshold-join rounds (0 if not certified) */
    uint64_t cells;             /* sum over m of n - m + 1                    */
    uint64_t indexed_cells;     /* non-constant windows put in the buckets    */
    uint64_t pass_candidates;   /* candidate inspections of the one pass      */
    uint64_t pass_verified;     /* exact distances of the one pass            */
    uint64_t join_candidates;   /* pairs kept by the join's filter            */
    uint64_t join_verified;     /* exact distances of the join                */
    uint64_t hot_buckets;       /* buckets holding more than R entries        */
    int32_t  max_depth;         /* deepest directory (bits)                   */
    int32_t  reserved;
    double   threshold;         /* final certified threshold T                */
    double   ms_total;          /* device time of the whole call              */
    double   ms_onepass;        /* moments + sketch + buckets + probe         */
    double   ms_certify;        /* selection + threshold join + exact rows
                                   (after the emit stage, ms_complete)        */
    double   ms_sketch;         /* the sketch kernel (FP64 sliding DFT, or the
                                   basis tables + MFMA projection)           */
    double   ms_sort;
    double   ms_probe;
    double   ms_join;
    double   ms_rows;
    uint64_t workspace_bytes;   /* device bytes used by the call              */
    uint64_t join_pairs;        /* pairs the join's MFMA filter evaluated     */
    uint64_t sieve_verified;    /* exact distances of the hot-class sieve     */
    uint64_t hint_verified;     /* exact distances re-cut from anchor hints   */
    uint64_t complete_verified; /* exact distances of local completion        */
    double   ms_complete;       /* sieve + hints + local completion           */
    int32_t  complete_rounds;   /* rounds of local completion run             */
    int32_t  anchors;           /* anchor lengths probed                      */
    double   ms_sieve;          /* the hot-class sieve (part of ms_complete)  */
    double   ms_hints;          /* the hints (part of ms_complete)            */
    double   ms_keys;           /* SimHash keys (after the sketch kernel,
                                   within the sketch phase)                  */
    uint64_t join_windows;      /* windows given join operands (the lengths
                                   up to the key bound of the last round)    */
    uint64_t probe_queries;     /* indexed windows of the anchor lengths (the
                                   probe's queries; when the first anchor's
                                   cells already settle the top-k at 0, the
                                   probe runs that anchor's only)            */
} pmp_stats;

/* Exact top-k pan-motifs of a host series.  lengths m_min..m_max (step 1),
 * valid pairs |i-j| >= exclusion, occupancy target budget (alpha, the paper's
 * only user knob).  out: caller-owned, capacity k; *n_out = number written
 * (< k when fewer finite cells exist).  The series is copied before return.
 * Errors: PMP_EINVAL unless 3 <= m_min <= m_max <= n, m_max <= 2048 (the
 * longest window supported), k >= 1, exclusion >= 1, budget >= 1, every
 * sample is finite and there are at most 2^31 - 1 cells (about 500 bytes of
 * workspace each bound the size one GPU holds well below that). */
int pmp_open(const double *series, int64_t n, int32_t m_min, int32_t m_max,
             int32_t k, int32_t exclusion, int32_t budget,
             pmp_motif *out, int32_t *n_out);

/* Same, with options (NULL = defaults) and optional stats (NULL = none). */
int pmp_open_ex(const double *series, int64_t n, int32_t m_min, int32_t m_max,
                int32_t k, int32_t exclusion, int32_t budget,
                const pmp_options *opt, pmp_motif *out, int32_t *n_out,
                pmp_stats *stats);

/* Upper bound of the device workspace pmp_run_device needs for a request
 * of these sizes, k reported motifs and any budget >= 1 (the deepest
 * directories, budget 1, bound every other budget).  The selection buffers
 * grow with k (k (m_max + 1) cells of the upper profile are selected, Sec. 2
 * top-k rule), so the bound depends on it.  0 on invalid arguments (the
 * checks of pmp_open on n, m_min, m_max and k, and on the options). */
size_t pmp_workspace_bytes(int64_t n, int32_t m_min, int32_t m_max, int32_t k,
                           const pmp_options *opt);

/* Device-resident form: d_series is a device pointer (FP64, n samples) on the
 * current HIP device; d_workspace/ws_bytes a caller-owned device buffer of at
 * least pmp_workspace_bytes(n, m_min, m_max, k, opt) bytes (256-byte
 * aligned; PMP_ENOMEM if smaller than the request needs); stream a hipStream_t
 * (NULL = default stream).  All work is enqueued on that stream; the call
 * returns after the results are in `out` (host memory).  The library
 * allocates no device memory in this form. */
int pmp_run_device(const double *d_series, int64_t n, int32_t m_min,
                   int32_t m_max, int32_t k, int32_t exclusion, int32_t budget,
                   const pmp_options *opt, void *d_workspace, size_t ws_bytes,
                   void *stream, pmp_motif *out, int32_t *n_out,
                   pmp_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and result as pmp_run_device, with the workspace taken from a
 * fixed device array of 256 MiB inside the library instead of a caller
 * buffer.  Each GPU the library runs on holds that array until the process
 * ends; its address is looked up on the first call on a device.  No device
 * memory is allocated and no HIP event is created (pmp_stats then carries
 * the counters but 0 for the phase times).
 * The array is shared by every call on the same GPU and keeps the last
 * call's contents (the pipeline initializes what it reads): calls that
 * overlap on one GPU, from any thread or stream, race and must be
 * serialized by the caller.
 * Errors: as pmp_run_device; PMP_ENOMEM when the request's workspace bound
 * (pmp_workspace_bytes) exceeds 256 MiB, about 500,000 cells in the FP64
 * form. */
int pmp_run_device_noalloc(const double *d_series, int64_t n, int32_t m_min,
                           int32_t m_max, int32_t k, int32_t exclusion,
                           int32_t budget, const pmp_options *opt, void *stream,
                           pmp_motif *out, int32_t *n_out, pmp_stats *stats);

/* ------------------------------------------------------------- serving */

typedef struct pmp_server pmp_server;

typedef struct {
    double submit_s;     /* host clock at pmp_submit (CLOCK_MONOTONIC, s) */
    double start_s;      /* admitted and first work enqueued              */
    double end_s;        /* results in host memory                        */
    uint64_t cells;
    uint64_t workspace_bytes;
} pmp_timing;

/* A request server on `device` that admits requests while their workspace
 * fits in hbm_budget_bytes and a slot (HIP stream) is free; admitted requests
 * run concurrently, each on its own stream.  Thread-safe.  NULL on error. */
pmp_server *pmp_server_create(int device, size_t hbm_budget_bytes,
                              int32_t max_slots);

/* Queue a request; the series is copied before return.  *req_id receives its
 * id.  PMP_EINVAL on bad arguments, PMP_ENOMEM if the request alone can never
 * fit the HBM budget. */
int pmp_submit(pmp_server *srv, const double *series, int64_t n,
               int32_t m_min, int32_t m_max, int32_t k, int32_t exclusion,
               int32_t budget, const pmp_options *opt, uint64_t *req_id);

/* PMP_EBUSY while pending; on completion copies the motifs (capacity k) and
 * timing and forgets the request.  Returns the request's own status. */
int pmp_poll(pmp_server *srv, uint64_t req_id, pmp_motif *out, int32_t *n_out,
             pmp_timing *timing);

/* Blocks until the request completes, then behaves as pmp_poll. */
int pmp_wait(pmp_server *srv, uint64_t req_id, pmp_motif *out, int32_t *n_out,
             pmp_timing *timing);

/* Waits for every admitted request and frees the server. */
void pmp_server_destroy(pmp_server *srv);

/* ----------------------------------------------------------- streaming */

/* A stream session (Sec. 3.1, 3.5, Algorithm 1): samples arrive in order and
 * are processed in batches of `batch` <= exclusion consecutive samples.  At
 * every anchor length (every anchor_stride-th length of m_min..m_max by
 * m_step, and the last, Sec. 3.3) each sample completes the window that ends
 * at it; a batch's windows get their features and SimHash keys, search the
 * earlier windows of their length in the anchor's directory (exact-prefix
 * bucket and Hamming-1 probes, budget gamma * budget, Parseval prune, exact
 * FP64 distances) and lower the upper profile of both ends.  Windows of one
 * batch never search each other (they are all within the exclusion zone).
 * The series and all state stay on the GPU; updates at sample tau use only
 * samples 0..tau.  The profile is deterministic for a given input, batch
 * size and options (Prop. 5): how the samples are split over append calls
 * does not change it, since batches are cut at multiples of `batch` from the
 * first sample (pmp_stream_flush cuts one early).
 * Sessions are not thread-safe; one session uses one device.
 *
 * Memory: about 330 bytes per (sample, anchor length) of `capacity` on the
 * device, 4 bytes per sample on the host; an exact query adds the
 * workspace pmp_run_device needs for the samples held. */
typedef struct pmp_stream pmp_stream;

typedef struct {
    uint64_t appended;      /* samples appended                              */
    uint64_t processed;     /* samples whose batch has run                   */
    uint64_t batches;       /* batches run                                   */
    uint64_t windows;       /* non-constant anchor windows completed         */
    uint64_t candidates;    /* candidates inspected (Parseval bound)         */
    uint64_t verified;      /* exact distances computed                      */
    uint64_t updates;       /* candidate-end improvements merged             */
    uint64_t dropped;       /* improvements lost to a full buffer (0: the
                               buffer holds R per window by construction)   */
    int32_t  anchors;       /* anchor lengths                                */
    int32_t  K;             /* spectral width (the option, 16 if 0: a stream
                               has no series to calibrate on in advance)    */
    int32_t  batch;         /* samples per batch                             */
    int32_t  reserved;
    double   ms_ingest;     /* device time of the batches so far             */
    uint64_t device_bytes;  /* device memory the session holds, with the
                               exact query's workspace once grown           */
} pmp_stream_stats;

/* Opens a session on `device` for up to `capacity` samples.  batch 0 means
 * batch = exclusion.  Options as pmp_open_ex (NULL = defaults); only the
 * FP64 form (precision 0) is accepted.  *out receives the session.
 * Errors: PMP_EINVAL unless 3 <= m_min <= m_max <= min(capacity, 2048),
 * k >= 1, exclusion >= 1, budget >= 1, 1 <= batch <= exclusion and the
 * anchor cells (capacity times anchor lengths) stay below 2^31;
 * PMP_EDEVICE for a bad device; PMP_ENOMEM when the device memory is not
 * there. */
int pmp_stream_create(int device, int64_t capacity, int32_t m_min, int32_t m_max,
                      int32_t k, int32_t exclusion, int32_t budget, int32_t batch,
                      const pmp_options *opt, pmp_stream **out);

/* Appends `count` samples (host memory, copied before return) and runs
 * every batch they complete; a remainder shorter than a batch waits for the
 * next append.  Returns after the batches ran.  PMP_EINVAL for a non-finite
 * sample (nothing is appended) or past the capacity. */
int pmp_stream_append(pmp_stream *s, const double *samples, int64_t count);

/* Runs the pending remainder as a batch of its own. */
int pmp_stream_flush(pmp_stream *s);

/* Top-k pan-motifs of the upper profile at the anchor lengths over the
 * samples processed so far (the one-pass result, Sec. 2 top-k rule):
 * each reported distance is the exact distance of a valid pair, which the
 * true profile can only undercut.  out: capacity k. */
int pmp_stream_topk(pmp_stream *s, pmp_motif *out, int32_t *n_out);

/* Exact top-k pan-motifs over all lengths of the samples appended so far:
 * the certified request path (pmp_run_device) on the resident series, with
 * the session's parameters; stats as pmp_run_device (NULL = none). */
int pmp_stream_exact(pmp_stream *s, pmp_motif *out, int32_t *n_out,
                     pmp_stats *stats);

/* The upper profile of anchor `anchor` (0-based, ascending lengths): *W
 * receives its windows so far (processed samples - m + 1, or 0); P (FP64,
 * +inf where no pair was evaluated or the window is constant) and I (the
 * neighbour, -1 where none) receive W values each when not NULL. */
int pmp_stream_profile(pmp_stream *s, int32_t anchor, double *P, int64_t *I,
                       int64_t *W);

/* Counters; lengths (when not NULL) receives up to `capacity` anchor
 * lengths. */
int pmp_stream_info(pmp_stream *s, pmp_stream_stats *st, int32_t *lengths,
                    int32_t capacity);

/* Waits for the session's work and frees it (NULL: nothing). */
void pmp_stream_destroy(pmp_stream *s);

/* Text of the last error on this thread ("" if none). */
const char *pmp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PMP_H */
