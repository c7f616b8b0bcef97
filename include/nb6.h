/*
 * nb6.h -- C ABI of the MI355X regular-force library.
 *
 * The library computes, for a block of active i-particles of a star cluster,
 * the regular part of the Ahmad-Cohen force split: the acceleration and its
 * time derivative (jerk) due to every j-particle outside the i-particle's
 * neighbour sphere, and the list of j-particles inside it (Nitadori &
 * Aarseth 2012, section 3.3 step 6, with the velocity neighbour criterion of
 * section 3.2).  It plays the part of the paper's regular-force library
 * (open / send / regular force / close, section 3.4 and Appendix C) with the
 * j-particle prediction (section 3.3 step 3) moved onto the GPU.
 *
 * Conventions for every entry point
 *   - Return value: NB6_OK (0) on success, a positive warning, or a negative
 *     error code.  Nothing throws across the ABI.  nb6_last_error() returns
 *     a text description of the last failure on a context.
 *   - Units: G = 1.  R_ij = R_j - R_i, V_ij = V_j - V_i.
 *   - Vectors are row-major [n][3] arrays of double (x, y, z per particle).
 *   - mem_kind NB6_MEM_HOST: every array argument of the call is host
 *     memory; the call returns when the results are in place.
 *     mem_kind NB6_MEM_DEVICE: every array argument is device memory of the
 *     context's GPU; the call is ordered on `stream` and returns without
 *     waiting for the GPU.  Validation that needs device data is then done on
 *     the GPU and reported by nb6_sync_status().
 *   - stream is a hipStream_t (NULL: the null stream).  Calls that share a
 *     context share its scratch buffers and must be ordered on one stream.
 *   - The caller owns every array it passes; the library reads inputs and
 *     writes outputs only during the call (HOST) or the stream-ordered work
 *     the call enqueues (DEVICE).  The context owns all device state and
 *     scratch and frees it in nb6_destroy().
 */
#ifndef NB6_H
#define NB6_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define NB6_OK                  0
#define NB6_WARN_NB_OVERFLOW    1   /* some i had more neighbours than cap   */
#define NB6_ERR_ARG           (-1)  /* bad argument (index, size, h2, mode)  */
#define NB6_ERR_STATE         (-2)  /* cluster missing or not predicted      */
#define NB6_ERR_NOMEM         (-3)  /* device allocation failed              */
#define NB6_ERR_ADMISSION     (-4)  /* request can never fit the HBM budget  */
#define NB6_ERR_UNKNOWN_TICKET (-5) /* nb6_poll on a ticket never issued     */
#define NB6_ERR_HIP           (-6)  /* HIP runtime error                     */
#define NB6_ERR_DEVICE_INPUT  (-7)  /* GPU-side validation found bad input   */
#define NB6_PENDING             2   /* nb6_poll: request not finished yet    */

/* ---- memory kinds and coordinate-difference modes --------------------- */
#define NB6_MEM_HOST    0
#define NB6_MEM_DEVICE  1

/*
 * How the coordinate difference R_j - R_i is formed before the FP32 force
 * arithmetic.  The paper's GPU default kept FP32 coordinates and left the
 * 'two-float' form as an option (section 3.4 and its footnote); GPUIRR always
 * uses two-float coordinates (section 3.5).
 */
#define NB6_DX_FF    1   /* float-float (hi + lo) coordinates             */
#define NB6_DX_FP64  2   /* double coordinates, difference in FP64       */
#define NB6_DX_FP32  4   /* plain float coordinates (the paper's default) */
#define NB6_DX_LOCAL 8   /* tile-local coordinates (below), the fastest form
                            that keeps the float-float accuracy            */
#define NB6_DX_ALL   15
/*
 * NB6_DX_LOCAL: the j-records follow a spatial (Morton) order of the
 * cluster, and each tile of 32 consecutive records carries the FP64 centre
 * of its predicted positions; a record holds its particle's offset from that
 * centre rounded to FP32.  R_j - R_i is formed as that offset plus the FP32
 * rounding of (centre - R_i), computed in FP64 once per tile and i.  The
 * error of a pair is about 2^-24 (|R_ij| + tile extent): the large
 * coordinates cancel in FP64, and only quantities of the pair's own scale
 * are rounded.  The order is rebuilt from the stored state by
 * nb6_load_particles after a full load and after a cluster's worth of subset
 * updates (it only sets how compact the tiles are, never which pairs are
 * summed).  A block small enough to share a wavefront's lanes among its
 * i-particles (at most 256 of them, up to 1024 in a cluster too small for
 * one lane per i to fill the GPU, or any when the context forces the lanes),
 * or a call whose j-slices are shorter than 256 particles (a small block in a
 * small cluster), is bound by memory latency, not arithmetic: in this mode it
 * takes the float-float differences, from the float-float prediction the
 * mode also writes (as its i-side).
 */

/* Largest neighbour-list capacity of nb6_regular_force. */
#define NB6_MAX_CAP  1023

/* Largest row of the neighbour lists a cluster stores for the irregular
 * force (nb6_set_lists). */
#define NB6_MAX_LIST_CAP  8192

typedef struct nb6_ctx nb6_ctx;

typedef struct nb6_options {
    int     device;        /* HIP device ordinal                              */
    int     slice_hint;    /* 0: choose the j-split per call; >0: force it    */
    int64_t hbm_budget;    /* bytes the serving queue may hold; 0: 1/4 of free */
    int     flags;         /* NB6_OPT_* bits                                  */
    int     ipl_hint;      /* i-particles per lane: 0 or 1 one (the default:
                              measured faster at every block size), 2 two   */
    int     jl_hint;       /* 0: choose the lanes that share one i-particle;
                              1, 2, 4, ..., 64: force it (not with ipl_hint 2) */
} nb6_options;

/* Record HIP events around every predictor, force, finalize and
 * irregular-force launch so that nb6_kernel_times() can report their GPU
 * durations. */
#define NB6_OPT_TIMING 1
/* Run every force call on its active particles in the caller's order.  By
 * default a plain call whose block holds at least 8192 particles and three
 * quarters of its cluster first sorts them by the cluster's spatial order (a
 * counting sort over the cluster's particles), so that the particles sharing
 * a wavefront lie close together and test fewer candidate pairs; every
 * output is the same bits either way. */
#define NB6_OPT_CALLER_ORDER 2

/*
 * Create a context on options->device (NULL options: device 0, defaults).
 * *out receives the context.  Errors: NB6_ERR_ARG, NB6_ERR_HIP.
 */
int nb6_create(nb6_ctx **out, const nb6_options *options);

/* Free every device buffer of the context.  NULL is accepted. */
int nb6_destroy(nb6_ctx *ctx);

/* Text of the last error on ctx (never NULL; "" when none). */
const char *nb6_last_error(const nb6_ctx *ctx);

/*
 * Load or update the state of cluster `cluster` (0 <= cluster < 4096): the
 * corrected mass, position, velocity, acceleration, jerk and time of each
 * particle -- the data the host integrator keeps per body and from which
 * the predictor works (section 3.3 step 3; Appendix C sends the predicted
 * j-particles to the regular-force library before each regular block).
 *
 *   idx == NULL: full load.  n is the cluster size; m[n], x/v/a/jerk[n][3],
 *                t[n].  Replaces any previous state of that cluster.
 *   idx != NULL: update n existing particles; entry k of every array
 *                belongs to particle idx[k].  0 <= idx[k] < cluster size.
 * The cluster must be predicted again (nb6_predict_j) before the next force
 * call.  A full load, and the update that brings the particles updated since
 * the last ordering to the cluster size, also rebuild the cluster's spatial
 * order (NB6_DX_LOCAL) from the stored positions, on the same stream.
 * Errors: NB6_ERR_ARG (n <= 0, bad idx, non-finite host data),
 * NB6_ERR_NOMEM, NB6_ERR_HIP.
 */
int nb6_load_particles(nb6_ctx *ctx, int cluster, int64_t n,
                       const double *m, const double *x, const double *v,
                       const double *a, const double *jerk, const double *t,
                       const int32_t *idx, int mem_kind, void *stream);

/*
 * Predict every particle of the cluster to t_block with the cubic Taylor
 * series (section 3.3 step 3):
 *   dt = t_block - t_j;  x_p = x + v dt + a dt^2/2 + jerk dt^3/6;
 *   v_p = v + a dt + jerk dt^2/2     (FP64),
 * and write the j-streams the force kernel reads for every coordinate mode
 * in the bit mask `modes` (NB6_DX_*; 0 means all).  NB6_DX_LOCAL also
 * writes the float-float prediction of every particle (the i-side of that
 * mode), but marks only its own stream current.  Errors: NB6_ERR_STATE (cluster
 * not loaded), NB6_ERR_ARG, NB6_ERR_HIP.
 */
int nb6_predict_j(nb6_ctx *ctx, int cluster, double t_block, int modes,
                  void *stream);

/*
 * Regular force, jerk and neighbour list of n_i active particles of the
 * cluster, against all N predicted particles (section 3.3 step 6 with the
 * velocity criterion of section 3.2):
 *   j (!= i) is a neighbour iff min(|R|^2, |R + dtr_i V|^2) < h2_i;
 *   otherwise it adds m_j R / r^3 to acc_i and
 *   m_j (V / r^3 - 3 (R.V) R / r^5) to jerk_i.
 * Inputs:  idx_i[n_i] (cluster indices, 0 <= idx_i < N), h2_i[n_i]
 *          (squared neighbour radii, > 0 and >= 2^-126 as floats),
 *          dtr_i[n_i] (regular time-steps, finite and >= 0: the offset of
 *          the criterion's second end point is forward in time; HOST mode
 *          refuses others with NB6_ERR_ARG, DEVICE mode gives that i a NaN
 *          row and nnb = -1 and nb6_sync_status reports
 *          NB6_ERR_DEVICE_INPUT), dx_mode (one NB6_DX_* value
 *          whose stream holds the cluster's latest prediction: the block
 *          time of the last nb6_predict_j or served request on the cluster,
 *          whichever came last; a stream still at an earlier block time is
 *          refused with NB6_ERR_STATE),
 *          0 <= cap <= NB6_MAX_CAP.
 * Outputs: acc[n_i][3], jerk[n_i][3] (double), nnb[n_i] (true neighbour
 *          count, self excluded), list[n_i][cap] (the first min(nnb, cap)
 *          neighbours in ascending cluster index; entries past that are
 *          left unspecified).  list may be NULL when cap == 0.
 *          pot[n_i] (may be NULL): the regular potential
 *          -sum m_j / |R_ij| over the same non-neighbour terms (the optional
 *          potential sum of the paper's kernel, Appendix B; section 4 quotes
 *          its use in the energy check).  Asking for it adds one FP32 add
 *          per pair and one partial-sum component.
 * The neighbour decision and the force arithmetic are done in FP32 (the
 * coordinate difference per dx_mode); the terms are summed in FP32 over
 * tiles of 32 j and the tile sums in FP64, and the outputs are double.
 * HOST mode copies only the first min(nnb, cap) entries of each list row
 * into `list`.
 * Returns NB6_OK, or NB6_WARN_NB_OVERFLOW (HOST mode only) when some nnb
 * exceeds cap.  Errors: NB6_ERR_ARG, NB6_ERR_STATE, NB6_ERR_NOMEM,
 * NB6_ERR_HIP.  n_i == 0 is a no-op.
 */
int nb6_regular_force(nb6_ctx *ctx, int cluster, int64_t n_i,
                      const int32_t *idx_i, const double *h2_i,
                      const double *dtr_i, int dx_mode, double *acc,
                      double *jerk, double *pot, int32_t *nnb, int32_t *list,
                      int32_t cap, int mem_kind, void *stream);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * nb6_regular_force with device arrays only (every array argument is device
 * memory; the call is ordered on `stream` and returns without waiting), whose
 * force-call scratch -- the slice partial sums, the per-i neighbour counters
 * and the unsorted list rows -- lives in one fixed device array of
 * NB6_NOALLOC_SCRATCH_BYTES per GPU, instead of buffers the context grows.
 * The call allocates nothing: the cluster must be loaded and predicted in
 * dx_mode (those calls allocate its records), and NB6_OPT_TIMING does not
 * record this call's launches.  The counters are cleared by the call itself,
 * with a kernel.
 *
 * The scratch of a call is 8 np S ceil(n_i / 64) 64 + 4 n_i + 4 n_i (cap + 1)
 * bytes (each part rounded up to 256 B; np = 6, or 7 with pot; S j-slices).
 * It runs in the caller's order (no spatial i-order, which would need scratch
 * of its own; see NB6_OPT_CALLER_ORDER).
 * When nb6_regular_force's plan on the same context fits the array, the call
 * takes it and both give the same bits; otherwise it takes the most slices
 * that fit (then the sums differ from nb6_regular_force's by rounding only),
 * e.g. about 1100 instead of 4096 for a block of 1024 at N = 2^20 with the
 * potential and cap 1023.  A block too large for one slice (n_i above about
 * 16000 at cap 1023, 62000 at cap 256) is refused with NB6_ERR_ARG, the
 * message giving the bytes it needs.
 *
 * The array is shared by every context on one GPU and keeps the last call's
 * contents: calls that overlap on one GPU (different streams, contexts or
 * threads without ordering between them) race and give undefined results.
 * Other errors are those of nb6_regular_force.
 */
#define NB6_NOALLOC_SCRATCH_BYTES (64u << 20)
int nb6_regular_force_noalloc(nb6_ctx *ctx, int cluster, int64_t n_i,
                              const int32_t *idx_i, const double *h2_i,
                              const double *dtr_i, int dx_mode, double *acc,
                              double *jerk, double *pot, int32_t *nnb,
                              int32_t *list, int32_t cap, void *stream);

/*
 * Wait for `stream` and return (and clear) the GPU-side validation state of
 * the context: NB6_OK, or NB6_ERR_DEVICE_INPUT when a DEVICE-mode call met
 * an out-of-range index, an h2 that is not a positive normal float, a
 * dtr that is negative or not finite, a non-finite predicted coordinate,
 * or an invalid neighbour list
 * (nb6_set_lists).  Results of such a call are NaN for the offending i.
 */
int nb6_sync_status(nb6_ctx *ctx, void *stream);

/*
 * Read back the predicted positions and velocities of every particle of the
 * cluster as the j-stream of `dx_mode` holds them (NB6_DX_FF and
 * NB6_DX_LOCAL: hi + lo, NB6_DX_FP64: the FP64 prediction, NB6_DX_FP32: the
 * float), widened to
 * double: x[N][3], v[N][3].  For checks of the predictor (section 3.3 step 3)
 * and for callers that want the predicted state.  Errors: NB6_ERR_STATE when
 * that stream is not current, NB6_ERR_ARG, NB6_ERR_NOMEM, NB6_ERR_HIP.
 */
int nb6_get_predicted(nb6_ctx *ctx, int cluster, int dx_mode, double *x, double *v,
                      int mem_kind, void *stream);

/*
 * With NB6_OPT_TIMING: wait for the recorded launches and return, for the
 * launches since the previous call, ms[0] = total predictor time,
 * ms[1] = total force-kernel time, ms[2] = total finalize time,
 * ms[3] = total irregular-force time, and counts[0..3] = the number of
 * launches of each (ms and counts hold 4 entries).  The record is then
 * cleared.  Errors: NB6_ERR_STATE when timing is off, NB6_ERR_HIP.
 */
int nb6_kernel_times(nb6_ctx *ctx, double *ms, int64_t *counts);

/* ---- irregular force over stored neighbour lists ----------------------- */

/*
 * Replace the stored neighbour lists of particles idx_i[0..n_i) of the
 * cluster.  The library keeps one list per particle between regular steps
 * and the host sends a particle's list after a regular step that changed it
 * (section 3.5; Appendix C sends each new list after the regular force of
 * its block).  Row k of `list` holds nnb_i[k] entries, list[k*cap + e] for
 * e < nnb_i[k]: particle indices of the cluster, in any order (the list of
 * nb6_regular_force is ascending and can be passed as it is, with the same
 * cap).  An entry equal to the particle itself adds nothing.
 *   1 <= cap <= NB6_MAX_LIST_CAP; 0 <= nnb_i[k] <= cap; the idx_i distinct.
 * A full nb6_load_particles of the cluster empties every stored list; lists
 * never set are empty.  HOST mode checks every argument (NB6_ERR_ARG); in
 * DEVICE mode an out-of-range particle, count or entry is reported by
 * nb6_sync_status (NB6_ERR_DEVICE_INPUT) and that particle's list is stored
 * empty; repeated idx_i then leave one of their lists (which is undefined).
 * Errors: NB6_ERR_ARG, NB6_ERR_STATE, NB6_ERR_NOMEM, NB6_ERR_HIP.
 */
int nb6_set_lists(nb6_ctx *ctx, int cluster, int64_t n_i, const int32_t *idx_i,
                  const int32_t *nnb_i, const int32_t *list, int32_t cap,
                  int mem_kind, void *stream);

/*
 * Irregular force and its time derivative (section 3.3 step 4) of the
 * active particles idx_i[0..n_i) at time t_block, over their stored lists:
 *   acc[q]  = sum_{j in L_i} m_j R_ij / |R_ij|^3
 *   jerk[q] = sum_{j in L_i} m_j (V_ij / |R_ij|^3 - 3 (R_ij.V_ij) R_ij / |R_ij|^5)
 * with i = idx_i[q], R_ij = R_j - R_i and V_ij = V_j - V_i.  Every particle
 * needed is predicted to t_block from the stored state by the cubic Taylor
 * series (section 3.3 step 3), inside the call and independently of
 * nb6_predict_j; all arithmetic is FP64.  acc, jerk: [n_i][3] doubles;
 * pot[n_i] (may be NULL): the irregular potential -sum_{j in L_i} m_j / |R_ij|.
 * Repeated idx_i are allowed.  An empty list gives zeros.  Out-of-range
 * idx_i: NB6_ERR_ARG (HOST) or NaN rows and NB6_ERR_DEVICE_INPUT from
 * nb6_sync_status (DEVICE).  Errors: NB6_ERR_ARG, NB6_ERR_STATE,
 * NB6_ERR_NOMEM, NB6_ERR_HIP, NB6_ERR_DEVICE_INPUT (HOST: a stored list that
 * held an invalid entry).  n_i == 0 is a no-op.
 */
int nb6_irregular_force(nb6_ctx *ctx, int cluster, double t_block, int64_t n_i,
                        const int32_t *idx_i, double *acc, double *jerk,
                        double *pot, int mem_kind, void *stream);

/* ---- regular corrector of a block -------------------------------------- */

/* Parameters of nb6_regular_correct. */
typedef struct nb6_corr_params {
    double eta;     /* accuracy parameter of the step criterion (> 0; the
                       paper's runs use 0.02)                                 */
    double dt_min;  /* smallest regular step, a power of two                  */
    double dt_max;  /* largest regular step, a power of two >= dt_min         */
    double f_lo;    /* limits of the radius factor of equation (1):           */
    double f_hi;    /*   0 < f_lo <= f_hi; f_hi is also used for empty lists  */
} nb6_corr_params;

/* One block of particles that reached their regular time t.  Vectors are
 * [n_i][3] doubles, scalars [n_i]; "old" regular values are those of the
 * previous regular step at t_old with the old list, "new" ones those of
 * the force call at t with the new list; the irregular values g are both at
 * t, with the old and with the new list (nb6_irregular_force before and
 * after nb6_set_lists). */
typedef struct nb6_corr_block {
    int64_t        n_i;
    double         t;
    const double  *t_old;
    const double  *f_old, *fd_old;   /* regular force and derivative at t_old */
    const double  *f_new, *fd_new;   /* regular force and derivative at t     */
    const double  *g_old, *gd_old;   /* irregular, at t, old list             */
    const double  *g_new, *gd_new;   /* irregular, at t, new list             */
    const double  *h_old;            /* neighbour radius of the new list      */
    const int32_t *nnb;              /* size of the new list                  */
    const double  *n_p;              /* neighbour number aimed at (eq. 1)     */
    double        *df, *dfd;         /* out: regular change, fixed list       */
    double        *f2, *f3;          /* out: 2nd derivative at t, 3rd         */
    double        *dt_new, *h_new;   /* out: next regular step, new radius    */
} nb6_corr_block;

/*
 * The regular corrector of a block (section 3.3 step 7):
 *   dF = (f_new - f_old) + (g_new - g_old), and dFd likewise: the regular
 *   force change over the step with the neighbour set held fixed (section
 *   3.6: the irregular-force change at t from the old to the new list);
 *   with h = t - t_old, the cubic through (f_old, fd_old) at t_old and
 *   (f_old + dF, fd_old + dFd) at t (fourth-order Hermite, Makino & Aarseth
 *   1992) gives f3 = (-12 dF + 6 h (2 fd_old + dFd)) / h^3 and
 *   f2 = (6 dF - h (6 fd_old + 2 dFd)) / h^2 + h f3 (the new-time value);
 *   dt_new: the step criterion sqrt(eta (|F||F2| + |Fd|^2) / (|Fd||F3| +
 *   |F2|^2)) on the new-time values, taken down to the largest power of two
 *   that is at most 2 h and dt_max and divides t, and at least dt_min;
 *   h_new = h_old (n_p / nnb)^(1/3) (equation 1), the factor limited to
 *   [f_lo, f_hi], f_hi when nnb == 0.
 * FP64 throughout.  Every pointer of *blk lives in mem_kind memory.
 * Errors: NB6_ERR_ARG (parameters; HOST mode: some t_old >= t, or
 * non-finite), NB6_ERR_NOMEM, NB6_ERR_HIP.  In DEVICE mode a particle with
 * t_old >= t gets NaN outputs and nb6_sync_status reports
 * NB6_ERR_DEVICE_INPUT.  n_i == 0 is a no-op.
 */
int nb6_regular_correct(nb6_ctx *ctx, const nb6_corr_block *blk,
                        const nb6_corr_params *params, int mem_kind, void *stream);

/* ---- serving: continuously batched requests ---------------------------- */

/*
 * One regular-force block of one cluster, for the serving queue.  The
 * fields mean what the arguments of nb6_regular_force mean; t_block is the
 * block time the cluster is predicted to before the force (section 3.3,
 * steps 3 and 6).  All arrays stay owned by the caller and must stay valid,
 * and untouched, until nb6_poll reports the request finished.
 */
typedef struct nb6_request {
    int            cluster;
    double         t_block;
    int            dx_mode;     /* one NB6_DX_* value                    */
    int64_t        n_i;
    const int32_t *idx_i;
    const double  *h2_i;
    const double  *dtr_i;
    double        *acc;         /* [n_i][3] */
    double        *jerk;        /* [n_i][3] */
    int32_t       *nnb;         /* [n_i]    */
    int32_t       *list;        /* [n_i][cap] */
    int32_t        cap;         /* 0 <= cap <= NB6_MAX_CAP */
    int            mem_kind;    /* NB6_MEM_HOST or NB6_MEM_DEVICE */
} nb6_request;

/* What nb6_poll reports about a finished request. */
typedef struct nb6_ticket_info {
    int    status;      /* the request's final status code                     */
    int    slices;      /* j-slices its force work was split into              */
    int    batch_size;  /* requests fused into the launch that served it       */
    double submit_us;   /* steady-clock microseconds since the queue started:  */
    double admit_us;    /*   submitted, admitted to a launch,                  */
    double done_us;     /*   and finished on the GPU                           */
} nb6_ticket_info;

/*
 * Queue one request; *ticket identifies it.  A scheduler thread of the
 * context admits queued requests in arrival order while their device scratch
 * (slice partials, lists, staging; the request's "footprint") fits the
 * context's HBM budget (nb6_options.hbm_budget) and no other request of the
 * same cluster is in flight; it fuses every admitted request into one
 * batch of persistent launches (up to four batches in flight, each on a
 * stream of its own), so requests that arrive while others run are served
 * as memory and batch slots free up.
 * A request's result does not depend on the other requests it is fused with.
 * There is no paper counterpart: the paper keeps two GPUs busy by running
 * two simulations at once (section 4); this queue serves many.
 * Errors: NB6_ERR_ARG, NB6_ERR_STATE (cluster not loaded),
 * NB6_ERR_ADMISSION (the footprint alone exceeds the budget), NB6_ERR_NOMEM,
 * NB6_ERR_HIP.
 */
int nb6_submit(nb6_ctx *ctx, const nb6_request *req, uint64_t *ticket);

/*
 * NB6_PENDING while the request runs (wait == 0), else its final status
 * (NB6_OK, NB6_WARN_NB_OVERFLOW, or an error code), after which the ticket is
 * released.  wait != 0 blocks until the request finishes.  info (may be
 * NULL) receives its timing.  NB6_ERR_UNKNOWN_TICKET for a ticket that was
 * never issued or was already released.
 */
int nb6_poll(nb6_ctx *ctx, uint64_t ticket, int wait, nb6_ticket_info *info);

/* Number of j-slices (the j-split across workgroups) the last force call
 * used; for diagnostics and tests. */
int nb6_last_slices(const nb6_ctx *ctx);

/* Work partition of the last force call, for diagnostics and tests:
 * out[0] i-particles per lane, out[1] lanes per i-particle, out[2] number of
 * j-slices, out[3] j-particles per slice (the last slice may be shorter).
 * Errors: NB6_ERR_ARG (NULL ctx or out). */
int nb6_last_plan(const nb6_ctx *ctx, int out[4]);

#ifdef __cplusplus
}
#endif
#endif /* NB6_H */
