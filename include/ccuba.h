/*
 * ccuba.h -- C ABI of libccuba: the DoSample hot path of Vegas and Cuhre
 * ("Concurrent Cuba", T. Hahn, MPP-2014-327) on one AMD Instinct MI355X.
 *
 * The paper states the problem every call here solves: integrate f over the
 * unit hypercube [0,1]^ndim to the requested relative or absolute accuracy,
 * max(epsabs, epsrel |I|), and return the integral, its error estimate and a
 * chi^2 probability, with neval, fail and nregions as further outputs
 * (Sect. 3.2.2, the Vegas and Cuhre prototypes).  All sampling goes through
 * one batched routine, DoSample (Sect. 2.1), which is what runs on the GPU.
 *
 * Differences from the paper's prototypes, all forced by the device:
 *  - the integrand is a device-side Genz family descriptor (ccuba_integrand)
 *    instead of a host callback, since the GPU cannot call host code per
 *    point; nvec and userdata therefore disappear;
 *  - the `spin' argument (Sect. 3.2.3) becomes a context handle with the same
 *    three cases (see ccuba_ctx);
 *  - two entry points are added: a batch of independent Vegas integrals that
 *    share the device launches of every iteration, and a submit/poll pair
 *    for a serving loop.
 *
 * Conventions for every function:
 *  - return value: CCUBA_OK (0) or a negative CCUBA_E* status; nothing is
 *    thrown across the ABI; ccuba_strerror() names a status;
 *  - host arrays belong to the caller and are read during the call only;
 *    outputs are written before a synchronous call returns;
 *  - the context owns all device memory it allocates (grids, region heaps,
 *    partial sums) and frees it in ccuba_shutdown;
 *  - a context may be used by one host thread at a time (the serving loop's
 *    own thread is internal and synchronised).
 */
#ifndef CCUBA_H
#define CCUBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum {
  CCUBA_OK = 0,
  CCUBA_EINVAL = -1,   /* an argument is out of range */
  CCUBA_EHIP = -2,     /* a HIP runtime call failed */
  CCUBA_ENOMEM = -3,   /* the request does not fit the context's HBM budget */
  CCUBA_ENOENT = -4,   /* unknown ticket or configuration key */
  CCUBA_ESTATE = -5    /* call not allowed in the context's current state */
};

/* ---- integrands ---------------------------------------------------------- */
/* Genz test families (Genz 1987) over [0,1]^d:
 *   GAUSSIAN      exp(-sum a_i^2 (x_i - u_i)^2)
 *   OSCILLATORY   cos(2 pi u_1 + sum a_i x_i)
 *   PRODUCT_PEAK  prod 1 / (a_i^-2 + (x_i - u_i)^2)
 *   CORNER_PEAK   (1 + sum a_i x_i)^-(d+1)
 *   C0            exp(-sum a_i |x_i - u_i|)                                  */
enum { CCUBA_GAUSSIAN = 0, CCUBA_OSCILLATORY = 1, CCUBA_PRODUCT_PEAK = 2,
       CCUBA_CORNER_PEAK = 3, CCUBA_C0 = 4 };

/* a[ndim] and u[ndim] are host arrays, copied during the call. */
typedef struct {
  int family;
  const double *a;
  const double *u;
} ccuba_integrand;

/* ---- flags --------------------------------------------------------------- */
/* bits 0-1: sampling precision.  FP64: points, map, integrand and sums in
 * FP64.  FP32_EVAL: point map and integrand in FP32, every sum, the grid
 * refinement and the final combination in FP64.
 * bit 4: FREEZE_GRID keeps the initial uniform grid (no refinement). */
enum { CCUBA_FP64 = 0, CCUBA_FP32_EVAL = 1, CCUBA_PRECISION_MASK = 3,
       CCUBA_FREEZE_GRID = 1 << 4 };

/* ---- context (the `spin' analog, Sect. 3.2.3) -----------------------------
 * Every integrator takes `ccuba_ctx **ctx':
 *   ctx == NULL  : a temporary context is created and destroyed in the call
 *                  (the paper's NULL / -1: workers started and stopped);
 *   *ctx == NULL : a context is created and returned in *ctx and kept
 *                  (the paper's zero-initialised spin variable);
 *   *ctx != NULL : the existing context is reused (a spin from an earlier
 *                  call or from cubafork).                                   */
typedef struct ccuba_ctx ccuba_ctx;

/* Create a context on HIP device `device' (negative: CCUBA_DEVICE from the
 * environment, else 0) that may allocate at most `hbm_budget' bytes of device
 * memory (0: CCUBA_HBM_BUDGET from the environment, else 90% of the free
 * memory).  The analog of cubafork (Sect. 3.2.3).  Errors: CCUBA_EINVAL
 * (ctx NULL or bad device), CCUBA_EHIP. */
int ccuba_init(ccuba_ctx **ctx, int device, size_t hbm_budget);

/* Stop the serving loop if running, free all device memory and set *ctx to
 * NULL.  The analog of cubawait (Sect. 3.2.3).  A NULL *ctx is accepted. */
int ccuba_shutdown(ccuba_ctx **ctx);

/* Override one setting of the context; explicit settings take precedence
 * over the environment, as cubacores/cubaaccel override CUBACORES and
 * CUBAACCEL (Sect. 3.2.4).  Keys:
 *   "block"          DoSample threads per workgroup (64, 128 or 256)
 *   "blocks_per_cu"  persistent DoSample workgroups per compute unit (1..16)
 *   "hist64"         FP32 path: 1 = FP64 LDS histogram, 0 = 64-bit fixed point
 *                    for every v^2 it holds exactly, FP64 for the rest
 *                    (default; same results up to summation order)
 *   "ilp"            points each lane carries per loop trip, 1 or 2 (default
 *                    2 for FP32, 1 for FP64; the key sets both)
 *   "min_tile"       smallest tile of points in a batched launch (>= 64)
 *   "autotune"       1 = pick the settings above by measurement: a single
 *                    integral times a fixed synthetic integral (cached in the
 *                    file named by CCUBA_TUNE_CACHE, if set); a batch times
 *                    a few iterations of its own jobs, with and without the
 *                    split into halves, once per context and precision
 *   "graph"          1 = replay iterations from a captured hipGraph
 *   "engine_cache"   1 = keep the engine of the last single-integral Vegas call
 *                    (its buffers and graphs) for the next call of its shape
 *   "serve_slots"    maximum requests resident in the serving loop
 *   "batch_streams"  2 = a ccuba_vegas_batch of two or more integrals runs as
 *                    two halves on two streams (default; CCUBA_BATCH_STREAMS),
 *                    1 = as one; per precision like the keys above (the
 *                    batch splits when all its precisions ask for it)
 *   "profile"        1 = time every kernel launch with HIP events (see
 *                    ccuba_stats_get)
 * Returns CCUBA_ENOENT for an unknown key, CCUBA_EINVAL for a bad value. */
int ccuba_config(ccuba_ctx *ctx, const char *key, long long value);

/* Read one setting into *value (the settings take the place of the
 * environment variables and cubaaccel/cubacores calls of Sect. 3.2.4, so a
 * caller can see what is in force): the keys of ccuba_config; the DoSample
 * launch settings ("block", "blocks_per_cu", "hist64", "ilp", "min_tile",
 * "batch_streams") are
 * those of `precision' (CCUBA_FP64 or CCUBA_FP32_EVAL), e.g. after an
 * autotuned batch.  Returns CCUBA_ENOENT for an unknown key. */
int ccuba_config_get(ccuba_ctx *ctx, const char *key, int precision, long long *value);

/* Vegas (Sect. 3.2.2 prototype; Lepage 1978).  Iteration t samples
 * n_t = nstart + t*nincrease points from Philox4x32-10 with counter
 * (i, (t<<8)|b, stream_id, 0) and key (seed mod 2^32, seed div 2^32), maps
 * them through the adaptive grid of nbins bins per dimension, and refines the
 * grid after every iteration.  Iterations combine with inverse-variance
 * weights; prob = P(dof/2, chi2/2) with dof = iterations - 1.  The run stops
 * when neval >= mineval and error <= max(epsabs, epsrel |integral|)
 * (fail = 0), or before an iteration that would take neval past maxeval, or
 * after 4096 iterations (fail = 1).  An iteration whose sums are not finite
 * (an integrand value that is not) ends the run with fail = -4 and zero
 * results; this applies to every integrator below, after the step whose
 * totals are not finite.  nbatch only partitions the sampling
 * internally and has no bearing on the results (Sect. 3.2.7); it must be
 * >= 1.  Ranges: 1 <= ndim <= 16, ncomp == 1, 2 <= nbins <= 256,
 * nstart >= 2, nincrease >= 0, every n_t < 2^32.  Outputs have ncomp = 1
 * entries.  Errors: CCUBA_EINVAL, CCUBA_EHIP, CCUBA_ENOMEM. */
int ccuba_vegas(ccuba_ctx **ctx, int ndim, int ncomp, const ccuba_integrand *f,
                double epsrel, double epsabs, int flags, unsigned long long seed,
                long long mineval, long long maxeval, long long nstart,
                long long nincrease, long long nbatch, int nbins,
                unsigned int stream_id, long long *neval, int *fail,
                double integral[], double error[], double prob[]);

/* Optional trace of a Vegas run (any pointer may be NULL). */
typedef struct {
  int max_iter;     /* capacity of iter_I and iter_var */
  int n_iter;       /* out: iterations done */
  double *iter_I;   /* out: I_t per iteration */
  double *iter_var; /* out: sigma_t^2 per iteration */
  double chi2;      /* out */
  int dof;          /* out */
  double *grid;     /* out: final grid, ndim * (nbins + 1) */
} ccuba_vegas_trace;

/* ccuba_vegas with a trace (trace may be NULL): besides the outputs of the
 * Sect. 3.2.2 prototype, each iteration's estimate and variance, the chi^2
 * that prob is taken from, and the final grid, written before return into
 * the caller's arrays (capacities as given in the struct). */
int ccuba_vegas_ex(ccuba_ctx **ctx, int ndim, int ncomp, const ccuba_integrand *f,
                   double epsrel, double epsabs, int flags,
                   unsigned long long seed, long long mineval, long long maxeval,
                   long long nstart, long long nincrease, long long nbatch,
                   int nbins, unsigned int stream_id, long long *neval,
                   int *fail, double integral[], double error[], double prob[],
                   ccuba_vegas_trace *trace);

/* ccuba_vegas_ex with the prototype's gridno and statefile (Sect. 3.2.2).
 * gridno: a slot of the context's grid table.  With gridno != 0 the run
 * starts from the grid kept in slot |gridno| when that grid has the same
 * ndim and nbins (else from the uniform grid); with gridno > 0 the final grid
 * is kept in the slot for later calls.  Iterations, sums and counters start
 * afresh: only the grid is reused.
 * statefile: a file path (NULL or "" for none).  After every iteration the
 * state, grid and per-iteration history are written to it (atomically, by a
 * rename).  A call that finds the file continues from it, provided it was
 * written for the same ndim, nbins, integrand, precision and flags, seed,
 * stream_id, nstart and nincrease (else CCUBA_EINVAL); tolerances, mineval
 * and maxeval may differ, so a run stopped by maxeval continues under a
 * larger one.  The file is removed once the integral converges (fail = 0).
 * A resumed run samples the same points as an uninterrupted one.  With a
 * state file iterations run one at a time (each is read back and saved).
 * Errors: those of ccuba_vegas, and CCUBA_EINVAL for a state file that does
 * not fit, cannot be read or cannot be written. */
int ccuba_vegas_stateful(ccuba_ctx **ctx, int ndim, int ncomp, const ccuba_integrand *f,
                         double epsrel, double epsabs, int flags, unsigned long long seed,
                         long long mineval, long long maxeval, long long nstart,
                         long long nincrease, long long nbatch, int gridno, const char *statefile,
                         int nbins, unsigned int stream_id, long long *neval, int *fail,
                         double integral[], double error[], double prob[],
                         ccuba_vegas_trace *trace);

/* ---- device integrands compiled at run time ------------------------------
 * Vegas of a caller's integrand written as HIP device code, evaluated per
 * point inside DoSample like the built-in families (the integrand of
 * Sect. 3.2.2, as GPU code).  `source' is a null-terminated string that
 * defines
 *   __device__ double ccuba_user(const double *x, int ndim, const double *a,
 *                                const double *u);
 * and, for CCUBA_FP32_EVAL, the same with float in place of double; x holds
 * the point, a and u the ndim parameters given here (NULL: zeros; in float
 * for FP32 evaluation).  The source may use the HIP device math functions
 * but no headers.  The library compiles the DoSample kernel with it for the
 * context's GPU on first use (hiprtc) and keeps it in the context until
 * ccuba_shutdown.  All other arguments, outputs, ranges and results are
 * those of ccuba_vegas.  Errors: CCUBA_EINVAL (also when the source does not
 * compile: ccuba_rtc_log returns the compiler's message), CCUBA_EHIP,
 * CCUBA_ENOMEM. */
int ccuba_vegas_source(ccuba_ctx **ctx, int ndim, const char *source, const double *a,
                       const double *u, double epsrel, double epsabs, int flags,
                       unsigned long long seed, long long mineval, long long maxeval,
                       long long nstart, long long nincrease, long long nbatch, int nbins,
                       unsigned int stream_id, long long *neval, int *fail, double integral[],
                       double error[], double prob[]);

/* The compiler's message of ctx's last run-time compilation of a caller's
 * integrand (the Sect. 3.2.2 integrand as device code), null-terminated and
 * cut to size bytes (empty if none), written into the caller's buf.
 * Errors: CCUBA_EINVAL. */
int ccuba_rtc_log(ccuba_ctx *ctx, char *buf, size_t size);

/* ---- caller-evaluated integrands ---------------------------------------
 * The integrand declaration of Sect. 3.2.2 with its nvec and core arguments:
 * x[*nvec][*ndim] points, f[*nvec][*ncomp] values for the integrand to fill.
 * Returning -999 aborts the integration at once; any other value goes on.
 * core is -1: the points come in the accelerator strategy of Sect. 3.2.4. */
typedef int (*ccuba_batch_integrand)(const int *ndim, const double x[], const int *ncomp,
                                     double f[], void *userdata, const int *nvec,
                                     const int *core);

/* where the batch's x and f live during the integrand call */
enum { CCUBA_POINTS_HOST = 0, CCUBA_POINTS_DEVICE = 1 };

/* Vegas of a caller's integrand (the same sampling, combination and stop rule
 * as ccuba_vegas, over ncomp components).  Each iteration's points are made
 * on the GPU and handed to the integrand in batches of exactly nvec points
 * (fewer only in an iteration's last batch; Sect. 3.2.4).  With
 * CCUBA_POINTS_HOST x and f are host arrays the library owns; with
 * CCUBA_POINTS_DEVICE they are device arrays on the context's GPU, and the
 * integrand's writes to f must be complete when it returns (for work it
 * launches itself, it synchronises first).  The integrand runs while the
 * context is held and must not call back into the same context.
 * Components: every one has its own sums, estimate, combination, chi^2 and
 * prob over the same points; the grid adapts to component 0's histogram;
 * the accuracy test needs every component within its tolerance.
 * fail: 0 accuracy reached, 1 maxeval reached first, -4 a value that is
 * not finite, -99 the integrand
 * returned -999 (then neval counts every point handed to it and the results
 * are 0).  Ranges: 1 <= ndim <= 16, 1 <= ncomp <= 16, 2 <= nbins <= 256,
 * nvec >= 1, nstart >= 2, nincrease >= 0, every n_t < 2^32.  integral, error
 * and prob have ncomp entries.  Errors: CCUBA_EINVAL, CCUBA_EHIP,
 * CCUBA_ENOMEM. */
int ccuba_vegas_batched(ccuba_ctx **ctx, int ndim, int ncomp, ccuba_batch_integrand integrand,
                        void *userdata, int nvec, int where, double epsrel, double epsabs,
                        int flags, unsigned long long seed, long long mineval,
                        long long maxeval, long long nstart, long long nincrease, int nbins,
                        unsigned int stream_id, long long *neval, int *fail, double integral[],
                        double error[], double prob[]);

/* ---- Suave -----------------------------------------------------------------
 * Subregion-adaptive Vegas: the Suave prototype of Sect. 3.2.2 (nnew,
 * flatness, nregions), whose steps the paper does not give.  Reading: every
 * region keeps its own Vegas grid and the values of its own nnew-point
 * sample.  The root [0,1]^d is sampled first; then each step bisects the K
 * regions of largest variance (ties: lower position), K = min(nsplit,
 * regions, (maxeval - neval) / (2 nnew)), at the midpoint of the dimension
 * whose halves have the least total fluctuation
 *   F_h = (n_h/n) ((1/n_h) sum_{i in h} |v_i - m_h|^p)^(1/p),  p = flatness.
 * A child's grid is its parent's, with the map along the cut restricted to
 * the child's half; its result combines (inverse-variance weights) the
 * estimate from its parent's sample points inside it with that of its own
 * nnew new points.  The j-th split of the run draws its children's points
 * with Philox iteration numbers 2j+1 and 2j+2 (the root: 0).  Totals: the sums
 * of the regions' estimates and variances; prob = P(dof/2, chi^2/2) over the
 * regions' combinations.  Stop when neval >= mineval and error <=
 * max(epsabs, epsrel |integral|) (fail 0), or when no split fits maxeval (fail
 * 1; maxeval < nnew samples nothing).  nsplit = 1 is one region at a time.
 * flags: CCUBA_FP64, optionally CCUBA_FREEZE_GRID.  Ranges: 1 <= ndim <= 16,
 * ncomp == 1, 2 <= nbins <= 256, 2 <= nnew < 2^32, flatness > 0,
 * 1 <= nsplit <= 1024, regions at most 2^23.  The device holds 10 bytes per
 * sampled point plus each region's grid.  Errors: CCUBA_EINVAL, CCUBA_EHIP,
 * CCUBA_ENOMEM (beyond the budget). */
typedef struct {
  int max_regions;    /* capacity of the per-region arrays */
  int max_splits;     /* capacity of cut */
  int nregions;       /* out */
  int nsplits;        /* out */
  double chi2;        /* out: summed over the regions */
  int dof;            /* out */
  double *lo, *hi;    /* out: [nregions][ndim] bounds, in position order */
  double *I, *var;    /* out: each region's combined estimate and variance */
  double *grid;       /* out: [nregions][ndim][nbins + 1] (may be NULL) */
  int *cut;           /* out: the dimension of every split, in order */
} ccuba_suave_trace;

int ccuba_suave(ccuba_ctx **ctx, int ndim, int ncomp, const ccuba_integrand *f, double epsrel,
                double epsabs, int flags, unsigned long long seed, long long mineval,
                long long maxeval, long long nnew, double flatness, int nbins, int nsplit,
                unsigned int stream_id, int *nregions, long long *neval, int *fail,
                double integral[], double error[], double prob[], ccuba_suave_trace *trace);

/* ---- Divonne's partitioning phase ------------------------------------------
 * Sect. 2.2: the integration region is split into subregions of about equal
 * spread, Spread(r) = 1/2 Vol(r) (sup_r f - inf_r f), with the extrema
 * sought by numerical optimisation; the parallel version gives each worker a
 * whole region to search and subdivide (here: one workgroup per region, all
 * regions of a step in one launch).  Reading of the unstated steps: a
 * region's extrema start from the largest and smallest value of nsearch
 * Philox points in it (search serial q: counter (i, (q<<8)|b, stream_id, 0))
 * and are refined by two compass searches of niter iterations (steps w/4,
 * 2d clipped candidates x +- h_j e_j, the best taken if it improves, else
 * all steps halve).  Each step bisects the K = min(nsplit, regions,
 * maxregions - regions) regions of largest spread (ties: lower position) at
 * the midpoint of the dimension j maximising fmax - f(xmax with x_j :=
 * xmin_j); the j-th split searches its children with serials 2j+1 and 2j+2
 * (the root: 0).  fail = 0 once every spread is <= spread_tol, 1 when
 * maxregions ends the phase.  neval counts every evaluation: nsearch + 4 d
 * niter per search and d per split.  total_spread is the sum of the spreads.
 * Ranges: 1 <= ndim <= 16, 1 <= nsearch <= 2^30, 0 <= niter <= 4096,
 * 1 <= maxregions <= 2^23, 1 <= nsplit <= 1024, spread_tol >= 0.  Errors:
 * CCUBA_EINVAL, CCUBA_EHIP, CCUBA_ENOMEM. */
typedef struct {
  int max_regions;           /* capacity of the per-region arrays */
  int max_splits;            /* capacity of cut */
  int nregions, nsplits;     /* out */
  double *lo, *hi;           /* out: [nregions][ndim] bounds, in position order */
  double *xmin, *xmax;       /* out: [nregions][ndim] the extrema's points */
  double *fmin, *fmax;       /* out: [nregions] */
  double *spread;            /* out: [nregions] */
  int *cut;                  /* out: the dimension of every split, in order */
} ccuba_partition_trace;

int ccuba_divonne_partition(ccuba_ctx **ctx, int ndim, const ccuba_integrand *f,
                            unsigned long long seed, unsigned int stream_id, int nsearch,
                            int niter, int maxregions, int nsplit, double spread_tol,
                            int *nregions, long long *neval, int *fail, double *total_spread,
                            ccuba_partition_trace *trace);

/* Cuhre (Sect. 3.2.2 prototype) with the degree-7 Genz-Malik rule and its
 * embedded degree-5 rule (Genz & Malik 1980), error |I7 - I5|, bisection of
 * each selected region along its largest fourth difference.  Each step splits
 * the K = min(max_regions_per_batch/2, regions) regions of largest error
 * (ties: lower region id) and evaluates the 2K children in one launch, until
 * neval >= mineval and error <= max(epsabs, epsrel |integral|) (fail = 0), or
 * until no child fits maxeval any more (fail = 1).  key must be 0 or 7.
 * prob is 0.  Ranges: 2 <= ndim <= 16, ncomp == 1,
 * max_regions_per_batch >= 2.  Errors: CCUBA_EINVAL, CCUBA_EHIP,
 * CCUBA_ENOMEM (region heap beyond the budget). */
int ccuba_cuhre(ccuba_ctx **ctx, int ndim, int ncomp, const ccuba_integrand *f,
                double epsrel, double epsabs, int flags, long long mineval,
                long long maxeval, int key, long long max_regions_per_batch,
                int *nregions, long long *neval, int *fail, double integral[],
                double error[], double prob[]);

/* The Cuhre rule alone on a batch of regions: the DoSample of Cuhre
 * (Sect. 2.1: the sampling routine every integrator calls), one launch for
 * all nreg regions.
 * c[ndim*nreg] and h[ndim*nreg] are host arrays of centres and half-widths,
 * structure-of-arrays (dimension-major: c[j*nreg + r]).  Outputs per region:
 * I7, I5, err = |I7 - I5|, split axis.  Any output may be NULL.
 * Errors: CCUBA_EINVAL, CCUBA_EHIP, CCUBA_ENOMEM. */
int ccuba_cuhre_rule(ccuba_ctx *ctx, int ndim, const ccuba_integrand *f,
                     long long nreg, const double *c, const double *h,
                     double *I7, double *I5, double *err, int *axis);

/* ---- batched Vegas (many independent integrals, one launch per iteration) */
typedef struct {
  int method;               /* 0 Vegas, 1 Cuhre (submit only) */
  int ndim;
  ccuba_integrand f;
  double epsrel, epsabs;
  int flags;
  unsigned long long seed;
  unsigned int stream_id;
  long long mineval, maxeval, nstart, nincrease;
  int nbins;                /* Vegas bins (0: 128) */
  long long max_regions_per_batch; /* Cuhre (0: 100000) */
} ccuba_job;

typedef struct {
  long long neval;
  int nregions, fail, status; /* status: CCUBA_OK or the job's error */
  double integral, error, prob;
  double t_submit, t_done;    /* seconds on the context's steady clock */
} ccuba_result;

/* Run njobs independent Vegas integrals together.  DoSample (Sect. 2.1) is
 * the one routine every integrator samples through, and the paper splits one
 * call's n points into batches for N workers; here the points of all jobs'
 * current iterations are split into tiles of (job, point range), and the
 * tiles of every job still running go out together: one sampling launch per
 * class of tile shape (precision, Philox blocks per point, bins a power of
 * two or not, tile full or ragged), each a persistent grid over that class's
 * tile list, then one fold of the partial sums and one refine launch for all
 * jobs.  The launches of an iteration are replayed from a captured hipGraph.
 * A batch of two or more jobs can be split into two halves of about equal
 * evaluations, each run so on a stream of its own (the context's and a
 * second one), so that one half's sampling has the compute units while the
 * other half folds and refines ("batch_streams"; the autotuner measures
 * both); the call returns when both are done.
 * Like nbatch (Sect. 3.2.7), the tiling partitions the sampling internally
 * and changes neither the points nor what the integrand sees: each job's
 * result is the one ccuba_vegas gives for it alone (same points; sums in
 * another order, within rounding).
 * jobs[njobs]: host array, read during the call; jobs[j].f's arrays are
 * copied.  out[njobs]: host array, written before the call returns; a job
 * that fails on its own (method != 0, or an argument out of range) gets
 * status CCUBA_EINVAL in its out[j] while the others run.
 * Errors: CCUBA_EINVAL (njobs < 0, a NULL array), CCUBA_EHIP, CCUBA_ENOMEM
 * (the jobs' grids and partial sums exceed the context's budget). */
int ccuba_vegas_batch(ccuba_ctx *ctx, int njobs, const ccuba_job jobs[],
                      ccuba_result out[]);

/* ---- serving loop -------------------------------------------------------
 * The spinning workers of Sect. 3.2.3 carried further: the context keeps a
 * background thread that stays up between integrations (it starts at the
 * first ccuba_submit and stops in ccuba_shutdown, the cubawait analog), and
 * requests reach it while others run, as batches reach the next free worker
 * in Sect. 3.2.4.  Each tick the thread admits queued requests while slots
 * and the HBM budget allow, keeps their grids and region heaps resident, runs
 * the next Vegas iteration of every resident Vegas request as one batch
 * (ccuba_vegas_batch's launches) and the next region batch of every resident
 * Cuhre request in one rule launch, and retires finished requests.  A
 * request's outputs are those of the Sect. 3.2.2 prototypes and equal what
 * ccuba_vegas or ccuba_cuhre gives it alone.
 *
 * ccuba_submit: *job is read during the call (its integrand arrays copied);
 * *ticket receives the request's id.  Errors: CCUBA_EINVAL (a NULL pointer,
 * method not 0 or 1, ndim outside 1..16), CCUBA_ENOMEM (host allocation of
 * the loop).  A request whose other arguments are out of range, or whose
 * memory can never fit the budget, is accepted and finishes with status
 * CCUBA_EINVAL or CCUBA_ENOMEM in its result.
 * ccuba_poll: returns 0 and fills *out once the ticket is done (the ticket is
 * then forgotten), 1 while pending, CCUBA_ENOENT for an unknown or already
 * collected ticket.
 * ccuba_drain: blocks until every submitted request is done (at once if
 * nothing was ever submitted).  If a tick of the loop fails on the device,
 * the requests it held finish with that status (CCUBA_EHIP, CCUBA_ENOMEM) in
 * their results. */
int ccuba_submit(ccuba_ctx *ctx, const ccuba_job *job, unsigned long long *ticket);
int ccuba_poll(ccuba_ctx *ctx, unsigned long long ticket, ccuba_result *out);
int ccuba_drain(ccuba_ctx *ctx);

/* ---- device-buffer entry points (for callers that own memory/streams) ---
 * One DoSample pass (Sect. 2.1: sample n points, here over every compute
 * unit at once) of Vegas iteration `iteration' over npts points on the FP64
 * grid grid_dev[ndim*(nbins+1)] (device memory, dimension-major, each row
 * nbins+1 ascending edges from 0 to 1), on the caller's HIP stream (NULL: the
 * default stream).  Writes sums_dev[2] = (sum w f, sum (w f)^2) and
 * hist_dev[ndim*nbins] = per-bin sums of (w f)^2, all FP64 device memory
 * owned by the caller and never freed here.  The job is given by its fields
 * (ndim, nbins, f, flags, seed, stream_id) rather than a ccuba_job, since
 * one pass needs none of the convergence settings.  Work already on the
 * stream runs first; the call returns once the pass has finished on it (the
 * partial sums it allocates are freed on return).
 * Ranges: 1 <= ndim <= 16, 2 <= nbins <= 256, npts >= 2,
 * 0 <= iteration < 2^24.
 * Errors: CCUBA_EINVAL (a range or a NULL pointer), CCUBA_EHIP,
 * CCUBA_ENOMEM. */
int ccuba_vegas_dosample_raw(ccuba_ctx *ctx, int ndim, int nbins,
                             const ccuba_integrand *f, int flags,
                             unsigned long long seed, unsigned int stream_id,
                             int iteration, long long npts, const double *grid_dev,
                             double *sums_dev, double *hist_dev, void *hip_stream);

/* ccuba_vegas_dosample_raw for callers that cannot allocate: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  The
 * same pass, arguments and outputs, but it calls no hipMalloc, hipFree or
 * other allocating routine and does not synchronise: the descriptors and the
 * partial sums (one row of 2 + ndim*nbins doubles per tile and per group of
 * 32 tiles) live in a 16 MiB device array that the library holds on every
 * GPU it runs on until the process ends, found at ccuba_init.  Tiles are
 * those of ccuba_vegas_dosample_raw, or fewer and larger when their rows
 * would not fit the array; a call that would need more (fewer than one tile
 * per compute unit) returns CCUBA_ENOMEM and launches nothing.  Every call on
 * a GPU uses that GPU's one array, which keeps the last call's contents, so
 * calls that overlap on one GPU (other streams, other contexts, other host
 * threads) race: serialise them, e.g. on one stream.  Errors: CCUBA_EINVAL,
 * CCUBA_EHIP, CCUBA_ENOMEM. */
int ccuba_vegas_dosample_raw_noalloc(ccuba_ctx *ctx, int ndim, int nbins,
                                     const ccuba_integrand *f, int flags,
                                     unsigned long long seed, unsigned int stream_id,
                                     int iteration, long long npts, const double *grid_dev,
                                     double *sums_dev, double *hist_dev, void *hip_stream);

/* The points DoSample draws (Sect. 2.1; steps: Philox words, uniform, grid
 * map, weight) for points [i0, i0+npts) of iteration `iteration' on the
 * host grid grid[ndim*(nbins+1)], computed on the device by the same code
 * as the sampling kernels.  The paper's master alone generates the samples,
 * so that no random number is used twice (Sect. 2); here point i's words
 * are a pure function of (seed, stream_id, iteration, i), which gives the
 * same guarantee without a master.  Outputs (host, any may be NULL, written
 * before return): words[npts*4*ceil(ndim/4)], x[npts*ndim] (point-major),
 * w[npts], bin[npts*ndim].  Errors: CCUBA_EINVAL, CCUBA_EHIP. */
int ccuba_vegas_points(ccuba_ctx *ctx, int ndim, int nbins, int flags,
                       unsigned long long seed, unsigned int stream_id,
                       int iteration, const double *grid, long long i0,
                       long long npts, uint32_t *words, double *x, double *w,
                       int *bin);

/* One Lepage grid refinement on the device, the step between two DoSample
 * passes of Vegas (Sect. 2.1 leaves the integrator's own algorithm
 * unchanged; the refinement is Lepage's): hist[ndim*nbins] accumulated
 * (w f)^2 per bin, grid_in[ndim*(nbins+1)] -> grid_out (host arrays, read
 * and written during the call; grid_out may equal grid_in).
 * Errors: CCUBA_EINVAL, CCUBA_EHIP. */
int ccuba_vegas_refine(ccuba_ctx *ctx, int ndim, int nbins, const double *hist,
                       const double *grid_in, double *grid_out);

/* Kernel timing of the context, for timing measurements like those of
 * Sect. 4.2 taken on the device side; measured with HIP events recorded on the
 * stream each kernel is launched on, around the sampling kernels, the fold of
 * their partial sums and the refine launch of every Vegas iteration, and
 * around every Cuhre rule launch, while the context's "profile" setting is 1
 * (iterations are then launched one by one rather than replayed from a
 * graph).  evals counts the points sampled by the timed sampling launches.
 * dosample_busy_ms is the time during which at least one sampling launch
 * ran: the sum of their durations, except for a batch run as two halves on
 * two streams, whose sampling launches can overlap: there it is the length of
 * the union of their intervals. */
typedef struct {
  long long dosample_launches; /* sampling kernel launches (one per tile class) */
  double dosample_ms;      /* summed sampling kernel time */
  long long refine_launches;
  double refine_ms;
  long long evals;
  long long rule_launches; /* Cuhre rule kernels */
  double rule_ms;
  long long rule_evals;
  double fold_ms;          /* summed time of the partial-sum folds */
  double dosample_busy_ms; /* time with a sampling launch running (see above) */
} ccuba_stats;

/* Copy the context's counters to *out (host, written before return) and reset
 * them when reset != 0.  Errors: CCUBA_EINVAL (NULL argument). */
int ccuba_stats_get(ccuba_ctx *ctx, ccuba_stats *out, int reset);

/* Name of a status code: a static string, never freed; "unknown status" for a
 * value that is no CCUBA_E* code.  The statuses are this library's; the
 * integrators' own outcome stays in `fail' (Sect. 3.2.2). */
const char *ccuba_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
