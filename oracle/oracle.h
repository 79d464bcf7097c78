/*
 * oracle.h -- plain, slow, serial FP64 CPU oracle for the DoSample hot path
 * of Vegas and Cuhre ("Concurrent Cuba", T. Hahn, MPP-2014-327).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant generator with
 * the device library, and it never includes anything from the package.
 *
 * The paper poses the problem (integrate f over the unit hypercube to a
 * requested relative/absolute accuracy, returning integral, error and a chi^2
 * probability; Sect. 3.2.2, the Vegas and Cuhre prototypes) and computes it
 * all through one sampling routine, DoSample (Sect. 2.1).  It defers the
 * integrators' internals to the literature; the oracle follows the published
 * methods:
 *   - random numbers : Philox4x32-10, Salmon, Moraes, Dror, Shaw,
 *                      "Parallel random numbers: as easy as 1, 2, 3", SC'11;
 *   - Vegas          : G. P. Lepage, J. Comput. Phys. 27 (1978) 192;
 *   - Cuhre rule     : A. C. Genz, A. A. Malik, J. Comput. Appl. Math. 6
 *                      (1980) 295, degree-7 rule with embedded degree-5 rule;
 *   - test integrands: the Genz families (Genz 1984).
 * Every place where the paper is silent carries the reading chosen for it in
 * the comment of the function that implements it.
 *
 * All entry points are serial (the analog of CUBACORES=0, Sect. 3.2.6), and
 * call the integrand through the paper's integrand_t with up to nvec points
 * per call (Sect. 3.2.2, Sect. 3.2.7).
 */
#ifndef CCUBA_ORACLE_H
#define CCUBA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The full integrand declaration of Sect. 3.2.2: x[*nvec][*ndim],
 * f[*nvec][*ncomp]; returning -999 aborts the integration at once. */
typedef int (*oracle_integrand_t)(const int *ndim, const double x[],
                                  const int *ncomp, double f[], void *userdata,
                                  const int *nvec, const int *core);

/* Philox4x32-10 block function (Salmon et al. 2011): out = philox(ctr, key). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]);

/* Precision of the sampling arithmetic (flags bits 0-1).
 *  ORACLE_FP64      : everything in FP64 (the reference).
 *  ORACLE_FP32_EVAL : point map and integrand evaluated in IEEE binary32
 *                     (emulated with C float), accumulation in FP64. */
enum { ORACLE_FP64 = 0, ORACLE_FP32_EVAL = 1 };
enum { ORACLE_PRECISION_MASK = 3, ORACLE_FREEZE_GRID = 1 << 4 };

/* Genz test families, Genz (1984). */
enum { ORACLE_GAUSSIAN = 0, ORACLE_OSCILLATORY = 1, ORACLE_PRODUCT_PEAK = 2,
       ORACLE_CORNER_PEAK = 3, ORACLE_C0 = 4 };

typedef struct {
  int family;      /* ORACLE_GAUSSIAN .. ORACLE_C0 */
  int ndim;
  const double *a; /* a[ndim] */
  const double *u; /* u[ndim] */
  int precision;   /* ORACLE_FP64 or ORACLE_FP32_EVAL */
} oracle_genz;

/* One Genz value at one point. */
double oracle_genz_eval(const oracle_genz *g, const double *x);
/* The same as an integrand_t; userdata points to an oracle_genz. */
int oracle_genz_integrand(const int *ndim, const double x[], const int *ncomp,
                          double f[], void *userdata, const int *nvec,
                          const int *core);

/* Vegas sample points of one iteration on a given grid (steps a1-a3).
 * grid[ndim*(nbins+1)], row j = edges of dimension j.  For points
 * i in [i0, i0+npts): words[(i-i0)*4*nblk + 4*b + q] (nblk = ceil(ndim/4)),
 * x[(i-i0)*ndim + j], w[i-i0], bin[(i-i0)*ndim + j].  Any output may be NULL. */
int oracle_vegas_points(int ndim, int nbins, int precision,
                        unsigned long long seed, unsigned int stream_id,
                        int iteration, const double *grid, long long i0,
                        long long npts, uint32_t *words, double *x, double *w,
                        int *bin);

/* One grid refinement of one dimension (Lepage 1978): H[nbins] accumulated
 * (w f)^2 per bin, E_in[nbins+1] old edges, E_out[nbins+1] new edges. */
void oracle_vegas_refine_dim(int nbins, const double *H, const double *E_in,
                             double *E_out);

/* Optional per-run trace of Vegas (any pointer may be NULL). */
typedef struct {
  int max_iter;       /* capacity of iter_I / iter_var */
  int n_iter;         /* out: iterations done */
  double *iter_I;     /* out: I_t */
  double *iter_var;   /* out: sigma_t^2 */
  double chi2;        /* out */
  int dof;            /* out */
  double *grid;       /* out: final grid, ndim*(nbins+1) */
  double *hist;       /* out: histogram of the last iteration, ndim*nbins */
} oracle_vegas_trace;

/* Vegas integrator with the paper's argument list (Sect. 3.2.2) plus the
 * bin count and the Philox stream id.  Returns 0, or -1 for bad arguments.
 * fail: 0 accuracy reached, 1 maxeval reached first, -99 integrand aborted.
 * 1 <= ncomp <= 16: integral/error/prob hold ncomp values; the grid adapts to
 * component 0; the trace records component 0. */
int oracle_vegas(int ndim, int ncomp, oracle_integrand_t integrand,
                 void *userdata, int nvec, double epsrel, double epsabs,
                 int flags, unsigned long long seed, long long mineval,
                 long long maxeval, long long nstart, long long nincrease,
                 long long nbatch, int nbins, unsigned int stream_id,
                 long long *neval, int *fail, double integral[],
                 double error[], double prob[], oracle_vegas_trace *trace);

/* oracle_vegas started from grid_in (ndim rows of nbins + 1 edges) instead of
 * the uniform grid; grid_in NULL is oracle_vegas. */
int oracle_vegas_from(const double *grid_in, int ndim, int ncomp,
                      oracle_integrand_t integrand, void *userdata, int nvec, double epsrel,
                      double epsabs, int flags, unsigned long long seed, long long mineval,
                      long long maxeval, long long nstart, long long nincrease,
                      long long nbatch, int nbins, unsigned int stream_id, long long *neval,
                      int *fail, double integral[], double error[], double prob[],
                      oracle_vegas_trace *trace);

/* Genz-Malik degree-7/5 rule over one region with centre c[ndim] and
 * half-widths h[ndim].  dfour[ndim] (may be NULL) receives the fourth
 * differences.  Returns 0, -1 bad arguments, -99 integrand aborted. */
int oracle_gm_rule(int ndim, oracle_integrand_t integrand, void *userdata,
                   int nvec, const double *c, const double *h, double *I7,
                   double *I5, double *err, int *axis, double *dfour);

/* Number of rule points, 2^d + 2d^2 + 2d + 1. */
long long oracle_gm_npoints(int ndim);

typedef struct {
  int n_batches;  /* out: rule batches evaluated after the root */
} oracle_cuhre_trace;

/* Cuhre: globally adaptive subdivision with the degree-7 Genz-Malik rule,
 * batches of up to max_regions_per_batch new regions.  key must be 0 or 7. */
int oracle_cuhre(int ndim, int ncomp, oracle_integrand_t integrand,
                 void *userdata, int nvec, double epsrel, double epsabs,
                 int flags, long long mineval, long long maxeval, int key,
                 long long max_regions_per_batch, int *nregions,
                 long long *neval, int *fail, double integral[],
                 double error[], double prob[], oracle_cuhre_trace *trace);

/* Lower regularized incomplete gamma function P(a, x). */
/* Suave (subregion-adaptive Vegas; the steps are listed in suave.cpp).
 * Regions are reported in position order. */
typedef struct {
  int max_regions;    /* capacity of the per-region arrays */
  int max_splits;     /* capacity of cut */
  int nregions;       /* out */
  int nsplits;        /* out: splits done */
  double chi2;        /* out: summed over regions */
  int dof;            /* out */
  double *lo, *hi;    /* out: [nregions][ndim] bounds */
  double *I, *var;    /* out: each region's combined estimate and variance */
  double *inh_I;      /* out: the estimate inherited from the parent (0: none) */
  double *inh_var;    /* out: its variance (0: none kept) */
  double *grid;       /* out: [nregions][ndim][nbins + 1] grids */
  int *cut;           /* out: the dimension of every split, in order */
} oracle_suave_trace;

/* The Suave prototype of Sect. 3.2.2 with ncomp = 1 (FP64), plus the bin
 * count, the regions split per step (nsplit = 1: one at a time) and the
 * Philox stream id.  Returns 0, or -1 for bad arguments.  fail: 0 accuracy
 * reached, 1 maxeval reached first, -99 integrand aborted. */
int oracle_suave(int ndim, int ncomp, oracle_integrand_t integrand, void *userdata, int nvec,
                 double epsrel, double epsabs, int flags, unsigned long long seed,
                 long long mineval, long long maxeval, long long nnew, double flatness,
                 int nbins, int nsplit, unsigned int stream_id, int *nregions,
                 long long *neval, int *fail, double integral[], double error[],
                 double prob[], oracle_suave_trace *trace);

/* Divonne's partitioning phase (Sect. 2.2; the steps are listed in
 * divonne.cpp).  Regions are reported in position order. */
typedef struct {
  int max_regions, max_splits;
  int nregions, nsplits;        /* out */
  double *lo, *hi;              /* out: [nregions][ndim] */
  double *xmin, *xmax;          /* out: [nregions][ndim] the extrema's points */
  double *fmin, *fmax, *spread; /* out: [nregions] */
  int *cut;                     /* out: the dimension of every split */
} oracle_partition_trace;

int oracle_divonne_partition(int ndim, oracle_integrand_t integrand, void *userdata, int nvec,
                             unsigned long long seed, unsigned int stream_id, int nsearch,
                             int niter, int maxregions, int nsplit, double spread_tol,
                             int *nregions, long long *neval, int *fail, double *total_spread,
                             oracle_partition_trace *trace);

double oracle_gammainc_lower(double a, double x);

#ifdef __cplusplus
}
#endif
#endif
