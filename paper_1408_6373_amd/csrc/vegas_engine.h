// vegas_engine.h -- host driver of the batched Vegas DoSample engine.
//
// One engine holds any number of independent Vegas integrals resident on the
// device (grids, parameters, partial sums, iteration history, state) and
// advances all of them one iteration per launch pair (DoSample + refine).
// A single integral is an engine with one job.
#pragma once
#include <functional>
#include <utility>
#include <vector>

#include "context.h"
#include "vegas.h"

namespace ccuba {

constexpr int kIterCap = 4096;  // iterations kept per integral

// Host description of one Vegas integral.
struct VegasSpec {
  int ndim = 1, nbins = 128, family = 0, prec = FP64, flags = 0;
  unsigned long long seed = 0;
  uint32_t sid = 0;
  long long nstart = 1000, nincrease = 0, mineval = 0, maxeval = 0;
  double epsrel = 0, epsabs = 0;
  double a[kMaxDim] = {0}, u[kMaxDim] = {0};
};

// Validate a spec; CCUBA_OK or CCUBA_EINVAL.
int validate_vegas(const VegasSpec &s);
// Iterations the budget allows and the largest n_t among them.
void vegas_budget(const VegasSpec &s, int *iters, long long *nmax);
// Where a batch splits into two halves of about equal evaluations (the
// budget's iterations): the first `cut' integrals and the rest, each holding
// at least one; specs.size() for fewer than two.
size_t batch_cut(const std::vector<VegasSpec> &specs);
// The per-dimension constants of the device Genz code (see genz.h).
void genz_constants(const VegasSpec &s, double p64[2][kParamRow], float p32[2][kParamRow]);

// A slice of a launch's tile list holding the tiles of every job of one
// (precision, Philox blocks per point) class, with the LDS it needs.
struct TileGroup {
  int prec, nb, pow2, full, first, count;
  size_t grid_bytes, lds;
  int hfx;  // 1: the fixed-point LDS histogram instance
};

// Whether the DoSample launch of a class takes the fixed-point LDS histogram:
// unless hist64 asks for the FP64 one, or (FP64 evaluation: 16-byte cells and
// three histogram words per bin) the class's largest d N would not fit the LDS.
bool fixed_hist(int prec, int hist64, long long dN);

// Order the tiles of `jobs' by class, set each job's tile0 to the position of
// its first tile, and describe the classes.  Also returns the refine LDS.
void plan_tile_groups(std::vector<VJob> &jobs, std::vector<int> &tiles,
                      std::vector<TileGroup> &groups, const int hist64[2], size_t *refine_lds);
// One DoSample launch per class; `user' (if given) is the run-time compiled
// kernel of the one class of a caller's device integrand.
int launch_tile_groups(ccuba_ctx *ctx, VegasArgs A, const std::vector<TileGroup> &groups,
                       hipStream_t s, hipFunction_t user = nullptr);
// Inclusive prefixes over jobs of their fold tasks, both levels (see
// FoldArgs); ends holds level 1 then level 2 (2 * njobs entries).
void fold_tasks(const std::vector<VJob> &jobs, std::vector<long long> &ends, long long *total,
                long long *total2);

class VegasEngine {
 public:
  explicit VegasEngine(ccuba_ctx *ctx) : ctx_(ctx) {}
  // Allocate and upload; `single' plans tiles for one large integral.
  int setup(const std::vector<VegasSpec> &specs, bool single, hipStream_t s);
  // One iteration of every unfinished job (async on s).
  int step(hipStream_t s);
  // Iterate until every job is done; replays a captured graph if enabled.
  // run = launch_run then finish_run.
  int run(hipStream_t s);
  // Capture ahead the graphs that launch_run replays when every job runs
  // its whole budget (nothing to do otherwise), so that launch_run then only
  // queues them.
  int prepare_run(hipStream_t s);
  // Launch the iterations: all without waiting when every job runs its
  // whole budget (fixed()), else in chunks with host checks of the states.
  int launch_run(hipStream_t s);
  // Wait for what launch_run queued; the profile-mode timings.
  int finish_run(hipStream_t s);
  // No job can stop before its budget (no epsrel or epsabs).
  bool fixed() const;
  // The same one iteration at a time, calling after(state of job 0) once each
  // iteration is done (a checkpoint); a nonzero return from it stops the run
  // with that status.
  int run_each(hipStream_t s, const std::function<int(const VState &)> &after);
  // Job 0 continues from a saved state, grid and history (T = st.T
  // iterations done); call after setup.
  int load_checkpoint(const VState &st, const double *grid, const double *I, const double *var,
                      hipStream_t s);
  // Job 0's history capacity (iterations the budget allows).
  int hist_cap() const { return hjobs_.empty() ? 0 : hjobs_[0].hist_cap; }
  int read_states(std::vector<VState> &out, hipStream_t s);
  int read_history(int job, int n, double *I, double *var, hipStream_t s);
  int read_grid(int job, double *grid, hipStream_t s);
  // The grid and iteration t's estimate and variance of one job, read with
  // one synchronisation (what a checkpoint needs after each iteration).
  int read_step(int job, int t, double *grid, double *I, double *var, hipStream_t s);
  // Raw pieces: set iteration index of job 0, run DoSample only, and sum the
  // group partials into caller buffers.
  int set_iteration(int job, int t, hipStream_t s);
  int load_grid(int job, const double *src, hipMemcpyKind kind, hipStream_t s);
  // the sampling kernels, then the fold (with level2 both levels, into
  // hsum); records `between` (if given) after the sampling kernels
  int dosample_only(hipStream_t s, bool level2 = false, hipEvent_t between = nullptr);
  int collect(double *sums_dev, double *hist_dev, hipStream_t s);
  // One refinement of job 0 from a given histogram and grid.
  int refine_only(const double *hist, const double *grid_in, double *grid_out, hipStream_t s);

  // A caller's device integrand (family USER): its compiled DoSample kernel,
  // set before setup.
  void set_user_kernel(hipFunction_t f) { user_fn_ = f; }

  // Profile mode with a reference event recorded before this engine's work
  // (on its stream or one it waits on): each iteration's sampling interval,
  // in ms after the reference, goes to dosample_intervals() instead of the
  // context's busy time, so that a caller running engines side by side can
  // take the union.
  void set_time_reference(hipEvent_t ref) { ref_ = ref; }
  const std::vector<std::pair<double, double>> &dosample_intervals() const { return ds_iv_; }

  int njobs() const { return (int)specs_.size(); }
  int max_iters() const { return max_iters_; }
  long long evals_per_iteration() const { return evals_iter_; }
  const std::vector<VegasSpec> &specs() const { return specs_; }
  // launch geometry actually used
  int grid_blocks(int prec) const { return nblocks_[prec]; }
  int block() const { return block_[1]; }

 private:
  int launch_iteration(hipStream_t s);
  int flush_timing();
  struct Timed {
    hipEvent_t e0, e1, e2, e3;
    int iter;
  };
  std::vector<Timed> pending_;
  hipEvent_t ref_ = nullptr;
  std::vector<std::pair<double, double>> ds_iv_;
  bool capturing_ = false;
  int iter_launched_ = 0;
  ccuba_ctx *ctx_;
  std::vector<VegasSpec> specs_;
  std::vector<VJob> hjobs_;
  DevBuf<VJob> jobs_;
  DevBuf<VState> state_;
  DevBuf<int> tile_job_;
  DevBuf<double> grids_, p64_, tile_sums_, tile_hist_, group_sums_, group_hist_, iter_I_,
      iter_var_;
  DevBuf<float> p32_;
  DevBuf<long long> fold_end_;
  DevBuf<double> hsum_;
  long long fold_total_ = 0, fold_total2_ = 0;
  VegasArgs args_{};
  int ntiles_ = 0, ngroups_ = 0;
  std::vector<TileGroup> tgroups_;
  int has_prec_[2] = {0, 0};
  int nblocks_[2] = {0, 0}, block_[2] = {256, 256};
  size_t lds_refine_ = 0;
  int hist64_[2] = {0, 0};  // per precision: the FP64 LDS histogram asked for
  hipFunction_t user_fn_ = nullptr;
  int max_iters_ = 0;
  int dmax_ = 1;  // the largest dimension among the jobs (refine launch)
  long long evals_iter_ = 0;
  // instantiated graphs of k consecutive iterations
  struct ChunkGraph {
    int k;
    hipGraphExec_t exec;
  };
  std::vector<ChunkGraph> graphs_;
  std::vector<long long> graph_sig_;  // the launch arguments the graphs hold
  static constexpr int kMaxGraphIters = 32;
  int graph_for(int k, hipStream_t s, hipGraphExec_t *out);

 public:
  ~VegasEngine();
};

}  // namespace ccuba
