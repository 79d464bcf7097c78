// serve.cpp -- the serving loop (see serve.h).
#include "serve.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace ccuba {

struct Server::Req {
  unsigned long long ticket = 0;
  ccuba_job job{};
  double a[kMaxDim] = {0}, u[kMaxDim] = {0};
  double t_submit = 0;
  int slot = -1;
  bool running = false;
  // Vegas
  VegasSpec vs;
  VJob hj{};
  bool vdone = false;
  DevBuf<double> grid, tsums, thist, gsums, ghist, hsum, iters, p64;
  DevBuf<float> p32;
  // host sources of the activation's uploads, alive while the copies are in
  // flight (the request outlives them)
  double a64[2][kParamRow];
  float a32[2][kParamRow];
  VState st0{};
  // Cuhre
  std::unique_ptr<CuhreRun> cuhre;
  bool cpending = false;
};

Server::Server(ccuba_ctx *ctx) : ctx_(ctx) {}

Server::~Server() {
  {
    std::lock_guard<std::mutex> g(qmu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (th_.joinable()) th_.join();
  std::lock_guard<std::mutex> g(ctx_->lock);
  (void)hipStreamSynchronize(ctx_->stream);
  for (auto &r : active_) release(*r);
  active_.clear();
  if (tot_host_) (void)hipHostFree(tot_host_);
}

int Server::submit(const ccuba_job &job, unsigned long long *ticket) {
  if (!ticket || (job.method != 0 && job.method != 1) || !job.f.a || !job.f.u ||
      job.ndim < 1 || job.ndim > kMaxDim)
    return CCUBA_EINVAL;
  auto r = std::make_unique<Req>();
  r->job = job;
  for (int j = 0; j < job.ndim; ++j) {
    r->a[j] = job.f.a[j];
    r->u[j] = job.f.u[j];
  }
  r->job.f.a = r->a;
  r->job.f.u = r->u;
  r->t_submit = ctx_->now();
  std::lock_guard<std::mutex> g(qmu_);
  if (!started_) {
    started_ = true;
    th_ = std::thread([this] { loop(); });
  }
  r->ticket = next_ticket_++;
  *ticket = r->ticket;
  live_.insert(r->ticket);
  queue_.push_back(std::move(r));
  ++outstanding_;
  cv_.notify_all();
  return CCUBA_OK;
}

int Server::poll(unsigned long long ticket, ccuba_result *out) {
  if (!out) return CCUBA_EINVAL;
  std::lock_guard<std::mutex> g(qmu_);
  auto it = done_.find(ticket);
  if (it != done_.end()) {
    *out = it->second;
    done_.erase(it);
    return 0;
  }
  return live_.count(ticket) ? 1 : CCUBA_ENOENT;
}

int Server::drain() {
  std::unique_lock<std::mutex> g(qmu_);
  cv_.wait(g, [this] { return outstanding_ == 0 || stop_; });
  return CCUBA_OK;
}

void Server::finish(Req &r, int status) {
  ccuba_result res{};
  res.status = status;
  res.t_submit = r.t_submit;
  res.t_done = ctx_->now();
  res.fail = 1;
  if (status == CCUBA_OK) {
    if (r.job.method == 0) {
      // filled by the caller from the device state
    } else if (r.cuhre) {
      res.neval = r.cuhre->neval();
      res.nregions = (int)std::min<long long>(r.cuhre->nregions(), 0x7fffffff);
      res.fail = r.cuhre->fail();
      res.integral = r.cuhre->integral();
      res.error = r.cuhre->error();
      res.prob = 0.0;
    }
  }
  std::lock_guard<std::mutex> g(qmu_);
  done_[r.ticket] = res;
  live_.erase(r.ticket);
  --outstanding_;
  cv_.notify_all();
}

void Server::release(Req &r) {
  r.grid.release();
  r.tsums.release();
  r.thist.release();
  r.gsums.release();
  r.ghist.release();
  r.hsum.release();
  r.iters.release();
  r.p64.release();
  r.p32.release();
  r.cuhre.reset();
  if (r.slot >= 0) free_slots_.push_back(r.slot);
  r.slot = -1;
}

int Server::activate(Req &r) {
  hipStream_t s = ctx_->stream;
  const ccuba_job &jb = r.job;
  if (jb.method == 1) {
    CuhreSpec sp;
    sp.ndim = jb.ndim;
    sp.family = jb.f.family;
    for (int j = 0; j < jb.ndim; ++j) {
      sp.a[j] = r.a[j];
      sp.u[j] = r.u[j];
    }
    sp.epsrel = jb.epsrel;
    sp.epsabs = jb.epsabs;
    sp.mineval = jb.mineval;
    sp.maxeval = jb.maxeval;
    sp.batch = jb.max_regions_per_batch > 0 ? jb.max_regions_per_batch : 100000;
    if (validate_cuhre(sp) || (jb.flags & CCUBA_PRECISION_MASK) != CCUBA_FP64)
      return CCUBA_EINVAL;
    if (free_slots_.empty()) return CCUBA_ENOMEM;
    r.slot = free_slots_.back();
    free_slots_.pop_back();
    r.cuhre = std::make_unique<CuhreRun>(ctx_);
    r.cuhre->set_mapped_totals(tot_host_ + 2 * r.slot, tot_dev_ + 2 * r.slot);
    int rc = r.cuhre->start(sp, s);
    if (rc) {
      r.cuhre.reset();
      return rc;
    }
    r.cpending = true;  // the root's rule was launched; totals next
    return r.cuhre->launch_totals(s);
  }
  VegasSpec &sp = r.vs;
  const int prec = jb.flags & CCUBA_PRECISION_MASK;
  if (prec != CCUBA_FP64 && prec != CCUBA_FP32_EVAL) return CCUBA_EINVAL;
  sp.ndim = jb.ndim;
  sp.nbins = jb.nbins > 0 ? jb.nbins : 128;
  sp.family = jb.f.family;
  sp.prec = prec == CCUBA_FP64 ? FP64 : FP32;
  sp.flags = jb.flags & CCUBA_FREEZE_GRID;
  sp.seed = jb.seed;
  sp.sid = jb.stream_id;
  sp.nstart = jb.nstart;
  sp.nincrease = jb.nincrease;
  sp.mineval = jb.mineval;
  sp.maxeval = jb.maxeval;
  sp.epsrel = jb.epsrel;
  sp.epsabs = jb.epsabs;
  for (int j = 0; j < jb.ndim; ++j) {
    sp.a[j] = r.a[j];
    sp.u[j] = r.u[j];
  }
  if (validate_vegas(sp)) return CCUBA_EINVAL;
  int iters;
  long long nmax;
  vegas_budget(sp, &iters, &nmax);
  const int bs = ctx_->tune[sp.prec].block;
  auto round_up = [](long long v, long long m) { return (v + m - 1) / m * m; };
  const long long P = std::max(round_up(ctx_->tune[sp.prec].min_tile, bs),
                               round_up((nmax + 63) / 64, bs));
  const int nt = (int)std::max<long long>(1, (nmax + P - 1) / P), ng = ngroups_of(nt);
  const long long dN = (long long)sp.ndim * sp.nbins, row = (long long)sp.ndim * (sp.nbins + 1);
  const int cap = std::max(1, iters);
  int rc;
  if ((rc = r.grid.alloc(ctx_, row)) || (rc = r.tsums.alloc(ctx_, 2 * nt)) ||
      (rc = r.thist.alloc(ctx_, nt * dN)) || (rc = r.gsums.alloc(ctx_, 2 * ng)) ||
      (rc = r.ghist.alloc(ctx_, ng * dN)) || (rc = r.hsum.alloc(ctx_, 2 + dN)) ||
      (rc = r.iters.alloc(ctx_, 2 * (size_t)cap)) ||
      (rc = r.p64.alloc(ctx_, 2 * kParamRow)) || (rc = r.p32.alloc(ctx_, 2 * kParamRow)))
    return rc;
  if (free_slots_.empty()) return CCUBA_ENOMEM;
  r.slot = free_slots_.back();
  free_slots_.pop_back();
  VJob &J = r.hj;
  J = VJob{};
  J.ndim = sp.ndim;
  J.nbins = sp.nbins;
  J.family = sp.family;
  J.prec = sp.prec;
  J.flags = sp.flags;
  J.key0 = (uint32_t)(sp.seed & 0xffffffffull);
  J.key1 = (uint32_t)(sp.seed >> 32);
  J.sid = sp.sid;
  J.nstart = sp.nstart;
  J.nincrease = sp.nincrease;
  J.mineval = sp.mineval;
  J.maxeval = sp.maxeval;
  J.epsrel = sp.epsrel;
  J.epsabs = sp.epsabs;
  J.ntiles = nt;
  J.tile_pts = P;
  J.hist_cap = cap;
  J.state = states_.p + r.slot;
  J.snap = states_.p + states_.n / 2 + r.slot;
  J.grid = r.grid.p;
  J.tsums = r.tsums.p;
  J.thist = r.thist.p;
  J.gsums = r.gsums.p;
  J.ghist = r.ghist.p;
  J.hsum = r.hsum.p;
  J.iter_I = r.iters.p;
  J.iter_var = r.iters.p + cap;
  J.p64 = r.p64.p;
  J.p32 = r.p32.p;
  genz_constants(sp, r.a64, r.a32);
  r.st0 = VState{};
  if (iters == 0) {
    r.st0.done = 1;
    r.st0.fail = 1;
  }
  r.vdone = iters == 0;
  (void)row;
  CCUBA_HIP(launch_init_grid(J.grid, sp.ndim, sp.nbins, s));
  CCUBA_HIP(hipMemcpyAsync(r.p64.p, r.a64, sizeof(r.a64), hipMemcpyHostToDevice, s));
  CCUBA_HIP(hipMemcpyAsync(r.p32.p, r.a32, sizeof(r.a32), hipMemcpyHostToDevice, s));
  CCUBA_HIP(hipMemcpyAsync(J.state, &r.st0, sizeof(r.st0), hipMemcpyHostToDevice, s));
  return CCUBA_OK;
}

int Server::admit_locked(std::unique_lock<std::mutex> &q) {
  while (!queue_.empty() && (int)active_.size() < ctx_->serve_slots) {
    std::unique_ptr<Req> r = std::move(queue_.front());
    queue_.pop_front();
    q.unlock();
    const int rc = activate(*r);
    q.lock();
    if (rc == CCUBA_OK) {
      r->running = true;
      active_.push_back(std::move(r));
      continue;
    }
    release(*r);
    if (rc == CCUBA_ENOMEM && !active_.empty()) {
      queue_.push_front(std::move(r));  // wait for memory to free up
      break;
    }
    q.unlock();
    finish(*r, rc);
    q.lock();
  }
  return CCUBA_OK;
}

int Server::tick() {
  std::lock_guard<std::mutex> dev(ctx_->lock);
  hipStream_t s = ctx_->stream;
  if (hipSetDevice(ctx_->device) != hipSuccess) return CCUBA_EHIP;
  int rc;
  if (!tables_ready_) {
    const int slots = ctx_->serve_slots;
    // (the states, then their snapshots for the refine kernel)
    if ((rc = states_.alloc(ctx_, 2 * slots)) || (rc = jobs_.alloc(ctx_, slots)) ||
        (rc = w7_.alloc(ctx_, 17 * 5)) || (rc = w5_.alloc(ctx_, 17 * 5)))
      return rc;
    for (int q = slots - 1; q >= 0; --q) free_slots_.push_back(q);
    CCUBA_HIP(hipHostMalloc((void **)&tot_host_, 2 * sizeof(double) * slots, 0));
    CCUBA_HIP(hipHostGetDevicePointer((void **)&tot_dev_, tot_host_, 0));
    const GMTables &T = gm_tables();
    CCUBA_HIP(hipMemcpy(w7_.p, T.w7, sizeof(T.w7), hipMemcpyHostToDevice));
    CCUBA_HIP(hipMemcpy(w5_.p, T.w5, sizeof(T.w5), hipMemcpyHostToDevice));
    tables_ready_ = true;
  }
  {
    std::unique_lock<std::mutex> q(qmu_);
    const size_t before = active_.size();
    admit_locked(q);
    // newly admitted requests' uploads and first launches (a Cuhre root's
    // totals among them) complete before this tick reads them
    if (active_.size() != before) CCUBA_HIP(hipStreamSynchronize(s));
  }
  if (active_.empty()) return CCUBA_OK;
  ++ticks_;
  // Cuhre: the totals launched last tick decide each request's next step
  std::vector<CSeg> segs;
  std::vector<Req *> stepping;
  for (auto &r : active_) {
    if (!r->cuhre || !r->cpending) continue;
    if ((rc = r->cuhre->read_totals(s))) return rc;
    r->cpending = false;
    rc = r->cuhre->plan_and_split(s);
    if (rc < 0) return rc;
    if (rc == 1) {
      segs.push_back(r->cuhre->pending_segment());
      stepping.push_back(r.get());
    }
  }
  // Vegas: one DoSample per (precision, dimension class) over every running
  // request, one refine over all of them
  std::vector<VJob> table;
  std::vector<long long> ends;  // host tables live until the tick's sync
  std::vector<int> tiles;
  std::vector<TileGroup> groups;
  for (auto &r : active_)
    if (r->job.method == 0 && !r->vdone) table.push_back(r->hj);
  if (!table.empty()) {
    size_t refb = 0;
    const int h64[2] = {ctx_->tune[0].hist64, ctx_->tune[1].hist64};
    plan_tile_groups(table, tiles, groups, h64, &refb);
    if (jobs_.n < table.size() && (rc = jobs_.alloc(ctx_, table.size() * 2))) return rc;
    if (tiles_.n < tiles.size() && (rc = tiles_.alloc(ctx_, tiles.size() * 2))) return rc;
    CCUBA_HIP(hipMemcpyAsync(jobs_.p, table.data(), table.size() * sizeof(VJob),
                             hipMemcpyHostToDevice, s));
    CCUBA_HIP(hipMemcpyAsync(tiles_.p, tiles.data(), tiles.size() * sizeof(int),
                             hipMemcpyHostToDevice, s));
    // the host tables above must outlive the copies: the tick syncs before
    // they go out of scope
    VegasArgs A{};
    A.jobs = jobs_.p;
    A.tile_job = tiles_.p;
    A.njobs = (int)table.size();
    if ((rc = launch_tile_groups(ctx_, A, groups, s))) return rc;
    long long ftot = 0, ftot2 = 0;
    fold_tasks(table, ends, &ftot, &ftot2);
    if (fold_end_.n < ends.size() && (rc = fold_end_.alloc(ctx_, ends.size() * 2))) return rc;
    CCUBA_HIP(hipMemcpyAsync(fold_end_.p, ends.data(), ends.size() * sizeof(long long),
                             hipMemcpyHostToDevice, s));
    FoldArgs F{jobs_.p, fold_end_.p, (int)table.size(), ftot, fold_end_.p + table.size(), ftot2};
    CCUBA_HIP(launch_fold(F, false, s));
    int dmax = 1;
    for (const VJob &J : table) dmax = std::max(dmax, J.ndim);
    CCUBA_HIP(launch_refine(A, (int)table.size(), dmax, s));
  }
  // Cuhre: one rule launch over the children of every stepping request
  if (!segs.empty()) {
    if ((rc = launch_rule_segments(ctx_, segs.data(), (int)segs.size(), segs_, seg_end_, w7_.p,
                                   w5_.p, s)))
      return rc;
    for (Req *r : stepping) {
      r->cuhre->commit_pending();
      if ((rc = r->cuhre->launch_totals(s))) return rc;
      r->cpending = true;
    }
  }
  CCUBA_HIP(hipStreamSynchronize(s));
  // retire finished requests
  std::vector<VState> st;
  if (!table.empty()) {
    st.resize(states_.n / 2);  // (the states; their snapshots follow)
    CCUBA_HIP(hipMemcpy(st.data(), states_.p, st.size() * sizeof(VState), hipMemcpyDeviceToHost));
  }
  std::vector<std::unique_ptr<Req>> keep;
  for (auto &r : active_) {
    bool fin = false;
    ccuba_result res{};
    if (r->job.method == 0) {
      const VState &x = st.empty() ? VState{} : st[r->slot];
      if (r->vdone || (!st.empty() && x.done)) {
        fin = true;
        VState v = x;
        if (r->vdone && st.empty()) {
          CCUBA_HIP(hipMemcpy(&v, r->hj.state, sizeof(VState), hipMemcpyDeviceToHost));
        }
        res.neval = v.neval;
        res.fail = v.fail;
        res.integral = v.integral;
        res.error = v.error;
        res.prob = v.prob;
      }
    } else if (r->cuhre && r->cuhre->done()) {
      fin = true;
    }
    if (!fin) {
      keep.push_back(std::move(r));
      continue;
    }
    if (r->job.method == 0) {
      res.status = CCUBA_OK;
      res.t_submit = r->t_submit;
      res.t_done = ctx_->now();
      release(*r);
      std::lock_guard<std::mutex> g(qmu_);
      done_[r->ticket] = res;
      live_.erase(r->ticket);
      --outstanding_;
      cv_.notify_all();
    } else {
      finish(*r, CCUBA_OK);
      release(*r);
    }
  }
  active_.swap(keep);
  return CCUBA_OK;
}

void Server::loop() {
  for (;;) {
    {
      std::unique_lock<std::mutex> g(qmu_);
      cv_.wait(g, [this] { return stop_ || !queue_.empty() || outstanding_ > 0; });
      if (stop_) return;
    }
    const int rc = tick();
    if (rc != CCUBA_OK) {
      // a device error fails every request in flight
      std::vector<std::unique_ptr<Req>> all;
      {
        std::lock_guard<std::mutex> dev(ctx_->lock);
        for (auto &r : active_) all.push_back(std::move(r));
        active_.clear();
      }
      {
        std::lock_guard<std::mutex> g(qmu_);
        while (!queue_.empty()) {
          all.push_back(std::move(queue_.front()));
          queue_.pop_front();
        }
      }
      for (auto &r : all) {
        finish(*r, rc);
        std::lock_guard<std::mutex> dev(ctx_->lock);
        release(*r);
      }
    }
    std::unique_lock<std::mutex> g(qmu_);
    if (active_.empty() && queue_.empty() && !stop_)
      cv_.wait_for(g, std::chrono::milliseconds(1));
  }
}

}  // namespace ccuba
