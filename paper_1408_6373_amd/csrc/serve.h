// serve.h -- the serving loop: continuous batching of Vegas and Cuhre
// requests on one device.
//
// A background thread admits queued requests while request slots and the
// context's HBM budget allow, keeps every admitted request's state resident
// on the device (Vegas grids, partial sums and iteration history; Cuhre
// region heaps), and advances all of them together, one tick at a time:
//   * one DoSample launch (per precision) over the tiles of every running
//     Vegas request, then one refine launch over all of them;
//   * the region step (select + split) of every running Cuhre request, then
//     one rule launch over the new children of all of them, then totals.
// A request that arrives while others run joins at the next tick, so its
// work overlaps theirs in the same launches.  Each request computes exactly
// what it computes alone (same points, same subdivisions); only the order of
// floating-point sums inside a launch can differ.
#pragma once
#include <condition_variable>
#include <deque>
#include <map>
#include <set>
#include <memory>
#include <thread>
#include <vector>

#include "context.h"
#include "cuhre_engine.h"
#include "vegas.h"
#include "vegas_engine.h"

namespace ccuba {

class Server {
 public:
  explicit Server(ccuba_ctx *ctx);
  ~Server();
  int submit(const ccuba_job &job, unsigned long long *ticket);
  int poll(unsigned long long ticket, ccuba_result *out);
  int drain();
  // counters since the server started
  long long ticks() const { return ticks_; }

 private:
  struct Req;
  void loop();
  int tick();
  int admit_locked(std::unique_lock<std::mutex> &q);
  int activate(Req &r);
  void finish(Req &r, int status);
  void release(Req &r);

  ccuba_ctx *ctx_;
  std::mutex qmu_;
  std::condition_variable cv_;
  std::thread th_;
  bool started_ = false, stop_ = false;
  unsigned long long next_ticket_ = 1;
  std::deque<std::unique_ptr<Req>> queue_;
  std::vector<std::unique_ptr<Req>> active_;
  std::map<unsigned long long, ccuba_result> done_;
  std::set<unsigned long long> live_;  // submitted, not yet finished
  long long outstanding_ = 0;
  long long ticks_ = 0;
  // device tables shared by all requests
  DevBuf<VState> states_;
  std::vector<int> free_slots_;
  DevBuf<VJob> jobs_;
  DevBuf<int> tiles_;
  DevBuf<long long> fold_end_;
  DevBuf<CSeg> segs_;
  DevBuf<long long> seg_end_;
  DevBuf<double> w7_, w5_;
  // per slot, the Cuhre totals in pinned host memory the device writes to
  double *tot_host_ = nullptr, *tot_dev_ = nullptr;
  bool tables_ready_ = false;
};

}  // namespace ccuba
