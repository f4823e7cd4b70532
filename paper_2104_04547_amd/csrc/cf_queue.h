// Request queue of the serving engine (host only, no HIP): arrival-order
// admission of queued requests into batches and cancellation of queued requests.
//
// A batch takes the oldest request's grid size and then, in arrival order, every
// queued request of that grid size that still fits the batch's pose and atom
// limits; requests that do not fit stay queued in their order.  A request leaves
// the queue either in a batch or by cancellation, never both.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <deque>
#include <vector>

namespace cf {

// R provides: int n_poses, int G, int64_t atoms() const.
template <class R>
class RequestQueue {
 public:
  void push(R *r) { q_.push_back(r); }
  bool empty() const { return q_.empty(); }
  size_t size() const { return q_.size(); }

  // Removes and returns the requests of the next batch (empty if none are queued).
  std::vector<R *> take_batch(int max_poses, int64_t max_atoms) {
    std::vector<R *> take;
    if (q_.empty()) return take;
    const int G = q_.front()->G;
    int np = 0;
    int64_t na = 0;
    for (auto it = q_.begin(); it != q_.end();) {
      R *r = *it;
      const int64_t ra = r->atoms();
      if (r->G == G && np + r->n_poses <= max_poses && na + ra <= max_atoms) {
        take.push_back(r);
        np += r->n_poses;
        na += ra;
        it = q_.erase(it);
      } else {
        ++it;
      }
    }
    return take;
  }

  // Removes r if it is still queued; false if it has already left the queue.
  bool cancel(R *r) {
    auto it = std::find(q_.begin(), q_.end(), r);
    if (it == q_.end()) return false;
    q_.erase(it);
    return true;
  }

  int64_t queued_poses() const {
    int64_t n = 0;
    for (const R *r : q_) n += r->n_poses;
    return n;
  }

 private:
  std::deque<R *> q_;
};

}  // namespace cf
