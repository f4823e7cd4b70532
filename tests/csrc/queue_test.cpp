// Host-only checks of the serving engine's request queue (arrival-order packing
// by grid size, pose and atom limits, cancellation).  Built with g++ by
// tests/test_engine_queue_cpu.py; prints "OK" and exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "cf_queue.h"

struct Req {
  int id, n_poses, G;
  long long na;
  int64_t atoms() const { return na; }
};

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAILED line %d: %s\n", __LINE__, #c);           \
      ++failures;                                                  \
    }                                                              \
  } while (0)

static std::vector<int> ids(const std::vector<Req *> &v) {
  std::vector<int> o;
  for (auto *r : v) o.push_back(r->id);
  return o;
}

int main() {
  Req a{0, 10, 48, 6000}, b{1, 5, 64, 3000}, c{2, 20, 48, 12000}, d{3, 300, 48, 200000}, e{4, 60, 48, 30000},
      f{5, 1, 48, 100};
  {
    cf::RequestQueue<Req> q;
    for (Req *r : {&a, &b, &c, &d, &e, &f}) q.push(r);
    CHECK(q.queued_poses() == 396);
    // head's grid size (48); d does not fit 100 poses; e fits after a and c (90)
    // but f then still fits (91); b (G = 64) stays
    auto t = q.take_batch(100, 1 << 20);
    CHECK((ids(t) == std::vector<int>{0, 2, 4, 5}));
    CHECK(q.size() == 2);
    // the next batch starts at the oldest remaining request (b, G = 64)
    t = q.take_batch(100, 1 << 20);
    CHECK((ids(t) == std::vector<int>{1}));
    t = q.take_batch(512, 1 << 20);
    CHECK((ids(t) == std::vector<int>{3}));
    CHECK(q.empty() && q.take_batch(512, 1 << 20).empty());
  }
  {
    // atom limit: a (6000) + c (12000) exceed 15000, f still fits
    cf::RequestQueue<Req> q;
    for (Req *r : {&a, &c, &f}) q.push(r);
    auto t = q.take_batch(512, 15000);
    CHECK((ids(t) == std::vector<int>{0, 5}));
    CHECK((ids(q.take_batch(512, 15000)) == std::vector<int>{2}));
  }
  {
    // cancellation: a queued request leaves the queue exactly once and is never
    // packed; a request already packed cannot be cancelled
    cf::RequestQueue<Req> q;
    for (Req *r : {&a, &b, &c, &e}) q.push(r);
    CHECK(q.cancel(&c));
    CHECK(!q.cancel(&c));
    CHECK(q.queued_poses() == 75);
    auto t = q.take_batch(512, 1 << 20);
    CHECK((ids(t) == std::vector<int>{0, 4}));
    CHECK(!q.cancel(&a));
    CHECK(q.cancel(&b));   // the G = 64 head, cancelled before its batch
    CHECK(q.empty() && q.queued_poses() == 0);
    // cancelling the head moves the next batch to the following request's grid size
    for (Req *r : {&b, &a, &f}) q.push(r);
    CHECK(q.cancel(&b));
    CHECK((ids(q.take_batch(512, 1 << 20)) == std::vector<int>{0, 5}));
  }
  if (failures) return 1;
  std::printf("OK\n");
  return 0;
}
