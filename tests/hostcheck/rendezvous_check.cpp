// CPU stress test of blr::Rendezvous (the server's shared collision rounds):
// participants join at different times, hand in items with random delays,
// and leave after different numbers of items.  Checks that every item runs
// exactly once, that no round holds two items of one participant or more
// items than participants joined, that with a fixed set of participants every
// round holds one item of each, that a failed round's outcome reaches every
// item in it, and that stop() releases the participants still waiting.
// Built with ThreadSanitizer.  Prints "ok" on success; any failure aborts.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <stdexcept>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "rendezvous.hpp"

namespace {

struct Item {
  int who;
  int seq;
};

#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      std::abort();                                                      \
    }                                                                    \
  } while (0)

void stress(int parts, int max_items, unsigned seed) {
  std::mutex log_mu;
  std::map<std::pair<int, int>, int> runs;  // (who, seq) -> times run
  std::atomic<int> joined{0};
  std::vector<std::set<int>> round_members;
  blr::Rendezvous<Item>* rvp = nullptr;
  blr::Rendezvous<Item> rv([&](const std::vector<Item*>& items) {
    std::set<int> who;
    std::lock_guard<std::mutex> lk(log_mu);
    for (Item* it : items) {
      CHECK(who.insert(it->who).second);  // one item per participant per round
      ++runs[{it->who, it->seq}];
    }
    // never more items than joined participants (one may have joined after
    // the round started, so not always equal)
    CHECK((int)items.size() <= joined.load());
    round_members.push_back(who);
    blr::Rendezvous<Item>::Outcome o;
    o.code = (int)items.size();
    return o;
  });
  rvp = &rv;
  std::vector<std::thread> th;
  std::vector<int> counts(parts);
  std::mt19937 rng(seed);
  for (int p = 0; p < parts; ++p) counts[p] = 1 + (int)(rng() % max_items);
  for (int p = 0; p < parts; ++p) {
    th.emplace_back([&, p] {
      std::mt19937 r(seed * 131 + p);
      std::this_thread::sleep_for(std::chrono::microseconds(r() % 2000));
      {
        // join and count under the log lock, so a round never sees a half-joined participant
        std::lock_guard<std::mutex> lk(log_mu);
        rvp->join();
        joined.fetch_add(1);
      }
      for (int k = 0; k < counts[p]; ++k) {
        std::this_thread::sleep_for(std::chrono::microseconds(r() % 300));
        Item it{p, k};
        blr::Rendezvous<Item>::Outcome o;
        CHECK(rvp->submit(&it, &o));
        CHECK(o.code >= 1);
      }
      {
        std::lock_guard<std::mutex> lk(log_mu);
        joined.fetch_sub(1);
      }
      rvp->leave();
    });
  }
  for (auto& t : th) t.join();
  // every item ran exactly once
  int total = 0;
  for (int p = 0; p < parts; ++p) {
    total += counts[p];
    for (int k = 0; k < counts[p]; ++k) CHECK((runs[{p, k}] == 1));
  }
  CHECK((int)runs.size() == total);
  CHECK(rv.items() == total);
  CHECK(rv.rounds() == (int64_t)round_members.size());
  std::printf("stress parts=%d items=%d rounds=%lld\n", parts, total, (long long)rv.rounds());
}

// All participants join before any item; each hands in k items: every round
// must hold exactly one item of each of them (k rounds of n items).
void fixed_set(int n, int k, unsigned seed) {
  std::mutex mu;
  std::vector<int> sizes;
  blr::Rendezvous<Item> rv([&](const std::vector<Item*>& items) {
    std::set<int> who;
    for (Item* it : items) CHECK(who.insert(it->who).second);
    std::lock_guard<std::mutex> lk(mu);
    sizes.push_back((int)items.size());
    return blr::Rendezvous<Item>::Outcome{};
  });
  for (int p = 0; p < n; ++p) rv.join();
  std::vector<std::thread> th;
  for (int p = 0; p < n; ++p)
    th.emplace_back([&, p] {
      std::mt19937 r(seed * 977 + p);
      for (int j = 0; j < k; ++j) {
        std::this_thread::sleep_for(std::chrono::microseconds(r() % 400));
        Item it{p, j};
        blr::Rendezvous<Item>::Outcome o;
        CHECK(rv.submit(&it, &o));
      }
      rv.leave();
    });
  for (auto& t : th) t.join();
  CHECK((int)sizes.size() == k);
  for (int s : sizes) CHECK(s == n);
  std::printf("fixed set n=%d k=%d ok\n", n, k);
}

void stop_releases_waiters() {
  blr::Rendezvous<Item> rv([](const std::vector<Item*>&) { return blr::Rendezvous<Item>::Outcome{}; });
  rv.join();
  rv.join();  // a second participant that never hands anything in
  std::atomic<int> released{0};
  std::thread t([&] {
    Item it{0, 0};
    blr::Rendezvous<Item>::Outcome o;
    const bool ran = rv.submit(&it, &o);
    CHECK(!ran);  // its round never started
    released.fetch_add(1);
  });
  std::this_thread::sleep_for(std::chrono::milliseconds(20));
  CHECK(released.load() == 0);  // still waiting for the second participant
  rv.stop();
  t.join();
  CHECK(released.load() == 1);
  Item late{1, 0};
  blr::Rendezvous<Item>::Outcome o;
  CHECK(!rv.submit(&late, &o));  // refused once stopped
  std::printf("stop ok\n");
}

void errors_reach_every_item() {
  blr::Rendezvous<Item> rv([](const std::vector<Item*>&) -> blr::Rendezvous<Item>::Outcome {
    throw std::runtime_error("round failed");
  });
  const int parts = 4;
  std::vector<std::thread> th;
  std::atomic<int> failed{0};
  for (int p = 0; p < parts; ++p) rv.join();
  for (int p = 0; p < parts; ++p)
    th.emplace_back([&, p] {
      Item it{p, 0};
      blr::Rendezvous<Item>::Outcome o;
      CHECK(rv.submit(&it, &o));
      if (o.code != 0 && o.err == "round failed") failed.fetch_add(1);
      rv.leave();
    });
  for (auto& t : th) t.join();
  CHECK(failed.load() == parts);
  CHECK(rv.rounds() == 1);
  std::printf("errors ok\n");
}

}  // namespace

int main() {
  stop_releases_waiters();
  errors_reach_every_item();
  fixed_set(1, 20, 1);
  fixed_set(5, 30, 2);
  fixed_set(16, 25, 3);
  for (unsigned seed = 1; seed <= 6; ++seed) stress(2 + (int)seed * 2, 40, seed);
  std::printf("ok\n");
  return 0;
}
