// Rounds of work from a changing set of participants (the server's shared
// collision launches).  A joined participant hands in one item at a time and
// waits for it; once every joined participant has an item in (or has left),
// the thread that completes the set runs the round: all pending items at once,
// outside the lock.  Every item of the round then gets the round's outcome.
//
// A participant has at most one item in at a time, so a round holds exactly
// one item of each participant joined when it starts, and rounds never
// overlap (a new round needs every joined participant to hand in again, and
// the members of the running round are still waiting for it).  stop() sends
// back the items no round has taken yet; an item a round has taken is waited
// for to the end, since the round holds it.  No GPU types: the logic is
// tested on the CPU.
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

namespace blr {

template <class Item>
class Rendezvous {
 public:
  // Outcome of a round, handed to every item in it (code 0: success).
  struct Outcome {
    int code = 0;
    std::string err;
  };
  // Runs one round's items (called without the lock held).
  using Runner = std::function<Outcome(const std::vector<Item*>&)>;

  explicit Rendezvous(Runner run) : run_(std::move(run)) {}

  void join() {
    std::lock_guard<std::mutex> lk(mu_);
    ++active_;
  }

  void leave() {
    std::unique_lock<std::mutex> lk(mu_);
    --active_;
    if (!stopping_ && !pending_.empty() && (int)pending_.size() >= active_) run_round(lk);
  }

  void stop() {
    std::lock_guard<std::mutex> lk(mu_);
    stopping_ = true;
    cv_.notify_all();
  }

  // Hands `item` in and waits for its round.  Returns false (and leaves *out
  // untouched) when the rendezvous stopped before a round took the item.
  bool submit(Item* item, Outcome* out) {
    std::unique_lock<std::mutex> lk(mu_);
    if (stopping_) return false;
    Slot s{item};
    pending_.push_back(&s);
    if ((int)pending_.size() >= active_) run_round(lk);
    auto queued = [&] { return std::find(pending_.begin(), pending_.end(), &s) != pending_.end(); };
    cv_.wait(lk, [&] { return s.done || (stopping_ && queued()); });
    if (!s.done) {
      pending_.erase(std::remove(pending_.begin(), pending_.end(), &s), pending_.end());
      return false;
    }
    *out = s.outcome;
    return true;
  }

  int64_t rounds() const {
    std::lock_guard<std::mutex> lk(mu_);
    return rounds_;
  }
  int64_t items() const {
    std::lock_guard<std::mutex> lk(mu_);
    return items_;
  }

 private:
  struct Slot {
    Item* item;
    bool done = false;
    Outcome outcome;
  };

  // mu_ held on entry and on return; released while the round runs.
  void run_round(std::unique_lock<std::mutex>& lk) {
    std::vector<Slot*> batch;
    batch.swap(pending_);
    ++rounds_;
    items_ += (int64_t)batch.size();
    lk.unlock();
    std::vector<Item*> its;
    its.reserve(batch.size());
    for (Slot* s : batch) its.push_back(s->item);
    Outcome o;
    {
      // rounds are serial by construction; the lock keeps them so
      std::lock_guard<std::mutex> lg(run_mu_);
      try {
        o = run_(its);
      } catch (const std::exception& e) {
        o.code = -1;
        o.err = e.what();
      }
    }
    lk.lock();
    for (Slot* s : batch) {
      s->done = true;
      s->outcome = o;
    }
    cv_.notify_all();
  }

  Runner run_;
  mutable std::mutex mu_;
  std::mutex run_mu_;
  std::condition_variable cv_;
  int active_ = 0;
  bool stopping_ = false;
  std::vector<Slot*> pending_;
  int64_t rounds_ = 0, items_ = 0;
};

}  // namespace blr
