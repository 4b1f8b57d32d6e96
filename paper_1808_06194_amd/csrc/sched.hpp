// Host-side scheduling policy of the matching server: device-memory arena,
// admission by free memory, continuous batching in arrival order, and
// least-recently-used eviction of resident CFOG volumes.  Pure C++ with no
// HIP calls: the server (server.hip) executes the batches it forms, and a host
// test drives it with a simulated executor.
//
// Model:
//   * The server owns one device region of `budget` bytes.  Every resident
//     image pair (CFOG volumes + FP64 SATs of both images and the scratch of
//     their extraction) occupies one block of it.  Request buffers live in
//     fixed per-slot staging sized by the per-batch limits.
//   * Requests are admitted strictly in arrival order.  A request is admitted
//     when its pair is resident or a block for the pair can be made free.
//     Making room evicts resident pairs that no admitted request uses, least
//     recently used first.  When the oldest waiting request cannot be
//     admitted, nothing behind it is (no starvation).
//   * A batch is the run of consecutive admitted requests that fits the
//     per-batch limits (control points, surface values, requests).
//   * A pair that became resident while forming a batch is listed in
//     Batch::extract: its volumes must be computed before the batch runs.
//   * complete() releases a batch's pair references.
#pragma once
#include <stddef.h>
#include <stdint.h>
#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

namespace cfog {
namespace serve {

constexpr size_t kGranule = 256;

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit allocator of offsets in [0, size).  Blocks are multiples of
// kGranule; freed neighbours coalesce.
class Arena {
 public:
  explicit Arena(size_t size = 0) { reset(size); }

  void reset(size_t size) {
    size_ = size / kGranule * kGranule;
    free_.clear();
    live_.clear();
    if (size_) free_[0] = size_;
    used_ = peak_ = 0;
  }

  bool alloc(size_t bytes, size_t* off) {
    const size_t n = round_up(std::max<size_t>(bytes, 1), kGranule);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t o = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[o + n] = len - n;
      live_[o] = n;
      used_ += n;
      peak_ = std::max(peak_, used_);
      *off = o;
      return true;
    }
    return false;
  }

  // Returns false for an offset that is not a live block.
  bool release(size_t off) {
    auto lt = live_.find(off);
    if (lt == live_.end()) return false;
    size_t o = off, n = lt->second;
    live_.erase(lt);
    used_ -= n;
    auto next = free_.lower_bound(o);
    if (next != free_.end() && next->first == o + n) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == o) {
        o = prev->first;
        n += prev->second;
        free_.erase(prev);
      }
    }
    free_[o] = n;
    return true;
  }

  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t blocks() const { return live_.size(); }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
  std::unordered_map<size_t, size_t> live_;
  size_t size_ = 0, used_ = 0, peak_ = 0;
};

struct PairState {
  size_t bytes = 0;          // arena bytes of the pair's volumes + SATs
  bool resident = false;     // holds an arena block
  size_t off = 0;
  int refs = 0;              // admitted, not completed requests using the pair
  uint64_t last_use = 0;
};

struct Request {
  int64_t id = 0;
  int pair = 0;
  int n_cps = 0;
  size_t surf_values = 0;    // surface values staged for the host
};

struct Batch {
  std::vector<Request> reqs;
  std::vector<int> extract;  // pairs to compute before the batch runs
  int n_cps = 0;
  size_t surf_values = 0;
};

struct Limits {
  int max_batch_cps = 8192;
  int max_batch_reqs = 256;
  size_t max_batch_surf = 1 << 22;
};

struct Stats {
  int64_t batches = 0, admitted = 0, completed = 0, evictions = 0, extractions = 0;
  int64_t blocked = 0;       // batch formations stopped by memory
};

class Scheduler {
 public:
  Scheduler(size_t budget, const Limits& lim) : arena_(budget), lim_(lim) {}

  int add_pair(size_t bytes) {
    PairState p;
    p.bytes = bytes;
    pairs_.push_back(p);
    return (int)pairs_.size() - 1;
  }

  // Whether a request can ever be admitted (alone, on an empty arena).
  bool feasible(int pair, int n_cps, size_t surf_values) const {
    if (pair < 0 || pair >= (int)pairs_.size()) return false;
    if (n_cps > lim_.max_batch_cps || surf_values > lim_.max_batch_surf) return false;
    return round_up(pairs_[pair].bytes, kGranule) <= arena_.size();
  }

  void submit(const Request& r) { pending_.push_back(r); }

  // Form the next batch from the oldest waiting requests; false if none can
  // be admitted now.
  bool next_batch(Batch* b) {
    *b = Batch{};
    while (!pending_.empty()) {
      const Request& r = pending_.front();
      if (!b->reqs.empty() && (b->n_cps + r.n_cps > lim_.max_batch_cps ||
                               b->surf_values + r.surf_values > lim_.max_batch_surf ||
                               (int)b->reqs.size() >= lim_.max_batch_reqs))
        break;
      PairState& p = pairs_[r.pair];
      if (!p.resident) {
        size_t off;
        if (!make_room(p.bytes, &off)) {
          ++stats_.blocked;
          break;
        }
        p.resident = true;
        p.off = off;
        b->extract.push_back(r.pair);
        ++stats_.extractions;
      }
      ++p.refs;
      p.last_use = ++clock_;
      b->reqs.push_back(r);
      b->n_cps += r.n_cps;
      b->surf_values += r.surf_values;
      pending_.pop_front();
    }
    if (b->reqs.empty()) return false;
    ++stats_.batches;
    stats_.admitted += (int64_t)b->reqs.size();
    return true;
  }

  // The batch's device work has finished.
  void complete(const Batch& b) {
    for (const Request& a : b.reqs) {
      --pairs_[a.pair].refs;
      ++stats_.completed;
    }
  }

  // Drop a resident pair that no admitted request uses (its volumes were not
  // computed, e.g. the batch that should have computed them failed).
  void forget(int pair) {
    PairState& p = pairs_[pair];
    if (!p.resident || p.refs > 0) return;
    arena_.release(p.off);
    p.resident = false;
  }

  // Remove every waiting request (after a device failure); returns them.
  std::vector<Request> drop_pending() {
    std::vector<Request> out(pending_.begin(), pending_.end());
    pending_.clear();
    return out;
  }

  size_t pending() const { return pending_.size(); }
  const PairState& pair(int i) const { return pairs_[i]; }
  int n_pairs() const { return (int)pairs_.size(); }
  const Arena& arena() const { return arena_; }
  const Stats& stats() const { return stats_; }
  const Limits& limits() const { return lim_; }

 private:
  // Allocate `bytes`, evicting unreferenced resident pairs (least recently
  // used first) until it fits.
  bool make_room(size_t bytes, size_t* off) {
    while (!arena_.alloc(bytes, off)) {
      int victim = -1;
      for (int i = 0; i < (int)pairs_.size(); ++i) {
        const PairState& q = pairs_[i];
        if (!q.resident || q.refs > 0) continue;
        if (victim < 0 || q.last_use < pairs_[victim].last_use) victim = i;
      }
      if (victim < 0) return false;
      PairState& v = pairs_[victim];
      arena_.release(v.off);
      v.resident = false;
      ++stats_.evictions;
    }
    return true;
  }

  Arena arena_;
  Limits lim_;
  std::vector<PairState> pairs_;
  std::deque<Request> pending_;
  Stats stats_;
  uint64_t clock_ = 0;
};

}  // namespace serve
}  // namespace cfog
