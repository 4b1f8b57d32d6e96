// Host simulation of the serving scheduler (sched.hpp) with a fake executor:
// random pair sizes, arrivals and batch durations; checks the invariants the
// server relies on after every step.
#include <stdio.h>
#include <stdlib.h>
#include <algorithm>
#include <map>
#include <random>
#include <set>
#include <vector>
#include "sched.hpp"

using namespace cfog::serve;

static int g_fail = 0;
#define CHECK(c, ...)                                     \
  do {                                                    \
    if (!(c)) {                                           \
      printf("FAIL %s:%d: %s  ", __FILE__, __LINE__, #c); \
      printf(__VA_ARGS__);                                \
      printf("\n");                                       \
      ++g_fail;                                           \
      return;                                             \
    }                                                     \
  } while (0)

// Arena against a byte-map model.
static void arena_random(unsigned seed) {
  std::mt19937 rng(seed);
  const size_t size = 1 << 20;
  Arena a(size);
  std::vector<int> owner(size / kGranule, -1);
  std::map<size_t, size_t> live;  // off -> bytes (rounded)
  int tag = 0;
  for (int step = 0; step < 4000; ++step) {
    if (live.empty() || rng() % 3) {
      const size_t want = 1 + rng() % 40000;
      size_t off;
      const bool ok = a.alloc(want, &off);
      const size_t n = round_up(want, kGranule) / kGranule;
      // does any free run of n granules exist in the model?
      size_t run = 0;
      bool exists = false;
      for (size_t g = 0; g < owner.size() && !exists; ++g) {
        run = owner[g] < 0 ? run + 1 : 0;
        exists = run >= n;
      }
      CHECK(ok == exists, "alloc %zu: arena says %d, model says %d", want, ok, exists);
      if (!ok) continue;
      CHECK(off % kGranule == 0 && off + n * kGranule <= size, "bad offset %zu", off);
      for (size_t g = off / kGranule; g < off / kGranule + n; ++g) {
        CHECK(owner[g] < 0, "overlap at granule %zu", g);
        owner[g] = tag;
      }
      ++tag;
      live[off] = n * kGranule;
    } else {
      auto it = live.begin();
      std::advance(it, rng() % live.size());
      CHECK(a.release(it->first), "release of a live block failed");
      for (size_t g = it->first / kGranule; g < (it->first + it->second) / kGranule; ++g) owner[g] = -1;
      live.erase(it);
    }
    size_t used = 0;
    for (auto& kv : live) used += kv.second;
    CHECK(a.used() == used, "used %zu vs %zu", a.used(), used);
  }
  CHECK(!a.release(12345 * kGranule + 1), "release of a non-block succeeded");
  for (auto& kv : live) a.release(kv.first);
  size_t off;
  CHECK(a.used() == 0 && a.alloc(size, &off) && off == 0, "free blocks did not coalesce");
}

struct InFlight {
  Batch b;
  int remaining;  // simulated steps until the device finishes
  std::map<int, size_t> pair_off;
};

// One simulated serving run.
static void serve_random(unsigned seed, size_t budget, int n_pairs, int n_slots, bool expect_evictions) {
  std::mt19937 rng(seed);
  Limits lim;
  lim.max_batch_cps = 700;
  lim.max_batch_reqs = 9;
  lim.max_batch_surf = 50000;
  Scheduler s(budget, lim);
  std::vector<size_t> bytes(n_pairs);
  for (int i = 0; i < n_pairs; ++i) {
    bytes[i] = 1000 + rng() % 200000;
    CHECK(s.add_pair(bytes[i]) == i, "pair id");
  }
  const int n_req = 3000;
  int64_t next_id = 0, next_admit = 0, completed = 0;
  std::vector<InFlight> slots;
  std::set<int> ever_resident_extracted;
  int step = 0;
  while (completed < n_req) {
    CHECK(++step < 1000000, "no progress (completed %lld)", (long long)completed);
    // arrivals
    const int arrivals = next_id < n_req ? (int)(rng() % 4) : 0;
    for (int k = 0; k < arrivals && next_id < n_req; ++k) {
      Request r;
      r.id = next_id++;
      r.pair = (int)(rng() % n_pairs);
      r.n_cps = 1 + (int)(rng() % 500);
      r.surf_values = (rng() % 4 == 0) ? (size_t)r.n_cps * (1 + rng() % 100) : 0;
      if (r.surf_values > lim.max_batch_surf) r.surf_values = 0;
      CHECK(s.feasible(r.pair, r.n_cps, r.surf_values), "feasible request rejected");
      s.submit(r);
    }
    // completions
    for (size_t i = 0; i < slots.size();) {
      if (--slots[i].remaining > 0) {
        ++i;
        continue;
      }
      for (auto& kv : slots[i].pair_off)
        CHECK(s.pair(kv.first).resident && s.pair(kv.first).off == kv.second,
              "pair %d moved or was evicted while a batch used it", kv.first);
      s.complete(slots[i].b);
      completed += (int64_t)slots[i].b.reqs.size();
      slots.erase(slots.begin() + i);
    }
    // launches
    while ((int)slots.size() < n_slots) {
      std::vector<bool> was_resident(n_pairs);
      for (int p = 0; p < n_pairs; ++p) was_resident[p] = s.pair(p).resident;
      InFlight f;
      const size_t pending_before = s.pending();
      if (!s.next_batch(&f.b)) {
        CHECK(!slots.empty() || pending_before == 0, "idle device but nothing admitted (%zu pending)",
              pending_before);
        break;
      }
      CHECK(!f.b.reqs.empty(), "empty batch");
      CHECK(f.b.n_cps <= lim.max_batch_cps || f.b.reqs.size() == 1, "cps limit");
      CHECK((int)f.b.reqs.size() <= lim.max_batch_reqs, "request limit");
      CHECK(f.b.surf_values <= lim.max_batch_surf, "surface limit");
      int ncp = 0;
      for (const Request& r : f.b.reqs) {
        CHECK(r.id == next_admit, "admitted %lld, expected %lld (FIFO)", (long long)r.id, (long long)next_admit);
        ++next_admit;
        ncp += r.n_cps;
        CHECK(s.pair(r.pair).resident && s.pair(r.pair).refs > 0, "admitted request's pair not resident");
        f.pair_off[r.pair] = s.pair(r.pair).off;
      }
      CHECK(ncp == f.b.n_cps, "cp count");
      // a pair that became resident must be extracted; a listed pair is
      // resident now (it may have been evicted and re-admitted while this
      // batch formed, with a new block); no pair is listed twice
      for (int p = 0; p < n_pairs; ++p) {
        const int listed = (int)std::count(f.b.extract.begin(), f.b.extract.end(), p);
        const bool became = !was_resident[p] && s.pair(p).resident;
        CHECK(listed <= 1, "pair %d listed %d times", p, listed);
        CHECK(!became || listed, "pair %d became resident without extraction", p);
        CHECK(!listed || (s.pair(p).resident && s.pair(p).refs > 0), "listed pair %d not resident", p);
      }
      // resident blocks never overlap and fit the budget
      std::vector<std::pair<size_t, size_t>> blk;
      for (int p = 0; p < n_pairs; ++p)
        if (s.pair(p).resident) blk.push_back({s.pair(p).off, round_up(bytes[p], kGranule)});
      std::sort(blk.begin(), blk.end());
      for (size_t i = 0; i + 1 < blk.size(); ++i)
        CHECK(blk[i].first + blk[i].second <= blk[i + 1].first, "resident pairs overlap");
      CHECK(s.arena().used() <= s.arena().size(), "arena over budget");
      f.remaining = 1 + (int)(rng() % 6);
      slots.push_back(f);
    }
  }
  CHECK(s.stats().completed == n_req && s.pending() == 0, "not all completed");
  for (int p = 0; p < n_pairs; ++p) CHECK(s.pair(p).refs == 0, "dangling reference on pair %d", p);
  if (expect_evictions) {
    CHECK(s.stats().evictions > 0 && s.stats().blocked > 0, "budget never gated (evictions %lld)",
          (long long)s.stats().evictions);
  } else {
    CHECK(s.stats().evictions == 0 && s.stats().extractions <= n_pairs, "unexpected eviction");
  }
  printf("serve seed %u budget %zu pairs %d slots %d: batches %lld evictions %lld extractions %lld blocked %lld "
         "peak %zu\n",
         seed, budget, n_pairs, n_slots, (long long)s.stats().batches, (long long)s.stats().evictions,
         (long long)s.stats().extractions, (long long)s.stats().blocked, s.arena().peak());
}

static void infeasible() {
  Limits lim;
  Scheduler s(10000, lim);
  const int big = s.add_pair(20000), small = s.add_pair(5000);
  CHECK(!s.feasible(big, 1, 0), "pair larger than the budget accepted");
  CHECK(s.feasible(small, 1, 0), "small pair rejected");
  CHECK(!s.feasible(small, lim.max_batch_cps + 1, 0), "too many control points accepted");
  CHECK(!s.feasible(7, 1, 0), "unknown pair accepted");
}

// Head-of-line: the oldest request blocks everything behind it while memory
// for its pair is held by in-flight work.
static void head_of_line() {
  Limits lim;
  lim.max_batch_reqs = 1;
  Scheduler s(2560, lim);  // a + b do not fit together, b + c do
  const int a = s.add_pair(1500), b = s.add_pair(1500), c = s.add_pair(500);
  s.submit(Request{0, a, 1, 0});
  s.submit(Request{1, b, 1, 0});
  s.submit(Request{2, c, 1, 0});
  Batch b0, b1;
  CHECK(s.next_batch(&b0) && b0.reqs[0].id == 0 && b0.extract == std::vector<int>{a}, "first batch");
  CHECK(!s.next_batch(&b1), "request 1 admitted while pair a is in use");
  CHECK(s.pending() == 2, "request 2 overtook the blocked request 1");
  s.complete(b0);
  CHECK(s.next_batch(&b1) && b1.reqs[0].id == 1 && s.stats().evictions == 1, "after completion");
  CHECK(!s.pair(a).resident && s.pair(b).resident, "LRU victim");
  s.complete(b1);
  Batch b2;
  CHECK(s.next_batch(&b2) && b2.reqs[0].id == 2 && s.pair(b).resident, "small pair fits beside b");
  s.complete(b2);
  s.forget(c);
  CHECK(!s.pair(c).resident, "forget");
}

int main() {
  for (unsigned seed = 1; seed <= 3; ++seed) arena_random(seed);
  infeasible();
  head_of_line();
  serve_random(11, 1 << 26, 12, 4, false);      // everything fits: no eviction
  serve_random(12, 450000, 12, 4, true);        // about two pairs fit: admission gates
  serve_random(13, 260000, 30, 2, true);        // about one pair fits
  serve_random(14, 900000, 30, 8, true);
  if (g_fail) {
    printf("%d FAILED\n", g_fail);
    return 1;
  }
  printf("ALL OK\n");
  return 0;
}
