// Host-only model of the served likelihood's slot protocol, for ThreadSanitizer.
//
// The device loop of the library (a poller workgroup, worker workgroups, the
// host thread publishing requests into slots) is modelled with std::threads
// over the same words and the same rules:
//   host     writes desc[s], then mail[s] = seq (release), then bumps gen;
//            takes a result once fin[s] == seq (acquire), then reuses the slot.
//   poller   on a new gen, for each slot whose mail word is newer than open[s]:
//            copies desc[s] to the device copy dd[s], stamps the opening
//            order, sets open/done/lim, publishes claim[s] = seq << 32
//            (release) and the slot's bit in the mask.
//   workers  take one claim (a run of consecutive items, chunk_of) with one
//            fetch_add on claim[s] of a slot in the
//            mask (from a per-worker starting slot, oldest stamp first, or
//            fewest unclaimed claims first, read from the claim and lim
//            words); the claim is valid iff lim[s] names the same sequence
//            number and the claim is below the request's claim count; the
//            last valid claim clears the mask bit; after a claim's items,
//            done[s] += 1 (acq_rel), and the worker completing the last claim
//            sums the partials in item order, writes out[s] and fin[s] = seq
//            (release).
// The device code gets the release/acquire pairs above from relaxed
// device-coherent atomics with the writer waiting for its stores to complete
// before the publishing atomic and the reader issuing its loads after the
// observing one; here they are C++ release/acquire so that ThreadSanitizer
// checks the happens-before chain that makes the plain data (descriptors,
// partials, results) race-free.
//
// Checks: every item of every request is processed exactly once, every
// request completes exactly once with the sum of its items, and the loop
// drains.  Modes:
//   stress <policy> <requests> <workers> <slots> <seed>
//   late <policy>      forces a late claim: a worker that chose a slot for a
//                      finishing request claims only after the next request
//                      was opened in the same slot.
// Built with -DOLD_PROTOCOL the claim is validated against the sequence
// number read before the fetch_add (the earlier, faulty rule): the forced
// interleaving then loses an item and the request never completes (exit 3).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

namespace {

constexpr int kMaxSlots = 64;
constexpr int kMaxItems = 64;

struct Desc {              // plain data: written by the host, copied by the poller
  uint64_t seq;
  int items;
  int req;                 // request index (for the checks)
};

struct Slot {
  std::atomic<uint64_t> claim{0}, lim{0}, open{0}, stamp{0};
  std::atomic<uint32_t> done{0};
};

struct Request {
  int items = 0;
  int slot = -1;
  uint64_t seq = 0;
  std::atomic<int> processed[kMaxItems];
  std::atomic<int> completions{0};
  double partial[kMaxItems];   // plain: written by the item's worker, read by the finisher
  Request() {
    for (auto& p : processed) p.store(0);
  }
};

struct Model {
  int nslots = 4;
  int policy = 0;            // 0 spread, 1 oldest first, 2 fewest unclaimed claims first
  int nworkers = 1;          // the device loop's chunk rule depends on it
  // host <-> device words
  std::atomic<uint64_t> gen{0}, stop{0};
  std::atomic<uint64_t> mail[kMaxSlots];
  std::atomic<uint64_t> fin[kMaxSlots];
  Desc desc[kMaxSlots];      // host-side descriptors (plain)
  double out[kMaxSlots];     // results (plain)
  // device words
  Desc dd[kMaxSlots];        // device copies of the descriptors (plain)
  Slot st[kMaxSlots];
  std::atomic<uint64_t> mask{0}, opened{0};
  std::atomic<uint32_t> quit{0}, live{0};
  std::vector<Request>* reqs = nullptr;
  // forced interleaving of the "late" mode
  std::atomic<int> late_phase{0};   // 0 idle, 1 the late worker chose its slot, 2 the next request is open
  int late_worker = -1;
  Model() {
    for (int s = 0; s < kMaxSlots; ++s) {
      mail[s].store(0);
      fin[s].store(0);
    }
  }
};

double item_value(int req, int item) { return 1.0 + req * 0.001 + item * 1e-6; }

// The device loop's claim size: a claim is a run of chunk_of(items, workers)
// consecutive items (about two claims per worker, at most 16 items).
int chunk_of(int items, int workers) {
  const int w2 = 2 * std::max(workers, 1);
  const int k = (items + w2 - 1) / w2;
  return std::min(std::max(k, 1), 16);
}
int claims_of(int items, int workers) {
  const int k = chunk_of(items, workers);
  return (items + k - 1) / k;
}

// Poller: open slot s for seq.
void poller_open(Model& M, int s, uint64_t seq) {
  M.dd[s] = M.desc[s];                       // ordered after the acquire of mail[s]
  const uint64_t stamp = M.opened.load(std::memory_order_relaxed) + 1;
  M.opened.store(stamp, std::memory_order_relaxed);
  M.st[s].stamp.store(stamp, std::memory_order_relaxed);
  M.st[s].open.store(seq, std::memory_order_relaxed);
  M.st[s].done.store(0, std::memory_order_relaxed);
  M.st[s].lim.store((seq << 32) | (uint64_t)claims_of(M.dd[s].items, M.nworkers), std::memory_order_release);
  M.st[s].claim.store(seq << 32, std::memory_order_release);
  M.mask.fetch_or(1ull << s, std::memory_order_acq_rel);
}

void poller(Model& M, int idle_limit) {
  uint64_t seen = 0;
  int idle = 0;
  for (;;) {
    if (M.stop.load(std::memory_order_acquire)) return;
    if (M.quit.load(std::memory_order_relaxed)) {
      if (M.live.load(std::memory_order_acquire) == 0) return;
      std::this_thread::yield();
      continue;
    }
    const uint64_t g = M.gen.load(std::memory_order_acquire);
    if (g != seen) {
      seen = g;
      idle = 0;
      for (int s = 0; s < M.nslots; ++s) {
        const uint64_t m = M.mail[s].load(std::memory_order_acquire);
        if (m > M.st[s].open.load(std::memory_order_relaxed)) poller_open(M, s, m);
      }
      if (M.late_phase.load() == 1) {
        // the late worker waits for a reopened slot: signal once one exists
        for (int s = 0; s < M.nslots; ++s)
          if (M.st[s].open.load(std::memory_order_relaxed) >= 2) M.late_phase.store(2);
      }
    } else if (M.mask.load(std::memory_order_acquire) != 0) {
      idle = 0;
    } else if (++idle > idle_limit) {
      M.quit.store(1, std::memory_order_release);
    }
    std::this_thread::yield();
  }
}

// One claim on slot s: true with the item if valid.
bool claim(Model& M, int s, uint64_t expected_seq, int* item) {
  const uint64_t old = M.st[s].claim.fetch_add(1, std::memory_order_acq_rel);
  const uint64_t lim = M.st[s].lim.load(std::memory_order_acquire);
  const unsigned it = (unsigned)(old & 0xffffffffull);
  const unsigned n = (unsigned)(lim & 0xffffffffull);
#ifdef OLD_PROTOCOL
  // the earlier rule: the claim counts only for the request the worker saw
  if ((old >> 32) != expected_seq || (lim >> 32) != (old >> 32) || it >= n) return false;
#else
  (void)expected_seq;
  if ((lim >> 32) != (old >> 32) || it >= n) return false;
#endif
  if (it == n - 1) M.mask.fetch_and(~(1ull << s), std::memory_order_acq_rel);
  *item = (int)it;
  return true;
}

void worker(Model& M, int id) {
  const unsigned rot = (unsigned)id & 63u;
  for (;;) {
    if (M.stop.load(std::memory_order_acquire) || M.quit.load(std::memory_order_acquire)) break;
    if (M.late_worker >= 0 && id != M.late_worker && M.late_phase.load() == 0) {
      // forced interleaving: the others start only once the late worker has
      // chosen its slot (else they could finish the first request before it
      // looks, and the host would wait for a choice that never comes)
      std::this_thread::yield();
      continue;
    }
    uint64_t m = M.mask.load(std::memory_order_acquire);
    int s = -1, item = -1;
    if (M.policy != 0) {
      while (m != 0 && s < 0) {
        int best = -1;
        uint64_t bst = ~0ull;
        for (int k = 0; k < M.nslots; ++k)
          if ((m >> k) & 1ull) {
            uint64_t v;
            if (M.policy == 1) {
              v = M.st[k].stamp.load(std::memory_order_relaxed);
            } else {
              const uint64_t c = M.st[k].claim.load(std::memory_order_relaxed);
              const uint64_t l = M.st[k].lim.load(std::memory_order_relaxed);
              const unsigned next = (unsigned)(c & 0xffffffffull), n = (unsigned)(l & 0xffffffffull);
              v = ((c >> 32) == (l >> 32) && next < n) ? (uint64_t)(n - next) : (1ull << 40);
            }
            if (v < bst) { bst = v; best = k; }
          }
        if (best < 0) break;
        const uint64_t seen = M.st[best].claim.load(std::memory_order_relaxed) >> 32;
        if (id == M.late_worker && M.late_phase.load() == 0) {
          M.late_phase.store(1);
          while (M.late_phase.load() != 2 && !M.stop.load()) std::this_thread::yield();
        }
        if (claim(M, best, seen, &item)) s = best;
        m &= ~(1ull << best);
      }
    } else {
      m = rot ? (m >> rot) | (m << (64u - rot)) : m;
      while (m != 0 && s < 0) {
        const int k = (int)((__builtin_ctzll(m) + rot) & 63u);
        m &= m - 1;
        if (k >= M.nslots) continue;
        const uint64_t seen = M.st[k].claim.load(std::memory_order_relaxed) >> 32;
        if (id == M.late_worker && M.late_phase.load() == 0) {
          M.late_phase.store(1);
          while (M.late_phase.load() != 2 && !M.stop.load()) std::this_thread::yield();
        }
        if (claim(M, k, seen, &item)) s = k;
      }
    }
    if (s < 0) {
      std::this_thread::yield();
      continue;
    }
    const Desc d = M.dd[s];                  // ordered after the claim's acquire
    Request& R = (*M.reqs)[d.req];
    // claim `item` covers the items chunk x item .. (the request's last)
    const int chunk = chunk_of(d.items, M.nworkers);
    for (int i = item * chunk; i < std::min(item * chunk + chunk, d.items); ++i) {
      R.processed[i].fetch_add(1, std::memory_order_relaxed);
      R.partial[i] = item_value(d.req, i);
    }
    const uint32_t prev = M.st[s].done.fetch_add(1, std::memory_order_acq_rel);
    if ((int)prev + 1 == claims_of(d.items, M.nworkers)) {
      double tot = 0.0;
      for (int i = 0; i < d.items; ++i) tot += R.partial[i];
      M.out[s] = tot;
      R.completions.fetch_add(1, std::memory_order_relaxed);
      M.fin[s].store(d.seq, std::memory_order_release);
    }
  }
  M.live.fetch_sub(1, std::memory_order_acq_rel);
}

int run(int policy, int nreq, int nworkers, int nslots, unsigned seed, bool late) {
  Model M;
  M.nslots = nslots;
  M.policy = policy;
  M.nworkers = nworkers;
  std::vector<Request> reqs(nreq);
  M.reqs = &reqs;
  std::mt19937 rng(seed);
  for (auto& r : reqs) r.items = late ? 3 : 1 + (int)(rng() % kMaxItems);
  if (late) M.late_worker = 0;
  M.live.store((uint32_t)nworkers);
  std::thread pol(poller, std::ref(M), 1 << 30);
  std::vector<std::thread> ws;
  for (int i = 0; i < nworkers; ++i) ws.emplace_back(worker, std::ref(M), i);

  // host: publish into free slots, collect results
  std::vector<int> in_slot(nslots, -1);
  std::vector<uint64_t> slot_seq(nslots, 0);
  int next = 0, finished = 0;
  const auto t0 = std::chrono::steady_clock::now();
  int status = 0;
  while (finished < nreq) {
    for (int s = 0; s < nslots; ++s) {
      const int r = in_slot[s];
      if (r >= 0 && M.fin[s].load(std::memory_order_acquire) == reqs[r].seq) {
        double want = 0.0;
        for (int i = 0; i < reqs[r].items; ++i) want += item_value(r, i);
        if (M.out[s] != want) {
          std::fprintf(stderr, "request %d: result %.17g, expected %.17g\n", r, M.out[s], want);
          status = 2;
        }
        in_slot[s] = -1;
        ++finished;
      }
    }
    for (int s = 0; s < nslots && next < nreq; ++s) {
      if (in_slot[s] >= 0) continue;
      if (late && next == 1 && M.late_phase.load() != 1) break;   // the late worker holds a choice first
      Request& R = reqs[next];
      R.slot = s;
      R.seq = ++slot_seq[s];
      M.desc[s] = Desc{R.seq, R.items, next};
      M.mail[s].store(R.seq, std::memory_order_release);
      M.gen.fetch_add(1, std::memory_order_acq_rel);
      in_slot[s] = next++;
      if (late) break;                                          // one request at a time
    }
    if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(late ? 4 : 30)) {
      std::fprintf(stderr, "stalled: %d of %d requests finished\n", finished, nreq);
      status = 3;
      break;
    }
    std::this_thread::yield();
  }
  M.stop.store(1, std::memory_order_release);
  M.late_phase.store(2);
  pol.join();
  for (auto& w : ws) w.join();
  for (int r = 0; r < nreq && status == 0; ++r) {
    for (int i = 0; i < reqs[r].items; ++i)
      if (reqs[r].processed[i].load() != 1) {
        std::fprintf(stderr, "request %d item %d processed %d times\n", r, i, reqs[r].processed[i].load());
        status = 4;
      }
    if (reqs[r].completions.load() != 1) {
      std::fprintf(stderr, "request %d completed %d times\n", r, reqs[r].completions.load());
      status = 4;
    }
  }
  return status;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc >= 2 && !std::strcmp(argv[1], "stress") && argc == 7) {
    const int st = run(std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4]), std::atoi(argv[5]),
                       (unsigned)std::atoi(argv[6]), false);
    std::printf("stress %s\n", st ? "FAILED" : "ok");
    return st;
  }
  if (argc == 3 && !std::strcmp(argv[1], "late")) {
    // one slot: request 0 (3 items) finishes while the late worker holds its
    // choice of the slot; request 1 is then opened in the same slot and the
    // late worker's claim lands on it
    const int st = run(std::atoi(argv[2]), 2, 3, 1, 1u, true);
    std::printf("late %s\n", st ? "FAILED" : "ok");
    return st;
  }
  std::fprintf(stderr, "usage: %s stress <policy> <requests> <workers> <slots> <seed> | late <policy>\n", argv[0]);
  return 1;
}
