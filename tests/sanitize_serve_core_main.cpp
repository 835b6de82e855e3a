// Drives the server's scheduling core through a seeded random scenario (submissions
// over a simulated clock, admission, up to three epochs in flight, failed epochs,
// cancellations, one device loss at the end), for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_sanitizers.py). Checks that every request
// becomes final, that admitted bytes return to zero and that the counts add up.
// Prints "ok" and returns 0; any violated check returns 1.
#include <cstdint>
#include <cstdio>
#include <deque>
#include <vector>

#include "serve_core.h"

using namespace dqj::serve;

namespace {

uint64_t rng_state = 0x9e3779b97f4a7c15ull;
uint32_t next_u32() {   // xorshift64*
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (uint32_t)((rng_state * 0x2545f4914f6cdd1dull) >> 32);
}

int fail(const char *what) {
  std::printf("FAILED: %s\n", what);
  return 1;
}

}  // namespace

int main() {
  CoreConfig cfg;
  cfg.budget_bytes = 1u << 20;
  cfg.max_inflight = 12;
  cfg.max_pending = 64;
  cfg.epoch_work = 5000.0;
  cfg.epoch_pixels = 1u << 14;
  cfg.max_chunks = 16;
  Core core(cfg);
  std::vector<uint64_t> tickets, finished;
  std::deque<uint64_t> inflight;
  double now = 0.0;
  int rejected = 0;
  for (int step = 0; step < 4000; ++step) {
    now += 1e-3;
    if (step < 3000 && next_u32() % 3 == 0) {
      RequestSpec s;
      s.tiles = 1 + next_u32() % 200;
      s.tile_pixels = 64;
      s.resident_bytes = (uint64_t)s.tiles * s.tile_pixels * 9u;
      s.work_per_tile = 10.0 + next_u32() % 90;
      uint64_t t = 0;
      const int32_t st = core.submit(s, now, &t);
      if (st == kOk)
        tickets.push_back(t);
      else if (st == kQueueFull || st == kBudget)
        ++rejected;
      else
        return fail("unexpected submit status");
    }
    if (!tickets.empty() && next_u32() % 17 == 0) {
      const uint64_t t = tickets[next_u32() % tickets.size()];
      const int32_t st = core.cancel(t, now, &finished);
      if (st != kOk && st != kState) return fail("unexpected cancel status");
    }
    core.admit(now);
    while (inflight.size() < 3) {
      Epoch e;
      if (!core.build_epoch(now, &e)) break;
      if (e.chunks.empty() || (int32_t)e.chunks.size() > cfg.max_chunks)
        return fail("epoch chunk count out of range");
      inflight.push_back(e.id);
    }
    if (!inflight.empty() && next_u32() % 2 == 0) {
      const bool ok = next_u32() % 50 != 0;   // now and then a launch fails
      core.finish_epoch(inflight.front(), ok, now, &finished);
      inflight.pop_front();
    }
  }
  // drain what is left, then lose the device with work still queued
  for (int guard = 0; guard < 100000 && !core.idle(); ++guard) {
    now += 1e-3;
    core.admit(now);
    Epoch e;
    if (core.build_epoch(now, &e)) inflight.push_back(e.id);
    if (!inflight.empty()) {
      core.finish_epoch(inflight.front(), true, now, &finished);
      inflight.pop_front();
    }
    if (guard == 50) {
      RequestSpec s;
      s.tiles = 10;
      s.tile_pixels = 64;
      s.resident_bytes = 640 * 9;
      s.work_per_tile = 20.0;
      uint64_t t = 0;
      if (core.submit(s, now, &t) == kOk) tickets.push_back(t);
      core.fail_all(now, &finished);
      inflight.clear();
    }
  }
  if (!core.idle()) return fail("scheduler never became idle");
  for (uint64_t t : tickets) {
    const RequestInfo *r = core.info(t);
    if (!r) return fail("unknown ticket");
    if (r->state == State::Pending || r->state == State::Admitted) return fail("request not final");
  }
  const CoreStats s = core.stats();
  if (s.resident_bytes != 0) return fail("admitted bytes not returned");
  if (s.completed + s.cancelled + s.failed != s.submitted) return fail("counts do not add up");
  std::printf("ok submitted %llu completed %llu cancelled %llu failed %llu rejected %d\n",
              (unsigned long long)s.submitted, (unsigned long long)s.completed,
              (unsigned long long)s.cancelled, (unsigned long long)s.failed, rejected);
  return 0;
}
