// C shim over the server's scheduling core, compiled with g++ by the CPU tests
// (no HIP): lets the tests drive admission, epochs, cancellation and failures with a
// simulated clock.
#include <cstdint>
#include <cstring>
#include <vector>

#include "serve_core.h"

using namespace dqj::serve;

extern "C" {

void *core_new(uint64_t budget, int32_t max_inflight, int32_t max_pending, double epoch_work,
               uint64_t epoch_pixels, int32_t max_chunks, int32_t oldest_first) {
  CoreConfig c;
  c.oldest_first = oldest_first != 0;
  c.budget_bytes = budget;
  c.max_inflight = max_inflight;
  c.max_pending = max_pending;
  c.epoch_work = epoch_work;
  c.epoch_pixels = epoch_pixels;
  c.max_chunks = max_chunks;
  return new Core(c);
}

void core_free(void *p) { delete (Core *)p; }

int32_t core_submit(void *p, uint64_t bytes, uint32_t tiles, uint32_t tile_px, double wpt,
                    double now, uint64_t *ticket) {
  RequestSpec s;
  s.resident_bytes = bytes;
  s.tiles = tiles;
  s.tile_pixels = tile_px;
  s.work_per_tile = wpt;
  return ((Core *)p)->submit(s, now, ticket);
}

void core_admit(void *p, double now) { ((Core *)p)->admit(now); }

// Returns the number of chunks (0 if no epoch); chunk arrays must hold `cap` entries.
int32_t core_build(void *p, double now, uint64_t *epoch_id, uint64_t *tickets, uint32_t *begins,
                   uint32_t *ntiles, int32_t cap) {
  Epoch e;
  if (!((Core *)p)->build_epoch(now, &e)) return 0;
  *epoch_id = e.id;
  const int32_t n = (int32_t)e.chunks.size() < cap ? (int32_t)e.chunks.size() : cap;
  for (int32_t i = 0; i < n; ++i) {
    tickets[i] = e.chunks[i].ticket;
    begins[i] = e.chunks[i].tile_begin;
    ntiles[i] = e.chunks[i].ntiles;
  }
  return (int32_t)e.chunks.size();
}

int32_t core_finish(void *p, uint64_t epoch, int32_t ok, double now, uint64_t *fin, int32_t cap) {
  std::vector<uint64_t> f;
  ((Core *)p)->finish_epoch(epoch, ok != 0, now, &f);
  for (size_t i = 0; i < f.size() && (int32_t)i < cap; ++i) fin[i] = f[i];
  return (int32_t)f.size();
}

int32_t core_cancel(void *p, uint64_t ticket, double now) {
  std::vector<uint64_t> f;
  return ((Core *)p)->cancel(ticket, now, &f);
}

int32_t core_fail_all(void *p, double now) {
  std::vector<uint64_t> f;
  ((Core *)p)->fail_all(now, &f);
  return (int32_t)f.size();
}

// state: 0 pending, 1 admitted, 2 done, 3 cancelled, 4 failed; -1 unknown ticket
int32_t core_state(void *p, uint64_t ticket, int32_t *status, double *t_admit, double *t_done,
                   int32_t *chunks) {
  const RequestInfo *r = ((Core *)p)->info(ticket);
  if (!r) return -1;
  *status = r->status;
  *t_admit = r->t_admit;
  *t_done = r->t_done;
  *chunks = r->chunks;
  return (int32_t)r->state;
}

// counts: submitted, admitted, completed, cancelled, failed, rejected, epochs, resident,
// pending, active; lat: p50, p99, max, mean
void core_stats(void *p, uint64_t *counts, double *lat) {
  const CoreStats s = ((Core *)p)->stats();
  const uint64_t c[10] = {s.submitted, s.admitted, s.completed, s.cancelled, s.failed,
                          s.rejected, s.epochs, s.resident_bytes, (uint64_t)s.pending,
                          (uint64_t)s.active};
  memcpy(counts, c, sizeof c);
  lat[0] = s.p50;
  lat[1] = s.p99;
  lat[2] = s.max;
  lat[3] = s.mean;
}

}  // extern "C"
