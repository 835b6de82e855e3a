// serve_core.h -- scheduling core of the render server (library-internal, no HIP).
//
// Continuous batching at tile granularity: admitted requests are cut into chunks of
// tiles, and every launch ("epoch") takes chunks from all active requests at once,
// so a request that arrives while others run joins the next epoch instead of
// waiting for them to finish, and a large request cannot hold the GPU for longer
// than one epoch at a time. Admission is first come, first served, limited by the
// device bytes the admitted requests keep resident (their framebuffers) and by a
// cap on requests in flight.
//
// Times are host steady-clock seconds supplied by the caller, so the core can be
// driven by a simulated clock in tests.
#pragma once
#include <cstddef>
#include <cstdint>
#include <deque>
#include <unordered_map>
#include <vector>

namespace dqj {
namespace serve {

// Status codes mirror the C ABI's dqj_status values.
enum : int32_t {
  kOk = 0,
  kPending = 1,
  kInvalid = -1,
  kBudget = -3,
  kQueueFull = -4,
  kDevice = -5,
  kCancelled = -7,
  kState = -9
};

struct CoreConfig {
  uint64_t budget_bytes = 8ull << 30;  // resident bytes of admitted requests at once
  int32_t max_inflight = 64;           // admitted, unfinished requests at once
  int32_t max_pending = 4096;          // queue length before submit is refused
  double epoch_work = 8e9;             // estimated DQ updates per epoch
  uint64_t epoch_pixels = 4u << 20;    // pixels per epoch (scratch capacity)
  int32_t max_chunks = 256;            // table entries per epoch
  bool oldest_first = false;           // fill epochs oldest request first (no fair share)
};

struct RequestSpec {
  uint64_t resident_bytes = 0;  // device bytes held while admitted
  uint32_t tiles = 0;           // tiles of the frame
  uint32_t tile_pixels = 0;     // pixels of one tile
  double work_per_tile = 0;     // estimated DQ updates of one tile
};

struct Chunk {
  uint64_t ticket;
  uint32_t tile_begin;  // first tile of the frame in this chunk
  uint32_t ntiles;
};

struct Epoch {
  uint64_t id = 0;
  std::vector<Chunk> chunks;
  uint64_t pixels = 0;
  double work = 0;
};

enum class State : int32_t { Pending, Admitted, Done, Cancelled, Failed };

struct RequestInfo {
  State state = State::Pending;
  int32_t status = kPending;      // final status once state is Done/Cancelled/Failed
  double t_submit = 0, t_admit = -1, t_first_launch = -1, t_done = -1;
  RequestSpec spec;
  uint32_t tiles_assigned = 0, tiles_done = 0;
  int32_t chunks_inflight = 0;
  int32_t chunks = 0;             // chunks launched so far
  bool cancel_requested = false;
  bool failed = false;
};

struct CoreStats {
  uint64_t submitted = 0, admitted = 0, completed = 0, cancelled = 0, failed = 0, rejected = 0;
  uint64_t epochs = 0;
  uint64_t resident_bytes = 0;
  int32_t pending = 0, active = 0;
  double p50 = 0, p99 = 0, max = 0, mean = 0;  // latency t_done - t_submit of completed requests
};

class Core {
 public:
  explicit Core(const CoreConfig &cfg);

  // kOk (ticket set), kInvalid, kBudget (alone exceeds the budget), kQueueFull.
  int32_t submit(const RequestSpec &spec, double now, uint64_t *ticket);
  // Admit pending requests in arrival order while budget and slots allow.
  void admit(double now);
  // Build the next epoch from active requests' unassigned tiles. False if none.
  bool build_epoch(double now, Epoch *out);
  // Retire an epoch (ok = its launch completed without error); appends requests that
  // became final to *finished.
  void finish_epoch(uint64_t epoch_id, bool ok, double now, std::vector<uint64_t> *finished);
  // kOk (final now or once its in-flight chunks retire), kState if already final,
  // kInvalid if unknown. Appends requests that became final to *finished.
  int32_t cancel(uint64_t ticket, double now, std::vector<uint64_t> *finished);
  // Fail every unfinished request (device lost); appends them to *finished.
  void fail_all(double now, std::vector<uint64_t> *finished);

  const RequestInfo *info(uint64_t ticket) const;
  CoreStats stats() const;
  bool idle() const { return pending_.empty() && active_.empty(); }
  size_t pending_count() const { return pending_.size(); }
  bool has_unassigned() const;

 private:
  void finalize(uint64_t ticket, RequestInfo &r, State st, int32_t status, double now,
                std::vector<uint64_t> *finished);

  CoreConfig cfg_;
  uint64_t next_ticket_ = 1, next_epoch_ = 1;
  uint64_t resident_ = 0;
  std::deque<uint64_t> pending_;
  std::vector<uint64_t> active_;   // admitted, not final, in admission order
  std::unordered_map<uint64_t, RequestInfo> reqs_;
  std::unordered_map<uint64_t, std::vector<Chunk>> epochs_;
  std::vector<double> latencies_;
  CoreStats counts_;
};

}  // namespace serve
}  // namespace dqj
