// serve_core.cpp -- scheduling core of the render server (see serve_core.h).
#include "serve_core.h"

#include <algorithm>
#include <cmath>

namespace dqj {
namespace serve {

Core::Core(const CoreConfig &cfg) : cfg_(cfg) {
  if (cfg_.max_inflight < 1) cfg_.max_inflight = 1;
  if (cfg_.max_pending < 1) cfg_.max_pending = 1;
  if (cfg_.max_chunks < 1) cfg_.max_chunks = 1;
  if (!(cfg_.epoch_work > 0)) cfg_.epoch_work = 1;
  if (cfg_.epoch_pixels < 1) cfg_.epoch_pixels = 1;
}

int32_t Core::submit(const RequestSpec &spec, double now, uint64_t *ticket) {
  if (spec.tiles == 0 || spec.tile_pixels == 0 || !(spec.work_per_tile >= 0)) return kInvalid;
  if (spec.tile_pixels > cfg_.epoch_pixels) return kInvalid;
  if (spec.resident_bytes > cfg_.budget_bytes) {
    ++counts_.rejected;
    return kBudget;
  }
  if ((int32_t)pending_.size() >= cfg_.max_pending) {
    ++counts_.rejected;
    return kQueueFull;
  }
  const uint64_t t = next_ticket_++;
  RequestInfo r;
  r.spec = spec;
  r.t_submit = now;
  reqs_.emplace(t, r);
  pending_.push_back(t);
  ++counts_.submitted;
  *ticket = t;
  return kOk;
}

void Core::admit(double now) {
  while (!pending_.empty()) {
    RequestInfo &r = reqs_.at(pending_.front());
    if ((int32_t)active_.size() >= cfg_.max_inflight) break;
    if (resident_ + r.spec.resident_bytes > cfg_.budget_bytes) break;  // first come, first served
    resident_ += r.spec.resident_bytes;
    r.state = State::Admitted;
    r.t_admit = now;
    active_.push_back(pending_.front());
    pending_.pop_front();
    ++counts_.admitted;
  }
}

bool Core::has_unassigned() const {
  for (uint64_t t : active_) {
    const RequestInfo &r = reqs_.at(t);
    if (r.tiles_assigned < r.spec.tiles) return true;
  }
  return false;
}

bool Core::build_epoch(double now, Epoch *out) {
  std::vector<uint64_t> cand;
  for (uint64_t t : active_) {
    const RequestInfo &r = reqs_.at(t);
    if (r.tiles_assigned < r.spec.tiles) cand.push_back(t);
  }
  if (cand.empty()) return false;
  Epoch e;
  e.id = next_epoch_++;
  double work_left = cfg_.epoch_work;
  uint64_t pix_left = cfg_.epoch_pixels;
  // chunk index per request within this epoch (tiles of one request stay contiguous)
  std::unordered_map<uint64_t, size_t> slot;
  auto take = [&](uint64_t t, double budget_work) {
    RequestInfo &r = reqs_.at(t);
    const uint32_t remaining = r.spec.tiles - r.tiles_assigned;
    if (remaining == 0) return;
    uint64_t by_work = r.spec.work_per_tile > 0
                           ? (uint64_t)std::floor(budget_work / r.spec.work_per_tile)
                           : (uint64_t)remaining;
    const uint64_t by_pix = pix_left / r.spec.tile_pixels;
    uint64_t n = std::min<uint64_t>({(uint64_t)remaining, by_work, by_pix});
    if (n == 0) return;
    auto it = slot.find(t);
    if (it == slot.end()) {
      if ((int32_t)e.chunks.size() >= cfg_.max_chunks) return;
      slot[t] = e.chunks.size();
      e.chunks.push_back(Chunk{t, r.tiles_assigned, (uint32_t)n});
    } else {
      e.chunks[it->second].ntiles += (uint32_t)n;   // contiguous with its first chunk
    }
    r.tiles_assigned += (uint32_t)n;
    const double w = (double)n * r.spec.work_per_tile;
    work_left -= w;
    e.work += w;
    pix_left -= n * r.spec.tile_pixels;
    e.pixels += n * r.spec.tile_pixels;
  };
  // pass 1 (fair policy): an equal share of the epoch for every request (at least one
  // tile each, so no request waits for another to drain)
  if (!cfg_.oldest_first) {
    const double share = cfg_.epoch_work / (double)cand.size();
    for (uint64_t t : cand) {
      const RequestInfo &r = reqs_.at(t);
      take(t, std::max(share, r.spec.work_per_tile));
    }
  }
  // pass 2: what is left of the epoch, first come first served
  for (uint64_t t : cand) {
    if (work_left <= 0 || pix_left == 0) break;
    take(t, work_left);
  }
  if (e.chunks.empty()) {
    // a single tile larger than the work cap: take one tile of the oldest request
    RequestInfo &r = reqs_.at(cand.front());
    e.chunks.push_back(Chunk{cand.front(), r.tiles_assigned, 1});
    r.tiles_assigned += 1;
    e.pixels = r.spec.tile_pixels;
    e.work = r.spec.work_per_tile;
  }
  for (const Chunk &c : e.chunks) {
    RequestInfo &r = reqs_.at(c.ticket);
    ++r.chunks_inflight;
    ++r.chunks;
    if (r.t_first_launch < 0) r.t_first_launch = now;
  }
  epochs_[e.id] = e.chunks;
  ++counts_.epochs;
  *out = std::move(e);
  return true;
}

void Core::finalize(uint64_t ticket, RequestInfo &r, State st, int32_t status, double now,
                    std::vector<uint64_t> *finished) {
  r.state = st;
  r.status = status;
  r.t_done = now;
  resident_ -= r.spec.resident_bytes;
  active_.erase(std::find(active_.begin(), active_.end(), ticket));
  if (st == State::Done) {
    ++counts_.completed;
    latencies_.push_back(now - r.t_submit);
  } else if (st == State::Cancelled) {
    ++counts_.cancelled;
  } else {
    ++counts_.failed;
  }
  if (finished) finished->push_back(ticket);
}

void Core::finish_epoch(uint64_t epoch_id, bool ok, double now, std::vector<uint64_t> *finished) {
  auto it = epochs_.find(epoch_id);
  if (it == epochs_.end()) return;
  const std::vector<Chunk> chunks = it->second;
  epochs_.erase(it);
  for (const Chunk &c : chunks) {
    RequestInfo &r = reqs_.at(c.ticket);
    --r.chunks_inflight;
    if (ok) {
      r.tiles_done += c.ntiles;
    } else {
      r.failed = true;
      r.tiles_assigned = r.spec.tiles;   // assign nothing more
    }
    if (r.state != State::Admitted || r.chunks_inflight > 0) continue;
    if (r.failed)
      finalize(c.ticket, r, State::Failed, kDevice, now, finished);
    else if (r.cancel_requested)
      finalize(c.ticket, r, State::Cancelled, kCancelled, now, finished);
    else if (r.tiles_done == r.spec.tiles)
      finalize(c.ticket, r, State::Done, kOk, now, finished);
  }
}

int32_t Core::cancel(uint64_t ticket, double now, std::vector<uint64_t> *finished) {
  auto it = reqs_.find(ticket);
  if (it == reqs_.end()) return kInvalid;
  RequestInfo &r = it->second;
  if (r.state == State::Pending) {
    pending_.erase(std::find(pending_.begin(), pending_.end(), ticket));
    r.state = State::Cancelled;
    r.status = kCancelled;
    r.t_done = now;
    ++counts_.cancelled;
    if (finished) finished->push_back(ticket);
    return kOk;
  }
  if (r.state != State::Admitted) return kState;
  r.cancel_requested = true;
  r.tiles_assigned = r.spec.tiles;
  if (r.chunks_inflight == 0) finalize(ticket, r, State::Cancelled, kCancelled, now, finished);
  return kOk;
}

void Core::fail_all(double now, std::vector<uint64_t> *finished) {
  epochs_.clear();
  const std::vector<uint64_t> act = active_;
  for (uint64_t t : act) {
    RequestInfo &r = reqs_.at(t);
    r.chunks_inflight = 0;
    finalize(t, r, State::Failed, kDevice, now, finished);
  }
  while (!pending_.empty()) {
    RequestInfo &r = reqs_.at(pending_.front());
    r.state = State::Failed;
    r.status = kDevice;
    r.t_done = now;
    ++counts_.failed;
    if (finished) finished->push_back(pending_.front());
    pending_.pop_front();
  }
}

const RequestInfo *Core::info(uint64_t ticket) const {
  auto it = reqs_.find(ticket);
  return it == reqs_.end() ? nullptr : &it->second;
}

CoreStats Core::stats() const {
  CoreStats s = counts_;
  s.resident_bytes = resident_;
  s.pending = (int32_t)pending_.size();
  s.active = (int32_t)active_.size();
  if (!latencies_.empty()) {
    std::vector<double> v = latencies_;
    std::sort(v.begin(), v.end());
    auto q = [&](double f) {
      const size_t i = (size_t)std::ceil(f * (double)v.size()) - 1;
      return v[std::min(i, v.size() - 1)];
    };
    s.p50 = q(0.50);
    s.p99 = q(0.99);
    s.max = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    s.mean = sum / (double)v.size();
  }
  return s;
}

}  // namespace serve
}  // namespace dqj
