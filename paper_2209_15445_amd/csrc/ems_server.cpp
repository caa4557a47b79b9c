// ems_server.cpp -- continuous-batching offload server over one transport
// context.
//
// The paper's hybrid workflow buffers particles entering the GPU region and
// processes a batch synchronously, with a Flush call to drain the rest
// (section 4), and observes that injecting new primaries at regular intervals
// would let staggered showers overlap on the device (section 5).  Here the
// device loop never waits for a batch to finish: a driver thread admits
// requests whenever a tally slot is free and the track-buffer budget allows,
// injects them between chunks of iterations into the same queues as the
// showers already in flight, and returns each event as soon as its last
// track is gone (per-event live-track counters kept by the kernels).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>

#include "ems_runtime.hpp"

using namespace ems;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  uint32_t key = 0;
  std::vector<ems_primary> tracks;
  uint64_t add[3] = {0, 0, 0};  // tracks per species
  uint64_t bytes = 0;           // admission estimate
  int slot = -1;
  bool done = false;
  Clock::time_point t_submit;
  std::vector<double> edep;
  ems_ledger ledger{};
  std::vector<ems_primary> exits;  // outgoing tracks (event field 0)
};

constexpr size_t kMaxQueued = 1u << 20;
constexpr uint32_t kMaxTracks = 65536;

}  // namespace

struct ems_server {
  ems_ctx* ctx = nullptr;
  uint64_t cap_bytes = 0;
  uint32_t chunk = 8;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
  std::set<uint64_t> unfinished;
  uint64_t next_ticket = 1;
  bool stop = false;
  bool failed = false;
  std::string fail_msg;

  // admission state (under mu)
  std::vector<std::shared_ptr<Request>> slots;
  std::vector<uint32_t> free_slots;
  uint64_t admitted_bytes = 0, peak_bytes = 0, in_flight = 0;

  // statistics (under mu)
  uint64_t submitted = 0, completed = 0, prim_completed = 0, chunks = 0, exits_dropped = 0;
  std::vector<double> lat_ms;
  Clock::time_point t0;

  std::thread driver;

  void fail_all(const std::string& msg) {
    std::lock_guard<std::mutex> lk(mu);
    failed = true;
    fail_msg = msg;
    cv_done.notify_all();
  }

  void run();
};

void ems_server::run() {
  if (hipSetDevice(ctx->device) != hipSuccess) {
    fail_all("driver thread cannot select the device");
    return;
  }
  const uint64_t cap = ctx->L.cap;
  std::vector<int32_t> live(ctx->cfg.max_events);
  // tracks in the current queues after the last chunk, plus those injected since
  uint64_t occupied[3] = {0, 0, 0};
  for (;;) {
    std::vector<std::shared_ptr<Request>> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (in_flight == 0 && queue.empty()) cv_work.wait(lk, [&] { return stop || !queue.empty(); });
      if (stop) return;
      while (!queue.empty() && !free_slots.empty()) {
        const std::shared_ptr<Request>& r = queue.front();
        if (in_flight > 0 && admitted_bytes + r->bytes > cap_bytes) break;
        bool room = true;
        for (int s = 0; s < 3; ++s) room = room && occupied[s] + r->add[s] <= cap;
        if (!room) break;
        for (int s = 0; s < 3; ++s) occupied[s] += r->add[s];
        r->slot = (int)free_slots.back();
        free_slots.pop_back();
        slots[r->slot] = r;
        admitted_bytes += r->bytes;
        peak_bytes = std::max(peak_bytes, admitted_bytes);
        in_flight += 1;
        admit.push_back(r);
        queue.pop_front();
      }
      if (in_flight == 0) continue;
    }
    // inject all admitted events into their slots with one row reset and
    // one enqueue (driver thread only)
    if (!admit.empty()) {
      std::vector<uint32_t> rows;
      std::vector<ems_primary> p;
      for (const std::shared_ptr<Request>& r : admit) {
        rows.push_back((uint32_t)r->slot);
        ctx->keys[r->slot] = r->key;
        for (ems_primary q : r->tracks) {
          q.event = (uint32_t)r->slot;
          p.push_back(q);
        }
      }
      ems_status st = rt_reset_rows(ctx, rows.data(), (uint32_t)rows.size());
      for (int s2 = 0; s2 < 3; ++s2) ctx->pending[s2] = 0;  // room was checked above
      if (!st) st = rt_enqueue(ctx, p.data(), p.size());
      if (st) {
        fail_all(std::string("injection failed: ") + ems_last_error());
        return;
      }
    }
    const ems_status st = rt_chunk(ctx, chunk);
    if (st) {
      fail_all(std::string("device loop failed: ") + ems_last_error());
      return;
    }
    for (int s2 = 0; s2 < 3; ++s2) occupied[s2] = ctx->pin_ctl->n_home[s2] + ctx->pin_ctl->n_sec[s2];
    if (rt_read_live(ctx, live.data())) {
      fail_all(std::string("live counters unreadable: ") + ems_last_error());
      return;
    }
    // outgoing tracks of this chunk, to their requests (slots change owner
    // only in this thread)
    if (ctx->cfg.exit_capacity) {
      std::vector<ems_primary> ex;
      uint64_t total = 0;
      if (rt_take_exits(ctx, ex, &total)) {
        fail_all(std::string("exit read-back failed: ") + ems_last_error());
        return;
      }
      for (ems_primary q : ex) {
        const uint32_t row = q.event;
        if (row < slots.size() && slots[row]) {
          q.event = 0;
          slots[row]->exits.push_back(q);
        }
      }
      if (total > ex.size()) {
        std::lock_guard<std::mutex> lk(mu);
        exits_dropped += total - ex.size();
      }
    }
    // events whose last track is gone: their rows come back in one transfer
    std::vector<std::shared_ptr<Request>> finished;
    {
      std::lock_guard<std::mutex> lk(mu);
      chunks += 1;
      for (size_t i = 0; i < slots.size(); ++i)
        if (slots[i] && live[i] == 0) finished.push_back(slots[i]);
    }
    if (!finished.empty()) {
      const uint32_t nf = (uint32_t)finished.size();
      std::vector<uint32_t> rows(nf);
      for (uint32_t i = 0; i < nf; ++i) rows[i] = (uint32_t)finished[i]->slot;
      std::vector<double> edep((size_t)nf * ctx->ncols);
      std::vector<ems_ledger> led(nf);
      if (rt_gather_rows(ctx, rows.data(), nf, edep.data(), led.data())) {
        fail_all(std::string("result read-back failed: ") + ems_last_error());
        return;
      }
      for (uint32_t i = 0; i < nf; ++i) {
        finished[i]->edep.assign(edep.begin() + (size_t)i * ctx->ncols,
                                 edep.begin() + (size_t)(i + 1) * ctx->ncols);
        finished[i]->ledger = led[i];
      }
    }
    if (!finished.empty()) {
      const Clock::time_point now = Clock::now();
      std::lock_guard<std::mutex> lk(mu);
      for (const std::shared_ptr<Request>& r : finished) {
        slots[r->slot].reset();
        free_slots.push_back((uint32_t)r->slot);
        admitted_bytes -= r->bytes;
        in_flight -= 1;
        r->done = true;
        completed += 1;
        prim_completed += r->tracks.size();
        lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
        unfinished.erase(r->ticket);
      }
      cv_done.notify_all();
    }
  }
}

extern "C" {

ems_status ems_server_create(const ems_config* cfg, const ems_geometry* geo, void* d_ws, uint64_t bytes,
                             void* stream, uint64_t admit_cap_bytes, ems_server** out) {
  if (!cfg || !out) return fail(EMS_E_INVALID, "null argument");
  if (cfg->flags & (EMS_F_STEPLOG | EMS_F_PROFILE)) return fail(EMS_E_INVALID, "server: no step log or profile");
  if (admit_cap_bytes == 0) return fail(EMS_E_INVALID, "admit_cap_bytes must be > 0");
  ems_config c2 = *cfg;
  c2.flags |= EMS_F_EVENT_LIVE;
  ems_ctx* ctx = nullptr;
  ems_status st = ems_create(&c2, geo, d_ws, bytes, stream, &ctx);
  if (st) return st;
  ems_server* s = new ems_server();
  s->ctx = ctx;
  s->cap_bytes = admit_cap_bytes;
  s->chunk = cfg->steps_per_launch ? cfg->steps_per_launch : 8;
  s->slots.resize(cfg->max_events);
  for (uint32_t i = cfg->max_events; i-- > 0;) s->free_slots.push_back(i);
  s->t0 = Clock::now();
  s->driver = std::thread([s] { s->run(); });
  *out = s;
  return EMS_OK;
}

ems_status ems_server_submit(ems_server* s, const ems_primary* tracks, uint32_t n, uint32_t key, uint64_t* ticket) {
  return ems_server_submit_at(s, tracks, n, key, 0, ticket);
}

ems_status ems_server_submit_at(ems_server* s, const ems_primary* tracks, uint32_t n, uint32_t key,
                                uint64_t arrival_ns, uint64_t* ticket) {
  if (!s || !ticket || !tracks) return fail(EMS_E_INVALID, "null argument");
  if (n < 1 || n > kMaxTracks) return fail(EMS_E_INVALID, "a request holds 1..65536 tracks");
  auto r = std::make_shared<Request>();
  r->tracks.assign(tracks, tracks + n);
  double etot = 0.0;
  const ems_geometry& g = s->ctx->geo;
  for (uint32_t i = 0; i < n; ++i) {
    ems_primary& q = r->tracks[i];
    q.event = 0;
    const double d2 = q.dir[0] * q.dir[0] + q.dir[1] * q.dir[1] + q.dir[2] * q.dir[2];
    bool ok = q.species <= EMS_POSITRON && q.ekin_MeV > 0.0 && std::isfinite(q.ekin_MeV) && d2 > 0.0 &&
              std::isfinite(d2);
    if (ok && g.n_boxes)
      ok = std::isfinite(q.pos_mm[0]) && std::isfinite(q.pos_mm[1]) && std::isfinite(q.pos_mm[2]) &&
           bvh_locate(s->ctx->nav, q.pos_mm, q.dir) >= 0;
    else if (ok)
      ok = q.pos_mm[2] >= g.z_mm[0] && q.pos_mm[2] <= g.z_mm[g.n_slabs] && std::fabs(q.pos_mm[0]) <= g.half_xy_mm &&
           std::fabs(q.pos_mm[1]) <= g.half_xy_mm;
    if (!ok) return fail(EMS_E_INVALID, "invalid track #" + std::to_string(i));
    r->add[q.species] += 1;
    etot += q.ekin_MeV;
  }
  for (int sp = 0; sp < 3; ++sp)
    if (r->add[sp] > s->ctx->L.cap) return fail(EMS_E_CAPACITY, "request exceeds the track capacity");
  // estimated peak tracks of the event in both queue buffers
  r->bytes = 2 * queue_track_bytes(&s->ctx->cfg) * (uint64_t)(n + 0.1 * etot + 1.0);
  r->key = key;
  // latency counts from the request's arrival (a monotonic-clock time the
  // caller gives, e.g. its scheduled arrival), or from now; never from later
  const Clock::time_point now = Clock::now();
  const Clock::time_point arrival{std::chrono::duration_cast<Clock::duration>(std::chrono::nanoseconds(arrival_ns))};
  r->t_submit = arrival_ns != 0 && arrival < now ? arrival : now;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed) return fail(EMS_E_STATE, s->fail_msg);
  if (s->queue.size() >= kMaxQueued) return fail(EMS_E_BUSY, "request queue full");
  r->ticket = s->next_ticket++;
  s->tickets[r->ticket] = r;
  s->unfinished.insert(r->ticket);
  s->queue.push_back(r);
  s->submitted += 1;
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return EMS_OK;
}

ems_status ems_server_wait(ems_server* s, uint64_t ticket, int64_t timeout_us, double* edep_out,
                           ems_ledger* ledger_out) {
  return ems_server_wait_exits(s, ticket, timeout_us, edep_out, ledger_out, nullptr, 0, nullptr);
}

ems_status ems_server_wait_exits(ems_server* s, uint64_t ticket, int64_t timeout_us, double* edep_out,
                                 ems_ledger* ledger_out, ems_primary* exits_out, uint64_t exits_cap,
                                 uint64_t* n_exits) {
  if (!s) return fail(EMS_E_INVALID, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(EMS_E_INVALID, "unknown ticket");
  std::shared_ptr<Request> r = it->second;
  auto ready = [&] { return r->done || s->failed; };
  if (timeout_us < 0) s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
    return fail(EMS_E_TIMEOUT, "request not finished yet");
  if (!r->done) return fail(EMS_E_STATE, s->fail_msg);
  if (n_exits) {
    *n_exits = r->exits.size();
    // too small a buffer: report the size and keep the result for a retry
    if (r->exits.size() > exits_cap) return fail(EMS_E_CAPACITY, "exit buffer too small");
    if (exits_out) std::copy(r->exits.begin(), r->exits.end(), exits_out);
  }
  if (edep_out) std::copy(r->edep.begin(), r->edep.end(), edep_out);
  if (ledger_out) *ledger_out = r->ledger;
  s->tickets.erase(ticket);
  return EMS_OK;
}

ems_status ems_server_poll(ems_server* s, uint64_t ticket, int* done) {
  if (!s || !done) return fail(EMS_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(EMS_E_INVALID, "unknown ticket");
  if (s->failed) return fail(EMS_E_STATE, s->fail_msg);
  *done = it->second->done ? 1 : 0;
  return EMS_OK;
}

ems_status ems_server_flush(ems_server* s) {
  if (!s) return fail(EMS_E_INVALID, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  const uint64_t target = s->next_ticket - 1;
  s->cv_done.wait(lk, [&] { return s->failed || s->unfinished.empty() || *s->unfinished.begin() > target; });
  if (s->failed) return fail(EMS_E_STATE, s->fail_msg);
  return EMS_OK;
}

ems_status ems_server_stats(ems_server* s, ems_server_info* out) {
  if (!s || !out) return fail(EMS_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  ems_server_info st{};
  st.submitted = s->submitted;
  st.completed = s->completed;
  st.in_flight = s->in_flight;
  st.queued = s->queue.size();
  st.admitted_bytes = s->admitted_bytes;
  st.admit_cap_bytes = s->cap_bytes;
  st.peak_admitted_bytes = s->peak_bytes;
  st.primaries_completed = s->prim_completed;
  st.chunks = s->chunks;
  st.exits_dropped = s->exits_dropped;
  std::vector<double> v = s->lat_ms;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto q = [&](double f) { return v[std::min(v.size() - 1, (size_t)(f * (v.size() - 1) + 0.5))]; };
    st.p50_ms = q(0.50);
    st.p99_ms = q(0.99);
    double sum = 0.0;
    for (double x : v) sum += x;
    st.mean_ms = sum / v.size();
    st.max_ms = v.back();
  }
  st.wall_s = std::chrono::duration<double>(Clock::now() - s->t0).count();
  st.primaries_per_s = st.wall_s > 0 ? st.primaries_completed / st.wall_s : 0.0;
  *out = st;
  return EMS_OK;
}

ems_status ems_server_reset_stats(ems_server* s) {
  if (!s) return fail(EMS_E_INVALID, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  s->lat_ms.clear();
  s->completed = s->prim_completed = s->submitted = s->chunks = 0;
  s->peak_bytes = s->admitted_bytes;
  s->t0 = Clock::now();
  return EMS_OK;
}

ems_status ems_server_drive(ems_server* s, const ems_load_request* reqs, const uint64_t* first,
                            uint32_t n_producers, uint32_t window, double* max_lag_ms, uint64_t* last_submit_ns) {
  if (!s || !reqs || !first || n_producers == 0 || window == 0) return fail(EMS_E_INVALID, "null argument or zero count");
  for (uint32_t p = 0; p < n_producers; ++p)
    if (first[p] > first[p + 1]) return fail(EMS_E_INVALID, "request ranges must not decrease");
  std::mutex mu;
  ems_status first_err = EMS_OK;
  std::string err_msg;
  int64_t lag_ns = 0, last_ns = 0;
  auto record = [&](ems_status st) {
    std::lock_guard<std::mutex> lk(mu);
    if (first_err == EMS_OK) {
      first_err = st;
      err_msg = ems_last_error();
    }
  };
  auto producer = [&](uint32_t p) {
    std::deque<uint64_t> out;
    int64_t my_lag = 0, my_last = 0;
    for (uint64_t i = first[p]; i < first[p + 1]; ++i) {
      const ems_load_request& r = reqs[i];
      if (r.arrival_ns == 0) {
        while (out.size() >= window) {
          const ems_status st = ems_server_wait(s, out.front(), -1, nullptr, nullptr);
          out.pop_front();
          if (st) return record(st);
        }
      } else {
        const Clock::time_point due{std::chrono::duration_cast<Clock::duration>(std::chrono::nanoseconds(r.arrival_ns))};
        std::this_thread::sleep_until(due);
        my_lag = std::max<int64_t>(my_lag, std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - due).count());
      }
      uint64_t t = 0;
      const ems_status st = ems_server_submit_at(s, r.tracks, r.n_tracks, r.event_key, r.arrival_ns, &t);
      if (st) return record(st);
      my_last = std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count();
      out.push_back(t);
    }
    for (uint64_t t : out) {
      const ems_status st = ems_server_wait(s, t, -1, nullptr, nullptr);
      if (st) return record(st);
    }
    std::lock_guard<std::mutex> lk(mu);
    lag_ns = std::max(lag_ns, my_lag);
    last_ns = std::max(last_ns, my_last);
  };
  std::vector<std::thread> th;
  for (uint32_t p = 0; p < n_producers; ++p) th.emplace_back(producer, p);
  for (std::thread& t : th) t.join();
  if (max_lag_ms) *max_lag_ms = lag_ns / 1e6;
  if (last_submit_ns) *last_submit_ns = (uint64_t)last_ns;
  if (first_err) return fail(first_err, err_msg);
  return EMS_OK;
}

ems_status ems_server_destroy(ems_server* s) {
  if (!s) return EMS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->driver.joinable()) s->driver.join();
  ems_destroy(s->ctx);
  delete s;
  return EMS_OK;
}

}  // extern "C"
