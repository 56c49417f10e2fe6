// Serving loop: continuous batching of uplink detection frames.
//
// Frames of mixed shapes arrive through dbp_server_submit (caller-owned pinned
// host buffers for H, y and the results).  A scheduler thread admits them in
// arrival order whenever a stream slot is free and the frame's device
// footprint fits in what is left of the HBM budget (a device arena allocated
// once at creation), then enqueues host-to-device copies, the detection kernel
// and device-to-host copies on the slot's stream.  Admitted frames run
// concurrently on the device; finished frames give their arena space and slot
// back, so a waiting frame is admitted as soon as resources free up.  Per-frame
// latency runs from submit to the completion of the result copy.
//
// Static channels: dbp_channel_load copies H into the arena and factors it
// once (B_c^{-1} per subcarrier and cluster, resident until dbp_channel_free);
// frames submitted with dbp_server_submit_factored carry only y and run the
// iterations against those resident factors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dbp.h"

namespace {

using Clock = std::chrono::steady_clock;

double us_since(Clock::time_point t0, Clock::time_point t1) {
  return std::chrono::duration<double, std::micro>(t1 - t0).count();
}

// First-fit allocator over one device block; offsets are 256-byte aligned.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t start = it->first + n;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Channel {
  size_t off = 0, footprint = 0;     // arena block: H (complex64 or packed FP16), then the factors
  size_t bytes_H = 0;
  bool h16 = false;                  // H kept as the packed FP16 channel
  int n_sc = 0, B = 0, U = 0, C = 0;
  float rho = 0.f;
  hipEvent_t ready = nullptr;        // recorded after the factorisation
  int refs = 0;                      // frames queued or in flight against it
};

struct Frame {
  uint64_t ticket;
  uint64_t channel = 0;              // nonzero: detect against a resident channel
  const void* H;
  const void* y;
  void* s_out;
  uint8_t* hard_out;
  int n_sc, n_sym, B, U, C, T, qam, prec, reg, flags;
  float rho, N0;
  size_t bytes_H, bytes_y, bytes_s, bytes_hard, bytes_ws, footprint;
  size_t off = 0;
  int slot = -1;
  int status = DBP_OK;
  bool done = false;
  Clock::time_point t_arrive, t_admit, t_done;
};

}  // namespace

struct dbp_server {
  int device = 0;
  void* base = nullptr;
  Arena* arena = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<std::vector<uint64_t>> slot_frames;   // frames in flight on each slot (empty = free)
  int max_batch = 8;                  // frames one launch may take (1: no batching)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::map<uint64_t, Frame> frames;
  uint64_t next_ticket = 1;
  std::map<uint64_t, Channel> channels;
  uint64_t next_channel = 1;
  size_t channel_bytes = 0;          // arena space held by resident channels
  hipStream_t load_stream = nullptr;
  std::atomic<bool> stop{false};
  std::thread worker;
  std::string error;
  size_t peak_used = 0;
  int peak_inflight = 0;
  uint64_t completed = 0;
};

namespace {

// Frames against a resident channel: wait for its factorisation, then copy y,
// run the factored iterations and copy the results back.
int launch_factored(dbp_server* s, Frame& f, hipStream_t st) {
  const Channel& ch = s->channels.at(f.channel);
  const char* cbase = static_cast<const char*>(s->base) + ch.off;
  const void* dH = cbase;
  const void* dF = cbase + ((ch.bytes_H + 255) & ~size_t(255));
  if (hipStreamWaitEvent(st, ch.ready, 0) != hipSuccess) return DBP_ERR_DEVICE;
  const void* y = f.y;
  void* so = f.s_out;
  uint8_t* ho = f.hard_out;
  char* ws = static_cast<char*>(s->base) + f.off;   // re-slice workspace first in the frame's block
  char* d = ws + f.bytes_ws;
  if (!(f.flags & DBP_SERVE_DEVICE_IO)) {
    char* dy = d;
    char* ds = dy + ((f.bytes_y + 255) & ~size_t(255));
    char* dh = ds + ((f.bytes_s + 255) & ~size_t(255));
    if (hipMemcpyAsync(dy, f.y, f.bytes_y, hipMemcpyHostToDevice, st) != hipSuccess) return DBP_ERR_DEVICE;
    y = dy;
    so = ds;
    ho = f.hard_out ? reinterpret_cast<uint8_t*>(dh) : nullptr;
  }
  int rc = ch.h16 ? dbp_detect_admm_factored_h16(dH, dF, y, so, ho, nullptr, f.n_sc, f.n_sym, f.B, f.U, f.C, f.T,
                                                  f.rho, 1.0f, f.N0, 1.0f, f.reg, f.qam, st)
                  : dbp_detect_admm_factored(dH, dF, y, so, ho, nullptr, f.bytes_ws ? ws : nullptr, f.bytes_ws,
                                             f.n_sc, f.n_sym, f.B, f.U, f.C, f.T, f.rho, 1.0f, f.N0, 1.0f, f.reg,
                                             f.qam, st);
  if (rc != DBP_OK) return rc;
  if (!(f.flags & DBP_SERVE_DEVICE_IO)) {
    if (hipMemcpyAsync(f.s_out, so, f.bytes_s, hipMemcpyDeviceToHost, st) != hipSuccess) return DBP_ERR_DEVICE;
    if (f.hard_out && hipMemcpyAsync(f.hard_out, ho, f.bytes_hard, hipMemcpyDeviceToHost, st) != hipSuccess)
      return DBP_ERR_DEVICE;
  }
  return hipEventRecord(s->events[f.slot], st) == hipSuccess ? DBP_OK : DBP_ERR_DEVICE;
}

// Enqueue copies + detection for an admitted frame on its slot's stream.
int launch_frame(dbp_server* s, Frame& f) {
  hipStream_t st = s->streams[f.slot];
  if (f.channel) return launch_factored(s, f, st);
  char* ws = static_cast<char*>(s->base) + f.off;   // re-slice workspace first in the frame's block
  void* wsp = f.bytes_ws ? ws : nullptr;
  if (f.flags & DBP_SERVE_DEVICE_IO) {
    // inputs and outputs already in device memory: beyond the workspace the
    // arena space only accounts for the frame's share of the budget
    int rc = dbp_detect_admm(f.H, f.y, f.s_out, f.hard_out, nullptr, wsp, f.bytes_ws, f.n_sc, f.n_sym, f.B, f.U,
                             f.C, f.T, f.rho, 1.0f, f.N0, 1.0f, f.reg, f.qam, f.prec, st);
    if (rc != DBP_OK) return rc;
    return hipEventRecord(s->events[f.slot], st) == hipSuccess ? DBP_OK : DBP_ERR_DEVICE;
  }
  char* d = ws + f.bytes_ws;
  char* dH = d;
  char* dy = dH + ((f.bytes_H + 255) & ~size_t(255));
  char* ds = dy + ((f.bytes_y + 255) & ~size_t(255));
  char* dh = ds + ((f.bytes_s + 255) & ~size_t(255));
  if (hipMemcpyAsync(dH, f.H, f.bytes_H, hipMemcpyHostToDevice, st) != hipSuccess) return DBP_ERR_DEVICE;
  if (hipMemcpyAsync(dy, f.y, f.bytes_y, hipMemcpyHostToDevice, st) != hipSuccess) return DBP_ERR_DEVICE;
  int rc = dbp_detect_admm(dH, dy, ds, f.hard_out ? reinterpret_cast<uint8_t*>(dh) : nullptr, nullptr, wsp,
                           f.bytes_ws, f.n_sc, f.n_sym, f.B, f.U, f.C, f.T, f.rho, 1.0f, f.N0, 1.0f, f.reg, f.qam,
                           f.prec, st);
  if (rc != DBP_OK) return rc;
  if (hipMemcpyAsync(f.s_out, ds, f.bytes_s, hipMemcpyDeviceToHost, st) != hipSuccess) return DBP_ERR_DEVICE;
  if (f.hard_out && hipMemcpyAsync(f.hard_out, dh, f.bytes_hard, hipMemcpyDeviceToHost, st) != hipSuccess)
    return DBP_ERR_DEVICE;
  if (hipEventRecord(s->events[f.slot], st) != hipSuccess) return DBP_ERR_DEVICE;
  return DBP_OK;
}

// The arena block of a frame starts with its re-slice workspace; a host-I/O
// frame's copies of H, y and the outputs follow.
struct DevIO {
  const void* H;
  const void* y;
  void* s;
  uint8_t* hard;
  void* ws;
};

DevIO device_io(dbp_server* s, const Frame& f) {
  char* ws = static_cast<char*>(s->base) + f.off;
  if (f.flags & DBP_SERVE_DEVICE_IO) return DevIO{f.H, f.y, f.s_out, f.hard_out, f.bytes_ws ? ws : nullptr};
  auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
  char* dH = ws + f.bytes_ws;
  char* dy = dH + al(f.bytes_H);
  char* ds = dy + al(f.bytes_y);
  char* dh = ds + al(f.bytes_s);
  return DevIO{dH, dy, ds, f.hard_out ? reinterpret_cast<uint8_t*>(dh) : nullptr, f.bytes_ws ? ws : nullptr};
}

// Several admitted frames of one U (FP32, not against a resident channel) in
// one dbp_detect_admm_batch launch on the slot's stream, with each host-I/O
// frame's copies before and after it.
int launch_batch(dbp_server* s, const std::vector<Frame*>& fs, int slot) {
  hipStream_t st = s->streams[slot];
  dbp_frame d[DBP_MAX_BATCH];
  for (size_t i = 0; i < fs.size(); ++i) {
    const Frame& f = *fs[i];
    const DevIO io = device_io(s, f);
    if (!(f.flags & DBP_SERVE_DEVICE_IO)) {
      if (hipMemcpyAsync(const_cast<void*>(io.H), f.H, f.bytes_H, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(const_cast<void*>(io.y), f.y, f.bytes_y, hipMemcpyHostToDevice, st) != hipSuccess)
        return DBP_ERR_DEVICE;
    }
    d[i] = dbp_frame{io.H, io.y, io.s, io.hard, nullptr, io.ws, f.bytes_ws, f.n_sc, f.n_sym, f.B, f.C, f.T,
                     f.reg, f.qam, f.rho, 1.0f, f.N0, 1.0f};
  }
  int rc = dbp_detect_admm_batch(d, int(fs.size()), fs[0]->U, st);
  if (rc != DBP_OK) return rc;
  for (size_t i = 0; i < fs.size(); ++i) {
    const Frame& f = *fs[i];
    if (f.flags & DBP_SERVE_DEVICE_IO) continue;
    if (hipMemcpyAsync(f.s_out, d[i].s_hat, f.bytes_s, hipMemcpyDeviceToHost, st) != hipSuccess) return DBP_ERR_DEVICE;
    if (f.hard_out && hipMemcpyAsync(f.hard_out, d[i].hard, f.bytes_hard, hipMemcpyDeviceToHost, st) != hipSuccess)
      return DBP_ERR_DEVICE;
  }
  return hipEventRecord(s->events[slot], st) == hipSuccess ? DBP_OK : DBP_ERR_DEVICE;
}

bool batchable(const Frame& f) { return f.channel == 0 && f.prec == DBP_PREC_FP32; }

void scheduler(dbp_server* s) {
  // dbp_server_create made this device current successfully before starting
  // the thread, so the call cannot fail here
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop.load()) {
    bool progressed = false;
    // completions
    int inflight = 0;
    for (size_t i = 0; i < s->slot_frames.size(); ++i) {
      std::vector<uint64_t>& ts = s->slot_frames[i];
      if (ts.empty()) continue;
      const hipError_t q = hipEventQuery(s->events[i]);
      if (q != hipErrorNotReady) {
        const auto now = Clock::now();
        for (uint64_t t : ts) {
          Frame& f = s->frames[t];
          f.t_done = now;
          f.done = true;
          if (q != hipSuccess) f.status = DBP_ERR_DEVICE;
          s->arena->release(f.off, f.footprint);
          if (f.channel) --s->channels[f.channel].refs;
          ++s->completed;
        }
        ts.clear();
        progressed = true;
      } else {
        inflight += int(ts.size());
      }
    }
    // admissions, in arrival order; a batchable frame at the head takes up
    // to max_batch - 1 more batchable frames of the same U and I/O mode from
    // the next queued ones into its launch
    while (!s->queue.empty()) {
      auto free_slot = std::find_if(s->slot_frames.begin(), s->slot_frames.end(),
                                    [](const std::vector<uint64_t>& v) { return v.empty(); });
      if (free_slot == s->slot_frames.end()) break;
      const int slot = int(free_slot - s->slot_frames.begin());
      Frame& f = s->frames[s->queue.front()];
      size_t off;
      if (!s->arena->alloc(f.footprint, &off)) break;
      f.off = off;
      f.slot = slot;
      f.t_admit = Clock::now();
      s->queue.pop_front();
      std::vector<Frame*> batch{&f};
      if (batchable(f) && s->max_batch > 1) {
        constexpr size_t kScan = 64;
        for (auto it = s->queue.begin(); it != s->queue.end() && int(batch.size()) < s->max_batch &&
                                         size_t(it - s->queue.begin()) < kScan;) {
          Frame& g = s->frames[*it];
          if (batchable(g) && g.U == f.U && g.flags == f.flags && s->arena->alloc(g.footprint, &off)) {
            g.off = off;
            g.slot = slot;
            g.t_admit = f.t_admit;
            batch.push_back(&g);
            it = s->queue.erase(it);
          } else {
            ++it;
          }
        }
      }
      const int rc = batch.size() > 1 ? launch_batch(s, batch, slot) : launch_frame(s, f);
      if (rc != DBP_OK) {
        // nothing more of these frames runs: drain what was enqueued before
        // the failure, then release and report (a failing drain leaves the
        // error in the status too)
        (void)hipStreamSynchronize(s->streams[slot]);
        for (Frame* g : batch) {
          s->arena->release(g->off, g->footprint);
          if (g->channel) --s->channels[g->channel].refs;
          g->status = rc;
          g->done = true;
          g->t_done = Clock::now();
        }
        progressed = true;   // wakes callers waiting on these tickets
        continue;
      }
      for (Frame* g : batch) free_slot->push_back(g->ticket);
      inflight += int(batch.size());
      progressed = true;
    }
    s->peak_used = std::max(s->peak_used, s->arena->used());
    s->peak_inflight = std::max(s->peak_inflight, inflight);
    if (progressed) s->cv.notify_all();
    if (inflight == 0 && s->queue.empty()) {
      s->cv.wait(lk, [&] { return s->stop.load() || !s->queue.empty(); });
    } else {
      // poll completions without holding the lock; yielding (instead of a
      // timed sleep) keeps completion timestamps within about a microsecond
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    }
  }
}

int qam_ok(int q) { return q == 4 || q == 16 || q == 64; }

// Releases everything a server holds (streams and events that exist, the
// arena, the object).  Returns DBP_ERR_DEVICE if a release call failed.
int release_server(dbp_server* s) {
  bool ok = true;
  for (auto st : s->streams)
    if (st) ok &= hipStreamDestroy(st) == hipSuccess;
  for (auto ev : s->events)
    if (ev) ok &= hipEventDestroy(ev) == hipSuccess;
  for (auto& kv : s->channels) ok &= hipEventDestroy(kv.second.ready) == hipSuccess;
  if (s->load_stream) ok &= hipStreamDestroy(s->load_stream) == hipSuccess;
  if (s->base) ok &= hipFree(s->base) == hipSuccess;
  delete s->arena;
  delete s;
  return ok ? DBP_OK : DBP_ERR_DEVICE;
}

}  // namespace

extern "C" {

int dbp_server_create(int device, size_t hbm_budget_bytes, int n_slots, dbp_server** out) {
  if (!out || n_slots < 1 || n_slots > 64 || hbm_budget_bytes < 4096) return DBP_ERR_INVALID;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return DBP_ERR_DEVICE;
  auto* s = new dbp_server();
  s->device = device;
  if (hipMalloc(&s->base, hbm_budget_bytes) != hipSuccess) {
    s->base = nullptr;
    release_server(s);
    return DBP_ERR_NOMEM;
  }
  s->arena = new Arena(hbm_budget_bytes);
  s->streams.assign(n_slots, nullptr);
  s->events.assign(n_slots, nullptr);
  s->slot_frames.assign(n_slots, {});
  for (int i = 0; i < n_slots; ++i) {
    if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->events[i], hipEventDisableTiming) != hipSuccess) {
      release_server(s);
      return DBP_ERR_DEVICE;
    }
  }
  if (hipStreamCreateWithFlags(&s->load_stream, hipStreamNonBlocking) != hipSuccess) {
    release_server(s);
    return DBP_ERR_DEVICE;
  }
  s->worker = std::thread(scheduler, s);
  *out = s;
  return DBP_OK;
}

int dbp_server_destroy(dbp_server* s) {
  if (!s) return DBP_ERR_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop.store(true);
  }
  s->cv.notify_all();
  s->worker.join();
  bool ok = true;
  for (auto st : s->streams) ok &= hipStreamSynchronize(st) == hipSuccess;
  ok &= hipStreamSynchronize(s->load_stream) == hipSuccess;
  const int rc = release_server(s);
  return ok ? rc : DBP_ERR_DEVICE;
}

int dbp_server_submit(dbp_server* s, const void* H_host, const void* y_host, void* s_hat_host, uint8_t* hard_host,
                      int n_sc, int n_sym, int B, int U, int C, int T, float rho, float N0, int reg, int qam,
                      int prec, int flags, uint64_t* ticket) {
  if (!s || !ticket || !H_host || !y_host || !s_hat_host) return DBP_ERR_INVALID;
  if (n_sc < 1 || n_sym < 1 || B < 1 || U < 1 || C < 1 || B % C || U > B / C || T < 1 || !qam_ok(qam) ||
      !(rho > 0.f) || !(N0 >= 0.f) || (flags & ~DBP_SERVE_DEVICE_IO))
    return DBP_ERR_INVALID;
  // every other argument check of the detection call (precision, regulariser,
  // built shapes): with n_sc = 0 it validates and queues nothing, so a frame
  // the library would refuse is refused here instead of at admission
  const int vrc = dbp_detect_admm(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, n_sym, B, U, C, T, rho,
                                  1.0f, N0, 1.0f, reg, qam, prec, nullptr);
  if (vrc != DBP_OK) return vrc;
  Frame f{};
  f.H = H_host;
  f.y = y_host;
  f.s_out = s_hat_host;
  f.hard_out = hard_host;
  f.n_sc = n_sc;
  f.n_sym = n_sym;
  f.B = B;
  f.U = U;
  f.C = C;
  f.T = T;
  f.qam = qam;
  f.prec = prec;
  f.reg = reg;
  f.flags = flags;
  f.rho = rho;
  f.N0 = N0;
  f.bytes_H = size_t(n_sc) * B * U * 8;
  f.bytes_y = size_t(n_sc) * n_sym * B * 8;
  f.bytes_s = size_t(n_sc) * n_sym * U * 8;
  f.bytes_hard = size_t(n_sc) * n_sym * U;
  auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
  f.bytes_ws = hard_host ? al(dbp_detect_workspace_bytes(n_sc, U, C)) : 0;
  f.footprint = f.bytes_ws + al(f.bytes_H) + al(f.bytes_y) + al(f.bytes_s) + al(f.bytes_hard);
  f.t_arrive = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (f.footprint > s->arena->size() - s->channel_bytes) return DBP_ERR_NOMEM;   // can never be admitted
  f.ticket = s->next_ticket++;
  *ticket = f.ticket;
  s->frames.emplace(f.ticket, f);
  s->queue.push_back(f.ticket);
  s->cv.notify_all();
  return DBP_OK;
}

int dbp_channel_load(dbp_server* s, const void* H, int n_sc, int B, int U, int C, float rho, int prec, int flags,
                     uint64_t* channel) {
  if (!s || !H || !channel) return DBP_ERR_INVALID;
  if (n_sc < 1 || B < 1 || U < 1 || C < 1 || B % C || U > B / C || !(rho > 0.f) ||
      (flags & ~(DBP_SERVE_DEVICE_IO | DBP_CHANNEL_H16)))
    return DBP_ERR_INVALID;
  Channel ch;
  ch.n_sc = n_sc;
  ch.B = B;
  ch.U = U;
  ch.C = C;
  ch.rho = rho;
  ch.h16 = (flags & DBP_CHANNEL_H16) != 0;
  const size_t bytes_H32 = size_t(n_sc) * B * U * 8;
  ch.bytes_H = ch.h16 ? dbp_channel_h16_bytes(n_sc, B, U, C) : bytes_H32;
  ch.footprint = ((ch.bytes_H + 255) & ~size_t(255)) + dbp_factor_bytes(n_sc, U, C);
  // a packed channel is made from a complex64 copy of H held in a second,
  // temporary block until the packing and the factorisation have run
  size_t tmp_off = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->arena->alloc(ch.footprint, &ch.off)) return DBP_ERR_NOMEM;
    if (ch.h16 && !s->arena->alloc(bytes_H32, &tmp_off)) {
      s->arena->release(ch.off, ch.footprint);
      return DBP_ERR_NOMEM;
    }
    s->peak_used = std::max(s->peak_used, s->arena->used());
  }
  // The blocks are reserved and known to no one else yet: copy H outside the
  // lock (synchronously, so the caller may release H on return), then queue
  // the factorisation (and the packing) and mark its completion.
  char* d = static_cast<char*>(s->base) + ch.off;
  char* d32 = ch.h16 ? static_cast<char*>(s->base) + tmp_off : d;
  void* dF = d + ((ch.bytes_H + 255) & ~size_t(255));
  const hipMemcpyKind kind = (flags & DBP_SERVE_DEVICE_IO) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  int rc = DBP_OK;
  if (hipEventCreateWithFlags(&ch.ready, hipEventDisableTiming) != hipSuccess ||
      hipMemcpyAsync(d32, H, bytes_H32, kind, s->load_stream) != hipSuccess ||
      hipStreamSynchronize(s->load_stream) != hipSuccess)
    rc = DBP_ERR_DEVICE;
  if (rc == DBP_OK)
    rc = ch.h16 ? dbp_factor_admm_h16(d32, dF, d, n_sc, B, U, C, rho, prec, s->load_stream)
                : dbp_factor_admm(d32, dF, n_sc, B, U, C, rho, prec, s->load_stream);
  if (rc == DBP_OK && hipEventRecord(ch.ready, s->load_stream) != hipSuccess) rc = DBP_ERR_DEVICE;
  // the temporary block is returned only once the load stream is past it
  if (ch.h16 && hipStreamSynchronize(s->load_stream) != hipSuccess && rc == DBP_OK) rc = DBP_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ch.h16) s->arena->release(tmp_off, bytes_H32);
  if (rc != DBP_OK) {
    // drain the load stream before its block is handed out again; rc already
    // reports the failure
    (void)hipStreamSynchronize(s->load_stream);
    if (ch.ready) (void)hipEventDestroy(ch.ready);
    s->arena->release(ch.off, ch.footprint);
    return rc;
  }
  s->channel_bytes += (ch.footprint + 255) & ~size_t(255);
  *channel = s->next_channel++;
  s->channels.emplace(*channel, ch);
  return DBP_OK;
}

int dbp_channel_free(dbp_server* s, uint64_t channel) {
  if (!s) return DBP_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->channels.find(channel);
  if (it == s->channels.end()) return DBP_ERR_NOTFOUND;
  if (it->second.refs > 0) return DBP_ERR_BUSY;
  // the factorisation must be finished before its memory can be handed out again
  const bool ok = hipEventSynchronize(it->second.ready) == hipSuccess &&
                  hipEventDestroy(it->second.ready) == hipSuccess;
  s->arena->release(it->second.off, it->second.footprint);
  s->channel_bytes -= (it->second.footprint + 255) & ~size_t(255);
  s->channels.erase(it);
  return ok ? DBP_OK : DBP_ERR_DEVICE;
}

int dbp_server_submit_factored(dbp_server* s, uint64_t channel, const void* y, void* s_hat, uint8_t* hard, int n_sym,
                               int T, float N0, int reg, int qam, int flags, uint64_t* ticket) {
  if (!s || !ticket || !y || !s_hat) return DBP_ERR_INVALID;
  if (n_sym < 1 || T < 1 || !qam_ok(qam) || !(N0 >= 0.f) || (flags & ~DBP_SERVE_DEVICE_IO)) return DBP_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->channels.find(channel);
  if (it == s->channels.end()) return DBP_ERR_NOTFOUND;
  Channel& ch = it->second;
  // argument checks of the detection call (n_sc = 0: validation only)
  const int vrc = dbp_detect_admm_factored(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0, n_sym,
                                           ch.B, ch.U, ch.C, T, ch.rho, 1.0f, N0, 1.0f, reg, qam, nullptr);
  if (vrc != DBP_OK) return vrc;
  Frame f{};
  f.channel = channel;
  f.H = nullptr;
  f.y = y;
  f.s_out = s_hat;
  f.hard_out = hard;
  f.n_sc = ch.n_sc;
  f.n_sym = n_sym;
  f.B = ch.B;
  f.U = ch.U;
  f.C = ch.C;
  f.T = T;
  f.qam = qam;
  f.prec = 0;
  f.reg = reg;
  f.flags = flags;
  f.rho = ch.rho;
  f.N0 = N0;
  f.bytes_H = 0;
  f.bytes_y = size_t(f.n_sc) * n_sym * f.B * 8;
  f.bytes_s = size_t(f.n_sc) * n_sym * f.U * 8;
  f.bytes_hard = size_t(f.n_sc) * n_sym * f.U;
  auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
  f.bytes_ws = (hard && !ch.h16) ? al(dbp_detect_workspace_bytes(f.n_sc, f.U, f.C)) : 0;
  f.footprint = f.bytes_ws + al(f.bytes_y) + al(f.bytes_s) + al(f.bytes_hard);
  f.t_arrive = Clock::now();
  // a frame that does not fit beside the resident channels could never be admitted
  if (f.footprint > s->arena->size() - s->channel_bytes) return DBP_ERR_NOMEM;
  ++ch.refs;
  f.ticket = s->next_ticket++;
  *ticket = f.ticket;
  s->frames.emplace(f.ticket, f);
  s->queue.push_back(f.ticket);
  s->cv.notify_all();
  return DBP_OK;
}

int dbp_server_poll(dbp_server* s, uint64_t ticket, int* done, double* latency_us) {
  if (!s || !done) return DBP_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->frames.find(ticket);
  if (it == s->frames.end()) return DBP_ERR_NOTFOUND;
  *done = it->second.done ? 1 : 0;
  if (latency_us) *latency_us = it->second.done ? us_since(it->second.t_arrive, it->second.t_done) : -1.0;
  return it->second.done ? it->second.status : DBP_OK;
}

int dbp_server_wait(dbp_server* s, uint64_t ticket, double* latency_us, double* queue_us) {
  if (!s) return DBP_ERR_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->frames.find(ticket);
  if (it == s->frames.end()) return DBP_ERR_NOTFOUND;
  s->cv.wait(lk, [&] { return it->second.done; });
  if (latency_us) *latency_us = us_since(it->second.t_arrive, it->second.t_done);
  if (queue_us) *queue_us = it->second.slot >= 0 ? us_since(it->second.t_arrive, it->second.t_admit) : -1.0;
  const int st = it->second.status;
  s->frames.erase(it);
  return st;
}

int dbp_server_set_batching(dbp_server* s, int max_frames) {
  if (!s || max_frames < 1 || max_frames > DBP_MAX_BATCH) return DBP_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  s->max_batch = max_frames;
  return DBP_OK;
}

int dbp_server_stats(dbp_server* s, size_t* peak_bytes, int* peak_inflight, uint64_t* completed) {
  if (!s) return DBP_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (peak_bytes) *peak_bytes = s->peak_used;
  if (peak_inflight) *peak_inflight = s->peak_inflight;
  if (completed) *completed = s->completed;
  return DBP_OK;
}

}  // extern "C"
