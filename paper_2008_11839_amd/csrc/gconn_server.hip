// gconn_server.hip -- continuous-batching request loop for incremental
// connectivity (gconn_server_* in include/gconn.h).  Host code only: the
// device work is the incremental insert / query kernels of gconn_static.hip.
//
// One worker thread owns every copy, launch, event and stream call after
// creation (submit only asks whether the caller's buffers are pinned).  Its
// loop:
//   1. admit the next pending request, in submission order, when the device
//      arena and the pinned staging area have room for it (first-fit
//      allocator, 256-byte granules); a request that does not fit stops
//      admission until earlier requests complete and free space;
//   2. on admission: copy the request's host data into pinned staging (unless
//      the caller's buffers are pinned already: then the copy engines read
//      and write them directly), pick the next stream round-robin; if its
//      kind differs from the current epoch's, open a new epoch by recording
//      one fence event on every stream; enqueue the H2D copies, make the
//      stream wait on the current epoch's fences, then enqueue the kernel,
//      (queries) the D2H of the answers, and a completion event;
//   3. poll completion events after every admission; for finished queries
//      copy the answers from staging into the caller's buffer; free the arena
//      space; publish the request record and wake waiters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gconn_internal.hpp"

namespace gconn {
namespace {

constexpr uint64_t kGranule = 256;
constexpr uint64_t kInsertChunk = 4u << 20;  // pairs per staged chunk of a large batch

// Host copy into pinned staging, split over a few threads for large requests:
// one thread's memcpy (~10 GB/s) would otherwise cap the host-fed rate well
// below what the host-to-device link carries.
void staged_copy(void* dst, const void* src, size_t bytes) {
  constexpr size_t kChunk = 2u << 20;
  const size_t parts = std::min<size_t>(8, bytes / kChunk);
  if (parts < 2) {
    std::memcpy(dst, src, bytes);
    return;
  }
  std::vector<std::thread> ts;
  const size_t per = (bytes + parts - 1) / parts;
  for (size_t i = 1; i < parts; ++i) {
    const size_t lo = i * per, len = std::min(bytes, lo + per) - lo;
    ts.emplace_back([=] {
      std::memcpy(static_cast<char*>(dst) + lo, static_cast<const char*>(src) + lo, len);
    });
  }
  std::memcpy(dst, src, std::min(per, bytes));
  for (auto& t : ts) t.join();
}

// Largest vertex id of a request's two host arrays, split over a few threads
// for large requests like the staging copy.  Every id reaches the device
// kernels unchecked, and the parent array is shared by every client of the
// server, so submission rejects ids >= n_max before anything is queued.
uint32_t host_max_id(const uint32_t* a, const uint32_t* b, uint64_t count) {
  auto part_max = [](const uint32_t* x, const uint32_t* y, uint64_t lo, uint64_t hi) {
    uint32_t m = 0;
    for (uint64_t i = lo; i < hi; ++i) {
      const uint32_t t = x[i] > y[i] ? x[i] : y[i];
      m = t > m ? t : m;
    }
    return m;
  };
  constexpr uint64_t kPart = 1u << 20;
  const uint64_t parts = std::min<uint64_t>(8, count / kPart);
  if (parts < 2) return part_max(a, b, 0, count);
  std::vector<uint32_t> got(parts, 0);
  std::vector<std::thread> ts;
  const uint64_t per = (count + parts - 1) / parts;
  for (uint64_t i = 1; i < parts; ++i) {
    const uint64_t lo = i * per, hi = std::min(count, lo + per);
    ts.emplace_back([&, i, lo, hi] { got[i] = part_max(a, b, lo, hi); });
  }
  got[0] = part_max(a, b, 0, std::min(count, per));
  for (auto& t : ts) t.join();
  return *std::max_element(got.begin(), got.end());
}

// First-fit allocator over [0, size) with coalescing of free ranges.
class RangeAlloc {
 public:
  explicit RangeAlloc(uint64_t size) { if (size) free_[0] = size; }
  bool alloc(uint64_t bytes, uint64_t* at) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        *at = it->first;
        const uint64_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    return false;
  }
  void release(uint64_t at, uint64_t bytes) {
    auto it = free_.emplace(at, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
 private:
  std::map<uint64_t, uint64_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  int kind = 0;
  const uint32_t* a = nullptr;
  const uint32_t* b = nullptr;
  uint8_t* out = nullptr;
  uint64_t count = 0;
  uint64_t bytes = 0;     // arena / staging footprint
  uint64_t at = 0;        // offset in the arena and staging area
  bool pinned_in = false;  // a and b are pinned host memory: copied without staging
  bool pinned_out = false; // out is pinned host memory: answers copied straight to it
  int stream = 0;
  hipEvent_t done = nullptr;
  gconn_request_info info{};
};

// Is p page-locked host memory the DMA engines can read directly (allocated
// with hipHostMalloc, or torch's pin_memory)?  Pageable memory is not.
bool is_pinned_host(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();  // pageable memory: leave no error for later calls
    return false;
  }
  return attr.type == hipMemoryTypeHost;
}

uint64_t footprint(int kind, uint64_t count) {
  const uint64_t raw = kind == GCONN_REQ_INSERT ? 8 * count : 9 * count;
  return align_up(raw ? raw : 1, kGranule);
}

}  // namespace
}  // namespace gconn

using namespace gconn;

struct gconn_server {
  gconn_server_config cfg{};
  uint32_t* P = nullptr;
  uint8_t* arena = nullptr;
  uint8_t* staging = nullptr;  // pinned host, same size as the arena
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> fences;
  std::vector<hipEvent_t> event_pool;
  RangeAlloc space{0};
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Request>> pending;  // submitted, not admitted
  // Admitted requests per stream, oldest first: a stream runs its work in
  // order, so its requests complete in this order.
  std::vector<std::deque<std::unique_ptr<Request>>> inflight;
  size_t inflight_count = 0;
  std::unordered_map<uint64_t, gconn_request_info> finished;
  uint64_t next_ticket = 1;
  uint64_t submitted = 0, completed = 0;
  bool stop = false;
  std::thread worker;

  int epoch_kind = -1;
  uint64_t epoch = 0;
  int rr = 0;

  // Frees the HIP resources the server created (also after a failed create).
  // The worker thread, if it was started, has been joined before this runs.
  ~gconn_server() {
    for (auto st : streams) (void)hipStreamDestroy(st);
    for (auto e : fences) (void)hipEventDestroy(e);
    for (auto e : event_pool) (void)hipEventDestroy(e);
    if (staging) (void)hipHostFree(staging);
  }

  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  }

  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }

  // Enqueue one admitted request on its stream (worker thread, HIP device set).
  gconn_status launch(Request& r) {
    hipStream_t s = streams[r.stream];
    if (r.kind != epoch_kind) {
      // new epoch: fence everything already enqueued on every stream
      for (size_t t = 0; t < streams.size(); ++t)
        GCONN_HIP(hipEventRecord(fences[t], streams[t]));
      epoch_kind = r.kind;
      ++epoch;
    }
    r.info.epoch = epoch;
    uint8_t* dev = arena + r.at;
    uint8_t* host = staging + r.at;
    uint32_t* da = reinterpret_cast<uint32_t*>(dev);
    uint32_t* db = da + r.count;
    // Transfers first: they touch only this request's arena range, so they
    // need not wait for earlier epochs and overlap the kernels still running
    // there.  Large pageable inputs are staged in chunks, so that the host
    // copy of one chunk overlaps the transfer of the previous one; pinned
    // inputs are read by the copy engines directly, one transfer per array.
    uint32_t* ha = reinterpret_cast<uint32_t*>(host);
    uint32_t* hb = ha + r.count;
    const uint32_t* sa = r.pinned_in ? r.a : ha;
    const uint32_t* sb = r.pinned_in ? r.b : hb;
    const uint64_t chunk = r.pinned_in ? std::max<uint64_t>(r.count, 1) : kInsertChunk;
    for (uint64_t lo = 0; lo < r.count; lo += chunk) {
      const uint64_t len = std::min<uint64_t>(chunk, r.count - lo);
      if (!r.pinned_in) {
        staged_copy(ha + lo, r.a + lo, 4 * len);
        staged_copy(hb + lo, r.b + lo, 4 * len);
      }
      GCONN_HIP(hipMemcpyAsync(da + lo, sa + lo, 4 * len, hipMemcpyHostToDevice, s));
      GCONN_HIP(hipMemcpyAsync(db + lo, sb + lo, 4 * len, hipMemcpyHostToDevice, s));
    }
    // The kernel waits on the fences of the current epoch, which order it
    // after every earlier epoch's work on every stream; waiting on a fence
    // older than the stream's own work is a no-op for correctness.
    if (epoch > 1)
      for (size_t t = 0; t < streams.size(); ++t) GCONN_HIP(hipStreamWaitEvent(s, fences[t], 0));
    if (r.kind == GCONN_REQ_INSERT) {
      uint32_t* H = nullptr;  // rules with a claim array are not offered by the server
      GCONN_TRY(launch_insert(cfg.options, P, H, da, db, r.count, s));
    } else {
      uint8_t* dout = dev + 8 * r.count;
      GCONN_TRY(launch_query(cfg.options, P, da, db, r.count, dout, s));
      GCONN_HIP(hipMemcpyAsync(r.pinned_out ? r.out : host + 8 * r.count, dout, r.count,
                               hipMemcpyDeviceToHost, s));
    }
    r.done = get_event();
    if (!r.done) return fail(GCONN_EDEVICE, "hipEventCreate failed");
    GCONN_HIP(hipEventRecord(r.done, s));
    return GCONN_OK;
  }

  void finish_request(std::unique_ptr<Request>& r, gconn_status st) {
    if (st == GCONN_OK && r->kind == GCONN_REQ_QUERY && r->out && !r->pinned_out)
      std::memcpy(r->out, staging + r->at + 8 * r->count, r->count);
    space.release(r->at, r->bytes);
    if (r->done) event_pool.push_back(r->done);
    r->info.status = st;
    r->info.done_us = now_us();
    std::lock_guard<std::mutex> lock(mu);
    finished[r->ticket] = r->info;
    ++completed;
    cv_done.notify_all();
  }

  // Publish every request whose completion event has fired: per stream, from
  // the oldest, up to the first that is still running.
  bool sweep_completions() {
    bool progressed = false;
    for (auto& q : inflight) {
      while (!q.empty()) {
        const hipError_t e = hipEventQuery(q.front()->done);
        if (e == hipErrorNotReady) break;
        const gconn_status st = e == hipSuccess ? GCONN_OK : hip_fail(e, "request");
        finish_request(q.front(), st);
        q.pop_front();
        --inflight_count;
        progressed = true;
      }
    }
    return progressed;
  }

  void run() {
    (void)hipSetDevice(device);
    for (;;) {
      // 1. admit at most one request, in submission order.  Completions are
      // swept after every admission: a steady arrival stream can keep the
      // pending queue non-empty for a long time, and finished requests must
      // not wait for it to drain.
      bool admitted = false;
      std::unique_ptr<Request> r;
      {
        std::lock_guard<std::mutex> lock(mu);
        uint64_t at = 0;
        if (!pending.empty() && space.alloc(pending.front()->bytes, &at)) {
          r = std::move(pending.front());
          pending.pop_front();
          r->at = at;
        }
      }
      if (r) {
        admitted = true;
        r->stream = rr;
        rr = (rr + 1) % (int)streams.size();
        r->info.admit_us = now_us();
        const gconn_status st = launch(*r);
        if (st != GCONN_OK) finish_request(r, st);
        else {
          const int sid = r->stream;
          inflight[sid].push_back(std::move(r));
          ++inflight_count;
        }
      }
      // 2. completions
      const bool progressed = sweep_completions() || admitted;
      // 3. sleep when idle
      std::unique_lock<std::mutex> lock(mu);
      if (stop && pending.empty() && inflight_count == 0) break;
      if (progressed) continue;
      if (inflight_count == 0 && pending.empty())
        cv_work.wait_for(lock, std::chrono::milliseconds(5));
      else
        cv_work.wait_for(lock, std::chrono::microseconds(20));
    }
  }
};

extern "C" {

gconn_status gconn_server_create(const gconn_server_config* cfg, uint32_t* parent_buf, void* arena,
                                 gconn_server** out) {
  clear_error();
  if (!cfg || !out) return fail(GCONN_EINVAL, "cfg and out are required");
  *out = nullptr;
  GCONN_TRY(check_options(cfg->options));
  if (!is_union_find(cfg->options.link) || needs_claims(cfg->options.link) ||
      cfg->options.link == GCONN_LINK_JTB)
    return fail(GCONN_EUNSUPPORTED,
                "the server runs Union-Async, Union-Early, Union-Rem-CAS, ECL-CC's rule or "
                "G_Afforest's link");
  if (cfg->n_max == 0 || cfg->n_max > 0xFFFFFFFEu) return fail(GCONN_EINVAL, "n_max out of range");
  if (cfg->streams > 16) return fail(GCONN_EINVAL, "streams must be 1..16");
  if (cfg->arena_bytes < kGranule) return fail(GCONN_EINVAL, "arena too small");
  GCONN_TRY(check_device_ready());
  GCONN_TRY(check_device_ptr(parent_buf, "parent_buf"));
  GCONN_TRY(check_device_ptr(arena, "arena"));
  if (reinterpret_cast<uintptr_t>(arena) % kGranule != 0)
    return fail(GCONN_EINVAL, "arena must be 256-byte aligned");
  std::unique_ptr<gconn_server> s(new (std::nothrow) gconn_server);
  if (!s) return fail(GCONN_EINVAL, "host allocation failed");
  s->cfg = *cfg;
  if (s->cfg.streams == 0) s->cfg.streams = 4;
  s->P = parent_buf;
  s->arena = static_cast<uint8_t*>(arena);
  s->space = RangeAlloc(cfg->arena_bytes / kGranule * kGranule);
  GCONN_HIP(hipGetDevice(&s->device));
  void* staging = nullptr;
  GCONN_HIP(hipHostMalloc(&staging, cfg->arena_bytes, hipHostMallocDefault));
  s->staging = static_cast<uint8_t*>(staging);
  for (uint32_t t = 0; t < s->cfg.streams; ++t) {
    hipStream_t st = nullptr;
    GCONN_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    s->streams.push_back(st);
    hipEvent_t e = nullptr;
    GCONN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    s->fences.push_back(e);  // on any failure above, s's destructor frees what exists
  }
  s->inflight.resize(s->streams.size());
  GCONN_TRY(launch_iota(parent_buf, cfg->n_max, s->streams[0]));
  GCONN_HIP(hipStreamSynchronize(s->streams[0]));
  s->t0 = std::chrono::steady_clock::now();
  gconn_server* raw = s.release();
  raw->worker = std::thread([raw] { raw->run(); });
  *out = raw;
  return GCONN_OK;
}

gconn_status gconn_server_submit(gconn_server* s, int kind, const uint32_t* a, const uint32_t* b,
                                 uint64_t count, uint8_t* out, uint64_t* ticket) {
  if (!s || !ticket) return fail(GCONN_EINVAL, "server and ticket are required");
  if (kind != GCONN_REQ_INSERT && kind != GCONN_REQ_QUERY)
    return fail(GCONN_EINVAL, "kind must be GCONN_REQ_INSERT or GCONN_REQ_QUERY");
  if (count > 0 && (!a || !b)) return fail(GCONN_EINVAL, "a and b are required");
  if (kind == GCONN_REQ_QUERY && count > 0 && !out) return fail(GCONN_EINVAL, "out is required");
  if (footprint(kind, count) > s->cfg.arena_bytes)
    return fail(GCONN_EINVAL, "request larger than the server arena");
  if (count > 0 && host_max_id(a, b, count) >= s->cfg.n_max)
    return fail(GCONN_EINVAL, "vertex id >= n_max in the request");
  auto r = std::make_unique<Request>();
  r->kind = kind;
  r->a = a;
  r->b = b;
  r->out = out;
  r->count = count;
  r->bytes = footprint(kind, count);
  r->info.kind = kind;
  r->info.count = count;
  if (count > 0) {
    r->pinned_in = is_pinned_host(a) && is_pinned_host(b);
    r->pinned_out = kind == GCONN_REQ_QUERY && is_pinned_host(out);
  }
  {
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) return fail(GCONN_EBUSY, "server is shutting down");
    r->ticket = s->next_ticket++;
    r->info.submit_us = s->now_us();
    *ticket = r->ticket;
    s->pending.push_back(std::move(r));
    ++s->submitted;
  }
  s->cv_work.notify_one();
  return GCONN_OK;
}

gconn_status gconn_server_wait(gconn_server* s, uint64_t ticket, double timeout_s,
                               gconn_request_info* info) {
  if (!s) return fail(GCONN_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lock(s->mu);
  if (ticket == 0 || ticket >= s->next_ticket) return fail(GCONN_EINVAL, "unknown ticket");
  auto ready = [&] { return s->finished.count(ticket) != 0; };
  if (timeout_s < 0) {
    s->cv_done.wait(lock, ready);
  } else if (!s->cv_done.wait_for(lock, std::chrono::duration<double>(timeout_s), ready)) {
    return fail(GCONN_ETIMEOUT, "request not done within the timeout");
  }
  const gconn_request_info rec = s->finished[ticket];
  if (info) *info = rec;
  return (gconn_status)rec.status;
}

gconn_status gconn_server_drain(gconn_server* s) {
  if (!s) return fail(GCONN_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lock(s->mu);
  s->cv_done.wait(lock, [&] { return s->completed == s->submitted; });
  return GCONN_OK;
}

gconn_status gconn_server_destroy(gconn_server* s) {
  if (!s) return GCONN_OK;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  delete s;
  return GCONN_OK;
}

}  // extern "C"
