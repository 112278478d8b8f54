// Serving runtime: admission against an output arena, one batched merge
// launch per scheduler step, completion reporting.  The merge work itself is
// cm_stable_merge_batch (Algorithm 2 over a batch of independent merges); this
// file is scheduling and, for requests whose data live in host memory, the
// copies in and out on two copy streams of the runtime's own.
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "corank_merge.h"
#include "internal.hpp"
#include "ring_alloc.hpp"

static_assert(sizeof(cm_server_done) == 80, "cm_server_done layout (mirrored by the Python binding)");
static_assert(sizeof(cm_server_stats) == 80, "cm_server_stats layout (mirrored by the Python binding)");

namespace {

using Clock = std::chrono::steady_clock;

uint64_t round256(uint64_t x) { return (x + 255) / 256 * 256; }

enum State { kFree, kPending, kAdmitted, kDone };

struct Request {
  uint64_t ticket = 0;
  State state = kFree;
  cm_merge_desc d{};
  bool wait_ready = false;
  hipEvent_t ready = nullptr;  // recorded on the client's stream at submit (host requests: on copy_in)
  uint64_t out_bytes = 0;      // arena bytes held: outputs (keys, then payloads), then staged inputs
  uint64_t keys_off = 0, vals_off = 0;
  // host request (cm_server_submit_host): inputs and outputs in host memory
  bool host = false;
  const void* hA = nullptr;
  const uint32_t* hAv = nullptr;
  const void* hB = nullptr;
  const uint32_t* hBv = nullptr;
  void* hC = nullptr;
  uint32_t* hCv = nullptr;
  int copy_status = CM_OK;        // enqueueing the copy in
  bool out_pending = false;       // outputs being copied back (done when out_done is)
  hipEvent_t out_done = nullptr;  // recorded on copy_out after this request's copies
  Clock::time_point t_submit, t_launch, t_ended;
  uint64_t device_ns = 0;  // device time of the batch that ran it
};

struct Slot {  // one batch in flight
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, end = nullptr;
  cm_merge_desc* host = nullptr;      // pinned, mapped for the device
  cm_merge_desc* host_dev = nullptr;  // its device address (the batch kernels read it there)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<uint32_t> reqs;
  int status = CM_OK;
  bool timed = false;  // start was recorded by this batch
  bool busy = false;
};

}  // namespace

struct cm_server {
  int kt = 0;
  bool val = false;
  uint64_t ks = 4;
  char* arena = nullptr;
  uint32_t max_batch = 0, max_inflight = 0, max_requests = 0;
  int device = 0;
  hipStream_t copy_in = nullptr, copy_out = nullptr;  // host requests' copies

  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  cm::RingAlloc ring{256};
  std::vector<Request> reqs;
  std::vector<uint32_t> free_slots;  // request slots
  std::deque<uint32_t> pending;      // submitted, in arrival order
  std::deque<cm_server_done> done;
  uint64_t seq = 0;
  bool stop = false;
  cm_server_stats st{};

  // scheduler thread only
  std::deque<uint32_t> admitted;
  std::vector<Slot> slots;
  std::vector<uint32_t> outgoing;  // host requests whose outputs are on their way back
  hipEvent_t ref = nullptr;  // time origin of the busy intervals
  std::vector<std::pair<float, float>> intervals;

  std::thread thread;
};

namespace {

void destroy_resources(cm_server* s) {
  for (Slot& b : s->slots) {
    if (b.stream) (void)hipStreamDestroy(b.stream);
    if (b.start) (void)hipEventDestroy(b.start);
    if (b.end) (void)hipEventDestroy(b.end);
    if (b.host) (void)hipHostFree(b.host);
    if (b.ws) (void)hipFree(b.ws);
  }
  if (s->copy_in) (void)hipStreamDestroy(s->copy_in);
  if (s->copy_out) (void)hipStreamDestroy(s->copy_out);
  for (Request& r : s->reqs) {
    if (r.ready) (void)hipEventDestroy(r.ready);
    if (r.out_done) (void)hipEventDestroy(r.out_done);
  }
  if (s->ref) (void)hipEventDestroy(s->ref);
}

// Keys then payloads of an N-output merge, each 256-byte aligned.
uint64_t out_bytes(const cm_server* s, uint64_t N) {
  return N ? round256(N * s->ks) + (s->val ? round256(N * 4) : 0) : 0;
}

// Arena bytes a host request's inputs take when staged (keys of A and B,
// then their payloads, each 256-byte aligned).
uint64_t in_bytes(const cm_server* s, uint64_t m, uint64_t n) {
  auto part = [](uint64_t b) { return b ? round256(b) : 0; };
  return part(m * s->ks) + part(n * s->ks) + (s->val ? part(m * 4) + part(n * 4) : 0);
}

// Enqueue a host request's copy in to the arena at `base` on copy_in and
// point its descriptor there; the merge waits for the copy (ready event).
void stage_inputs(cm_server* s, Request& r, uint64_t base) {
  char* p = s->arena + base;
  auto put = [&](const void* src, uint64_t bytes) -> void* {
    if (!bytes) return nullptr;
    void* dst = p;
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->copy_in) != hipSuccess) r.copy_status = CM_EHIP;
    p += round256(bytes);
    return dst;
  };
  r.d.A = put(r.hA, r.d.m * s->ks);
  r.d.B = put(r.hB, r.d.n * s->ks);
  if (s->val) {
    r.d.A_val = (const uint32_t*)put(r.hAv, r.d.m * 4);
    r.d.B_val = (const uint32_t*)put(r.hBv, r.d.n * 4);
  }
  if (hipEventRecord(r.ready, s->copy_in) != hipSuccess) r.copy_status = CM_EHIP;
  r.wait_ready = r.copy_status == CM_OK;
  // on a failure, copies already enqueued must not outlive the report (the
  // client may free its host arrays once the request is reported)
  if (r.copy_status != CM_OK) (void)hipStreamSynchronize(s->copy_in);
}

// Admit pending requests in arrival order while their outputs (and, for host
// requests, their staged inputs) fit (mu held).
void admit(cm_server* s) {
  while (!s->pending.empty()) {
    Request& r = s->reqs[s->pending.front()];
    const int64_t off = s->ring.alloc(r.out_bytes, r.ticket);
    if (off < 0) break;
    const uint64_t N = r.d.m + r.d.n;
    r.keys_off = (uint64_t)off;
    r.vals_off = s->val && N ? (uint64_t)off + round256(N * s->ks) : 0;
    r.d.C = N ? s->arena + r.keys_off : nullptr;
    r.d.C_val = s->val && N ? (uint32_t*)(s->arena + r.vals_off) : nullptr;
    if (r.host && N) stage_inputs(s, r, (uint64_t)off + out_bytes(s, N));
    r.state = kAdmitted;
    s->admitted.push_back(s->pending.front());
    s->pending.pop_front();
    s->st.arena_peak_bytes = std::max(s->st.arena_peak_bytes, s->ring.used());
  }
}

// Inputs in place: no producer to wait for, or its work (the client's, or
// the runtime's copy in) has completed.
bool inputs_ready(const Request& r) {
  return !r.wait_ready || hipEventQuery(r.ready) != hipErrorNotReady;
}

// Launch up to max_batch admitted requests whose inputs are in place, in
// admission order, on slot b (scheduler thread, mu not held: the batch
// counters are the caller's to update under mu); requests still waiting
// for their inputs stay admitted, so a batch never holds a slot while it
// waits for a copy.  Returns the number launched.
uint32_t launch(cm_server* s, Slot& b) {
  b.reqs.clear();
  const Clock::time_point now = Clock::now();
  uint32_t n = 0;
  for (auto it = s->admitted.begin(); it != s->admitted.end() && n < s->max_batch;) {
    Request& r = s->reqs[*it];  // stays kAdmitted (not releasable) until reported
    if (!inputs_ready(r)) {
      ++it;
      continue;
    }
    r.t_launch = now;
    b.host[n++] = r.d;
    b.reqs.push_back(*it);
    it = s->admitted.erase(it);
  }
  if (n == 0) return 0;
  uint64_t total = 0;
  int rc = cm_batch_prepare(s->kt, s->val ? 1 : 0, b.host, n, &total);
  for (uint32_t idx : b.reqs)
    if (rc == CM_OK && s->reqs[idx].copy_status != CM_OK) rc = s->reqs[idx].copy_status;
  for (uint32_t idx : b.reqs)
    if (rc == CM_OK && s->reqs[idx].wait_ready && hipStreamWaitEvent(b.stream, s->reqs[idx].ready, 0) != hipSuccess)
      rc = CM_EHIP;
  b.timed = false;
  if (rc == CM_OK) {
    if (hipEventRecord(b.start, b.stream) == hipSuccess)
      b.timed = true;
    else
      rc = CM_EHIP;
  }
  // no upload: a small batch's descriptors travel in the kernel arguments,
  // a larger one's are read from the pinned host array by the batch's first
  // kernel (a copy engine's transfer of a few kilobytes took ~22 us)
  const bool inline_descs = n <= CM_BATCH_INLINE_MAX;
  if (rc == CM_OK)
    rc = cm_stable_merge_batch(s->kt, s->val ? 1 : 0, b.host, inline_descs ? nullptr : b.host_dev, n, total, b.ws,
                               b.ws_bytes, b.stream);
  // the end event is recorded whatever happened, so completion is detected the same way
  if (hipEventRecord(b.end, b.stream) != hipSuccess && rc == CM_OK) rc = CM_EHIP;
  // host requests: their outputs go back on copy_out once the batch has
  // ended; each is reported when its own copies are done, and the slot is
  // free again at the batch's end
  bool waited = false;
  for (uint32_t idx : b.reqs) {
    Request& r = s->reqs[idx];
    r.out_pending = false;
    const uint64_t N = r.d.m + r.d.n;
    if (!r.host || !N || rc != CM_OK) continue;
    if (!waited && hipStreamWaitEvent(s->copy_out, b.end, 0) != hipSuccess) rc = CM_EHIP;
    waited = true;
    if (rc == CM_OK && hipMemcpyAsync(r.hC, r.d.C, N * s->ks, hipMemcpyDeviceToHost, s->copy_out) != hipSuccess)
      rc = CM_EHIP;
    if (rc == CM_OK && s->val &&
        hipMemcpyAsync(r.hCv, r.d.C_val, N * 4, hipMemcpyDeviceToHost, s->copy_out) != hipSuccess)
      rc = CM_EHIP;
    if (rc == CM_OK && hipEventRecord(r.out_done, s->copy_out) != hipSuccess) rc = CM_EHIP;
    r.out_pending = rc == CM_OK;
  }
  if (rc != CM_OK) {
    // reported with the error at the batch's end; copies already enqueued
    // must finish before that (the client may then free its host arrays)
    if (waited) (void)hipStreamSynchronize(s->copy_out);
    for (uint32_t idx : b.reqs) s->reqs[idx].out_pending = false;
  }
  b.status = rc;
  b.busy = true;
  return n;
}

// Report one finished request (mu held).
void finish_request(cm_server* s, uint32_t idx, int status, Clock::time_point now) {
  {
    Request& r = s->reqs[idx];
    r.state = kDone;
    cm_server_done e{};
    e.ticket = r.ticket;
    e.status = status;
    e.C = r.host ? r.hC : r.d.C;
    e.C_val = r.host ? r.hCv : r.d.C_val;
    e.keys_offset = r.keys_off;
    e.vals_offset = r.vals_off;
    e.queued_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(r.t_launch - r.t_submit).count();
    e.latency_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(now - r.t_submit).count();
    e.ended_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(r.t_ended - r.t_submit).count();
    e.device_ns = r.device_ns;
    s->done.push_back(e);
    if (status == CM_OK)
      s->st.completed += 1;
    else
      s->st.failed += 1;
  }
}

// A slot's batch has ended (mu held; seen at `ended`, device time
// device_ns): report its requests, except host requests whose outputs are
// still on their way back, and free the slot.
void finish(cm_server* s, Slot& b, int status, Clock::time_point ended, uint64_t device_ns) {
  const Clock::time_point now = Clock::now();
  for (uint32_t idx : b.reqs) {
    s->reqs[idx].t_ended = ended;
    s->reqs[idx].device_ns = device_ns;
    if (status == CM_OK && s->reqs[idx].out_pending)
      s->outgoing.push_back(idx);
    else
      finish_request(s, idx, status, now);
  }
  b.reqs.clear();
  b.busy = false;
}

void cancel_pending(cm_server* s) {  // mu held
  const Clock::time_point now = Clock::now();
  while (!s->pending.empty()) {
    Request& r = s->reqs[s->pending.front()];
    s->pending.pop_front();
    r.state = kDone;
    r.d.C = nullptr;
    r.d.C_val = nullptr;
    r.out_bytes = 0;  // nothing allocated
    cm_server_done e{};
    e.ticket = r.ticket;
    e.status = CM_ECANCELED;
    e.latency_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(now - r.t_submit).count();
    s->done.push_back(e);
    s->st.canceled += 1;
  }
}

void scheduler(cm_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    admit(s);
    int inflight = s->outgoing.empty() ? 0 : 1;
    for (const Slot& b : s->slots) inflight += b.busy ? 1 : 0;
    if (s->stop && s->admitted.empty() && inflight == 0) {
      if (s->pending.empty()) break;
      cancel_pending(s);  // the arena is held by outputs nobody will release
      s->cv_done.notify_all();
      continue;
    }
    lk.unlock();
    std::vector<uint32_t> launched;  // batch sizes, counted under mu below
    for (Slot& b : s->slots) {
      if (s->admitted.empty()) break;
      if (b.busy) continue;
      const uint32_t n = launch(s, b);
      if (n > 0) launched.push_back(n);
    }
    bool progressed = !launched.empty();
    struct Finished {
      Slot* b;
      int status;
      bool timed;
      float t0, t1;
      Clock::time_point seen;
    };
    std::vector<Finished> finished;
    for (Slot& b : s->slots) {
      if (!b.busy) continue;
      const hipError_t q = hipEventQuery(b.end);
      if (q == hipErrorNotReady) continue;
      Finished f{&b, b.status, false, 0.f, 0.f, Clock::now()};
      if (q != hipSuccess && f.status == CM_OK) f.status = CM_EHIP;
      f.timed = b.timed && hipEventElapsedTime(&f.t0, s->ref, b.start) == hipSuccess &&
                hipEventElapsedTime(&f.t1, s->ref, b.end) == hipSuccess;
      finished.push_back(f);
    }
    // host requests whose outputs were on their way back (scheduler-owned list)
    std::vector<std::pair<uint32_t, int>> back;
    for (size_t k = 0; k < s->outgoing.size();) {
      const hipError_t q = hipEventQuery(s->reqs[s->outgoing[k]].out_done);
      if (q == hipErrorNotReady) {
        ++k;
        continue;
      }
      back.emplace_back(s->outgoing[k], q == hipSuccess ? CM_OK : CM_EHIP);
      s->outgoing[k] = s->outgoing.back();
      s->outgoing.pop_back();
    }
    lk.lock();
    for (const uint32_t n : launched) {
      s->st.batches += 1;
      s->st.max_batch_seen = std::max<uint64_t>(s->st.max_batch_seen, n);
    }
    for (const Finished& f : finished) {
      if (f.timed) s->intervals.emplace_back(f.t0, f.t1);
      finish(s, *f.b, f.status, f.seen, f.timed ? (uint64_t)((double)(f.t1 - f.t0) * 1e6) : 0);
    }
    const Clock::time_point now = Clock::now();
    for (const auto& rb : back) finish_request(s, rb.first, rb.second, now);
    if (!finished.empty() || !back.empty()) {
      progressed = true;
      s->cv_done.notify_all();
    }
    if (!progressed) {
      bool in_flight = !s->outgoing.empty();
      for (const Slot& b : s->slots) in_flight = in_flight || b.busy;
      // batches or copies in flight: poll their events again at once (a
      // timed wait would oversleep by tens of microseconds, each added to
      // the latency of every request in the batch); admitted requests still
      // waiting for their inputs: poll every 20 us; otherwise sleep until woken
      if (in_flight) {
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else if (!s->admitted.empty())
        s->cv_sched.wait_for(lk, std::chrono::microseconds(20));
      else if (!s->stop && s->pending.empty())
        s->cv_sched.wait(lk);
      else if (!s->stop)
        s->cv_sched.wait_for(lk, std::chrono::milliseconds(1));  // waiting for arena space
    }
  }
}

double union_ms(std::vector<std::pair<float, float>> iv, double* span) {
  *span = 0;
  if (iv.empty()) return 0;
  std::sort(iv.begin(), iv.end());
  double total = 0, lo = iv[0].first, hi = iv[0].second, last = iv[0].second;
  for (size_t k = 1; k < iv.size(); ++k) {
    if (iv[k].first > hi) {
      total += hi - lo;
      lo = iv[k].first;
      hi = iv[k].second;
    } else {
      hi = std::max<double>(hi, iv[k].second);
    }
    last = std::max<double>(last, iv[k].second);
  }
  *span = last - iv[0].first;
  return total + (hi - lo);
}

}  // namespace

namespace {

bool host_overlap(const void* a, uint64_t na, const void* b, uint64_t nb) {
  if (!a || !b || !na || !nb) return false;
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// Queues request `idx` (filled in by the caller, which owns it until here).
int queue_request(cm_server* s, uint32_t idx, uint64_t* ticket) {
  Request& r = s->reqs[idx];
  r.t_submit = Clock::now();
  uint64_t t;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    t = r.ticket;
    r.state = kPending;
    s->pending.push_back(idx);
    s->st.submitted += 1;
  }
  s->cv_sched.notify_one();
  *ticket = t;
  return CM_OK;
}

// Takes a free request slot and gives it a ticket (state stays kFree until queued).
int take_slot(cm_server* s, uint32_t* idx) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return CM_ECANCELED;
  if (s->free_slots.empty()) return CM_EBUSY;
  *idx = s->free_slots.back();
  s->free_slots.pop_back();
  s->seq += 1;
  s->reqs[*idx].ticket = (s->seq << 16) | *idx;
  return CM_OK;
}

}  // namespace

extern "C" {

int cm_server_create(int key_type, int with_payload, void* arena, uint64_t arena_bytes, uint32_t max_batch,
                     uint32_t max_inflight, uint32_t max_requests, cm_server** server) {
  if (!server) return CM_EINVAL;
  *server = nullptr;
  if (key_type < CM_KEY_U32 || key_type > CM_KEY_F32_DESC) return CM_EDTYPE;
  if (!arena || arena_bytes < 256 || max_batch < 1 || max_batch > 65536 || max_inflight < 1 || max_inflight > 16 ||
      max_requests < 1 || max_requests > 65535)
    return CM_EINVAL;
  cm_server* s = new cm_server();
  s->kt = key_type;
  s->val = with_payload != 0;
  s->ks = key_type == CM_KEY_U64 || key_type == CM_KEY_U64_DESC ? 8 : 4;
  s->arena = (char*)arena;
  s->max_batch = max_batch;
  s->max_inflight = max_inflight;
  s->max_requests = max_requests;
  s->ring = cm::RingAlloc(arena_bytes);
  s->st.arena_bytes = s->ring.size();
  s->reqs.resize(max_requests);
  for (uint32_t k = max_requests; k > 0; --k) s->free_slots.push_back(k - 1);
  s->slots.resize(max_inflight);
  // A batch's outputs all lie in the arena, so it has at most
  // arena / (bytes per output) outputs and that / smallest tile + count blocks.
  const uint64_t per_out = s->ks + (s->val ? 4 : 0);
  const uint64_t max_blocks = arena_bytes / per_out / cm::kMinTile + max_batch;
  int rc = hipGetDevice(&s->device) == hipSuccess ? CM_OK : CM_EHIP;
  for (Slot& b : s->slots) {
    if (rc != CM_OK) break;
    b.ws_bytes = cm_batch_workspace_size(max_blocks, max_batch);
    if (hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&b.start) != hipSuccess || hipEventCreate(&b.end) != hipSuccess ||
        hipHostMalloc((void**)&b.host, (size_t)max_batch * sizeof(cm_merge_desc), hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void**)&b.host_dev, b.host, 0) != hipSuccess ||
        hipMalloc(&b.ws, b.ws_bytes) != hipSuccess)
      rc = CM_EHIP;
  }
  if (rc == CM_OK && (hipStreamCreateWithFlags(&s->copy_in, hipStreamNonBlocking) != hipSuccess ||
                      hipStreamCreateWithFlags(&s->copy_out, hipStreamNonBlocking) != hipSuccess))
    rc = CM_EHIP;
  for (Request& r : s->reqs) {
    if (rc != CM_OK) break;
    if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&r.out_done, hipEventDisableTiming) != hipSuccess)
      rc = CM_EHIP;
  }
  if (rc == CM_OK && (hipEventCreate(&s->ref) != hipSuccess || hipEventRecord(s->ref, s->slots[0].stream) != hipSuccess ||
                      hipEventSynchronize(s->ref) != hipSuccess))
    rc = CM_EHIP;
  if (rc != CM_OK) {
    destroy_resources(s);
    delete s;
    return rc;
  }
  s->thread = std::thread(scheduler, s);
  *server = s;
  return CM_OK;
}


int cm_server_submit_host(cm_server* s, const void* A, const uint32_t* A_val, uint64_t m, const void* B,
                          const uint32_t* B_val, uint64_t n, void* C, uint32_t* C_val, uint64_t* ticket) {
  if (!s || !ticket) return CM_EINVAL;
  if (!cm::lengths_ok(m, n)) return CM_EINVAL;
  const uint64_t N = m + n;
  if ((m && !A) || (n && !B) || (N && !C)) return CM_EINVAL;
  if (s->val ? ((m && !A_val) || (n && !B_val) || (N && !C_val)) : (A_val || B_val || C_val)) return CM_EINVAL;
  const uint64_t kb = N * s->ks, vb = s->val ? N * 4 : 0;
  for (const auto& in : {std::make_pair(A, m * s->ks), std::make_pair(B, n * s->ks),
                         std::make_pair((const void*)A_val, s->val ? m * 4 : 0),
                         std::make_pair((const void*)B_val, s->val ? n * 4 : 0)})
    if (host_overlap(C, kb, in.first, in.second) || host_overlap(C_val, vb, in.first, in.second)) return CM_EALIAS;
  if (host_overlap(C, kb, C_val, vb)) return CM_EALIAS;
  const uint64_t bytes = out_bytes(s, N) + in_bytes(s, m, n);
  if (bytes > s->ring.size()) return CM_ENOSPC;
  uint32_t idx;
  const int rc = take_slot(s, &idx);
  if (rc != CM_OK) return rc;
  Request& r = s->reqs[idx];
  r.d = cm_merge_desc{};
  r.d.m = m;
  r.d.n = n;
  r.out_bytes = bytes;
  r.wait_ready = false;  // set when the copy in is enqueued at admission
  r.host = true;
  r.hA = A;
  r.hAv = A_val;
  r.hB = B;
  r.hBv = B_val;
  r.hC = C;
  r.hCv = C_val;
  r.copy_status = CM_OK;
  return queue_request(s, idx, ticket);
}

int cm_server_submit(cm_server* s, const void* A, const uint32_t* A_val, uint64_t m, const void* B,
                     const uint32_t* B_val, uint64_t n, hipStream_t inputs_stream, int inputs_pending,
                     uint64_t* ticket) {
  if (!s || !ticket) return CM_EINVAL;
  if (!cm::lengths_ok(m, n)) return CM_EINVAL;
  const uint64_t N = m + n;
  if ((m && !A) || (n && !B)) return CM_EINVAL;
  if (s->val ? ((m && !A_val) || (n && !B_val)) : (A_val || B_val)) return CM_EINVAL;
  const uint64_t bytes = out_bytes(s, N);
  if (bytes > s->ring.size()) return CM_ENOSPC;
  uint32_t idx;
  const int rc = take_slot(s, &idx);
  if (rc != CM_OK) return rc;
  Request& r = s->reqs[idx];  // only this thread touches it until it is queued
  r.d = cm_merge_desc{};
  r.d.A = A;
  r.d.A_val = A_val;
  r.d.m = m;
  r.d.B = B;
  r.d.B_val = B_val;
  r.d.n = n;
  r.out_bytes = bytes;
  r.host = false;
  r.copy_status = CM_OK;
  r.wait_ready = inputs_pending != 0;
  if (r.wait_ready && hipEventRecord(r.ready, inputs_stream) != hipSuccess) {
    std::lock_guard<std::mutex> lk(s->mu);
    r.ticket = 0;
    s->free_slots.push_back(idx);
    return CM_EHIP;
  }
  return queue_request(s, idx, ticket);
}

int cm_server_poll(cm_server* s, cm_server_done* done, uint32_t capacity, uint32_t* count, int64_t wait_us) {
  if (!s || !count || (capacity && !done)) return CM_EINVAL;
  *count = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_us > 0)
    s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [s] { return !s->done.empty(); });
  uint32_t k = 0;
  while (k < capacity && !s->done.empty()) {
    done[k++] = s->done.front();
    s->done.pop_front();
  }
  *count = k;
  return CM_OK;
}

int cm_server_release(cm_server* s, uint64_t ticket) {
  if (!s) return CM_EINVAL;
  const uint32_t idx = (uint32_t)(ticket & 0xffff);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (idx >= s->max_requests) return CM_EINVAL;
    Request& r = s->reqs[idx];
    if (r.ticket != ticket || r.state != kDone) return CM_EINVAL;
    if (r.out_bytes) s->ring.release(ticket);
    r.state = kFree;
    r.ticket = 0;
    s->free_slots.push_back(idx);
  }
  s->cv_sched.notify_one();  // arena space may admit a waiting request
  return CM_OK;
}

int cm_server_get_stats(cm_server* s, cm_server_stats* out) {
  if (!s || !out) return CM_EINVAL;
  std::vector<std::pair<float, float>> iv;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    iv = s->intervals;
  }
  double span = 0;
  out->busy_ms = union_ms(std::move(iv), &span);
  out->span_ms = span;
  return CM_OK;
}

int cm_server_destroy(cm_server* s) {
  if (!s) return CM_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_sched.notify_one();
  if (s->thread.joinable()) s->thread.join();
  destroy_resources(s);
  delete s;
  return CM_OK;
}

}  // extern "C"
