// Served form of the runtime: continuous batching of tenant requests with
// admission by device-memory budget (declared in include/gxbpf.h).
//
// A host thread owns every HIP call of the server.  Submissions land in
// per-tenant FIFO queues.  A tenant's programs own its maps, so its
// requests must run in order: they all go to stream (tenant mod streams),
// whose order keeps them in sequence; in continuous mode a stream holds up
// to four unfinished launches, each taking the head request of each of its
// tenants, so one tenant may have several requests queued on the device
// (one per launch, in order).  Only the per-request mode keeps at most one
// request per tenant in flight.  Whenever the thread finds requests whose
// buffers fit in the free part of the device pool, it admits them; a
// request whose buffers do not fit waits without blocking smaller requests
// of other tenants.  Completion is detected with HIP events, after the
// return codes have been copied back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gxbpf.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit range allocator over [0, size) with 256-byte granules.
class RangeAlloc {
 public:
  explicit RangeAlloc(size_t size) { free_[0] = size; }
  bool alloc(size_t len, size_t* off) {
    len = (len + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      *off = it->first;
      size_t rest = it->second - len, at = it->first + len;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += len;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t len) {
    len = (len + 255) & ~(size_t)255;
    used_ -= len;
    auto it = free_.emplace(off, len).first;
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

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

struct Req {
  uint64_t id = 0;
  int32_t tenant = 0;
  int prog = -1;
  uint64_t n = 0;
  uint32_t rs = 0;
  size_t ev_bytes = 0, dev_len = 0, dev_off = 0, pin_off = 0, pin_len = 0;
  bool pinned = false;
  const void* borrowed = nullptr;  // caller-owned events (submit_borrowed)
  std::vector<uint8_t> heap;   // events when the pinned pool was full
  std::vector<uint32_t> rc;    // return codes when not pinned
  uint32_t* rc_host = nullptr;
  int status = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Group {
  std::vector<Req*> reqs;
  hipEvent_t done = nullptr;
  uint32_t stream = 0;
};

}  // namespace

struct gx_server {
  gx_rt* rt = nullptr;
  gx_server_cfg cfg{};
  int dev = 0;
  uint8_t* d_pool = nullptr;
  uint8_t* h_pool = nullptr;
  RangeAlloc* dev_alloc = nullptr;
  RangeAlloc* pin_alloc = nullptr;
  std::mutex pin_mu;  // pinned pool: submit allocates, the thread frees
  std::vector<hipStream_t> streams;
  std::vector<uint32_t> inflight;  // unfinished groups per stream
  std::vector<hipEvent_t> free_events;
  uint32_t next_stream = 0;
  // queues
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Req*> incoming;
  std::vector<gx_completion> completed;
  uint64_t outstanding = 0;  // submitted and not yet completed
  bool stop = false;
  std::thread th;
  // thread-owned state
  std::unordered_map<int32_t, std::deque<Req*>> fifo;
  std::unordered_map<int32_t, bool> busy;
  std::vector<int32_t> tenants;  // round-robin order
  size_t rr = 0;
  std::vector<Group> groups;
};

namespace {

hipEvent_t take_event(gx_server* s) {
  if (!s->free_events.empty()) {
    hipEvent_t e = s->free_events.back();
    s->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
  return e;
}

void finish(gx_server* s, Req* r, int status) {
  r->status = status;
  r->t_done = now_s();
  s->dev_alloc->release(r->dev_off, r->dev_len);
  s->busy[r->tenant] = false;
  gx_completion c{};
  c.req_id = r->id;
  c.tenant = r->tenant;
  c.status = status;
  c.n_events = r->n;
  c.rc = r->pinned ? r->rc_host : r->rc.data();
  c.t_submit = r->t_submit;
  c.t_admit = r->t_admit;
  c.t_done = r->t_done;
  c.priv = r;
  std::lock_guard<std::mutex> g(s->mu);
  s->completed.push_back(c);
  s->outstanding--;
  s->cv_done.notify_all();
}

void launch(gx_server* s, std::vector<Req*>& grp, uint32_t k) {
  hipStream_t st = s->streams[k];
  std::vector<gx_batch> descs;
  int status = 0;
  for (Req* r : grp) {
    uint8_t* d_ev = s->d_pool + r->dev_off;
    const void* src = r->borrowed ? r->borrowed
                      : r->pinned ? (const void*)(s->h_pool + r->pin_off) : (const void*)r->heap.data();
    if (hipMemcpyAsync(d_ev, src, r->ev_bytes, hipMemcpyHostToDevice, st) != hipSuccess) status = -EIO;
    uint32_t* d_rc = (uint32_t*)(s->d_pool + r->dev_off + ((r->ev_bytes + 255) & ~(size_t)255));
    descs.push_back(gx_batch{r->prog, r->rs, d_ev, r->n, d_rc});
  }
  if (!status) {
    if (s->cfg.mode == GX_SERVE_PER_REQUEST) {
      for (auto& d : descs)
        if (!status) status = gx_run_batch(s->rt, d.prog_fd, d.d_events, d.n_events, d.record_size, d.d_rc, st);
    } else {
      status = gx_run_batches(s->rt, descs.data(), (uint32_t)descs.size(), st);
    }
  }
  for (size_t i = 0; i < grp.size(); i++) {
    Req* r = grp[i];
    if (r->pinned) {
      // the pinned range holds the copied events (consumed by now) or, for a
      // borrowed request, was sized for the return codes alone
      r->rc_host = (uint32_t*)(s->h_pool + r->pin_off);
      (void)hipMemcpyAsync(r->rc_host, descs[i].d_rc, 4 * r->n, hipMemcpyDeviceToHost, st);
    }
  }
  Group g;
  g.reqs = grp;
  g.stream = k;
  g.done = take_event(s);
  (void)hipEventRecord(g.done, st);
  if (status) {
    (void)hipEventSynchronize(g.done);
    for (Req* r : grp) finish(s, r, status);
    s->free_events.push_back(g.done);
    return;
  }
  s->inflight[k]++;
  s->groups.push_back(std::move(g));
}

void thread_main(gx_server* s) {
  (void)hipSetDevice(s->dev);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->incoming.empty() && s->groups.empty())
        s->cv.wait_for(lk, std::chrono::microseconds(200), [&] { return s->stop || !s->incoming.empty(); });
      while (!s->incoming.empty()) {
        Req* r = s->incoming.front();
        s->incoming.pop_front();
        if (!s->fifo.count(r->tenant)) s->tenants.push_back(r->tenant);
        s->fifo[r->tenant].push_back(r);
      }
      if (s->stop && s->outstanding == 0) break;
    }
    // completions
    for (size_t i = 0; i < s->groups.size();) {
      Group& g = s->groups[i];
      if (hipEventQuery(g.done) == hipSuccess) {
        for (Req* r : g.reqs) {
          if (!r->pinned) {
            r->rc.resize(r->n);
            uint32_t* d_rc = (uint32_t*)(s->d_pool + r->dev_off + ((r->ev_bytes + 255) & ~(size_t)255));
            if (hipMemcpy(r->rc.data(), d_rc, 4 * r->n, hipMemcpyDeviceToHost) != hipSuccess) r->status = -EIO;
          }
          finish(s, r, r->status);
        }
        s->free_events.push_back(g.done);
        s->inflight[g.stream]--;
        s->groups.erase(s->groups.begin() + i);
      } else {
        i++;
      }
    }
    if (s->cfg.mode == GX_SERVE_PER_REQUEST) {
      // baseline: every idle tenant's head request whose buffers fit, each
      // its own plain launch
      std::vector<Req*> grp;
      const size_t nt = s->tenants.size();
      for (size_t k = 0; k < nt; k++) {
        int32_t t = s->tenants[(s->rr + k) % nt];
        auto& q = s->fifo[t];
        if (s->busy[t] || q.empty()) continue;
        Req* r = q.front();
        if (!s->dev_alloc->alloc(r->dev_len, &r->dev_off)) continue;
        q.pop_front();
        s->busy[t] = true;
        r->t_admit = now_s();
        grp.push_back(r);
      }
      if (nt) s->rr = (s->rr + 1) % nt;
      if (grp.empty() && !s->groups.empty()) std::this_thread::yield();
      for (Req* r : grp) {
        std::vector<Req*> one{r};
        launch(s, one, s->next_stream++ % (uint32_t)s->streams.size());
      }
      continue;
    }
    // continuous batching: tenant t's requests all go to stream t mod S, so
    // they run in submission order across launches (the stream orders them)
    // and a tenant's next request can be queued on the device before its
    // previous one is done.  A stream with fewer than kStreamDepth
    // unfinished launches takes the head request of each of its tenants
    // (buffers fitting) as one batched launch: one request per tenant keeps
    // the launch one phase wide, and while the stream is busy requests
    // gather into the next launch.
    constexpr uint32_t kStreamDepth = 4;
    bool launched = false;
    const uint32_t S = (uint32_t)s->streams.size();
    const uint32_t cap = s->cfg.max_group ? s->cfg.max_group : 0xffffffffu;
    const size_t nt = s->tenants.size();
    for (uint32_t k = 0; k < S; k++) {
      if (s->inflight[k] >= kStreamDepth) continue;
      std::vector<Req*> grp;
      for (size_t j = 0; j < nt && grp.size() < cap; j++) {
        const int32_t t = s->tenants[(s->rr + j) % nt];
        if ((uint32_t)t % S != k) continue;
        auto& q = s->fifo[t];
        if (q.empty()) continue;
        Req* r = q.front();
        if (!s->dev_alloc->alloc(r->dev_len, &r->dev_off)) continue;
        q.pop_front();
        r->t_admit = now_s();
        grp.push_back(r);
      }
      if (!grp.empty()) {
        launch(s, grp, k);
        launched = true;
      }
    }
    if (nt) s->rr = (s->rr + 1) % nt;
    if (!launched && !s->groups.empty()) std::this_thread::yield();
  }
}

}  // namespace

extern "C" {

int gx_server_create(gx_rt* rt, const gx_server_cfg* cfg, gx_server** out) {
  if (!rt || !cfg || !out || cfg->hbm_budget_bytes == 0) return -EINVAL;
  *out = nullptr;
  gx_server* s = new (std::nothrow) gx_server();
  if (!s) return -ENOMEM;
  s->rt = rt;
  s->cfg = *cfg;
  if (s->cfg.streams == 0) s->cfg.streams = 1;
  if (s->cfg.mode == GX_SERVE_PER_REQUEST) s->cfg.streams = 1;
  (void)hipGetDevice(&s->dev);
  size_t bud = (size_t)cfg->hbm_budget_bytes;
  if (hipMalloc((void**)&s->d_pool, bud) != hipSuccess ||
      hipHostMalloc((void**)&s->h_pool, bud, hipHostMallocDefault) != hipSuccess) {
    if (s->d_pool) (void)hipFree(s->d_pool);
    delete s;
    return -ENOMEM;
  }
  s->dev_alloc = new RangeAlloc(bud);
  s->pin_alloc = new RangeAlloc(bud);
  for (uint32_t i = 0; i < s->cfg.streams; i++) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      gx_server_destroy(s);
      return -ENOMEM;
    }
    s->streams.push_back(st);
  }
  s->inflight.assign(s->streams.size(), 0);
  s->th = std::thread(thread_main, s);
  *out = s;
  return 0;
}

namespace {

int submit(gx_server* s, int32_t tenant, int prog_fd, const void* host_events, uint64_t n_events,
           uint32_t record_size, uint64_t req_id, bool borrow) {
  if (!s || !host_events || n_events == 0) return -EINVAL;
  gx_prog_info info;
  if (gx_prog_info_get(s->rt, prog_fd, &info)) return -EINVAL;
  uint32_t want_rs = info.hook == GX_HOOK_MEM_ACCESS ? 24 : 16;
  if (record_size != want_rs) return -EINVAL;
  Req* r = new (std::nothrow) Req();
  if (!r) return -ENOMEM;
  r->id = req_id;
  r->tenant = tenant;
  r->prog = prog_fd;
  r->n = n_events;
  r->rs = record_size;
  r->ev_bytes = (size_t)n_events * record_size;
  r->dev_len = ((r->ev_bytes + 255) & ~(size_t)255) + 4 * n_events;
  if (r->dev_len > s->cfg.hbm_budget_bytes) {
    delete r;
    return -E2BIG;
  }
  {
    std::lock_guard<std::mutex> g(s->pin_mu);
    r->pin_len = borrow ? 4 * n_events : r->ev_bytes;
    r->pinned = s->pin_alloc->alloc(r->pin_len, &r->pin_off);
  }
  if (borrow)
    r->borrowed = host_events;
  else if (r->pinned)
    std::memcpy(s->h_pool + r->pin_off, host_events, r->ev_bytes);
  else
    r->heap.assign((const uint8_t*)host_events, (const uint8_t*)host_events + r->ev_bytes);
  r->t_submit = now_s();
  std::lock_guard<std::mutex> g(s->mu);
  s->incoming.push_back(r);
  s->outstanding++;
  s->cv.notify_one();
  return 0;
}

}  // namespace

int gx_server_submit(gx_server* s, int32_t tenant, int prog_fd, const void* host_events, uint64_t n_events,
                     uint32_t record_size, uint64_t req_id) {
  return submit(s, tenant, prog_fd, host_events, n_events, record_size, req_id, false);
}

int gx_server_submit_borrowed(gx_server* s, int32_t tenant, int prog_fd, const void* host_events,
                              uint64_t n_events, uint32_t record_size, uint64_t req_id) {
  return submit(s, tenant, prog_fd, host_events, n_events, record_size, req_id, true);
}

int gx_server_poll(gx_server* s, gx_completion* out, uint32_t max, int wait_ms) {
  if (!s || (!out && max)) return -EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->completed.empty() && wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->completed.empty(); });
  uint32_t n = (uint32_t)std::min<size_t>(max, s->completed.size());
  for (uint32_t i = 0; i < n; i++) out[i] = s->completed[i];
  s->completed.erase(s->completed.begin(), s->completed.begin() + n);
  return (int)n;
}

void gx_server_release(gx_server* s, gx_completion* c) {
  if (!s || !c || !c->priv) return;
  Req* r = (Req*)c->priv;
  if (r->pinned) {
    std::lock_guard<std::mutex> g(s->pin_mu);
    s->pin_alloc->release(r->pin_off, r->pin_len);
  }
  delete r;
  c->priv = nullptr;
  c->rc = nullptr;
}

int gx_server_drain(gx_server* s) {
  if (!s) return -EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
  return 0;
}

void gx_server_destroy(gx_server* s) {
  if (!s) return;
  if (s->th.joinable()) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->stop = true;
      s->cv.notify_all();
    }
    s->th.join();
  }
  for (auto& c : s->completed) gx_server_release(s, &c);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  for (auto e : s->free_events) (void)hipEventDestroy(e);
  if (s->d_pool) (void)hipFree(s->d_pool);
  if (s->h_pool) (void)hipHostFree(s->h_pool);
  delete s->dev_alloc;
  delete s->pin_alloc;
  delete s;
}

}  // extern "C"
