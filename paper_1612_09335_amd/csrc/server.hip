// Serving loop: registered meshes whose operators live in host memory and
// move in and out of HBM under a byte budget, with reconstruction requests
// batched as they arrive.
//
// * Registration runs the host precompute once and keeps one host image of
//   the mesh's whole device layout (operators in the server's precision,
//   index tables, block halos), so that residency is one copy.  Images are
//   pinned up to the server's pinned limit (default 32 GiB) and pageable
//   beyond it.
// * HBM: one arena of `budget` bytes, allocated when the server is created;
//   meshes are placed first-fit (256-byte granules) and the least recently
//   used mesh with no request in flight is evicted when a placement fails.
//   The serving loop never allocates or frees device memory.
// * Continuous batching: whenever a launch may start (fewer than max_inflight
//   launches in flight), a scheduler thread takes the queued requests in
//   arrival order, as many as fit one launch (at most max_batch requests and
//   one launch table), makes their meshes resident (uploads on two copy
//   streams, each recorded in an event) and pins them.  A lone request runs
//   as the ordinary per-mesh launch; several run as one launch of the batched
//   persistent kernel per (dimension, degree, variable block) group over a
//   work list of (request block, 256-cell block) items, whose kernel
//   parameters come from a launch table (pinned host slot copied to a device
//   slot on the launch stream).  Requests that arrive while launches are in
//   flight queue up and leave together in the next launch.
// * Launches go round robin over several compute streams, each behind the
//   upload events of its meshes, so work of different launches overlaps on
//   the device and a launch waiting for an upload holds back no other.
// * A completion thread polls the in-flight launches' events, records each
//   request's latency (completion seen by the host minus submission), unpins
//   meshes, frees the launch's table slot and wakes waiters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cweno.h"
#include "mesh.hpp"
#include "pack.hpp"

using cweno_abi::fail;

namespace {

constexpr size_t kGranule = 256;
constexpr int kCopyStreams = 2;   // uploads alternate between two copy streams

size_t round_up(size_t x) { return (x + kGranule - 1) / kGranule * kGranule; }

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device allocation.
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  size_t alloc(size_t bytes) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        const size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return off;
      }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    auto it = free_.emplace(off, bytes).first;
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
  std::map<size_t, size_t> free_;   // offset -> size, disjoint, coalesced
};

// Byte offsets of the arrays in a mesh's device image.
struct Layout {
  size_t pinv = 0, binv = 0, gidx = 0, secpos = 0, mask = 0, halo = 0, hoff = 0, lidx = 0, total = 0;
};

struct SMesh {
  std::unique_ptr<cweno_mesh> m;   // metadata, tables, kernel variants
  Layout lay;
  void* image = nullptr;           // host copy of the device image
  bool pinned = true;              // image in pinned memory (else pageable: slower uploads)
  bool resident = false;
  size_t off = 0;                  // arena offset while resident
  hipEvent_t ready = nullptr;      // the latest upload has completed
  int pins = 0;                    // admitted requests not yet complete
  uint64_t last_use = 0;
};

void free_image(SMesh& sm) {
  if (!sm.image) return;
  if (sm.pinned) (void)hipHostFree(sm.image);
  else std::free(sm.image);
  sm.image = nullptr;
}

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2, kCancelled = 3, kFailed = 4 };

struct Req {
  int64_t mesh = 0;
  int n_vars = 0;
  const void* q = nullptr;
  void* coeffs = nullptr;
  double t_submit = 0.0;
  int state = kQueued;
  int waiters = 0;                 // threads blocked in cweno_server_wait on this ticket
  double latency = 0.0;
};

// One launch: the requests it carries, its completion event and its table slot.
struct Launch {
  std::vector<int64_t> tickets;
  hipEvent_t done = nullptr;
  int slot = -1;                   // -1: a lone request launched as the per-mesh kernel
};

constexpr int kDefaultBatch = 64;       // requests one launch may carry
constexpr int kSlotEntries = 512;       // (request, variable block) entries of one launch table
constexpr int kSlotItems = 1 << 16;     // (entry, 256-cell block) work items of one launch table

}  // namespace

struct cweno_server {
  bool f32 = true;
  int device = -1;
  int max_inflight = 8;              // launches in flight
  int max_batch = kDefaultBatch;     // requests per launch
  size_t budget = 0;
  void* arena_base = nullptr;
  Arena arena;
  std::vector<hipStream_t> copy;     // uploads, round robin (several DMA engines)
  int next_copy = 0;
  std::vector<hipStream_t> comp;
  int next_stream = 0;
  std::vector<std::unique_ptr<SMesh>> meshes;
  size_t pin_limit = size_t(32) << 30;      // pinned image bytes at most (the rest pageable)
  size_t pinned_bytes = 0;
  std::unordered_map<int64_t, Req> reqs;   // element addresses survive rehashing
  std::deque<int64_t> queue;
  std::vector<Launch> running;
  std::vector<hipEvent_t> event_pool;
  // launch tables: one slot per launch in flight, pinned host and device copies
  size_t param_bytes = 0, slot_bytes = 0;
  char* h_slots = nullptr;
  char* d_slots = nullptr;
  std::vector<int> free_slots;
  int64_t next_ticket = 1;
  uint64_t clock = 0;
  // statistics
  std::vector<double> latencies;
  int64_t evictions = 0, uploads = 0, completed = 0, upload_bytes = 0;
  int64_t launches = 0, shared_requests = 0, largest_launch = 0;
  std::string async_error;
  // threads
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_inflight;
  bool stop = false;
  bool paused = false;               // admission held (requests stay queued)
  std::thread scheduler, completer;

  ~cweno_server();
  void schedule_loop();
  void complete_loop();
  bool make_resident(SMesh& sm);
  void point_buffers(SMesh& sm, char* base);
  hipError_t launch_lone(const Req& r, hipStream_t s);
  hipError_t launch_table(const std::vector<int64_t>& pack, int slot, hipStream_t s);
  void release(int64_t ticket);
};

namespace {

template <typename T>
void copy_rows(const std::vector<double>& src, char* dst) {
  T* d = reinterpret_cast<T*>(dst);
  for (size_t t = 0; t < src.size(); ++t) d[t] = (T)src[t];
}

}  // namespace

void cweno_server::point_buffers(SMesh& sm, char* base) {
  cweno_mesh* m = sm.m.get();
  const Layout& L = sm.lay;
  cweno_abi::DevBuf& pinv = f32 ? m->pinv32 : m->pinv64;
  cweno_abi::DevBuf& binv = f32 ? m->binv32 : m->binv64;
  pinv.p = base ? base + L.pinv : nullptr;
  binv.p = base ? base + L.binv : nullptr;
  m->gidx.p = base ? base + L.gidx : nullptr;
  m->secpos.p = base ? base + L.secpos : nullptr;
  m->mask.p = base ? base + L.mask : nullptr;
  m->halo.p = base && m->maxH > 0 ? base + L.halo : nullptr;
  m->hoff.p = base && m->maxH > 0 ? base + L.hoff : nullptr;
  m->lidx.p = base && m->maxH > 0 ? base + L.lidx : nullptr;
}

// Place sm in the arena, evicting least recently used idle meshes as needed,
// and start its upload.  Returns false if it cannot be placed yet (every other
// resident mesh is in use); the caller waits for a completion and retries.
bool cweno_server::make_resident(SMesh& sm) {
  if (sm.resident) return true;
  size_t off = arena.alloc(sm.lay.total);
  while (off == SIZE_MAX) {
    SMesh* victim = nullptr;
    for (auto& x : meshes)
      if (x->resident && x->pins == 0 && x.get() != &sm && (!victim || x->last_use < victim->last_use))
        victim = x.get();
    if (!victim) return false;
    arena.release(victim->off, victim->lay.total);
    victim->resident = false;
    point_buffers(*victim, nullptr);
    ++evictions;
    off = arena.alloc(sm.lay.total);
  }
  sm.off = off;
  sm.resident = true;
  char* base = static_cast<char*>(arena_base) + off;
  point_buffers(sm, base);
  hipStream_t cs = copy[next_copy];
  next_copy = (next_copy + 1) % (int)copy.size();
  hipError_t e = hipMemcpyAsync(base, sm.image, sm.lay.total, hipMemcpyHostToDevice, cs);
  if (e == hipSuccess) e = hipEventRecord(sm.ready, cs);
  if (e != hipSuccess) async_error = std::string("upload failed: ") + hipGetErrorString(e);
  ++uploads;
  upload_bytes += (int64_t)sm.lay.total;
  return true;
}

// A lone request: the per-mesh kernel with the mesh's own variant choice.
hipError_t cweno_server::launch_lone(const Req& r, hipStream_t s) {
  const cweno_mesh* m = meshes[r.mesh]->m.get();
  hipError_t e = hipSuccess;
  for (int v0 = 0; v0 < r.n_vars && e == hipSuccess;) {
    const int vb = cweno_abi::pick_vb_mesh(m, r.n_vars - v0, f32);
    e = cweno_abi::launch_block(m, f32, r.q, r.coeffs, nullptr, nullptr, v0, vb, m->variant[f32][vb], s);
    v0 += vb;
  }
  return e;
}

// Several requests in one launch, packed into the slot's table (the batched
// persistent kernel, one launch per (dimension, degree, block size) group).
hipError_t cweno_server::launch_table(const std::vector<int64_t>& pack, int slot, hipStream_t s) {
  std::vector<cweno_abi::PackRequest> rq;
  for (int64_t t : pack) {
    const Req& r = reqs.at(t);
    rq.push_back({meshes[r.mesh]->m.get(), r.q, r.coeffs, r.n_vars});
  }
  char* h = h_slots + (size_t)slot * slot_bytes;
  char* d = d_slots + (size_t)slot * slot_bytes;
  const size_t items_off = (size_t)kSlotEntries * param_bytes;
  std::vector<cweno_abi::PackGroup> groups;
  int n_entries = 0;
  int64_t n_items = 0;
  cweno_abi::pack_requests(rq.data(), (int)rq.size(), f32, h, reinterpret_cast<cweno::BatchItem*>(h + items_off),
                           groups, n_entries, n_items);
  hipError_t e = hipMemcpyAsync(d, h, (size_t)n_entries * param_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d + items_off, h + items_off, (size_t)n_items * sizeof(cweno::BatchItem),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = cweno_abi::launch_packed(groups, f32, d, reinterpret_cast<const cweno::BatchItem*>(d + items_off), s);
  return e;
}

void cweno_server::schedule_loop() {
  if (hipSetDevice(device) != hipSuccess) return;
  std::unique_lock<std::mutex> lk(mu);
  std::vector<int64_t> pack;
  std::vector<SMesh*> used;
  while (true) {
    cv_sched.wait(lk, [&] { return stop || (!paused && !queue.empty() && (int)running.size() < max_inflight); });
    if (stop) break;
    // the longest prefix of the queue that fits one launch and whose meshes
    // can be made resident now
    pack.clear();
    used.clear();
    int entries = 0;
    int64_t items = 0;
    bool table = false;
    for (size_t at = 0; at < queue.size() && (int)pack.size() < max_batch; ++at) {
      const Req& r = reqs.at(queue[at]);
      SMesh& sm = *meshes[r.mesh];
      const cweno_abi::PackFootprint f = cweno_abi::pack_footprint(sm.m.get(), r.n_vars, f32);
      const bool fits = f.halo_ok && entries + f.entries <= kSlotEntries && items + f.items <= kSlotItems;
      if (!pack.empty() && !fits) break;
      if (!make_resident(sm)) break;
      sm.pins++;
      sm.last_use = ++clock;
      used.push_back(&sm);
      pack.push_back(queue[at]);
      entries += f.entries;
      items += f.items;
      if (!fits) break;             // runs alone as the per-mesh kernel
      table = pack.size() > 1;
    }
    if (pack.empty()) {
      // every other resident mesh is in use: a completion will free one
      cv_sched.wait_for(lk, std::chrono::milliseconds(1));
      continue;
    }
    queue.erase(queue.begin(), queue.begin() + (std::ptrdiff_t)pack.size());
    for (int64_t t : pack) reqs.at(t).state = kRunning;
    hipStream_t s = comp[next_stream];
    next_stream = (next_stream + 1) % (int)comp.size();
    if (event_pool.empty()) {
      hipEvent_t ev;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
      event_pool.push_back(ev);
    }
    Launch L;
    L.tickets = pack;
    L.done = event_pool.back();
    event_pool.pop_back();
    hipError_t e = L.done ? hipSuccess : hipErrorInvalidValue;
    std::sort(used.begin(), used.end());
    used.erase(std::unique(used.begin(), used.end()), used.end());
    for (SMesh* sm : used)
      if (e == hipSuccess) e = hipStreamWaitEvent(s, sm->ready, 0);
    if (e == hipSuccess) {
      if (table) {
        L.slot = free_slots.back();   // one slot per launch in flight: never empty here
        free_slots.pop_back();
        e = launch_table(pack, L.slot, s);
      } else {
        e = launch_lone(reqs.at(pack[0]), s);
      }
    }
    if (e == hipSuccess) e = hipEventRecord(L.done, s);
    if (e != hipSuccess) {
      // the launch did not start as a whole: its requests fail (work that did
      // start finishes before the stream is used again)
      async_error = std::string("launch failed: ") + hipGetErrorString(e);
      (void)hipStreamSynchronize(s);
      for (int64_t t : pack) {
        reqs.at(t).state = kFailed;
        meshes[reqs.at(t).mesh]->pins--;
      }
      if (L.slot >= 0) free_slots.push_back(L.slot);
      if (L.done) event_pool.push_back(L.done);
      cv_done.notify_all();
      continue;
    }
    ++launches;
    if (pack.size() > 1) shared_requests += (int64_t)pack.size();
    largest_launch = std::max(largest_launch, (int64_t)pack.size());
    running.push_back(std::move(L));
    cv_inflight.notify_all();
  }
}

void cweno_server::complete_loop() {
  if (hipSetDevice(device) != hipSuccess) return;
  std::vector<hipEvent_t> snapshot;
  std::vector<size_t> finished;
  while (true) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_inflight.wait(lk, [&] { return !running.empty() || stop; });
      if (running.empty() && stop) break;
      snapshot.clear();
      for (const Launch& L : running) snapshot.push_back(L.done);
    }
    // only this thread removes launches, so the first snapshot.size() entries
    // of `running` are still the ones polled here
    finished.clear();
    for (size_t k = 0; k < snapshot.size(); ++k)
      if (hipEventQuery(snapshot[k]) != hipErrorNotReady) finished.push_back(k);
    if (finished.empty()) {
      std::this_thread::yield();
      continue;
    }
    const double t_done = now_s();
    {
      std::lock_guard<std::mutex> g(mu);
      for (auto it = finished.rbegin(); it != finished.rend(); ++it) {
        Launch& L = running[*it];
        const hipError_t e = hipEventQuery(L.done);
        if (e != hipSuccess) async_error = std::string("request failed: ") + hipGetErrorString(e);
        for (int64_t t : L.tickets) {
          Req& r = reqs.at(t);
          r.state = e == hipSuccess ? kDone : kFailed;
          r.latency = t_done - r.t_submit;
          if (r.state == kDone) {
            latencies.push_back(r.latency);
            ++completed;
          }
          meshes[r.mesh]->pins--;
        }
        event_pool.push_back(L.done);
        if (L.slot >= 0) free_slots.push_back(L.slot);
        running.erase(running.begin() + (std::ptrdiff_t)*it);
      }
    }
    cv_sched.notify_all();
    cv_done.notify_all();
  }
}

// Forget a request whose final state has been reported (caller holds mu).
void cweno_server::release(int64_t ticket) {
  auto it = reqs.find(ticket);
  if (it != reqs.end() && it->second.state >= kDone && it->second.waiters == 0) reqs.erase(it);
}

cweno_server::~cweno_server() {
  {
    std::lock_guard<std::mutex> g(mu);
    stop = true;
    for (int64_t t : queue) reqs[t].state = kCancelled;
    queue.clear();
  }
  cv_sched.notify_all();
  cv_inflight.notify_all();
  if (scheduler.joinable()) scheduler.join();
  cv_inflight.notify_all();
  if (completer.joinable()) completer.join();
  for (hipStream_t s : comp)
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  for (hipStream_t s : copy)
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  for (hipEvent_t e : event_pool)
    if (e) (void)hipEventDestroy(e);
  for (auto& sm : meshes) {
    if (sm->ready) (void)hipEventDestroy(sm->ready);
    free_image(*sm);
  }
  if (arena_base) (void)hipFree(arena_base);
  if (d_slots) (void)hipFree(d_slots);
  if (h_slots) (void)hipHostFree(h_slots);
}

namespace {

cweno_status build_image(cweno_server* srv, SMesh& sm) {
  cweno_mesh* m = sm.m.get();
  const cweno::Operators& op = m->op;
  const size_t es = srv->f32 ? 4 : 8;
  cweno::Halo h;
  try {
    cweno::build_halo(op, cweno::kHaloBlock, h);
    m->maxH = h.max_len;
  } catch (const cweno::Error&) {
    m->maxH = 0;
  }
  Layout& L = sm.lay;
  size_t at = 0;
  auto place = [&](size_t bytes) {
    const size_t o = at;
    at += round_up(bytes);
    return o;
  };
  L.pinv = place(op.pinv.size() * es);
  L.binv = place(op.binv.size() * es);
  L.gidx = place(op.gidx.size() * 4);
  L.secpos = place(op.secpos.size());
  L.mask = place(op.mask.size());
  L.halo = place(m->maxH > 0 ? h.cells.size() * 4 : 0);
  L.hoff = place(m->maxH > 0 ? h.offset.size() * 4 : 0);
  L.lidx = place(m->maxH > 0 ? h.lidx.size() * 2 : 0);
  L.total = at;
  if (L.total > srv->budget) return fail(CWENO_E_BUDGET, "mesh larger than the server's HBM budget");
  // pinned memory up to the server's pinned limit (uploads at full bus speed),
  // pageable memory beyond it: the images of a large registered set can
  // exceed what the host may pin, and the runtime's own copies of pageable
  // memory need pinned staging memory that must stay available
  bool reserved = false;
  {
    // registrations may run concurrently: reserve the pinned bytes first
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->pinned_bytes + L.total <= srv->pin_limit) {
      srv->pinned_bytes += L.total;
      reserved = true;
    }
  }
  sm.pinned = reserved && hipHostMalloc(&sm.image, L.total, hipHostMallocDefault) == hipSuccess;
  if (!sm.pinned) {
    if (reserved) {
      std::lock_guard<std::mutex> g(srv->mu);
      srv->pinned_bytes -= L.total;
    }
    (void)hipGetLastError();
    sm.image = std::malloc(L.total);
    if (!sm.image) return fail(CWENO_E_NOMEM, "host allocation of the mesh image failed");
  }
  char* img = static_cast<char*>(sm.image);
  if (srv->f32) {
    copy_rows<float>(op.pinv, img + L.pinv);
    copy_rows<float>(op.binv, img + L.binv);
  } else {
    std::memcpy(img + L.pinv, op.pinv.data(), op.pinv.size() * 8);
    std::memcpy(img + L.binv, op.binv.data(), op.binv.size() * 8);
  }
  std::memcpy(img + L.gidx, op.gidx.data(), op.gidx.size() * 4);
  std::memcpy(img + L.secpos, op.secpos.data(), op.secpos.size());
  std::memcpy(img + L.mask, op.mask.data(), op.mask.size());
  if (m->maxH > 0) {
    std::memcpy(img + L.halo, h.cells.data(), h.cells.size() * 4);
    std::memcpy(img + L.hoff, h.offset.data(), h.offset.size() * 4);
    std::memcpy(img + L.lidx, h.lidx.data(), h.lidx.size() * 2);
  }
  return CWENO_OK;
}

}  // namespace

extern "C" {

cweno_status cweno_server_create(int64_t hbm_budget_bytes, cweno_dtype op_dtype, int max_inflight, int n_streams,
                                 cweno_server** out) {
  if (!out) return fail(CWENO_E_ARG, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes <= 0) return fail(CWENO_E_ARG, "budget must be positive");
  if (op_dtype != CWENO_F32 && op_dtype != CWENO_F64) return fail(CWENO_E_ARG, "bad dtype");
  if (max_inflight < 1 || max_inflight > 256) return fail(CWENO_E_ARG, "max_inflight must be in 1..256");
  if (n_streams < 1 || n_streams > 16) return fail(CWENO_E_ARG, "n_streams must be in 1..16");
  std::unique_ptr<cweno_server> s(new (std::nothrow) cweno_server());
  if (!s) return fail(CWENO_E_NOMEM, "host allocation failed");
  s->f32 = op_dtype == CWENO_F32;
  s->max_inflight = max_inflight;
  s->budget = round_up((size_t)hbm_budget_bytes);
  if (hipGetDevice(&s->device) != hipSuccess) return fail(CWENO_E_HIP, "no HIP device");
  if (cweno_status st = cweno_abi::configure_device_kernels()) return st;
  if (hipMalloc(&s->arena_base, s->budget) != hipSuccess)
    return fail(CWENO_E_NOMEM, "cannot allocate an HBM arena of the requested budget");
  s->arena.reset(s->budget);
  // launch tables: one slot per launch in flight
  s->param_bytes = s->f32 ? sizeof(cweno::KParams<float>) : sizeof(cweno::KParams<double>);
  s->slot_bytes = round_up((size_t)kSlotEntries * s->param_bytes + (size_t)kSlotItems * sizeof(cweno::BatchItem));
  if (hipMalloc(&s->d_slots, s->slot_bytes * (size_t)max_inflight) != hipSuccess ||
      hipHostMalloc(&s->h_slots, s->slot_bytes * (size_t)max_inflight, hipHostMallocDefault) != hipSuccess)
    return fail(CWENO_E_NOMEM, "cannot allocate the launch tables");
  for (int k = max_inflight - 1; k >= 0; --k) s->free_slots.push_back(k);
  s->copy.assign(kCopyStreams, nullptr);
  for (hipStream_t& x : s->copy)
    if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess)
      return fail(CWENO_E_HIP, "stream creation failed");
  s->comp.assign(n_streams, nullptr);
  for (hipStream_t& x : s->comp)
    if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess)
      return fail(CWENO_E_HIP, "stream creation failed");
  try {
    s->scheduler = std::thread([p = s.get()] { p->schedule_loop(); });
    s->completer = std::thread([p = s.get()] { p->complete_loop(); });
  } catch (const std::exception&) {
    return fail(CWENO_E_NOMEM, "thread creation failed");
  }
  *out = s.release();
  return CWENO_OK;
}

namespace {

// Take over a host-only mesh (its FP64 operators present) as a server mesh.
cweno_status adopt(cweno_server* s, cweno_mesh* raw, int64_t* mesh_id) {
  std::unique_ptr<SMesh> sm(new (std::nothrow) SMesh());
  if (!sm) {
    cweno_mesh_destroy(raw);
    return fail(CWENO_E_NOMEM, "host allocation failed");
  }
  sm->m.reset(raw);
  cweno_mesh* m = raw;
  if (cweno_status st = build_image(s, *sm)) {
    if (sm->image && sm->pinned) {
      // give back the pinned reservation of the failed registration
      std::lock_guard<std::mutex> g(s->mu);
      s->pinned_bytes -= sm->lay.total;
    }
    free_image(*sm);
    return st;
  }
  // the image holds everything the device needs; keep only the host tables
  std::vector<double>().swap(m->op.pinv);
  std::vector<double>().swap(m->op.binv);
  std::vector<int32_t>().swap(m->op.gidx);
  std::vector<uint8_t>().swap(m->op.secpos);
  m->flags &= ~(unsigned)CWENO_FLAG_HOST_ONLY;
  m->ops = s->f32 ? CWENO_OPS_F32 : CWENO_OPS_F64;
  m->device = s->device;
  m->owns_device = false;
  m->device_bytes = (int64_t)sm->lay.total;
  for (int t = 0; t < 2; ++t)
    for (int vb = 0; vb < 10; ++vb) m->variant[t][vb] = vb == 0 ? -1 : cweno_abi::default_variant(m, vb, t == 1);
  if (hipEventCreateWithFlags(&sm->ready, hipEventDisableTiming) != hipSuccess) {
    free_image(*sm);
    return fail(CWENO_E_HIP, "event creation failed");
  }
  std::lock_guard<std::mutex> g(s->mu);
  *mesh_id = (int64_t)s->meshes.size();
  s->meshes.push_back(std::move(sm));
  return CWENO_OK;
}

}  // namespace

cweno_status cweno_server_register(cweno_server* s, int dim, int64_t n_vertices, const double* vertices,
                                   int64_t n_cells, const int32_t* cells, int degree, const cweno_options* opt,
                                   int64_t* mesh_id) {
  if (!s || !mesh_id) return fail(CWENO_E_ARG, "server and mesh_id must not be NULL");
  cweno_options o{};
  if (opt) o = *opt;
  if (o.flags & (CWENO_FLAG_WENO | CWENO_FLAG_MOVING))
    return fail(CWENO_E_ARG, "the server holds stored CWENO operators only (no WENO or moving meshes)");
  o.flags |= CWENO_FLAG_HOST_ONLY;
  o.ops = s->f32 ? CWENO_OPS_F32 : CWENO_OPS_F64;
  cweno_mesh* raw = nullptr;
  if (cweno_status st = cweno_mesh_create(dim, n_vertices, vertices, n_cells, cells, degree, &o, nullptr, &raw))
    return st;
  return adopt(s, raw, mesh_id);
}

cweno_status cweno_server_register_mesh(cweno_server* s, const cweno_mesh* host_mesh, int64_t* mesh_id) {
  if (!s || !mesh_id || !host_mesh) return fail(CWENO_E_ARG, "server, mesh and mesh_id must not be NULL");
  if (!(host_mesh->flags & CWENO_FLAG_HOST_ONLY) || host_mesh->op.pinv.empty())
    return fail(CWENO_E_ARG, "register_mesh takes a host-only mesh (built with CWENO_FLAG_HOST_ONLY)");
  cweno_mesh* copy = nullptr;
  try {
    copy = new cweno_mesh(*host_mesh);
  } catch (const std::bad_alloc&) {
    return fail(CWENO_E_NOMEM, "host allocation failed");
  }
  return adopt(s, copy, mesh_id);
}

cweno_status cweno_server_mesh_info(cweno_server* s, int64_t mesh_id, int64_t* n_cells, int* n_basis,
                                    int64_t* image_bytes, int* resident) {
  if (!s) return fail(CWENO_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  if (mesh_id < 0 || mesh_id >= (int64_t)s->meshes.size()) return fail(CWENO_E_ARG, "unknown mesh id");
  const SMesh& sm = *s->meshes[mesh_id];
  if (n_cells) *n_cells = sm.m->nc;
  if (n_basis) *n_basis = sm.m->nb;
  if (image_bytes) *image_bytes = (int64_t)sm.lay.total;
  if (resident) *resident = sm.resident ? 1 : 0;
  return CWENO_OK;
}

cweno_status cweno_server_submit(cweno_server* s, int64_t mesh_id, int n_vars, cweno_dtype dtype, const void* q,
                                 void* coeffs, int64_t* ticket) {
  if (!s || !ticket) return fail(CWENO_E_ARG, "server and ticket must not be NULL");
  if ((dtype == CWENO_F32) != s->f32 || (dtype != CWENO_F32 && dtype != CWENO_F64))
    return fail(CWENO_E_ARG, "dtype differs from the server's operator precision");
  if (n_vars < 1) return fail(CWENO_E_ARG, "n_vars must be >= 1");
  if (!q || !coeffs) return fail(CWENO_E_ARG, "q and coeffs must be device pointers");
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) return fail(CWENO_E_CANCELLED, "server is shutting down");
  if (mesh_id < 0 || mesh_id >= (int64_t)s->meshes.size()) return fail(CWENO_E_ARG, "unknown mesh id");
  const cweno_mesh* m = s->meshes[mesh_id]->m.get();
  const uint64_t es = s->f32 ? 4 : 8, nq = (uint64_t)n_vars * m->nc * es, nco = nq * m->nb;
  const uintptr_t x = (uintptr_t)q, y = (uintptr_t)coeffs;
  if (x < y + nco && y < x + nq) return fail(CWENO_E_ARG, "q overlaps coeffs");
  if ((uint64_t)m->nc * m->nb * es >= (uint64_t(1) << 32))
    return fail(CWENO_E_ARG, "too many cells for 32-bit offsets within one variable's coefficients");
  const int64_t t = s->next_ticket++;
  Req& r = s->reqs[t];
  r.mesh = mesh_id;
  r.n_vars = n_vars;
  r.q = q;
  r.coeffs = coeffs;
  r.t_submit = now_s();
  r.state = kQueued;
  s->queue.push_back(t);
  *ticket = t;
  s->cv_sched.notify_one();
  return CWENO_OK;
}

cweno_status cweno_server_poll(cweno_server* s, int64_t ticket, int* done) {
  if (!s || !done) return fail(CWENO_E_ARG, "server and done must not be NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(CWENO_E_ARG, "unknown ticket");
  const int state = it->second.state;
  *done = state >= kDone ? 1 : 0;
  s->release(ticket);                // a reported final state ends the ticket
  if (state == kCancelled) return fail(CWENO_E_CANCELLED, "request was cancelled");
  if (state == kFailed) return fail(CWENO_E_HIP, "request failed: " + s->async_error);
  return CWENO_OK;
}

cweno_status cweno_server_wait(cweno_server* s, int64_t ticket, double timeout_s) {
  if (!s) return fail(CWENO_E_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(CWENO_E_ARG, "unknown ticket");
  // the element itself (not the iterator) stays valid while the map grows;
  // it is erased only once no thread waits on it
  Req* r = &it->second;
  r->waiters++;
  const auto pred = [&] { return r->state >= kDone; };
  bool finished = true;
  if (timeout_s < 0) s->cv_done.wait(lk, pred);
  else finished = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
  r->waiters--;
  const int state = r->state;
  if (!finished) return fail(CWENO_E_BUSY, "timed out");
  s->release(ticket);
  if (state == kCancelled) return fail(CWENO_E_CANCELLED, "request was cancelled");
  if (state == kFailed) return fail(CWENO_E_HIP, "request failed: " + s->async_error);
  return CWENO_OK;
}

cweno_status cweno_server_cancel(cweno_server* s, int64_t ticket) {
  if (!s) return fail(CWENO_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(CWENO_E_ARG, "unknown ticket");
  if (it->second.state != kQueued) return fail(CWENO_E_BUSY, "request already running or finished");
  s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
  it->second.state = kCancelled;
  s->cv_done.notify_all();
  return CWENO_OK;
}

cweno_status cweno_server_set_pinned_limit(cweno_server* s, int64_t bytes) {
  if (!s) return fail(CWENO_E_ARG, "server is NULL");
  if (bytes < 0) return fail(CWENO_E_ARG, "the pinned limit must not be negative");
  std::lock_guard<std::mutex> g(s->mu);
  s->pin_limit = (size_t)bytes;
  return CWENO_OK;
}

cweno_status cweno_server_set_batch(cweno_server* s, int max_batch) {
  if (!s) return fail(CWENO_E_ARG, "server is NULL");
  if (max_batch < 1 || max_batch > kSlotEntries) return fail(CWENO_E_ARG, "max_batch must be in 1..512");
  std::lock_guard<std::mutex> g(s->mu);
  s->max_batch = max_batch;
  return CWENO_OK;
}

cweno_status cweno_server_launch_stats(cweno_server* s, int64_t* launches, int64_t* shared_requests,
                                       int64_t* largest_launch, int64_t* tickets_held) {
  if (!s) return fail(CWENO_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  if (launches) *launches = s->launches;
  if (shared_requests) *shared_requests = s->shared_requests;
  if (largest_launch) *largest_launch = s->largest_launch;
  if (tickets_held) *tickets_held = (int64_t)s->reqs.size();
  return CWENO_OK;
}

cweno_status cweno_server_stats(cweno_server* s, double* p50_s, double* p99_s, double* p999_s, int64_t* completed,
                                int64_t* evictions, int64_t* uploads, int64_t* upload_bytes) {
  if (!s) return fail(CWENO_E_ARG, "server is NULL");
  std::vector<double> lat;
  {
    std::lock_guard<std::mutex> g(s->mu);
    lat = s->latencies;
    if (completed) *completed = s->completed;
    if (evictions) *evictions = s->evictions;
    if (uploads) *uploads = s->uploads;
    if (upload_bytes) *upload_bytes = s->upload_bytes;
  }
  auto quant = [&](double q) {
    if (lat.empty()) return 0.0;
    const size_t k = std::min(lat.size() - 1, (size_t)(q * (double)(lat.size() - 1) + 0.5));
    std::nth_element(lat.begin(), lat.begin() + k, lat.end());
    return lat[k];
  };
  if (p50_s) *p50_s = quant(0.5);
  if (p99_s) *p99_s = quant(0.99);
  if (p999_s) *p999_s = quant(0.999);
  return CWENO_OK;
}

cweno_status cweno_server_reset_stats(cweno_server* s) {
  if (!s) return fail(CWENO_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> g(s->mu);
  s->latencies.clear();
  s->completed = s->evictions = s->uploads = s->upload_bytes = 0;
  s->launches = s->shared_requests = s->largest_launch = 0;
  return CWENO_OK;
}

cweno_status cweno_server_pause(cweno_server* s, int paused) {
  if (!s) return fail(CWENO_E_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->paused = paused != 0;
  }
  s->cv_sched.notify_all();
  return CWENO_OK;
}

cweno_status cweno_server_destroy(cweno_server* s) {
  delete s;
  return CWENO_OK;
}

}  // extern "C"
