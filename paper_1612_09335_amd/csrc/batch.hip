// Batched reconstruction: many registered meshes in one graph launch.
//
// The meshes' variable blocks are grouped by (dimension, degree, block size);
// every group runs as one persistent kernel (reconstruct_batch_kernel) over a
// work list of (table entry, block of 256 cells) items, the table holding the
// kernel parameters of each (mesh, variable block).  The group kernels are
// captured into one HIP graph as parallel branches.  The caller's input and
// output pointers change from run to run, so they live in the device table,
// refreshed by one small host-to-device copy (from pinned memory) before each
// graph launch; the graph itself holds kernel nodes only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "cweno.h"
#include "mesh.hpp"
#include "pack.hpp"

using cweno_abi::fail;

namespace {

struct Entry {            // one (mesh, variable block)
  int mesh, v0, vb;
};

struct Group {            // meshes sharing (d, M, vb): one persistent kernel
  int d, M, vb;
  std::vector<int> entries;
  int item0 = 0, n_items = 0;
  size_t lds = 0;
  int variant = -1, grid = 0;
  float ms = 0.0f;
};

constexpr int kSlots = 2;        // pinned host copies of the table
constexpr int kSideStreams = 4;  // graph branches are recorded on these

}  // namespace

struct cweno_batch {
  bool f32 = false;
  int device = -1;
  std::vector<const cweno_mesh*> meshes;
  std::vector<int> n_vars;
  std::vector<Entry> entries;
  std::vector<Group> groups;
  size_t param_bytes = 0;            // sizeof(KParams<T>)
  void* d_table = nullptr;           // [entries] KParams<T>
  void* d_items = nullptr;           // [items] BatchItem
  void* h_table[kSlots] = {nullptr, nullptr};
  hipEvent_t slot_done[kSlots] = {nullptr, nullptr};
  int slot = 0;
  hipEvent_t last_run = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double tuned_ms = 0.0;

  ~cweno_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (int t = 0; t < kSlots; ++t) {
      if (slot_done[t]) {
        (void)hipEventSynchronize(slot_done[t]);
        (void)hipEventDestroy(slot_done[t]);
      }
      if (h_table[t]) (void)hipHostFree(h_table[t]);
    }
    if (last_run) (void)hipEventDestroy(last_run);
    if (d_table) (void)hipFree(d_table);
    if (d_items) (void)hipFree(d_items);
  }
};

namespace {

// Kernel parameters of every entry, with the given per-mesh buffers.
template <typename T>
void fill_table(const cweno_batch* b, const void* const* q, void* const* coeffs, void* dst) {
  auto* tab = static_cast<cweno::KParams<T>*>(dst);
  for (size_t e = 0; e < b->entries.size(); ++e) {
    const Entry& en = b->entries[e];
    tab[e] = cweno_abi::make_params<T>(b->meshes[en.mesh], q[en.mesh], coeffs[en.mesh], nullptr, nullptr, en.v0);
  }
}

hipError_t launch_group(const cweno_batch* b, const Group& g, int variant, int grid, hipStream_t s) {
  const int n = g.n_items;
  grid = std::max(1, std::min(grid, n));
  const auto* items = static_cast<const cweno::BatchItem*>(b->d_items) + g.item0;
  if (b->f32)
    return cweno::launch_batch<float>(g.d, g.M, static_cast<const cweno::KParams<float>*>(b->d_table), items, n,
                                      grid, g.lds, g.vb, variant, s);
  return cweno::launch_batch<double>(g.d, g.M, static_cast<const cweno::KParams<double>*>(b->d_table), items, n,
                                     grid, g.lds, g.vb, variant, s);
}

std::string group_key(const cweno_batch* b, const Group& g) {
  std::ostringstream k;
  k << "d" << g.d << "_M" << g.M << "_vb" << g.vb << "_" << (b->f32 ? "f32" : "f64") << "_items" << g.n_items
    << "_lds" << g.lds;
  return k.str();
}

// Tune cache: one line per group, "<key> <variant> <grid>".
void read_cache(const char* path, std::vector<std::pair<std::string, std::pair<int, int>>>& out) {
  if (!path) return;
  std::ifstream f(path);
  std::string key;
  int k, grid;
  while (f >> key >> k >> grid) out.push_back({key, {k, grid}});
}

cweno_status tune_groups(cweno_batch* b, const char* cache_path, hipStream_t s) {
  std::vector<std::pair<std::string, std::pair<int, int>>> cache;
  read_cache(cache_path, cache);
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess || n_cu < 1)
    n_cu = 256;
  const int grids[] = {n_cu, 2 * n_cu, 3 * n_cu, 4 * n_cu, 8 * n_cu};
  bool any_new = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(CWENO_E_HIP, "hipEventCreate failed");
  }
  cweno_status st = CWENO_OK;
  b->tuned_ms = 0.0;
  for (Group& g : b->groups) {
    const std::string key = group_key(b, g);
    bool cached = false;
    for (auto& c : cache)
      if (c.first == key) {
        g.variant = c.second.first;
        g.grid = c.second.second;
        cached = true;
      }
    float best = 0.0f;
    for (int k = 0; k < cweno::kNumVariants && st == CWENO_OK; ++k) {
      if (cweno::kVariants[k].kind != 1) continue;
      if (cached && k != g.variant) continue;
      for (int grid : grids) {
        if (cached && grid != g.grid) continue;
        hipError_t e = launch_group(b, g, k, grid, s);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int t = 0; t < 3 && e == hipSuccess; ++t) e = launch_group(b, g, k, grid, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          st = fail(CWENO_E_HIP, std::string("batch tuning launch failed: ") + hipGetErrorString(e));
          break;
        }
        ms /= 3.0f;
        if (g.variant < 0 || ms < best || (cached && k == g.variant && grid == g.grid)) {
          best = ms;
          g.variant = k;
          g.grid = grid;
        }
        if (grid >= g.n_items) break;   // larger grids add nothing
      }
    }
    if (st != CWENO_OK) break;
    g.ms = best;
    b->tuned_ms += best;
    if (!cached) {
      cache.push_back({key, {g.variant, g.grid}});
      any_new = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == CWENO_OK && cache_path && any_new) {
    std::ofstream f(cache_path, std::ios::trunc);
    for (auto& c : cache) f << c.first << " " << c.second.first << " " << c.second.second << "\n";
  }
  return st;
}

cweno_status capture_graph(cweno_batch* b) {
  hipStream_t cap = nullptr, side[kSideStreams] = {};
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins(b->groups.size(), nullptr);
  cweno_status st = CWENO_OK;
  auto cleanup = [&]() {
    for (hipEvent_t e : joins)
      if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (hipStream_t x : side)
      if (x) (void)hipStreamDestroy(x);
    if (cap) (void)hipStreamDestroy(cap);
  };
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
    cleanup();
    return fail(CWENO_E_HIP, "stream/event creation failed");
  }
  for (hipStream_t& x : side)
    if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) {
      cleanup();
      return fail(CWENO_E_HIP, "stream creation failed");
    }
  for (hipEvent_t& e : joins)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return fail(CWENO_E_HIP, "event creation failed");
    }
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) e = hipEventRecord(fork, cap);
  for (size_t gi = 0; gi < b->groups.size() && e == hipSuccess; ++gi) {
    hipStream_t x = side[gi % kSideStreams];
    e = hipStreamWaitEvent(x, fork, 0);
    if (e == hipSuccess) e = launch_group(b, b->groups[gi], b->groups[gi].variant, b->groups[gi].grid, x);
    if (e == hipSuccess) e = hipEventRecord(joins[gi], x);
    if (e == hipSuccess) e = hipStreamWaitEvent(cap, joins[gi], 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(cap, &graph);
  if (e == hipSuccess) e = e_end;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    st = fail(CWENO_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e));
  } else {
    b->graph = graph;
  }
  cleanup();
  return st;
}

template <typename T>
size_t param_size() { return sizeof(cweno::KParams<T>); }

}  // namespace

extern "C" {

cweno_status cweno_batch_create(int n, cweno_mesh* const* meshes, const int* n_vars, cweno_dtype dtype,
                                const char* tune_cache_path, void* hip_stream, cweno_batch** out) {
  if (!out) return fail(CWENO_E_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || !meshes || !n_vars) return fail(CWENO_E_ARG, "need at least one mesh");
  if (dtype != CWENO_F64 && dtype != CWENO_F32) return fail(CWENO_E_ARG, "bad dtype");
  const bool f32 = dtype == CWENO_F32;
  std::unique_ptr<cweno_batch> b(new (std::nothrow) cweno_batch());
  if (!b) return fail(CWENO_E_NOMEM, "host allocation failed");
  b->f32 = f32;
  b->param_bytes = f32 ? param_size<float>() : param_size<double>();
  if (hipGetDevice(&b->device) != hipSuccess) return fail(CWENO_E_HIP, "no HIP device");
  if (cweno_status cst = cweno_abi::configure_device_kernels()) return cst;
  hipStream_t s = (hipStream_t)hip_stream;

  // entries (mesh, variable block) and their groups
  for (int i = 0; i < n; ++i) {
    const cweno_mesh* m = meshes[i];
    if (!m) return fail(CWENO_E_ARG, "mesh " + std::to_string(i) + " is NULL");
    if (m->flags & CWENO_FLAG_HOST_ONLY) return fail(CWENO_E_ARG, "mesh " + std::to_string(i) + " is host-only");
    if (m->device != b->device) return fail(CWENO_E_ARG, "mesh " + std::to_string(i) + " lives on another device");
    if ((f32 && !m->pinv32.p) || (!f32 && !m->pinv64.p))
      return fail(CWENO_E_ARG, "mesh " + std::to_string(i) + " holds no operators of this precision");
    if (n_vars[i] < 1) return fail(CWENO_E_ARG, "n_vars must be >= 1");
    if ((uint64_t)m->nc * (uint64_t)m->nb * (f32 ? 4u : 8u) >= (uint64_t(1) << 32))
      return fail(CWENO_E_ARG, "mesh " + std::to_string(i) + " too large for 32-bit coefficient offsets");
    b->meshes.push_back(m);
    b->n_vars.push_back(n_vars[i]);
    for (int v0 = 0; v0 < n_vars[i];) {
      const int vb = cweno_abi::pick_vb_mesh(m, n_vars[i] - v0, f32, true);
      bool halo_ok = false;
      for (int k = 0; k < cweno::kNumVariants; ++k)
        if (cweno::kVariants[k].kind == 1 && cweno_abi::variant_ok(m, vb, k, f32)) halo_ok = true;
      if (!halo_ok)
        return fail(CWENO_E_ARG, "mesh " + std::to_string(i) + ": its block halos do not fit in LDS (the batch "
                                 "runs the LDS-halo kernel only; reconstruct this mesh on its own)");
      const int e = (int)b->entries.size();
      b->entries.push_back({i, v0, vb});
      Group* g = nullptr;
      for (Group& x : b->groups)
        if (x.d == m->d && x.M == m->M && x.vb == vb) g = &x;
      if (!g) {
        b->groups.push_back(Group{m->d, m->M, vb, {}, 0, 0, 0, -1, 0, 0.0f});
        g = &b->groups.back();
      }
      g->entries.push_back(e);
      g->lds = std::max(g->lds, (size_t)m->maxH * vb * (f32 ? 4 : 8));
      v0 += vb;
    }
  }
  // work list: per group, the blocks of its entries, interleaved entry by entry
  std::vector<cweno::BatchItem> items;
  for (Group& g : b->groups) {
    g.item0 = (int)items.size();
    std::vector<int64_t> nblk;
    int64_t most = 0;
    for (int e : g.entries) {
      nblk.push_back((b->meshes[b->entries[e].mesh]->nc + cweno::kHaloBlock - 1) / cweno::kHaloBlock);
      most = std::max(most, nblk.back());
    }
    for (int64_t blk = 0; blk < most; ++blk)
      for (size_t t = 0; t < g.entries.size(); ++t)
        if (blk < nblk[t]) items.push_back({g.entries[t], (int32_t)blk});
    g.n_items = (int)items.size() - g.item0;
    if ((int64_t)items.size() >= (int64_t(1) << 31)) return fail(CWENO_E_ARG, "work list too long");
  }

  // device table and work list, pinned host copies of the table
  const size_t tab_bytes = b->entries.size() * b->param_bytes;
  hipError_t e = hipMalloc(&b->d_table, tab_bytes);
  if (e == hipSuccess) e = hipMalloc(&b->d_items, items.size() * sizeof(cweno::BatchItem));
  if (e != hipSuccess) return fail(CWENO_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(cweno::BatchItem), hipMemcpyHostToDevice);
  for (int t = 0; t < kSlots && e == hipSuccess; ++t) {
    e = hipHostMalloc(&b->h_table[t], tab_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->slot_done[t], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->last_run, hipEventDisableTiming);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("batch set-up failed: ") + hipGetErrorString(e));

  // autotune on scratch buffers (zero averages), then capture
  {
    std::vector<void*> sq(n, nullptr), so(n, nullptr);
    const size_t es = f32 ? 4 : 8;
    cweno_status st = CWENO_OK;
    for (int i = 0; i < n && st == CWENO_OK; ++i) {
      const cweno_mesh* m = b->meshes[i];
      const size_t qb = (size_t)n_vars[i] * m->nc * es, ob = qb * m->nb;
      if (hipMalloc(&sq[i], qb) != hipSuccess || hipMalloc(&so[i], ob) != hipSuccess)
        st = fail(CWENO_E_NOMEM, "scratch allocation for tuning failed");
      else if (hipMemsetAsync(sq[i], 0, qb, s) != hipSuccess)
        st = fail(CWENO_E_HIP, "hipMemsetAsync failed");
    }
    if (st == CWENO_OK) {
      if (f32) fill_table<float>(b.get(), sq.data(), so.data(), b->h_table[0]);
      else fill_table<double>(b.get(), sq.data(), so.data(), b->h_table[0]);
      if (hipMemcpyAsync(b->d_table, b->h_table[0], tab_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        st = fail(CWENO_E_HIP, "table copy failed");
    }
    if (st == CWENO_OK) st = tune_groups(b.get(), tune_cache_path, s);
    (void)hipStreamSynchronize(s);
    for (int i = 0; i < n; ++i) {
      if (sq[i]) (void)hipFree(sq[i]);
      if (so[i]) (void)hipFree(so[i]);
    }
    if (st) return st;
  }
  if (cweno_status st = capture_graph(b.get())) return st;
  *out = b.release();
  return CWENO_OK;
}

cweno_status cweno_batch_run(cweno_batch* b, const void* const* q, void* const* coeffs, void* hip_stream) {
  if (!b) return fail(CWENO_E_ARG, "batch is NULL");
  if (!q || !coeffs) return fail(CWENO_E_ARG, "q and coeffs must be arrays of device pointers");
  const size_t es = b->f32 ? 4 : 8;
  for (size_t i = 0; i < b->meshes.size(); ++i) {
    if (!q[i] || !coeffs[i]) return fail(CWENO_E_ARG, "mesh " + std::to_string(i) + ": NULL buffer");
    const uint64_t nq = (uint64_t)b->n_vars[i] * b->meshes[i]->nc * es, nco = nq * b->meshes[i]->nb;
    const uintptr_t x = (uintptr_t)q[i], y = (uintptr_t)coeffs[i];
    if (x < y + nco && y < x + nq) return fail(CWENO_E_ARG, "mesh " + std::to_string(i) + ": q overlaps coeffs");
  }
  hipStream_t s = (hipStream_t)hip_stream;
  const int slot = b->slot;
  b->slot = (b->slot + 1) % kSlots;
  // the pinned slot may still be read by an earlier copy
  hipError_t e = hipEventSynchronize(b->slot_done[slot]);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("hipEventSynchronize failed: ") + hipGetErrorString(e));
  if (b->f32) fill_table<float>(b, q, coeffs, b->h_table[slot]);
  else fill_table<double>(b, q, coeffs, b->h_table[slot]);
  // runs on different streams are ordered: the table is rewritten only after the previous graph
  e = hipStreamWaitEvent(s, b->last_run, 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_table, b->h_table[slot], b->entries.size() * b->param_bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(b->slot_done[slot], s);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, s);
  if (e == hipSuccess) e = hipEventRecord(b->last_run, s);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("batch launch failed: ") + hipGetErrorString(e));
  return CWENO_OK;
}

cweno_status cweno_batch_info(const cweno_batch* b, int* n_groups, int64_t* n_items, double* tuned_ms) {
  if (!b) return fail(CWENO_E_ARG, "batch is NULL");
  if (n_groups) *n_groups = (int)b->groups.size();
  if (n_items) {
    int64_t t = 0;
    for (const Group& g : b->groups) t += g.n_items;
    *n_items = t;
  }
  if (tuned_ms) *tuned_ms = b->tuned_ms;
  return CWENO_OK;
}

cweno_status cweno_batch_group(const cweno_batch* b, int g, int* dim, int* degree, int* vb, int* n_entries,
                               int* n_items, int* variant, int* grid, double* ms) {
  if (!b) return fail(CWENO_E_ARG, "batch is NULL");
  if (g < 0 || g >= (int)b->groups.size()) return fail(CWENO_E_ARG, "group out of range");
  const Group& x = b->groups[g];
  if (dim) *dim = x.d;
  if (degree) *degree = x.M;
  if (vb) *vb = x.vb;
  if (n_entries) *n_entries = (int)x.entries.size();
  if (n_items) *n_items = x.n_items;
  if (variant) *variant = x.variant;
  if (grid) *grid = std::min(x.grid, x.n_items);
  if (ms) *ms = x.ms;
  return CWENO_OK;
}

cweno_status cweno_batch_destroy(cweno_batch* b) {
  delete b;
  return CWENO_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched reconstruction without allocation (cweno_batch_run_noalloc).
//
// The launch table and work list live in `scratch`, a static device array of
// kNoAllocBytes that each GPU holds for the life of the process.  Host code
// never uses the array's name as an address: on a device's first call its
// address on that device is looked up once with hipGetSymbolAddress and kept
// per device.  The table is packed into a static host stage and copied into
// the device array on the caller's stream; an event recorded after the copy
// guards the host stage against the next call.  Every call on one GPU uses
// the same device array: calls that overlap on one GPU (different streams,
// not ordered) race.

namespace {

constexpr int kNoAllocEntries = 256;       // (mesh, variable block) entries
constexpr int kNoAllocItems = 1 << 16;     // 256-cell blocks over all meshes
constexpr size_t kNoAllocTable = (size_t)kNoAllocEntries * sizeof(cweno::KParams<double>);
constexpr size_t kNoAllocBytes = kNoAllocTable + (size_t)kNoAllocItems * sizeof(cweno::BatchItem);
static_assert(sizeof(cweno::KParams<float>) <= sizeof(cweno::KParams<double>), "table slot size");
static_assert(kNoAllocTable % 256 == 0, "work list alignment");

constexpr int kMaxDevices = 64;

struct NoAllocDevice {
  char* scratch = nullptr;        // the array's address on this device
  hipEvent_t staged = nullptr;    // the last call's copy out of the host stage has finished
};

std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[kMaxDevices];
alignas(256) char g_noalloc_stage[kNoAllocBytes];

}  // namespace

static __device__ __align__(256) char scratch[kNoAllocBytes];

extern "C" cweno_status cweno_batch_run_noalloc(int n, const cweno_mesh* const* meshes, const int* n_vars,
                                                cweno_dtype dtype, const void* const* q, void* const* coeffs,
                                                void* hip_stream) {
  if (n < 1 || !meshes || !n_vars || !q || !coeffs) return fail(CWENO_E_ARG, "need at least one mesh and its buffers");
  if (dtype != CWENO_F64 && dtype != CWENO_F32) return fail(CWENO_E_ARG, "bad dtype");
  const bool f32 = dtype == CWENO_F32;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(CWENO_E_HIP, "no HIP device");
  if (dev >= kMaxDevices) return fail(CWENO_E_ARG, "device index beyond the supported 64");
  const size_t es = f32 ? 4 : 8;
  std::vector<cweno_abi::PackRequest> rq;
  int entries = 0;
  int64_t items = 0;
  for (int i = 0; i < n; ++i) {
    const cweno_mesh* m = meshes[i];
    const std::string who = "mesh " + std::to_string(i);
    if (!m) return fail(CWENO_E_ARG, who + " is NULL");
    if (m->flags & CWENO_FLAG_HOST_ONLY) return fail(CWENO_E_ARG, who + " is host-only");
    if (m->device != dev) return fail(CWENO_E_ARG, who + " lives on another device");
    if ((f32 && !m->pinv32.p) || (!f32 && !m->pinv64.p))
      return fail(CWENO_E_ARG, who + " holds no operators of this precision");
    if (n_vars[i] < 1) return fail(CWENO_E_ARG, "n_vars must be >= 1");
    if (!q[i] || !coeffs[i]) return fail(CWENO_E_ARG, who + ": NULL buffer");
    if ((uint64_t)m->nc * (uint64_t)m->nb * es >= (uint64_t(1) << 32))
      return fail(CWENO_E_ARG, who + " too large for 32-bit coefficient offsets");
    const uint64_t nq = (uint64_t)n_vars[i] * m->nc * es, nco = nq * m->nb;
    if (cweno_abi::overlap(q[i], nq, coeffs[i], nco)) return fail(CWENO_E_ARG, who + ": q overlaps coeffs");
    const cweno_abi::PackFootprint f = cweno_abi::pack_footprint(m, n_vars[i], f32);
    if (!f.halo_ok)
      return fail(CWENO_E_ARG, who + ": its block halos do not fit in LDS (reconstruct this mesh on its own)");
    entries += f.entries;
    items += f.items;
    rq.push_back({m, q[i], coeffs[i], n_vars[i]});
  }
  if (entries > kNoAllocEntries || items > kNoAllocItems)
    return fail(CWENO_E_ARG, "batch too large for the static scratch: " + std::to_string(entries) +
                                 " variable blocks (at most 256) and " + std::to_string(items) +
                                 " blocks of 256 cells (at most 65536)");
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  NoAllocDevice& D = g_noalloc[dev];
  if (!D.scratch) {
    // set-up on this device's first call: kernel attributes, the array's address, the stage event
    if (cweno_status st = cweno_abi::configure_device_kernels()) return st;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CWENO_E_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    if (!D.staged && hipEventCreateWithFlags(&D.staged, hipEventDisableTiming) != hipSuccess)
      return fail(CWENO_E_HIP, "event creation failed");
    D.scratch = static_cast<char*>(ptr);
  }
  hipStream_t s = (hipStream_t)hip_stream;
  // the previous call's copy out of the host stage must be complete
  hipError_t e = hipEventSynchronize(D.staged);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("hipEventSynchronize failed: ") + hipGetErrorString(e));
  std::vector<cweno_abi::PackGroup> groups;
  int n_entries = 0;
  int64_t n_items = 0;
  auto* h_items = reinterpret_cast<cweno::BatchItem*>(g_noalloc_stage + kNoAllocTable);
  cweno_abi::pack_requests(rq.data(), (int)rq.size(), f32, g_noalloc_stage, h_items, groups, n_entries, n_items);
  const size_t pb = f32 ? sizeof(cweno::KParams<float>) : sizeof(cweno::KParams<double>);
  e = hipMemcpyAsync(D.scratch, g_noalloc_stage, (size_t)n_entries * pb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(D.scratch + kNoAllocTable, h_items, (size_t)n_items * sizeof(cweno::BatchItem),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(D.staged, s);
  if (e == hipSuccess)
    e = cweno_abi::launch_packed(groups, f32, D.scratch,
                                 reinterpret_cast<const cweno::BatchItem*>(D.scratch + kNoAllocTable), s);
  if (e != hipSuccess) return fail(CWENO_E_HIP, std::string("batched launch failed: ") + hipGetErrorString(e));
  return CWENO_OK;
}
