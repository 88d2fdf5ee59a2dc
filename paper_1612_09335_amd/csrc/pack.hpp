// Packing several reconstructions (meshes with their own inputs and outputs)
// into one launch table for the batched persistent kernel, and launching it.
//
// Each request's variable blocks become entries of the table (one KParams
// each); entries sharing (dimension, degree, block size) form a group, run as
// one launch of reconstruct_batch_kernel over the group's work items, one
// item per 256-cell block and one workgroup per item.  Within a group the
// items are placed so that each XCD takes one contiguous run of blocks (the
// order the per-mesh kernel gives its blocks), which keeps the halo re-reads
// of neighbouring blocks in one L2.  The results are the same bits as the
// per-mesh kernel's.
#pragma once

#include <algorithm>
#include <vector>

#include "mesh.hpp"

namespace cweno_abi {

struct PackRequest {
  const cweno_mesh* m;
  const void* q;
  void* coeffs;
  int n_vars;
};

struct PackGroup {
  int d = 0, M = 0, vb = 0, variant = -1;
  size_t lds = 0;
  int64_t first = 0, n = 0;     // items [first, first + n) of the table's work list
};

// Entries and work items one request needs, and whether the batched (LDS
// halo) kernel can run every one of its variable blocks.
struct PackFootprint {
  int entries = 0;
  int64_t items = 0;
  bool halo_ok = true;
};

inline PackFootprint pack_footprint(const cweno_mesh* m, int n_vars, bool f32) {
  PackFootprint f;
  const int64_t nblk = (m->nc + cweno::kHaloBlock - 1) / cweno::kHaloBlock;
  for (int v0 = 0; v0 < n_vars;) {
    const int vb = pick_vb_mesh(m, n_vars - v0, f32, true);
    bool ok = false;
    for (int k = 0; k < cweno::kNumVariants; ++k)
      if (cweno::kVariants[k].kind == 1 && variant_ok(m, vb, k, f32)) ok = true;
    f.halo_ok = f.halo_ok && ok;
    f.entries += 1;
    f.items += nblk;
    v0 += vb;
  }
  return f;
}

// Write the table (n_entries KParams at h_table) and the work list (h_items)
// of reqs[0..n) and describe the groups.  The caller has checked every
// request with pack_footprint (halo_ok) and that the totals fit its buffers.
inline void pack_requests(const PackRequest* reqs, int n, bool f32, char* h_table, cweno::BatchItem* h_items,
                          std::vector<PackGroup>& groups, int& n_entries, int64_t& n_items) {
  struct Ent {
    const PackRequest* r;
    int v0, vb;
  };
  std::vector<Ent> ents;
  std::vector<std::vector<int>> members;
  groups.clear();
  for (int t = 0; t < n; ++t) {
    const cweno_mesh* m = reqs[t].m;
    for (int v0 = 0; v0 < reqs[t].n_vars;) {
      const int vb = pick_vb_mesh(m, reqs[t].n_vars - v0, f32, true);
      size_t g = 0;
      while (g < groups.size() && !(groups[g].d == m->d && groups[g].M == m->M && groups[g].vb == vb)) ++g;
      if (g == groups.size()) {
        PackGroup x;
        x.d = m->d;
        x.M = m->M;
        x.vb = vb;
        groups.push_back(x);
        members.emplace_back();
      }
      members[g].push_back((int)ents.size());
      groups[g].lds = std::max(groups[g].lds, (size_t)m->maxH * vb * (f32 ? 4 : 8));
      ents.push_back({&reqs[t], v0, vb});
      v0 += vb;
    }
  }
  for (size_t e = 0; e < ents.size(); ++e) {
    const PackRequest& r = *ents[e].r;
    if (f32)
      reinterpret_cast<cweno::KParams<float>*>(h_table)[e] =
          make_params<float>(r.m, r.q, r.coeffs, nullptr, nullptr, ents[e].v0);
    else
      reinterpret_cast<cweno::KParams<double>*>(h_table)[e] =
          make_params<double>(r.m, r.q, r.coeffs, nullptr, nullptr, ents[e].v0);
  }
  int64_t at = 0;
  std::vector<cweno::BatchItem> nat;
  for (size_t g = 0; g < groups.size(); ++g) {
    nat.clear();
    for (int e : members[g]) {
      const int64_t nblk = (ents[e].r->m->nc + cweno::kHaloBlock - 1) / cweno::kHaloBlock;
      for (int64_t b = 0; b < nblk; ++b) nat.push_back({e, (int32_t)b});
    }
    const int64_t cnt = (int64_t)nat.size();
    // workgroup w runs on XCD w % 8: give XCD x one contiguous run of items
    const int64_t q8 = cnt >> 3, r8 = cnt & 7;
    for (int64_t w = 0; w < cnt; ++w) {
      const int64_t x = w & 7, k = w >> 3;
      h_items[at + w] = nat[x * q8 + (x < r8 ? x : r8) + k];
    }
    // any LDS-halo variant runs every mesh of the group (each one's halos fit);
    // the first mesh's own choice if it is one
    const cweno_mesh* m0 = ents[members[g][0]].r->m;
    int k = m0->variant[f32][groups[g].vb];
    if (k < 0 || cweno::kVariants[k].kind != 1) {
      k = -1;
      for (int c = 0; c < cweno::kNumVariants && k < 0; ++c)
        if (cweno::kVariants[c].kind == 1 && variant_ok(m0, groups[g].vb, c, f32)) k = c;
    }
    groups[g].variant = k;
    groups[g].first = at;
    groups[g].n = cnt;
    at += cnt;
  }
  n_entries = (int)ents.size();
  n_items = at;
}

// Launch every group of a packed table whose device copies are d_table and
// d_items (grid = the group's items: one workgroup per 256-cell block).
inline hipError_t launch_packed(const std::vector<PackGroup>& groups, bool f32, const void* d_table,
                                const cweno::BatchItem* d_items, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (const PackGroup& g : groups) {
    if (e != hipSuccess) break;
    if (g.n == 0) continue;
    const int n = (int)g.n;
    if (f32)
      e = cweno::launch_batch<float>(g.d, g.M, static_cast<const cweno::KParams<float>*>(d_table), d_items + g.first,
                                     n, n, g.lds, g.vb, g.variant, s);
    else
      e = cweno::launch_batch<double>(g.d, g.M, static_cast<const cweno::KParams<double>*>(d_table),
                                      d_items + g.first, n, n, g.lds, g.vb, g.variant, s);
  }
  return e;
}

}  // namespace cweno_abi
