// Per-block halos of the gather lists (host).
//
// A block of B consecutive cells reads the averages of every cell in its
// cells' gather lists (central stencils and sector cells).  Neighbouring
// cells share most of those, so the block loads each referenced cell once
// into LDS and reads the stencils from there; this file builds, per block,
// the sorted list of referenced cells and the 16-bit position of each gather
// entry in that list.
#include <algorithm>

#include "host.hpp"

namespace cweno {

void build_halo(const Operators& op, int B, Halo& h) {
  const int64_t nc = op.nc, Np = op.Np;
  const int G = op.G;
  const int64_t nblk = (nc + B - 1) / B;
  h.B = B;
  h.offset.assign(nblk + 1, 0);
  h.lidx.assign((size_t)(G + 1) * Np, 0);
  std::vector<std::vector<int32_t>> lists(nblk);
  parallel_for(nblk, [&](int64_t b0, int64_t b1) {
    std::vector<int32_t> u;
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t c0 = b * B, c1 = std::min(nc, c0 + B);
      u.clear();
      for (int64_t i = c0; i < c1; ++i) {
        u.push_back((int32_t)i);
        for (int k = 0; k < G; ++k) u.push_back(op.gidx[(size_t)k * Np + i]);
      }
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      if (u.size() > 65535) throw Error(CWENO_E_ARG, "block halo larger than 65535 cells");
      for (int64_t i = c0; i < c1; ++i) {
        for (int k = 0; k < G; ++k) {
          const int32_t j = op.gidx[(size_t)k * Np + i];
          h.lidx[(size_t)k * Np + i] = (uint16_t)(std::lower_bound(u.begin(), u.end(), j) - u.begin());
        }
        h.lidx[(size_t)G * Np + i] = (uint16_t)(std::lower_bound(u.begin(), u.end(), (int32_t)i) - u.begin());
      }
      lists[b] = u;
    }
  });
  int64_t tot = 0;
  int mx = 0;
  for (int64_t b = 0; b < nblk; ++b) {
    h.offset[b] = (int32_t)tot;
    tot += (int64_t)lists[b].size();
    mx = std::max(mx, (int)lists[b].size());
  }
  if (tot >= (int64_t(1) << 31)) throw Error(CWENO_E_ARG, "halo lists too long");
  h.offset[nblk] = (int32_t)tot;
  h.max_len = mx;
  h.cells.resize(tot);
  for (int64_t b = 0; b < nblk; ++b) std::copy(lists[b].begin(), lists[b].end(), h.cells.begin() + h.offset[b]);
}

}  // namespace cweno
