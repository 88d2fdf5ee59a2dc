// Geometry, face adjacency and stencil selection (host, FP64).
//
// Integer tables (neighbours, stencils, sectors) are decided by floating-point
// comparisons.  To make them reproducible bit for bit by any implementation
// of the same rule, every such value is computed by a fixed sequence of IEEE
// operations with no contraction (this file is compiled with
// -ffp-contract=off):
//   min image      mi(x) = x - L * floor(x / L + 0.5)            (L = period)
//   unwrap         X_k  := X_0 + mi(X_k - X_0)                    per axis
//   barycentre     c = (((X_0 + X_1) + X_2) [+ X_3]) / (d + 1)
//   offset         o = mi(c_j - c_i);  squared distance o_x*o_x + o_y*o_y [+ o_z*o_z]
//   determinant    of [W_1-W_0 | ... | W_d-W_0] by the explicit cofactor expansion
//   barycentric    b_m = det(W with vertex m replaced by p) / det(W)
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

#include "host.hpp"

namespace cweno {

namespace {

constexpr double kConeTol = 1e-12;     // open cone: b_m > kConeTol
constexpr int kMaxRings = 16;
constexpr double kPeriodicReach = 0.375;

using P3 = std::array<double, 3>;

double det_columns(int d, const P3* W) {
  if (d == 2) {
    double ux = W[1][0] - W[0][0];
    double uy = W[1][1] - W[0][1];
    double vx = W[2][0] - W[0][0];
    double vy = W[2][1] - W[0][1];
    return ux * vy - vx * uy;
  }
  double ux = W[1][0] - W[0][0];
  double uy = W[1][1] - W[0][1];
  double uz = W[1][2] - W[0][2];
  double vx = W[2][0] - W[0][0];
  double vy = W[2][1] - W[0][1];
  double vz = W[2][2] - W[0][2];
  double wx = W[3][0] - W[0][0];
  double wy = W[3][1] - W[0][1];
  double wz = W[3][2] - W[0][2];
  return ux * (vy * wz - vz * wy) - uy * (vx * wz - vz * wx) + uz * (vx * wy - vy * wx);
}

// Small open-addressing set of cell ids, cleared in O(inserted).
struct IdSet {
  std::vector<int32_t> slot;
  std::vector<int32_t> used;
  uint32_t mask = 0;
  IdSet() { grow(1024); }
  void grow(uint32_t n) {
    slot.assign(n, -1);
    mask = n - 1;
    used.clear();
  }
  void clear() {
    for (int32_t u : used) slot[u] = -1;
    used.clear();
  }
  bool insert(int32_t j) {  // true if newly inserted
    if (used.size() * 2 >= slot.size()) {
      std::vector<int32_t> old;
      for (int32_t u : used) old.push_back(slot[u]);
      grow((uint32_t)slot.size() * 2);
      for (int32_t v : old) insert(v);
    }
    uint32_t h = ((uint32_t)j * 2654435761u) & mask;
    while (slot[h] != -1) {
      if (slot[h] == j) return false;
      h = (h + 1) & mask;
    }
    slot[h] = j;
    used.push_back((int32_t)h);
    return true;
  }
};

}  // namespace

int n_basis(int M, int d) {
  long num = 1, den = 1;
  for (int l = 1; l <= d; ++l) { num *= (M + l); den *= l; }
  return (int)(num / den);
}

double min_image(double delta, double L) {
  if (L == 0.0) return delta;
  return delta - L * std::floor(delta / L + 0.5);
}

void build_geometry(const MeshInput& in, Geometry& g) {
  const int d = in.d;
  g.d = d;
  g.nc = in.nc;
  for (int a = 0; a < 3; ++a) g.box[a] = in.box[a];
  g.X.assign((size_t)in.nc * (d + 1) * d, 0.0);
  g.cen.assign((size_t)in.nc * d, 0.0);
  parallel_for(in.nc, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      const int32_t* ids = in.C + i * (d + 1);
      for (int k = 0; k <= d; ++k)
        if (ids[k] < 0 || ids[k] >= in.nv)
          throw Error(CWENO_E_MESH, "cell " + std::to_string(i) + " references vertex id out of range");
      double* X = &g.X[(size_t)i * (d + 1) * d];
      for (int a = 0; a < d; ++a) X[a] = in.V[(size_t)ids[0] * d + a];
      for (int k = 1; k <= d; ++k)
        for (int a = 0; a < d; ++a) {
          double xk = in.V[(size_t)ids[k] * d + a];
          X[k * d + a] = X[a] + min_image(xk - X[a], in.box[a]);
        }
      double* c = &g.cen[(size_t)i * d];
      for (int a = 0; a < d; ++a) {
        double s = X[a];
        for (int k = 1; k <= d; ++k) s = s + X[k * d + a];
        c[a] = s / (double)(d + 1);
      }
      P3 W[4];
      double scale = 0.0;
      for (int k = 0; k <= d; ++k) {
        W[k] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
          W[k][a] = X[k * d + a];
          scale = std::max(scale, std::fabs(X[k * d + a] - X[a]));
        }
      }
      double det = det_columns(d, W);
      if (!(std::fabs(det) > 1e-12 * std::pow(scale, d)))
        throw Error(CWENO_E_MESH, "cell " + std::to_string(i) + " is degenerate (zero volume)");
    }
  });
}

void face_adjacency(const MeshInput& in, std::vector<int32_t>& nbr) {
  const int d = in.d, nv = d + 1;
  struct Rec { int32_t v[3]; int32_t cell; int32_t k; };
  std::vector<Rec> rec((size_t)in.nc * nv);
  parallel_for(in.nc, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      const int32_t* ids = in.C + i * nv;
      for (int k = 0; k < nv; ++k) {
        Rec r{{-1, -1, -1}, (int32_t)i, k};
        int t = 0;
        for (int m = 0; m < nv; ++m)
          if (m != k) r.v[t++] = ids[m];
        std::sort(r.v, r.v + d);
        rec[(size_t)i * nv + k] = r;
      }
    }
  });
  auto key_less = [](const Rec& a, const Rec& b) {
    if (a.v[0] != b.v[0]) return a.v[0] < b.v[0];
    if (a.v[1] != b.v[1]) return a.v[1] < b.v[1];
    return a.v[2] < b.v[2];
  };
  auto key_eq = [](const Rec& a, const Rec& b) {
    return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2];
  };
  std::sort(rec.begin(), rec.end(), key_less);
  nbr.assign((size_t)in.nc * nv, -1);
  size_t n = rec.size();
  for (size_t t = 0; t < n;) {
    size_t u = t + 1;
    while (u < n && key_eq(rec[t], rec[u])) ++u;
    if (u - t > 2)
      throw Error(CWENO_E_MESH, "a face is shared by more than two cells (cell " +
                                    std::to_string(rec[t].cell) + ")");
    if (u - t == 2) {
      const Rec& a = rec[t];
      const Rec& b = rec[t + 1];
      if (a.cell == b.cell) throw Error(CWENO_E_MESH, "cell " + std::to_string(a.cell) + " repeats a vertex");
      nbr[(size_t)a.cell * nv + a.k] = b.cell;
      nbr[(size_t)b.cell * nv + b.k] = a.cell;
    }
    t = u;
  }
}

namespace {

struct StencilCtx {
  const Geometry& g;
  const std::vector<int32_t>& nbr;
  IdSet visited;
  std::vector<int32_t> frontier, cand;
  std::vector<std::pair<double, int32_t>> ring;

  StencilCtx(const Geometry& g_, const std::vector<int32_t>& n_) : g(g_), nbr(n_) {}

  void offset(int64_t i, int64_t j, double* o) const {
    const int d = g.d;
    for (int a = 0; a < d; ++a)
      o[a] = min_image(g.cen[(size_t)j * d + a] - g.cen[(size_t)i * d + a], g.box[a]);
  }
  double dist2(int64_t i, int64_t j) const {
    double o[3] = {0.0, 0.0, 0.0};
    offset(i, j, o);
    double s = o[0] * o[0];
    for (int a = 1; a < g.d; ++a) s = s + o[a] * o[a];
    return s;
  }
  void check_reach(int64_t i, int64_t j) const {
    double o[3] = {0.0, 0.0, 0.0};
    offset(i, j, o);
    for (int a = 0; a < g.d; ++a)
      if (g.box[a] != 0.0 && std::fabs(o[a]) > kPeriodicReach * g.box[a])
        throw Error(CWENO_E_PERIODIC, "stencil of cell " + std::to_string(i) +
                                          " reaches too far across the periodic box");
  }
  // Cone s of cell i (apex at vertex s, spanned by the edges to the other
  // vertices): b_m > tol for every m != s; with reverse, the opposite cone at
  // vertex s: b_m < -tol for every m != s.
  bool in_cone(int64_t i, int s, int64_t j, bool reverse = false) const {
    const int d = g.d;
    P3 W[4];
    const double* X = &g.X[(size_t)i * (d + 1) * d];
    for (int k = 0; k <= d; ++k) {
      W[k] = {0, 0, 0};
      for (int a = 0; a < d; ++a) W[k][a] = X[k * d + a];
    }
    double o[3] = {0.0, 0.0, 0.0};
    offset(i, j, o);
    P3 p = {0, 0, 0};
    for (int a = 0; a < d; ++a) p[a] = g.cen[(size_t)i * d + a] + o[a];
    double D = det_columns(d, W);
    for (int m = 0; m <= d; ++m) {
      if (m == s) continue;
      P3 keep = W[m];
      W[m] = p;
      double b = det_columns(d, W) / D;
      W[m] = keep;
      if (reverse ? !(b < -kConeTol) : !(b > kConeTol)) return false;
    }
    return true;
  }

  // Breadth-first ring fill (cone sector s, or s < 0 for the central stencil;
  // reverse: the opposite cone of vertex s).
  bool fill(int64_t i, int n_target, int s, std::vector<int32_t>& sel, bool reverse = false) {
    const int nvx = g.d + 1;
    sel.clear();
    sel.push_back((int32_t)i);
    if (n_target <= 1) return true;
    visited.clear();
    visited.insert((int32_t)i);
    frontier.assign(1, (int32_t)i);
    for (int r = 0; r < kMaxRings; ++r) {
      cand.clear();
      for (int32_t f : frontier)
        for (int k = 0; k < nvx; ++k) {
          int32_t j = nbr[(size_t)f * nvx + k];
          if (j >= 0 && visited.insert(j)) cand.push_back(j);
        }
      if (cand.empty()) return false;
      ring.clear();
      for (int32_t j : cand) ring.emplace_back(dist2(i, j), j);
      std::sort(ring.begin(), ring.end(), [](const std::pair<double, int32_t>& a,
                                             const std::pair<double, int32_t>& b) {
        return a.first < b.first || (a.first == b.first && a.second < b.second);
      });
      frontier.clear();
      for (auto& pr : ring) {
        frontier.push_back(pr.second);
        if (s < 0 || in_cone(i, s, pr.second, reverse)) {
          sel.push_back(pr.second);
          if ((int)sel.size() == n_target) return true;
        }
      }
    }
    return false;
  }
};

}  // namespace

void build_stencils(const Geometry& g, const std::vector<int32_t>& nbr, int n_e, int rule,
                    Stencils& st) {
  const int d = g.d, ns = d + 1;
  st.n_e = n_e;
  st.central.assign((size_t)g.nc * n_e, -1);
  st.sectors.assign((size_t)g.nc * ns * ns, -1);
  parallel_for(g.nc, [&](int64_t b, int64_t e) {
    StencilCtx ctx(g, nbr);
    std::vector<int32_t> sel;
    for (int64_t i = b; i < e; ++i) {
      if (!ctx.fill(i, n_e, -1, sel))
        throw Error(CWENO_E_STENCIL, "cannot fill the central stencil of cell " + std::to_string(i));
      for (size_t t = 1; t < sel.size(); ++t) ctx.check_reach(i, sel[t]);
      std::copy(sel.begin(), sel.end(), &st.central[(size_t)i * n_e]);
      for (int s = 0; s < ns; ++s) {
        bool ok;
        if (rule == CWENO_SECTOR_FACE) {
          sel.assign(1, (int32_t)i);
          ok = true;
          for (int k = 0; k < ns; ++k) {
            if (k == s) continue;
            int32_t j = nbr[(size_t)i * ns + k];
            if (j < 0) { ok = false; break; }
            sel.push_back(j);
          }
        } else {
          ok = ctx.fill(i, ns, s, sel);
        }
        if (!ok) continue;
        for (size_t t = 1; t < sel.size(); ++t) ctx.check_reach(i, sel[t]);
        std::copy(sel.begin(), sel.end(), &st.sectors[((size_t)i * ns + s) * ns]);
      }
    }
  });
}

void build_weno_stencils(const Geometry& g, const std::vector<int32_t>& nbr, const Stencils& st,
                         WenoStencils& ws) {
  const int d = g.d, ns = d + 1, n_e = st.n_e, n_s = 1 + 2 * ns;
  ws.n_s = n_s;
  ws.n_e = n_e;
  ws.cells.assign((size_t)g.nc * n_s * n_e, -1);
  parallel_for(g.nc, [&](int64_t b, int64_t e) {
    StencilCtx ctx(g, nbr);
    std::vector<int32_t> sel;
    for (int64_t i = b; i < e; ++i) {
      int32_t* out = &ws.cells[(size_t)i * n_s * n_e];
      std::copy(&st.central[(size_t)i * n_e], &st.central[(size_t)i * n_e] + n_e, out);
      for (int rev = 0; rev < 2; ++rev)
        for (int s = 0; s < ns; ++s) {
          if (!ctx.fill(i, n_e, s, sel, rev == 1)) continue;
          for (size_t t = 1; t < sel.size(); ++t) ctx.check_reach(i, sel[t]);
          std::copy(sel.begin(), sel.end(), out + (size_t)(1 + rev * ns + s) * n_e);
        }
    }
  });
}

}  // namespace cweno
