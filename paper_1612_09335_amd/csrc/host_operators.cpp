// Per-cell reconstruction operators (host, FP64).
//
// P_opt (Sec. 2.1, eq. CWENO:Popt) minimises the squared misfit of the
// stencil averages subject to matching the cell's own average exactly.  In
// the orthonormal basis every psi_l with l >= 1 has zero mean on T_E, hence
// on T_i (the map is affine), so the constraint fixes p_0 = Q_i and the rest
// is the unconstrained problem  min || A' p' - (Q_j - Q_i) ||  with
// A'[k][l] = average over stencil cell j(k) of psi_l (l >= 1) in cell i's
// reference frame.  Its solution p' = pinv(A') dQ; pinv(A') is what is stored.
//
// Sector s (eq. CWENO:Ps) is the P1 polynomial matching the d+1 averages of
// its cells exactly; again p_0 = Q_i and the linear coefficients solve the
// d x d system B_s p = dQ with B_s[a][l] = average of psi_{l+1} over the
// a-th sector cell (the value at its barycentre, psi being linear).  B_s^{-1}
// is stored.  A sector whose B_s has 2-norm condition number above 1e10
// (or that could not be filled) is dropped.
//
// The averages are integrated with a Grundmann-Moller rule exact to degree M
// in the reference coordinates of cell i (Sec. 2.1 evaluates these
// integrals by Gaussian quadrature in the reference system to avoid scaling
// ill-conditioning).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.hpp"

namespace cweno {

namespace {

constexpr double kSectorCondMax = 1e10;

// Inverse of a small dense matrix (Gauss-Jordan, partial pivoting).  Returns
// false if a pivot vanishes.
bool invert(int n, const double* A, double* Ainv) {
  double W[8][16];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) W[r][c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(W[r][c]) > std::fabs(W[p][c])) p = r;
    if (W[p][c] == 0.0) return false;
    if (p != c)
      for (int k = 0; k < 2 * n; ++k) std::swap(W[p][k], W[c][k]);
    double piv = W[c][c];
    for (int k = 0; k < 2 * n; ++k) W[c][k] /= piv;
    for (int r = 0; r < n; ++r) {
      if (r == c || W[r][c] == 0.0) continue;
      double f = W[r][c];
      for (int k = 0; k < 2 * n; ++k) W[r][k] -= f * W[c][k];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Ainv[r * n + c] = W[r][n + c];
  return true;
}

// 2-norm condition number of a small square matrix via the eigenvalues of
// B^T B (cyclic Jacobi rotations).
double cond2(int n, const double* B) {
  double S[3][3] = {{0}};
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += B[k * n + i] * B[k * n + j];
      S[i][j] = s;
    }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += S[i][j] * S[i][j];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (S[p][q] == 0.0) continue;
        double th = (S[q][q] - S[p][p]) / (2.0 * S[p][q]);
        double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double a = S[k][p], b = S[k][q];
          S[k][p] = c * a - s * b;
          S[k][q] = s * a + c * b;
        }
        for (int k = 0; k < n; ++k) {
          double a = S[p][k], b = S[q][k];
          S[p][k] = c * a - s * b;
          S[q][k] = s * a + c * b;
        }
      }
  }
  double lo = S[0][0], hi = S[0][0];
  for (int i = 1; i < n; ++i) { lo = std::min(lo, S[i][i]); hi = std::max(hi, S[i][i]); }
  if (!(lo > 0.0)) return INFINITY;
  return std::sqrt(hi / lo);
}

// pinv of A (m x n, m >= n, row-major) into P (n x m, row-major) by
// Householder QR of the column-equilibrated matrix: A D^{-1} = Q1 R, so
// pinv(A) = D^{-1} R^{-1} Q1^T.  Columns are stored contiguously so that every
// inner loop runs over consecutive memory; Q1 is accumulated backwards from
// the first n columns of the identity (only columns >= k change under H_k).
// Returns false when the matrix is rank deficient.
bool pseudo_inverse(int m, int n, const double* A, double* P) {
  thread_local std::vector<double> R, V, Q, scale;
  R.assign((size_t)m * n, 0.0);       // column-major: R[c * m + r]
  V.assign((size_t)n * m, 0.0);       // reflector k: V[k * m + r], r >= k, unit norm
  Q.assign((size_t)n * m, 0.0);       // Q1 column-major: Q[c * m + r]
  scale.assign(n, 0.0);
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c) R[(size_t)c * m + r] = A[(size_t)r * n + c];
  for (int c = 0; c < n; ++c) {
    double* col = &R[(size_t)c * m];
    double s = 0.0;
    for (int r = 0; r < m; ++r) s += col[r] * col[r];
    s = std::sqrt(s);
    if (!(s > 0.0)) return false;
    scale[c] = s;
    for (int r = 0; r < m; ++r) col[r] /= s;
  }
  double rmax = 0.0;
  for (int k = 0; k < n; ++k) {
    double* ck = &R[(size_t)k * m];
    double nrm = 0.0;
    for (int r = k; r < m; ++r) nrm += ck[r] * ck[r];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return false;
    double* v = &V[(size_t)k * m];
    const double alpha = ck[k] > 0 ? -nrm : nrm;
    for (int r = k; r < m; ++r) v[r] = ck[r];
    v[k] -= alpha;
    double vn = 0.0;
    for (int r = k; r < m; ++r) vn += v[r] * v[r];
    vn = std::sqrt(vn);
    for (int r = k; r < m; ++r) v[r] /= vn;
    for (int c = k; c < n; ++c) {
      double* cc = &R[(size_t)c * m];
      double dot = 0.0;
      for (int r = k; r < m; ++r) dot += v[r] * cc[r];
      const double t = 2.0 * dot;
      for (int r = k; r < m; ++r) cc[r] -= t * v[r];
    }
    rmax = std::max(rmax, std::fabs(ck[k]));
  }
  for (int k = 0; k < n; ++k)
    if (!(std::fabs(R[(size_t)k * m + k]) > 1e-12 * rmax)) return false;
  // Q1 = H_0 H_1 ... H_{n-1} [I_n; 0]
  for (int c = 0; c < n; ++c) Q[(size_t)c * m + c] = 1.0;
  for (int k = n - 1; k >= 0; --k) {
    const double* v = &V[(size_t)k * m];
    for (int c = k; c < n; ++c) {
      double* qc = &Q[(size_t)c * m];
      double dot = 0.0;
      for (int r = k; r < m; ++r) dot += v[r] * qc[r];
      const double t = 2.0 * dot;
      for (int r = k; r < m; ++r) qc[r] -= t * v[r];
    }
  }
  // R X = Q1^T row by row from the bottom (row k of Q1^T is column k of Q1),
  // then undo the column scaling
  for (int k = n - 1; k >= 0; --k) {
    double* pk = &P[(size_t)k * m];
    const double* qk = &Q[(size_t)k * m];
    for (int j = 0; j < m; ++j) pk[j] = qk[j];
    for (int c = k + 1; c < n; ++c) {
      const double rkc = R[(size_t)c * m + k];
      const double* pc = &P[(size_t)c * m];
      for (int j = 0; j < m; ++j) pk[j] -= rkc * pc[j];
    }
    const double rkk = R[(size_t)k * m + k];
    for (int j = 0; j < m; ++j) pk[j] /= rkk;
  }
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < m; ++j) P[(size_t)k * m + j] /= scale[k];
  return true;
}

// Row k of A' (k < nl): the averages of psi_1 .. psi_{nb-1} over cell list[k]
// in cell i's reference frame (Jinv: inverse of its map), by the quadrature
// (qlam, qw); A is row-major [nl][nb-1], psi a scratch of nb values.
void stencil_rows(const Geometry& g, int64_t i, const double* Jinv, const int32_t* list, int nl, int M,
                  const std::vector<double>& qlam, const std::vector<double>& qw, double* psi, double* A) {
  const int d = g.d, ns = d + 1, nb = n_basis(M, d), nq = (int)qw.size();
  const double* Xi = &g.X[(size_t)i * ns * d];
  for (int k = 0; k < nl; ++k) {
    int64_t j = list[k];
    const double* Xj = &g.X[(size_t)j * ns * d];
    double shift[3];
    for (int a = 0; a < d; ++a) {
      double dc = g.cen[(size_t)j * d + a] - g.cen[(size_t)i * d + a];
      shift[a] = min_image(dc, g.box[a]) - dc;
    }
    double Y[4][3];
    for (int v = 0; v < ns; ++v) {
      double y[3];
      for (int a = 0; a < d; ++a) y[a] = Xj[v * d + a] + shift[a] - Xi[a];
      for (int r = 0; r < d; ++r) {
        double s = 0.0;
        for (int a = 0; a < d; ++a) s += Jinv[r * d + a] * y[a];
        Y[v][r] = s;
      }
    }
    double* row = &A[(size_t)k * (nb - 1)];
    std::fill(row, row + nb - 1, 0.0);
    for (int q = 0; q < nq; ++q) {
      double xi[3] = {0, 0, 0};
      for (int v = 0; v < ns; ++v)
        for (int r = 0; r < d; ++r) xi[r] += qlam[(size_t)q * ns + v] * Y[v][r];
      basis_eval(d, M, xi, psi);
      for (int l = 1; l < nb; ++l) row[l - 1] += qw[q] * psi[l];
    }
  }
}

}  // namespace

void build_gather(const Geometry& g, const Stencils& st, int M, Operators& op) {
  const int d = g.d, ns = d + 1, nb = n_basis(M, d), n_e = st.n_e, NE1 = n_e - 1;
  op.d = d;
  op.M = M;
  op.nb = nb;
  op.n_e = n_e;
  // gather lists: S0 without the cell, then sector cells outside S0
  std::vector<std::vector<int32_t>> extras(g.nc);
  int G = NE1;
  for (int64_t i = 0; i < g.nc; ++i) {
    const int32_t* S0 = &st.central[(size_t)i * n_e];
    for (int s = 0; s < ns; ++s) {
      const int32_t* sec = &st.sectors[((size_t)i * ns + s) * ns];
      if (sec[0] < 0) continue;
      for (int a = 1; a < ns; ++a) {
        int32_t j = sec[a];
        if (std::find(S0 + 1, S0 + n_e, j) != S0 + n_e) continue;
        if (std::find(extras[i].begin(), extras[i].end(), j) != extras[i].end()) continue;
        extras[i].push_back(j);
      }
    }
    G = std::max(G, NE1 + (int)extras[i].size());
  }
  if (G > 255) throw Error(CWENO_E_ARG, "gather list longer than 255 entries");
  op.G = G;
  op.nc = g.nc;
  op.Np = (g.nc + 63) / 64 * 64;
  const size_t Np = (size_t)op.Np;
  op.gidx.assign((size_t)G * Np, 0);
  op.secpos.assign((size_t)ns * d * Np, 0);
  op.mask.assign(Np, 0);
  parallel_for(g.nc, [&](int64_t b, int64_t e) {
    std::vector<int32_t> list(G);
    for (int64_t i = b; i < e; ++i) {
      const int32_t* S0 = &st.central[(size_t)i * n_e];
      int nl = 0;
      for (int k = 1; k < n_e; ++k) list[nl++] = S0[k];
      for (int32_t j : extras[i]) list[nl++] = j;
      for (int k = nl; k < G; ++k) list[k] = (int32_t)i;
      for (int k = 0; k < G; ++k) op.gidx[(size_t)k * Np + i] = list[k];
      for (int s = 0; s < ns; ++s) {
        const int32_t* sec = &st.sectors[((size_t)i * ns + s) * ns];
        if (sec[0] < 0) continue;
        for (int a = 0; a < d; ++a) {
          const int k = (int)(std::find(list.begin(), list.begin() + nl, sec[a + 1]) - list.begin());
          op.secpos[(size_t)(s * d + a) * Np + i] = (uint8_t)k;
        }
      }
    }
  });
  sigma_matrix(d, M, op.sigma);
  {  // drop row/column 0 (the constant has no derivatives)
    std::vector<double> s2((size_t)(nb - 1) * (nb - 1));
    for (int l = 1; l < nb; ++l)
      for (int m = 1; m < nb; ++m) s2[(size_t)(l - 1) * (nb - 1) + (m - 1)] = op.sigma[(size_t)l * nb + m];
    op.sigma.swap(s2);
  }
}

void build_operators(const Geometry& g, const Stencils& st, int M, Operators& op) {
  build_gather(g, st, M, op);
  const int d = g.d, ns = d + 1, nb = op.nb, n_e = st.n_e, NE1 = n_e - 1, G = op.G;
  const size_t Np = (size_t)op.Np;
  op.pinv.assign((size_t)(nb - 1) * NE1 * Np, 0.0);
  op.binv.assign((size_t)ns * d * d * Np, 0.0);
  std::vector<double> qlam, qw;
  grundmann_moller(d, M, qlam, qw);
  std::vector<int64_t> dropped_per_cell(g.nc, 0);

  parallel_for(g.nc, [&](int64_t b, int64_t e) {
    std::vector<double> A((size_t)G * (nb - 1)), P((size_t)(nb - 1) * NE1), psi(nb);
    std::vector<int32_t> list(G);
    for (int64_t i = b; i < e; ++i) {
      const double* Xi = &g.X[(size_t)i * ns * d];
      double J[9], Jinv[9];
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) J[r * d + c] = Xi[(c + 1) * d + r] - Xi[r];
      if (!invert(d, J, Jinv)) throw Error(CWENO_E_MESH, "singular cell map at cell " + std::to_string(i));
      for (int k = 0; k < G; ++k) list[k] = op.gidx[(size_t)k * Np + i];
      int nl = G;
      while (nl > NE1 && list[nl - 1] == (int32_t)i) --nl;   // padding entries are the cell itself
      // averages of psi_1.. over every gathered cell, in cell i's frame
      stencil_rows(g, i, Jinv, list.data(), nl, M, qlam, qw, psi.data(), A.data());
      if (!pseudo_inverse(NE1, nb - 1, A.data(), P.data()))
        throw Error(CWENO_E_RANK, "rank-deficient least-squares system at cell " + std::to_string(i));
      for (int l = 0; l < nb - 1; ++l)   // device layout is k-major: row k*(nb-1) + l
        for (int k = 0; k < NE1; ++k) op.pinv[((size_t)k * (nb - 1) + l) * Np + i] = P[(size_t)l * NE1 + k];
      uint8_t mask = 0;
      for (int s = 0; s < ns; ++s) {
        const int32_t* sec = &st.sectors[((size_t)i * ns + s) * ns];
        if (sec[0] < 0) { dropped_per_cell[i]++; continue; }
        double B[9], Binv[9];
        for (int a = 0; a < d; ++a) {
          const int k = op.secpos[(size_t)(s * d + a) * Np + i];
          for (int l = 0; l < d; ++l) B[a * d + l] = A[(size_t)k * (nb - 1) + l];
        }
        if (!(cond2(d, B) <= kSectorCondMax) || !invert(d, B, Binv)) { dropped_per_cell[i]++; continue; }
        mask |= (uint8_t)(1u << s);
        for (int l = 0; l < d; ++l)
          for (int a = 0; a < d; ++a) op.binv[(size_t)((s * d + l) * d + a) * Np + i] = Binv[l * d + a];
      }
      op.mask[i] = mask;
    }
  });
  op.n_dropped = 0;
  for (int64_t x : dropped_per_cell) op.n_dropped += x;
}

}  // namespace cweno

namespace cweno {

void build_weno_operators(const Geometry& g, const WenoStencils& ws, int M, WenoOperators& op) {
  const int d = g.d, ns = d + 1, nb = n_basis(M, d), NL = nb - 1, n_e = ws.n_e, NE1 = n_e - 1, n_s = ws.n_s;
  if (n_s > 16) throw Error(CWENO_E_ARG, "too many WENO stencils");
  op.n_s = n_s;
  op.Np = (g.nc + 63) / 64 * 64;
  const size_t Np = (size_t)op.Np;
  op.pinv.assign((size_t)n_s * NE1 * NL * Np, 0.0);
  op.gidx.assign((size_t)n_s * NE1 * Np, 0);
  op.alive.assign(Np, 0);
  std::vector<double> qlam, qw;
  grundmann_moller(d, M, qlam, qw);
  std::vector<int64_t> dropped(g.nc, 0);
  parallel_for(g.nc, [&](int64_t b, int64_t e) {
    std::vector<double> A((size_t)NE1 * NL), P((size_t)NL * NE1), psi(nb);
    for (int64_t i = b; i < e; ++i) {
      const double* Xi = &g.X[(size_t)i * ns * d];
      double J[9], Jinv[9];
      for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) J[r * d + c] = Xi[(c + 1) * d + r] - Xi[r];
      if (!invert(d, J, Jinv)) throw Error(CWENO_E_MESH, "singular cell map at cell " + std::to_string(i));
      uint16_t alive = 0;
      for (int j = 0; j < n_s; ++j) {
        const int32_t* S = &ws.cells[((size_t)i * n_s + j) * n_e];
        if (S[0] < 0) {   // unfillable: dropped, gathers point at the cell itself
          dropped[i]++;
          for (int k = 0; k < NE1; ++k) op.gidx[((size_t)j * NE1 + k) * Np + i] = (int32_t)i;
          continue;
        }
        stencil_rows(g, i, Jinv, S + 1, NE1, M, qlam, qw, psi.data(), A.data());
        if (!pseudo_inverse(NE1, NL, A.data(), P.data()))
          throw Error(CWENO_E_RANK, "rank-deficient WENO stencil " + std::to_string(j) + " at cell " +
                                        std::to_string(i));
        alive = (uint16_t)(alive | (1u << j));
        for (int k = 0; k < NE1; ++k) {
          op.gidx[((size_t)j * NE1 + k) * Np + i] = S[k + 1];
          for (int l = 0; l < NL; ++l) op.pinv[(((size_t)j * NE1 + k) * NL + l) * Np + i] = P[(size_t)l * NE1 + k];
        }
      }
      op.alive[i] = alive;
    }
  });
  op.n_dropped = 0;
  for (int64_t x : dropped) op.n_dropped += x;
}

}  // namespace cweno
