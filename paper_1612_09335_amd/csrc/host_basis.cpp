// Orthonormal Dubiner basis, Grundmann-Moller quadrature and the universal
// oscillation-indicator matrix (host, FP64).
//
// Basis (Sec. 2.1, eq. recpolydef names an orthogonal Dubiner-type basis on
// the reference simplex; the collapsed-coordinate family is used):
//   2-D  psi_pq  = s * F_p(u1, v1) * P_q^(2p+1,0)(2 eta - 1)
//   3-D  psi_pqr = s * F_p(u1, v1) * H_pq(u2, v2) * P_r^(2p+2q+2,0)(2 zeta - 1)
// with u1 = 2 xi + eta (+ zeta) - 1, v1 = 1 - eta (- zeta), u2 = 2 eta + zeta - 1,
// v2 = 1 - zeta, and F_p = v1^p P_p(u1/v1), H_pq = v2^q P_q^(2p+1,0)(u2/v2)
// evaluated by the *homogenised* three-term recurrences (Legendre and Jacobi
// recurrences multiplied through by powers of v), so no collapsed coordinate
// is ever divided by v and the functions are polynomials valid everywhere.
// Normalisation (1/|T_E|) int psi^2 = 1 uses the closed forms
//   2-D  int psi_pq^2  = 1 / (2 (2p+1) (p+q+1))
//   3-D  int psi_pqr^2 = 1 / ((2p+1) (2p+2q+2) (2p+2q+2r+3)).
// Order: total degree, then p descending, then q descending.
//
// Sigma_lm = sum over distinct multi-indices alpha with 1 <= |alpha| <= M of
// int_{T_E} d^alpha psi_l d^alpha psi_m (Sec. 2.1).  Here psi is expanded in
// monomials by running the same recurrences on dense polynomials, the
// derivatives are taken exactly and the products integrated with a
// Grundmann-Moller rule of sufficient degree.
#include <cmath>
#include <functional>
#include <vector>

#include "host.hpp"

namespace cweno {

namespace {

struct Idx { int p, q, r; };

std::vector<Idx> index_list(int d, int M) {
  std::vector<Idx> out;
  for (int n = 0; n <= M; ++n)
    for (int p = n; p >= 0; --p) {
      if (d == 2) out.push_back({p, n - p, 0});
      else
        for (int q = n - p; q >= 0; --q) out.push_back({p, q, n - p - q});
    }
  return out;
}

double norm_scale(int d, const Idx& t) {
  if (d == 2) return std::sqrt((2.0 * t.p + 1.0) * (t.p + t.q + 1.0));
  return std::sqrt((2.0 * t.p + 1.0) * (2.0 * t.p + 2.0 * t.q + 2.0) *
                   (2.0 * t.p + 2.0 * t.q + 2.0 * t.r + 3.0) / 6.0);
}

// Dense polynomial in d variables, total degree <= deg; coefficient of
// x^a y^b z^c at index (a*(deg+1) + b)*(deg+1) + c.
struct Poly {
  int d = 2, deg = 0;
  std::vector<double> c;
  Poly() = default;
  Poly(int d_, int deg_) : d(d_), deg(deg_), c((size_t)(deg_ + 1) * (deg_ + 1) * (deg_ + 1), 0.0) {}
  size_t at(int a, int b, int e) const { return ((size_t)a * (deg + 1) + b) * (deg + 1) + e; }
};

Poly padd(const Poly& x, const Poly& y, double sx, double sy) {
  Poly o(x.d, x.deg);
  for (size_t t = 0; t < o.c.size(); ++t) o.c[t] = sx * x.c[t] + sy * y.c[t];
  return o;
}
Poly pmul(const Poly& x, const Poly& y) {
  Poly o(x.d, x.deg);
  const int D = x.deg;
  for (int a = 0; a <= D; ++a)
    for (int b = 0; a + b <= D; ++b)
      for (int e = 0; a + b + e <= D; ++e) {
        double cx = x.c[x.at(a, b, e)];
        if (cx == 0.0) continue;
        for (int a2 = 0; a + a2 <= D; ++a2)
          for (int b2 = 0; a + a2 + b + b2 <= D; ++b2)
            for (int e2 = 0; a + a2 + b + b2 + e + e2 <= D; ++e2) {
              double cy = y.c[y.at(a2, b2, e2)];
              if (cy != 0.0) o.c[o.at(a + a2, b + b2, e + e2)] += cx * cy;
            }
      }
  return o;
}
Poly plin(int d, int deg, double c0, double cx, double cy, double cz) {
  Poly o(d, deg);
  o.c[o.at(0, 0, 0)] = c0;
  if (deg >= 1) {
    o.c[o.at(1, 0, 0)] = cx;
    o.c[o.at(0, 1, 0)] = cy;
    if (d == 3) o.c[o.at(0, 0, 1)] = cz;
  }
  return o;
}

// The recurrences, written once for T = double (point values) and T = Poly.
struct NumAlg {
  using T = double;
  T add(const T& a, const T& b, double sa, double sb) const { return sa * a + sb * b; }
  T mul(const T& a, const T& b) const { return a * b; }
};
struct PolyAlg {
  using T = Poly;
  T add(const T& a, const T& b, double sa, double sb) const { return padd(a, b, sa, sb); }
  T mul(const T& a, const T& b) const { return pmul(a, b); }
};

// H_n = v^n P_n^(alpha,0)(u/v) for n = 0..nmax via the homogenised Jacobi
// recurrence (alpha = 0 gives Legendre):
//   H_1 = ((alpha+2) u + alpha v) / 2
//   a1 H_{n+1} = (a3 u + a2 v) H_n - a4 v^2 H_{n-1},
//   a1 = 2(n+1)(n+alpha+1)(2n+alpha), a2 = (2n+alpha+1) alpha^2,
//   a3 = (2n+alpha)(2n+alpha+1)(2n+alpha+2), a4 = 2 n (n+alpha)(2n+alpha+2).
template <class Alg>
std::vector<typename Alg::T> jacobi_h(const Alg& A, const typename Alg::T& one, const typename Alg::T& u,
                                      const typename Alg::T& v, int nmax, int alpha) {
  std::vector<typename Alg::T> H;
  H.push_back(one);
  if (nmax >= 1) H.push_back(A.add(u, v, (alpha + 2) / 2.0, alpha / 2.0));
  typename Alg::T v2 = A.mul(v, v);
  for (int n = 1; n < nmax; ++n) {
    double a1 = 2.0 * (n + 1) * (n + alpha + 1) * (2.0 * n + alpha);
    double a2 = (2.0 * n + alpha + 1) * alpha * alpha;
    double a3 = (2.0 * n + alpha) * (2.0 * n + alpha + 1) * (2.0 * n + alpha + 2);
    double a4 = 2.0 * n * (n + alpha) * (2.0 * n + alpha + 2);
    typename Alg::T lin = A.add(u, v, a3 / a1, a2 / a1);
    typename Alg::T t1 = A.mul(lin, H[n]);
    typename Alg::T t2 = A.mul(v2, H[n - 1]);
    H.push_back(A.add(t1, t2, 1.0, -a4 / a1));
  }
  return H;
}

template <class Alg>
std::vector<typename Alg::T> dubiner(const Alg& A, int d, int M, const typename Alg::T& one,
                                     const typename Alg::T& X, const typename Alg::T& Y,
                                     const typename Alg::T& Z) {
  auto idx = index_list(d, M);
  std::vector<typename Alg::T> out;
  out.reserve(idx.size());
  if (d == 2) {
    typename Alg::T u1 = A.add(A.add(X, Y, 2.0, 1.0), one, 1.0, -1.0);   // 2x + y - 1
    typename Alg::T v1 = A.add(one, Y, 1.0, -1.0);                        // 1 - y
    typename Alg::T t = A.add(Y, one, 2.0, -1.0);                         // 2y - 1
    auto F = jacobi_h(A, one, u1, v1, M, 0);
    std::vector<std::vector<typename Alg::T>> G(M + 1);
    for (int p = 0; p <= M; ++p) G[p] = jacobi_h(A, one, t, one, M - p, 2 * p + 1);
    for (const Idx& k : idx) {
      typename Alg::T v = A.mul(F[k.p], G[k.p][k.q]);
      out.push_back(A.add(v, v, norm_scale(2, k), 0.0));
    }
    return out;
  }
  typename Alg::T u1 = A.add(A.add(A.add(X, Y, 2.0, 1.0), Z, 1.0, 1.0), one, 1.0, -1.0);  // 2x+y+z-1
  typename Alg::T v1 = A.add(A.add(one, Y, 1.0, -1.0), Z, 1.0, -1.0);                    // 1-y-z
  typename Alg::T u2 = A.add(A.add(Y, Z, 2.0, 1.0), one, 1.0, -1.0);                     // 2y+z-1
  typename Alg::T v2 = A.add(one, Z, 1.0, -1.0);                                         // 1-z
  typename Alg::T t = A.add(Z, one, 2.0, -1.0);                                          // 2z-1
  auto F = jacobi_h(A, one, u1, v1, M, 0);
  for (const Idx& k : idx) {
    auto H = jacobi_h(A, one, u2, v2, k.q, 2 * k.p + 1);
    auto K = jacobi_h(A, one, t, one, k.r, 2 * k.p + 2 * k.q + 2);
    typename Alg::T v = A.mul(A.mul(F[k.p], H[k.q]), K[k.r]);
    out.push_back(A.add(v, v, norm_scale(3, k), 0.0));
  }
  return out;
}

}  // namespace

namespace {

// Coefficients of the three-term recurrence below, divided by its leading
// factor, for n < 8 and alpha < 24 (computed once).
struct JacobiTable {
  double c2[8][24], c3[8][24], c4[8][24];
  JacobiTable() {
    for (int n = 1; n < 8; ++n)
      for (int alpha = 0; alpha < 24; ++alpha) {
        const double a1 = 2.0 * (n + 1) * (n + alpha + 1) * (2.0 * n + alpha);
        c2[n][alpha] = (2.0 * n + alpha + 1) * alpha * alpha / a1;
        c3[n][alpha] = (2.0 * n + alpha) * (2.0 * n + alpha + 1) * (2.0 * n + alpha + 2) / a1;
        c4[n][alpha] = 2.0 * n * (n + alpha) * (2.0 * n + alpha + 2) / a1;
      }
  }
};
const JacobiTable kJac;

// Allocation-free homogenised Jacobi recurrence for point values
// (nmax < 8, alpha < 24).
inline void jacobi_h_pt(double u, double v, int nmax, int alpha, double* H) {
  H[0] = 1.0;
  if (nmax >= 1) H[1] = ((alpha + 2) * u + alpha * v) / 2.0;
  const double v2 = v * v;
  for (int n = 1; n < nmax; ++n)
    H[n + 1] = (kJac.c3[n][alpha] * u + kJac.c2[n][alpha] * v) * H[n] - kJac.c4[n][alpha] * v2 * H[n - 1];
}

}  // namespace

// Normalisation factors norm_scale(d, {p, q, r}) for p + q + r < 8, computed
// once (the same expression, so the same bits) instead of one square root
// per basis function and point.
namespace {
struct NormTable {
  double t2[8][8];
  double t3[8][8][8];
  NormTable() {
    for (int p = 0; p < 8; ++p)
      for (int q = 0; q < 8; ++q) {
        t2[p][q] = norm_scale(2, {p, q, 0});
        for (int r = 0; r < 8; ++r) t3[p][q][r] = norm_scale(3, {p, q, r});
      }
  }
};
const NormTable kNorm;
}  // namespace

void basis_eval(int d, int M, const double* xi, double* out) {
  constexpr int MX = 8;
  if (M >= MX) throw Error(CWENO_E_ARG, "degree too large");
  double F[MX + 1];
  int l = 0;
  if (d == 2) {
    const double x = xi[0], y = xi[1];
    jacobi_h_pt(2.0 * x + y - 1.0, 1.0 - y, M, 0, F);
    double G[MX + 1][MX + 1];
    for (int p = 0; p <= M; ++p) jacobi_h_pt(2.0 * y - 1.0, 1.0, M - p, 2 * p + 1, G[p]);
    for (int n = 0; n <= M; ++n)
      for (int p = n; p >= 0; --p) {
        int q = n - p;
        out[l++] = kNorm.t2[p][q] * F[p] * G[p][q];
      }
    return;
  }
  const double x = xi[0], y = xi[1], z = xi[2];
  jacobi_h_pt(2.0 * x + y + z - 1.0, 1.0 - y - z, M, 0, F);
  double H[MX + 1][MX + 1], K[MX + 1][MX + 1][MX + 1];
  for (int p = 0; p <= M; ++p) {
    jacobi_h_pt(2.0 * y + z - 1.0, 1.0 - z, M - p, 2 * p + 1, H[p]);
    for (int q = 0; p + q <= M; ++q) jacobi_h_pt(2.0 * z - 1.0, 1.0, M - p - q, 2 * p + 2 * q + 2, K[p][q]);
  }
  for (int n = 0; n <= M; ++n)
    for (int p = n; p >= 0; --p)
      for (int q = n - p; q >= 0; --q) {
        int r = n - p - q;
        out[l++] = kNorm.t3[p][q][r] * F[p] * H[p][q] * K[p][q][r];
      }
}

void grundmann_moller(int d, int degree, std::vector<double>& lam, std::vector<double>& w) {
  // Degree 2s+1 rule on the d-simplex (Grundmann & Moller, 1978):
  //   int_T f = sum_{i=0..s} (-1)^i 2^{-2s} (d+2s+1-2i)^{2s+1} / (i! (d+2s+1-i)!)
  //             * sum_{|beta| = s-i} f(barycentric (2 beta_k + 1)/(d+2s+1-2i))
  // over the unit simplex of volume 1/d!; weights are rescaled to sum to 1.
  int s = degree / 2;   // smallest s with 2s + 1 >= degree
  lam.clear();
  w.clear();
  auto fact = [](int n) { double f = 1; for (int k = 2; k <= n; ++k) f *= k; return f; };
  double vol = 1.0 / fact(d);
  for (int i = 0; i <= s; ++i) {
    int den = d + 2 * s + 1 - 2 * i;
    double coef = ((i % 2) ? -1.0 : 1.0) * std::pow(2.0, -2.0 * s) * std::pow((double)den, 2 * s + 1) /
                  (fact(i) * fact(d + 2 * s + 1 - i));
    int m = s - i;
    // enumerate beta in N^{d+1}, |beta| = m
    std::vector<int> beta(d + 1, 0);
    std::function<void(int, int)> rec = [&](int pos, int left) {
      if (pos == d) {
        beta[d] = left;
        for (int k = 0; k <= d; ++k) lam.push_back((2.0 * beta[k] + 1.0) / den);
        w.push_back(coef / vol);
        return;
      }
      for (int b = 0; b <= left; ++b) { beta[pos] = b; rec(pos + 1, left - b); }
    };
    rec(0, m);
  }
}

void sigma_matrix(int d, int M, std::vector<double>& S) {
  PolyAlg A;
  const int deg = M;
  Poly one = plin(d, deg, 1, 0, 0, 0);
  Poly X = plin(d, deg, 0, 1, 0, 0), Y = plin(d, deg, 0, 0, 1, 0), Z = plin(d, deg, 0, 0, 0, 1);
  auto P = dubiner(A, d, M, one, X, Y, Z);
  const int nb = (int)P.size();
  std::vector<double> lam, w;
  grundmann_moller(d, 2 * M, lam, w);
  const int nq = (int)w.size();
  const double vol = d == 2 ? 0.5 : 1.0 / 6.0;
  S.assign((size_t)nb * nb, 0.0);
  std::vector<double> vals((size_t)nb * nq);
  for (int n = 1; n <= M; ++n)
    for (int a = 0; a <= n; ++a)
      for (int b = 0; a + b <= n; ++b) {
        int e = n - a - b;
        if (d == 2 && e != 0) continue;
        // d^alpha psi_l at the quadrature points
        for (int l = 0; l < nb; ++l) {
          const Poly& p = P[l];
          for (int q = 0; q < nq; ++q) {
            const double* L = &lam[(size_t)q * (d + 1)];
            double x = L[1], y = L[2], z = d == 3 ? L[3] : 0.0;
            double acc = 0.0;
            for (int i = a; i <= deg; ++i)
              for (int j = b; i + j <= deg; ++j)
                for (int k = e; i + j + k <= deg; ++k) {
                  double c = p.c[p.at(i, j, k)];
                  if (c == 0.0) continue;
                  double f = c;
                  for (int t = 0; t < a; ++t) f *= (i - t);
                  for (int t = 0; t < b; ++t) f *= (j - t);
                  for (int t = 0; t < e; ++t) f *= (k - t);
                  acc += f * std::pow(x, i - a) * std::pow(y, j - b) * std::pow(z, k - e);
                }
            vals[(size_t)l * nq + q] = acc;
          }
        }
        for (int l = 0; l < nb; ++l)
          for (int m = 0; m < nb; ++m) {
            double acc = 0.0;
            for (int q = 0; q < nq; ++q) acc += w[q] * vals[(size_t)l * nq + q] * vals[(size_t)m * nq + q];
            S[(size_t)l * nb + m] += acc * vol;
          }
      }
}

}  // namespace cweno
