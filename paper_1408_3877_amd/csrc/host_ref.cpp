// Reference element on the host: modal basis (Sec. 2.4.1; orders 5 and 6 by
// recursion), Gauss rules
// (Sec. 3.3), reference tensors (Sec. 3.6), computed once per context.
#include <cmath>
#include <stdexcept>

#include "ldg_internal.h"

namespace ldg {

int num_basis(int p) { return (p + 1) * (p + 2) / 2; }

namespace {
// Each basis function is a scale times sum c * x1^a * x2^b; the polynomials
// are the paper's closed forms multiplied out.
struct Term { int c, a, b; };
struct Poly { double scale; int nt; Term t[15]; };

const Poly& poly(int i) {
  static const Poly P[15] = {
    {std::sqrt(2.0), 1, {{1, 0, 0}}},
    {1.0, 2, {{2, 0, 0}, {-6, 1, 0}}},
    {2 * std::sqrt(3.0), 3, {{1, 0, 0}, {-1, 1, 0}, {-2, 0, 1}}},
    {std::sqrt(6.0), 3, {{1, 0, 0}, {-8, 1, 0}, {10, 2, 0}}},
    {std::sqrt(3.0), 5, {{-1, 0, 0}, {-4, 1, 0}, {12, 0, 1}, {5, 2, 0}, {-15, 0, 2}}},
    {3 * std::sqrt(5.0), 6, {{1, 0, 0}, {-4, 1, 0}, {-4, 0, 1}, {3, 2, 0}, {8, 1, 1}, {3, 0, 2}}},
    {2 * std::sqrt(2.0), 4, {{-1, 0, 0}, {15, 1, 0}, {-45, 2, 0}, {35, 3, 0}}},
    {2 * std::sqrt(6.0), 7,
     {{-1, 0, 0}, {13, 1, 0}, {2, 0, 1}, {-33, 2, 0}, {-24, 1, 1}, {21, 3, 0}, {42, 2, 1}}},
    {2 * std::sqrt(10.0), 9,
     {{-1, 0, 0}, {9, 1, 0}, {6, 0, 1}, {-15, 2, 0}, {-48, 1, 1}, {-6, 0, 2}, {7, 3, 0},
      {42, 2, 1}, {42, 1, 2}}},
    {2 * std::sqrt(14.0), 10,
     {{-1, 0, 0}, {3, 1, 0}, {12, 0, 1}, {-3, 2, 0}, {-24, 1, 1}, {-30, 0, 2}, {1, 3, 0},
      {12, 2, 1}, {30, 1, 2}, {20, 0, 3}}},
    {std::sqrt(10.0), 5, {{1, 0, 0}, {-24, 1, 0}, {126, 2, 0}, {-224, 3, 0}, {126, 4, 0}}},
    {std::sqrt(30.0), 9,
     {{1, 0, 0}, {-22, 1, 0}, {-2, 0, 1}, {105, 2, 0}, {42, 1, 1}, {-168, 3, 0}, {-168, 2, 1},
      {84, 4, 0}, {168, 3, 1}}},
    {5 * std::sqrt(2.0), 12,
     {{1, 0, 0}, {-18, 1, 0}, {-6, 0, 1}, {69, 2, 0}, {102, 1, 1}, {6, 0, 2}, {-88, 3, 0},
      {-312, 2, 1}, {-96, 1, 2}, {36, 4, 0}, {216, 3, 1}, {216, 2, 2}}},
    {std::sqrt(70.0), 14,
     {{1, 0, 0}, {-12, 1, 0}, {-12, 0, 1}, {30, 2, 0}, {132, 1, 1}, {30, 0, 2}, {-28, 3, 0},
      {-228, 2, 1}, {-300, 1, 2}, {-20, 0, 3}, {9, 4, 0}, {108, 3, 1}, {270, 2, 2},
      {180, 1, 3}}},
    {3 * std::sqrt(10.0), 15,
     {{1, 0, 0}, {-4, 1, 0}, {-20, 0, 1}, {6, 2, 0}, {60, 1, 1}, {90, 0, 2}, {-4, 3, 0},
      {-60, 2, 1}, {-180, 1, 2}, {-140, 0, 3}, {1, 4, 0}, {20, 3, 1}, {90, 2, 2},
      {140, 1, 3}, {70, 0, 4}}},
  };
  if (i < 0 || i >= 15) throw std::out_of_range("basis index");
  return P[i];
}

double ipow(double x, int a) {
  double r = 1.0;
  for (int k = 0; k < a; ++k) r *= x;
  return r;
}
}  // namespace

// Orders 5 and 6 (basis indices 15..27): the orthonormal collapsed-coordinate
// polynomials of total degree d = a + q, q = 0..d in that order,
//   psi = c A_a(x1, x2) J_q(2 x2 - 1),  c = sqrt(2 (2a+1) (a+q+1)),
// A_a = (1 - x2)^a P_a(2 x1 / (1 - x2) - 1) (P_a Legendre), J_q the Jacobi
// polynomial P_q^{(2a+1,0)}.  Each is orthogonal to all polynomials of lower
// degree, so the paper's fifteen functions followed by these are orthonormal
// (the recursion alternative to Gram-Schmidt of Sec. 2.4.1).  Both factors
// come from three-term recurrences; A_a is carried as a polynomial, so the
// vertex x2 = 1 needs no special case.
namespace {
constexpr int kPaperFunctions = 15;

void collapsed_index(int i, int& a, int& q) {
  int j = i - kPaperFunctions;
  for (int d = 5; d <= 6; ++d) {
    if (j <= d) {
      a = d - j;
      q = j;
      return;
    }
    j -= d + 1;
  }
  throw std::out_of_range("basis index");
}

// value v = psi, gradient (gx, gy)
void collapsed_psi(int i, double x1, double x2, double& v, double& gx, double& gy) {
  int a, q;
  collapsed_index(i, a, q);
  // A_n: (n+1) A_{n+1} = (2n+1) s A_n - n t^2 A_{n-1},  s = 2 x1 - t, t = 1 - x2
  const double t = 1.0 - x2, s = 2.0 * x1 - t;
  double A = 1.0, Ax = 0.0, Ay = 0.0;            // A_0
  if (a >= 1) {
    double Am = 1.0, Amx = 0.0, Amy = 0.0;       // A_{n-1}
    A = s; Ax = 2.0; Ay = 1.0;                   // A_1
    for (int n = 1; n < a; ++n) {
      const double t2 = t * t, t2y = -2.0 * t;
      const double An = ((2 * n + 1) * s * A - n * t2 * Am) / (n + 1);
      const double Anx = ((2 * n + 1) * (2.0 * A + s * Ax) - n * t2 * Amx) / (n + 1);
      const double Any = ((2 * n + 1) * (A + s * Ay) - n * (t2y * Am + t2 * Amy)) / (n + 1);
      Am = A; Amx = Ax; Amy = Ay;
      A = An; Ax = Anx; Ay = Any;
    }
  }
  // J_n = P_n^{(al,0)}(e), e = 2 x2 - 1:
  // 2n(n+al)(2n+al-2) J_n = (2n+al-1)((2n+al)(2n+al-2) e + al^2) J_{n-1}
  //                         - 2(n+al-1)(n-1)(2n+al) J_{n-2}
  const double al = 2.0 * a + 1.0, e = 2.0 * x2 - 1.0;
  double J = 1.0, Je = 0.0;                      // J_0 and d/de
  if (q >= 1) {
    double Jm = 1.0, Jme = 0.0;
    J = (al + 1.0) + (al + 2.0) * (e - 1.0) / 2.0;
    Je = (al + 2.0) / 2.0;
    for (int n = 2; n <= q; ++n) {
      const double c0 = 2.0 * n * (n + al) * (2 * n + al - 2);
      const double c1 = (2 * n + al - 1) * (2 * n + al) * (2 * n + al - 2);
      const double c2 = (2 * n + al - 1) * al * al;
      const double c3 = 2.0 * (n + al - 1) * (n - 1) * (2 * n + al);
      const double Jn = ((c1 * e + c2) * J - c3 * Jm) / c0;
      const double Jne = (c1 * J + (c1 * e + c2) * Je - c3 * Jme) / c0;
      Jm = J; Jme = Je;
      J = Jn; Je = Jne;
    }
  }
  const double c = std::sqrt(2.0 * (2 * a + 1) * (a + q + 1));
  v = c * A * J;
  gx = c * Ax * J;
  gy = c * (Ay * J + A * 2.0 * Je);
}
}  // namespace

double phi_hat(int i, double x1, double x2) {
  if (i >= kPaperFunctions) {
    double v, gx, gy;
    collapsed_psi(i, x1, x2, v, gx, gy);
    return v;
  }
  const Poly& P = poly(i);
  double v = 0.0;
  for (int t = 0; t < P.nt; ++t) v += P.t[t].c * ipow(x1, P.t[t].a) * ipow(x2, P.t[t].b);
  return P.scale * v;
}

double dphi_hat(int i, int m, double x1, double x2) {
  if (i >= kPaperFunctions) {
    double v, gx, gy;
    collapsed_psi(i, x1, x2, v, gx, gy);
    return m == 0 ? gx : gy;
  }
  const Poly& P = poly(i);
  double v = 0.0;
  for (int t = 0; t < P.nt; ++t) {
    const Term& T = P.t[t];
    if (m == 0 && T.a > 0) v += T.c * T.a * ipow(x1, T.a - 1) * ipow(x2, T.b);
    if (m == 1 && T.b > 0) v += T.c * T.b * ipow(x1, T.a) * ipow(x2, T.b - 1);
  }
  return P.scale * v;
}

// Gauss-Legendre on (0,1): Newton iteration on P_n from the Chebyshev guess.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double t = std::cos(M_PI * (k + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = t; p0 = 1.0; }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    // recompute derivative at the converged node for the weight
    double p0 = 1.0, p1 = t;
    for (int j = 2; j <= n; ++j) {
      double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = t; p0 = 1.0; }
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    double wt = 2.0 / ((1.0 - t * t) * dp * dp);
    x[n - 1 - k] = 0.5 * (t + 1.0);   // ascending
    w[n - 1 - k] = 0.5 * wt;
  }
}

// Gauss-Jacobi on (0,1) for the weight (1 - u): the roots of the Jacobi
// polynomial P_n^(1,0)(x), x = 2u - 1, by Newton's method from the
// Gauss-Legendre nodes, with the three-term recurrence
//   (k+1)(2k-1) P_k = ((2k+1)(2k-1) x + 1) P_{k-1} - (k-1)(2k+1) P_{k-2},
// P_0 = 1, P_1 = (3x + 1)/2, and the weights 4 / ((1 - x^2) P_n'(x)^2) on
// (-1,1) for (1 - x), i.e. 1 / ((1 - x^2) P_n'(x)^2) on (0,1) for (1 - u)
// (Golub and Welsch's weights for this family in closed form).
void gauss_jacobi10(int n, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> g, gw;
  gauss_legendre(n, g, gw);
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  auto eval = [n](double t, double& P, double& dP) {
    double p0 = 1.0, d0 = 0.0, p1 = 0.5 * (3.0 * t + 1.0), d1 = 1.5;
    if (n == 0) { P = p0; dP = d0; return; }
    for (int k = 2; k <= n; ++k) {
      const double a = (2.0 * k + 1.0) * (2.0 * k - 1.0), b = (k - 1.0) * (2.0 * k + 1.0);
      const double c = (k + 1.0) * (2.0 * k - 1.0);
      const double p2 = ((a * t + 1.0) * p1 - b * p0) / c;
      const double d2 = (a * p1 + (a * t + 1.0) * d1 - b * d0) / c;
      p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    P = p1;
    dP = d1;
  };
  for (int k = 0; k < n; ++k) {
    double t = 2.0 * g[k] - 1.0, P = 0.0, dP = 1.0;
    for (int it = 0; it < 100; ++it) {
      eval(t, P, dP);
      const double dt = P / dP;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    eval(t, P, dP);
    x[k] = 0.5 * (t + 1.0);
    w[k] = 1.0 / ((1.0 - t * t) * dP * dP);
  }
}

namespace {
// Gauss points of the unit square collapsed onto the reference triangle:
// x1 = u, x2 = (1-u) v, Jacobian 1-u, n points per direction.
void collapsed(int n, std::vector<double>& q1, std::vector<double>& q2, std::vector<double>& w) {
  std::vector<double> u, wu;
  gauss_legendre(n, u, wu);
  q1.clear(); q2.clear(); w.clear();
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      q1.push_back(u[a]);
      q2.push_back((1.0 - u[a]) * u[b]);
      w.push_back(wu[a] * wu[b] * (1.0 - u[a]));
    }
}
}  // namespace

// Volume rule of order max(2p,1) used for the L2 projection (main script):
// the printed rules of orders 1, 2, 4 and 6 (Sec. 3.3, quadRule2D) and, for
// the orders 8, 10, 12 of p = 4, 5, 6, the n x n collapsed Gauss rule, n = order.
void projection_rule(int p, std::vector<double>& q1, std::vector<double>& q2,
                     std::vector<double>& w) {
  const int ord = p == 0 ? 1 : 2 * p;
  if (ord == 1) {
    q1 = {1.0 / 3}; q2 = {1.0 / 3}; w = {0.5};
  } else if (ord == 2) {
    q1 = {1.0 / 6, 2.0 / 3, 1.0 / 6};
    q2 = {1.0 / 6, 1.0 / 6, 2.0 / 3};
    w = {1.0 / 6, 1.0 / 6, 1.0 / 6};
  } else if (ord == 4) {
    const double a = 0.445948490915965, a2 = 0.108103018168070;
    const double b = 0.091576213509771, b2 = 0.816847572980458;
    const double wa = 0.111690794839005, wb = 0.054975871827661;
    q1 = {a, a2, a, b, b2, b};
    q2 = {a2, a, a, b2, b, b};
    w = {wa, wa, wa, wb, wb, wb};
  } else if (ord == 6) {
    const double a = 0.063089014491502, a2 = 0.873821971016996;
    const double b = 0.249286745170910, b2 = 0.501426509658179;
    const double c = 0.310352451033785, d = 0.053145049844816, e = 0.636502499121399;
    const double wa = 0.025422453185103, wb = 0.058393137863189, wc = 0.041425537809187;
    q1 = {a, a2, a, b, b2, b, c, d, e, d, e, c};
    q2 = {a, a, a2, b, b, b2, d, c, d, e, c, e};
    w = {wa, wa, wa, wb, wb, wb, wc, wc, wc, wc, wc, wc};
  } else {
    collapsed(ord, q1, q2, w);
  }
}

namespace {
void edge_point(int n, double s, double& x1, double& x2) {
  // reference edge n runs from vertex n+1 to vertex n+2 (counter-clockwise)
  if (n == 0) { x1 = 1.0 - s; x2 = s; }
  else if (n == 1) { x1 = 0.0; x2 = 1.0 - s; }
  else { x1 = s; x2 = 0.0; }
}
}  // namespace

RefData build_refdata(int p, int policy) {
  RefData r;
  r.p = p;
  const int N = r.N = num_basis(p);
  const int NN = r.NN = N * N;
  std::vector<double> q1, q2, w, s, ws;
  if (policy == LDG_QUAD_PAPER) {
    // the paper's routines: order max(2p, 1) on the triangle (the projection
    // rule) and 2p + 1 on edges, below the degree 3p of the three-factor
    // integrands for p >= 2 (exact for M, H and the two-factor edge terms)
    projection_rule(p, q1, q2, w);
    gauss_legendre(p + 1, s, ws);
  } else {
    // exact integration: 12 x 12 collapsed points (degree 22) on the triangle,
    // 12 Gauss points (degree 23) on edges; integrands have degree <= 3p.
    collapsed(12, q1, q2, w);
    gauss_legendre(12, s, ws);
  }
  const int R = (int)w.size();
  std::vector<double> ph(R * N), dph[2];
  dph[0].resize(R * N);
  dph[1].resize(R * N);
  for (int q = 0; q < R; ++q)
    for (int i = 0; i < N; ++i) {
      ph[q * N + i] = phi_hat(i, q1[q], q2[q]);
      dph[0][q * N + i] = dphi_hat(i, 0, q1[q], q2[q]);
      dph[1][q * N + i] = dphi_hat(i, 1, q1[q], q2[q]);
    }
  r.M.assign(NN, 0.0);
  for (int m = 0; m < 2; ++m) { r.H[m].assign(NN, 0.0); r.G[m].assign(N * NN, 0.0); }
  for (int q = 0; q < R; ++q)
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const double pp = w[q] * ph[q * N + i] * ph[q * N + j];
        r.M[i * N + j] += pp;
        for (int m = 0; m < 2; ++m) {
          const double dp = w[q] * dph[m][q * N + i] * ph[q * N + j];
          r.H[m][i * N + j] += dp;
          for (int l = 0; l < N; ++l) r.G[m][(l * N + i) * N + j] += dp * ph[q * N + l];
        }
      }
  const int Q = (int)s.size();
  for (int a = 0; a < 3; ++a) {
    r.Sd[a].assign(NN, 0.0);
    r.Rd[a].assign(N * NN, 0.0);
    std::vector<double> pa(Q * N);
    for (int q = 0; q < Q; ++q) {
      double x1, x2;
      edge_point(a, s[q], x1, x2);
      for (int i = 0; i < N; ++i) pa[q * N + i] = phi_hat(i, x1, x2);
    }
    for (int q = 0; q < Q; ++q)
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          const double v = ws[q] * pa[q * N + i] * pa[q * N + j];
          r.Sd[a][i * N + j] += v;
          for (int l = 0; l < N; ++l) r.Rd[a][(l * N + i) * N + j] += v * pa[q * N + l];
        }
    for (int b = 0; b < 3; ++b) {
      // the neighbour's trace: a point at parameter s on edge a of T- is the
      // point at parameter 1-s on edge b of T+ (both triangles counter-clockwise)
      std::vector<double> pb(Q * N);
      for (int q = 0; q < Q; ++q) {
        double x1, x2;
        edge_point(b, 1.0 - s[q], x1, x2);
        for (int i = 0; i < N; ++i) pb[q * N + i] = phi_hat(i, x1, x2);
      }
      r.So[a][b].assign(NN, 0.0);
      r.Ro[a][b].assign(N * NN, 0.0);
      for (int q = 0; q < Q; ++q)
        for (int i = 0; i < N; ++i)
          for (int j = 0; j < N; ++j) {
            const double v = ws[q] * pa[q * N + i] * pb[q * N + j];
            r.So[a][b][i * N + j] += v;
            for (int l = 0; l < N; ++l) r.Ro[a][b][(l * N + i) * N + j] += v * pb[q * N + l];
          }
    }
  }
  projection_rule(p, r.q1, r.q2, r.w);
  r.R = (int)r.w.size();
  gauss_legendre(p + 1, r.s, r.ws);   // order 2p+1 on boundary edges
  r.R1 = p + 1;
  return r;
}

}  // namespace ldg
