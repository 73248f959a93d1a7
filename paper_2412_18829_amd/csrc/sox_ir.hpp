// In-house intermediate-representation (IR) imaginary-time grid (host code).
//
// The paper's computational details run every calculation on sparse IR
// grids (beta, Lambda and the number of tau points are listed there).  The IR
// basis is the singular value expansion of the analytic-continuation kernel;
// this file builds the grid the library's plans take (tau nodes, quadrature
// weights, the bosonic transform pair) from that definition:
//
//  * kernel: in x = 2 tau / beta - 1 and y = beta omega / Lambda, the logistic
//    kernel K(x, y) = exp(-Lambda y (x + 1) / 2) / (1 + exp(-Lambda y)); it is
//    centrosymmetric, so the expansion splits into an even and an odd part
//    on [0, 1]^2, K_+-(x, y) = K(x, y) +- K(x, -y), whose singular functions
//    are the even and odd u_l;
//  * discretisation: composite Gauss-Legendre quadrature, kIrP nodes per
//    segment, segments graded geometrically towards x = 1 and y = 0 (where
//    the kernel varies on the scale 1 / Lambda) and at most kIrHmax wide;
//  * singular values and left vectors of sqrt(w_x) K_+- sqrt(w_y) by
//    one-sided (Hestenes) Jacobi rotations, which keep small singular values
//    to high relative accuracy; u_l = column / sqrt(w_x) / sqrt(2), sign
//    fixed by u_l(x -> 1) > 0, parities merged by singular value, basis size
//    L = #{s_l >= eps s_0};
//  * u_l between nodes from per-segment Legendre series;
//  * sampling times: the L roots of u_L (the first function left out has
//    exactly L roots), ascending and mirror symmetric;
//  * Matsubara transforms U^_l(i Omega_m) per segment from
//    int_{-1}^{1} e^{i a t} P_k(t) dt = 2 i^k j_k(a) (spherical Bessel j_k by
//    upward recurrence for a >= 16, normalised downward recurrence below);
//  * bosonic frequencies: m = 0 and, for the first even and the first odd
//    function left out, the integer just below each sign change of Re U^
//    (even) or Im U^ (odd) for m <= 4 Lambda, found on every integer up to
//    1024 and on steps of m / 32 beyond (the sign changes there are at least
//    0.15 m apart for eps >= 1e-12), each bracket closed by bisection;
//  * fermionic pair: the odd frequencies and the sign changes of Im U^ (even)
//    and Re U^ (odd) instead, plus the row t_beta that evaluates the fitted
//    expansion at tau = beta^-;
//  * transform pair for functions real in imaginary time: T_fwd = U^ U_s^-1,
//    T_bwd from the least-squares inverse of [Re U^; Im U^] (Householder QR),
//    f(tau_i) = Re sum_m T_bwd[i][m] f(i Omega_m); weights w = U_s^-T I with
//    I_l = int_0^beta U_l(tau) dtau.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

namespace sox_ir {

constexpr int kIrP = 16;
constexpr double kIrHmax = 0.25;

using cplx = std::complex<double>;

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton on P_n.
inline void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w) {
  t.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) {
        p0 = 1.0;
        p1 = x;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        break;
      }
    }
    t[n - 1 - i] = x;
    w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

// Legendre P_0 .. P_{n-1} at t
inline void legendre_all(double t, int n, double* p) {
  p[0] = 1.0;
  if (n > 1) p[1] = t;
  for (int k = 2; k < n; ++k) p[k] = ((2.0 * k - 1.0) * t * p[k - 1] - (k - 1.0) * p[k - 2]) / k;
}

// Spherical Bessel j_0 .. j_{n-1} at a >= 0.
inline void sph_bessel_all(double a, int n, double* j) {
  if (a == 0.0) {
    j[0] = 1.0;
    for (int k = 1; k < n; ++k) j[k] = 0.0;
    return;
  }
  const double s = std::sin(a), c = std::cos(a);
  if (a >= 16.0) {
    // upward recurrence, stable for a >= the order
    j[0] = s / a;
    if (n > 1) j[1] = s / (a * a) - c / a;
    for (int k = 1; k + 1 < n; ++k) j[k + 1] = (2.0 * k + 1.0) / a * j[k] - j[k - 1];
    return;
  }
  // Miller: downward recurrence from far above the order, normalised by the
  // exact j_0 or j_1, whichever is larger in the recurrence
  const int top = n + 40 + (int)a;
  std::vector<double> f(top + 2, 0.0);
  f[top + 1] = 0.0;
  f[top] = 1e-300;
  for (int k = top; k >= 1; --k) {
    f[k - 1] = (2.0 * k + 1.0) / a * f[k] - f[k + 1];
    if (std::fabs(f[k - 1]) > 1e250) {
      for (int q = k - 1; q <= top + 1; ++q) f[q] *= 1e-250;
    }
  }
  const double j0 = s / a;
  const double j1 = a < 1e-3 ? a / 3.0 - a * a * a / 30.0 : s / (a * a) - c / a;
  const double scale = std::fabs(f[0]) >= std::fabs(f[1]) ? j0 / f[0] : j1 / f[1];
  for (int k = 0; k < n; ++k) j[k] = f[k] * scale;
}

inline double kernel(double x, double y, double lam) {
  const double a = std::fabs(y);
  const double num = y >= 0.0 ? std::exp(-lam * a * (x + 1.0) / 2.0) : std::exp(-lam * a * (1.0 - x) / 2.0);
  return num / (1.0 + std::exp(-lam * a));
}

inline std::vector<double> segments(double lam, bool towards_one) {
  std::vector<double> b{0.0, 1.0};
  for (int j = 0; std::ldexp(1.0, j) / lam < 1.0; ++j) {
    const double d = std::ldexp(1.0, j) / lam;
    b.push_back(towards_one ? 1.0 - d : d);
  }
  std::sort(b.begin(), b.end());
  b.erase(std::unique(b.begin(), b.end()), b.end());
  std::vector<double> out{b[0]};
  for (size_t i = 0; i + 1 < b.size(); ++i) {
    const double a = b[i], c = b[i + 1];
    const int m = (int)std::ceil((c - a) / kIrHmax - 1e-12);
    for (int q = 1; q <= m; ++q) out.push_back(a + (c - a) * ((double)q / m));
  }
  return out;
}

inline void quadrature(const std::vector<double>& br, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> t, wt;
  gauss_legendre(kIrP, t, wt);
  x.clear();
  w.clear();
  for (size_t s = 0; s + 1 < br.size(); ++s) {
    const double a = br[s], b = br[s + 1];
    for (int i = 0; i < kIrP; ++i) {
      x.push_back((a + b) / 2.0 + (b - a) / 2.0 * t[i]);
      w.push_back((b - a) / 2.0 * wt[i]);
    }
  }
}

// One-sided Jacobi: the columns of A (rows x cols, column-major) are rotated
// until pairwise orthogonal; then column l = s_l u_l.  Returns the singular
// values (column norms) and the normalised columns.
inline void jacobi_svd(std::vector<double>& A, int rows, int cols, std::vector<double>& s) {
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < cols - 1; ++p) {
      double* ap = A.data() + (size_t)p * rows;
      for (int q = p + 1; q < cols; ++q) {
        double* aq = A.data() + (size_t)q * rows;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = 0; i < rows; ++i) {
          al += ap[i] * ap[i];
          be += aq[i] * aq[i];
          ga += ap[i] * aq[i];
        }
        if (al == 0.0 || be == 0.0 || std::fabs(ga) <= 1e-15 * std::sqrt(al * be)) continue;
        rotated = true;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < rows; ++i) {
          const double u = ap[i], v = aq[i];
          ap[i] = c * u - sn * v;
          aq[i] = sn * u + c * v;
        }
      }
    }
    if (!rotated) break;
  }
  s.assign(cols, 0.0);
  for (int l = 0; l < cols; ++l) {
    double* a = A.data() + (size_t)l * rows;
    double nrm = 0.0;
    for (int i = 0; i < rows; ++i) nrm += a[i] * a[i];
    nrm = std::sqrt(nrm);
    s[l] = nrm;
    if (nrm > 0.0)
      for (int i = 0; i < rows; ++i) a[i] /= nrm;
  }
}

struct Func {
  double s;
  int par;                   // +1 even, -1 odd
  std::vector<double> u;     // at the x nodes of [0, 1]
  std::vector<double> coef;  // [segment][k]
};

struct Sve {
  std::vector<double> bx, x, wx;
  std::vector<Func> f;  // descending singular value
};

inline void legendre_coeffs(const Sve& sv, Func& fn) {
  std::vector<double> t, w, pk(kIrP);
  gauss_legendre(kIrP, t, w);
  const int nseg = (int)sv.bx.size() - 1;
  fn.coef.assign((size_t)nseg * kIrP, 0.0);
  for (int sg = 0; sg < nseg; ++sg)
    for (int i = 0; i < kIrP; ++i) {
      legendre_all(t[i], kIrP, pk.data());
      const double wu = w[i] * fn.u[(size_t)sg * kIrP + i];
      for (int k = 0; k < kIrP; ++k) fn.coef[(size_t)sg * kIrP + k] += wu * pk[k];
    }
  for (int sg = 0; sg < nseg; ++sg)
    for (int k = 0; k < kIrP; ++k) fn.coef[(size_t)sg * kIrP + k] *= (2.0 * k + 1.0) / 2.0;
}

inline Sve compute_sve(double lam) {
  Sve sv;
  sv.bx = segments(lam, true);
  const std::vector<double> by = segments(lam, false);
  std::vector<double> y, wy;
  quadrature(sv.bx, sv.x, sv.wx);
  quadrature(by, y, wy);
  const int nx = (int)sv.x.size(), ny = (int)y.size();
  for (int par = 1; par >= -1; par -= 2) {
    // columns indexed by y: A[:, j] = sqrt(w_x) K_par(x, y_j) sqrt(w_y)
    std::vector<double> A((size_t)nx * ny);
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        A[(size_t)j * nx + i] = std::sqrt(sv.wx[i]) *
                                (kernel(sv.x[i], y[j], lam) + par * kernel(sv.x[i], -y[j], lam)) *
                                std::sqrt(wy[j]);
    std::vector<double> s;
    jacobi_svd(A, nx, ny, s);
    for (int l = 0; l < ny; ++l) {
      Func fn;
      fn.s = s[l];
      fn.par = par;
      fn.u.resize(nx);
      for (int i = 0; i < nx; ++i) fn.u[i] = A[(size_t)l * nx + i] / std::sqrt(sv.wx[i]) / std::sqrt(2.0);
      if (fn.u[nx - 1] < 0.0)
        for (double& v : fn.u) v = -v;
      sv.f.push_back(std::move(fn));
    }
  }
  std::stable_sort(sv.f.begin(), sv.f.end(), [](const Func& a, const Func& b) { return a.s > b.s; });
  return sv;
}

// u(x) for x in [-1, 1]
inline double evaluate(const Sve& sv, const Func& fn, double x) {
  const double ax = std::fabs(x);
  const int nseg = (int)sv.bx.size() - 1;
  int sg = (int)(std::upper_bound(sv.bx.begin(), sv.bx.end(), ax) - sv.bx.begin()) - 1;
  sg = std::min(std::max(sg, 0), nseg - 1);
  const double a = sv.bx[sg], b = sv.bx[sg + 1];
  const double t = (2.0 * ax - a - b) / (b - a);
  double pk[kIrP];
  legendre_all(t, kIrP, pk);
  double v = 0.0;
  for (int k = 0; k < kIrP; ++k) v += fn.coef[(size_t)sg * kIrP + k] * pk[k];
  return x < 0.0 ? fn.par * v : v;
}

inline std::vector<double> roots(const Sve& sv, const Func& fn) {
  std::vector<double> grid;
  for (size_t sg = 0; sg + 1 < sv.bx.size(); ++sg)
    for (int i = 0; i < 64; ++i) grid.push_back(sv.bx[sg] + (sv.bx[sg + 1] - sv.bx[sg]) * (i / 64.0));
  grid.push_back(1.0);
  // an odd u vanishes at 0: its rounded value there carries no sign
  const size_t first = fn.par < 0 ? 1 : 0;
  std::vector<double> rs;
  double vprev = evaluate(sv, fn, grid[first]);
  for (size_t i = first; i + 1 < grid.size(); ++i) {
    const double vnext = evaluate(sv, fn, grid[i + 1]);
    if (grid[i] > 0.0 && vprev == 0.0) {
      rs.push_back(grid[i]);
    } else if (vprev * vnext < 0.0) {
      double a = grid[i], b = grid[i + 1], fa = vprev;
      for (int it = 0; it < 100; ++it) {
        const double m = 0.5 * (a + b);
        const double fm = evaluate(sv, fn, m);
        if (fa * fm <= 0.0) {
          b = m;
        } else {
          a = m;
          fa = fm;
        }
      }
      rs.push_back(0.5 * (a + b));
    }
    vprev = vnext;
  }
  std::vector<double> out;
  for (auto it = rs.rbegin(); it != rs.rend(); ++it)
    if (*it > 0.0) out.push_back(-*it);
  if (fn.par < 0) out.push_back(0.0);
  for (double r : rs)
    if (r > 0.0) out.push_back(r);
  return out;
}

// U^(i Omega) = sqrt(beta / 2) int_{-1}^{1} e^{i pi m (x + 1)} u(x) dx with
// Omega = 2 pi m / beta: m integer for bosons, m = n + 1/2 for fermions
inline cplx matsubara(const Sve& sv, const Func& fn, double beta, double m) {
  cplx acc(0.0, 0.0);
  double jb[kIrP];
  const cplx ipow[4] = {cplx(1, 0), cplx(0, 1), cplx(-1, 0), cplx(0, -1)};
  for (size_t sg = 0; sg + 1 < sv.bx.size(); ++sg) {
    const double a = sv.bx[sg], b = sv.bx[sg + 1];
    const double cc = (a + b) / 2.0, h = (b - a) / 2.0;
    sph_bessel_all(M_PI * m * h, kIrP, jb);
    cplx plus(0.0, 0.0), minus(0.0, 0.0);
    for (int k = 0; k < kIrP; ++k) {
      const double cj = fn.coef[sg * kIrP + k] * jb[k];
      plus += ipow[k & 3] * cj;
      minus += ipow[(4 - (k & 3)) & 3] * cj;
    }
    const cplx e1 = std::polar(1.0, M_PI * m * (cc + 1.0));
    const cplx e2 = std::polar(1.0, M_PI * m * (1.0 - cc));
    acc += 2.0 * h * (e1 * plus + (double)fn.par * e2 * minus);
  }
  return std::sqrt(beta / 2.0) * acc;
}

// integers m with g(m) g(m + 1) < 0 for m < mmax
template <class G>
inline void sign_changes(G&& g, long mmax, std::vector<long>& out) {
  long m = 0;
  double gm = g(0);
  while (m < mmax) {
    const long step = m < 1024 ? 1 : std::max(1L, m / 32);
    const long m2 = std::min(mmax, m + step);
    const double g2 = g(m2);
    if (gm * g2 < 0.0) {
      long lo = m, hi = m2;
      double glo = gm;
      while (hi - lo > 1) {
        const long mid = lo + (hi - lo) / 2;
        const double gmid = g(mid);
        if (glo * gmid < 0.0) {
          hi = mid;
        } else {
          lo = mid;
          glo = gmid;
        }
      }
      out.push_back(lo);
    }
    m = m2;
    gm = g2;
  }
}

// Solve A X = B in place (A n x n row-major, B n x r row-major), partial pivoting.
inline bool lu_solve(std::vector<double> A, int n, std::vector<double>& B, int r) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + c]) > std::fabs(A[(size_t)piv * n + c])) piv = i;
    if (A[(size_t)piv * n + c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[(size_t)c * n + k], A[(size_t)piv * n + k]);
      for (int k = 0; k < r; ++k) std::swap(B[(size_t)c * r + k], B[(size_t)piv * r + k]);
    }
    for (int i = c + 1; i < n; ++i) {
      const double f = A[(size_t)i * n + c] / A[(size_t)c * n + c];
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) A[(size_t)i * n + k] -= f * A[(size_t)c * n + k];
      for (int k = 0; k < r; ++k) B[(size_t)i * r + k] -= f * B[(size_t)c * r + k];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int k = 0; k < r; ++k) {
      double v = B[(size_t)c * r + k];
      for (int j = c + 1; j < n; ++j) v -= A[(size_t)c * n + j] * B[(size_t)j * r + k];
      B[(size_t)c * r + k] = v / A[(size_t)c * n + c];
    }
  }
  return true;
}

// Least-squares inverse of B (rows x cols, rows >= cols, full column rank,
// row-major) by Householder QR: returns P (cols x rows) with P B = I.
inline bool lsq_inverse(std::vector<double> B, int rows, int cols, std::vector<double>& P) {
  std::vector<double> Q((size_t)rows * rows, 0.0);  // accumulate Q^T as rows x rows
  for (int i = 0; i < rows; ++i) Q[(size_t)i * rows + i] = 1.0;
  for (int c = 0; c < cols; ++c) {
    double nrm = 0.0;
    for (int i = c; i < rows; ++i) nrm += B[(size_t)i * cols + c] * B[(size_t)i * cols + c];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return false;
    const double alpha = B[(size_t)c * cols + c] > 0.0 ? -nrm : nrm;
    std::vector<double> v(rows, 0.0);
    for (int i = c; i < rows; ++i) v[i] = B[(size_t)i * cols + c];
    v[c] -= alpha;
    double vv = 0.0;
    for (int i = c; i < rows; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int k = c; k < cols; ++k) {
      double d = 0.0;
      for (int i = c; i < rows; ++i) d += v[i] * B[(size_t)i * cols + k];
      d = 2.0 * d / vv;
      for (int i = c; i < rows; ++i) B[(size_t)i * cols + k] -= d * v[i];
    }
    for (int k = 0; k < rows; ++k) {
      double d = 0.0;
      for (int i = c; i < rows; ++i) d += v[i] * Q[(size_t)i * rows + k];
      d = 2.0 * d / vv;
      for (int i = c; i < rows; ++i) Q[(size_t)i * rows + k] -= d * v[i];
    }
  }
  // P = R^-1 (Q^T)[:cols, :]
  P.assign((size_t)cols * rows, 0.0);
  for (int k = 0; k < rows; ++k)
    for (int c = cols - 1; c >= 0; --c) {
      double v = Q[(size_t)c * rows + k];
      for (int j = c + 1; j < cols; ++j) v -= B[(size_t)c * cols + j] * P[(size_t)j * rows + k];
      P[(size_t)c * rows + k] = v / B[(size_t)c * cols + c];
    }
  return true;
}

struct Grid {
  int L = 0;
  std::vector<double> tau, weights, sv;  // sv: s_l / s_0
  std::vector<double> t_beta;            // f(beta^-) = sum_i t_beta[i] f(tau_i)
  std::vector<long> m;
  std::vector<cplx> t_fwd;  // [n_omega][L]
  std::vector<cplx> t_bwd;  // [L][n_omega]
  std::string error;
};

// fermion: the odd frequencies nu_n = (2n + 1) pi / beta (m = n + 1/2), the
// sign changes of Im U^ of the first omitted even function and Re U^ of the
// first omitted odd one (a function even about beta / 2 has an imaginary
// fermionic transform); bosons: the even frequencies, Re and Im swapped.
inline Grid build(double beta, double lam, double eps, bool fermion = false) {
  Grid g;
  Sve sv = compute_sve(lam);
  const double s0 = sv.f[0].s;
  int L = 0;
  while (L < (int)sv.f.size() && sv.f[L].s >= eps * s0) ++L;
  int le = -1, lo = -1;
  for (int l = L; l < (int)sv.f.size(); ++l) {
    if (le < 0 && sv.f[l].par > 0) le = l;
    if (lo < 0 && sv.f[l].par < 0) lo = l;
  }
  if (le < 0 || lo < 0) {
    g.error = "the discretisation holds no function beyond the basis";
    return g;
  }
  for (int l = 0; l <= std::max(le, lo); ++l) legendre_coeffs(sv, sv.f[l]);
  const std::vector<double> xr = roots(sv, sv.f[L]);
  if ((int)xr.size() != L) {
    g.error = "u_L has " + std::to_string(xr.size()) + " roots instead of " + std::to_string(L) +
              ": the basis is not resolved in float64 at this Lambda and eps";
    return g;
  }
  g.L = L;
  for (int l = 0; l < L; ++l) g.sv.push_back(sv.f[l].s / s0);
  for (double x : xr) g.tau.push_back(beta * (x + 1.0) / 2.0);
  // sampling matrix U_s[i][l] = sqrt(2 / beta) u_l(x_i)
  std::vector<double> Us((size_t)L * L);
  for (int i = 0; i < L; ++i)
    for (int l = 0; l < L; ++l) Us[(size_t)i * L + l] = std::sqrt(2.0 / beta) * evaluate(sv, sv.f[l], xr[i]);
  // bosonic frequencies
  const long mmax = (long)(4.0 * lam);
  std::vector<long> sc{0};
  const double sh = fermion ? 0.5 : 0.0;
  sign_changes(
      [&](long m) {
        const cplx v = matsubara(sv, sv.f[le], beta, (double)m + sh);
        return fermion ? v.imag() : v.real();
      },
      mmax, sc);
  sign_changes(
      [&](long m) {
        const cplx v = matsubara(sv, sv.f[lo], beta, (double)m + sh);
        return fermion ? v.real() : v.imag();
      },
      mmax, sc);
  std::sort(sc.begin(), sc.end());
  sc.erase(std::unique(sc.begin(), sc.end()), sc.end());
  g.m = sc;
  const int nm = (int)sc.size();
  if (2 * nm - 1 < L) {
    g.error = "too few Matsubara samples for the basis";
    g.L = 0;
    return g;
  }
  std::vector<cplx> Uh((size_t)nm * L);
  for (int q = 0; q < nm; ++q)
    for (int l = 0; l < L; ++l) Uh[(size_t)q * L + l] = matsubara(sv, sv.f[l], beta, (double)sc[q] + sh);
  // inverse of U_s: solve U_s X = I
  std::vector<double> Inv((size_t)L * L, 0.0);
  for (int i = 0; i < L; ++i) Inv[(size_t)i * L + i] = 1.0;
  if (!lu_solve(Us, L, Inv, L)) {
    g.error = "singular tau sampling matrix";
    g.L = 0;
    return g;
  }
  g.t_fwd.assign((size_t)nm * L, cplx(0.0, 0.0));
  for (int q = 0; q < nm; ++q)
    for (int i = 0; i < L; ++i) {
      cplx v(0.0, 0.0);
      for (int l = 0; l < L; ++l) v += Uh[(size_t)q * L + l] * Inv[(size_t)l * L + i];
      g.t_fwd[(size_t)q * L + i] = v;
    }
  // T_bwd = U_s pinv([Re U^; Im U^])
  std::vector<double> Bm((size_t)2 * nm * L);
  for (int q = 0; q < nm; ++q)
    for (int l = 0; l < L; ++l) {
      Bm[(size_t)q * L + l] = Uh[(size_t)q * L + l].real();
      Bm[(size_t)(nm + q) * L + l] = Uh[(size_t)q * L + l].imag();
    }
  std::vector<double> Pinv;
  if (!lsq_inverse(Bm, 2 * nm, L, Pinv)) {
    g.error = "rank-deficient Matsubara sampling matrix";
    g.L = 0;
    return g;
  }
  g.t_bwd.assign((size_t)L * nm, cplx(0.0, 0.0));
  for (int i = 0; i < L; ++i)
    for (int q = 0; q < nm; ++q) {
      double re = 0.0, im = 0.0;
      for (int l = 0; l < L; ++l) {
        re += Us[(size_t)i * L + l] * Pinv[(size_t)l * 2 * nm + q];
        im += Us[(size_t)i * L + l] * Pinv[(size_t)l * 2 * nm + nm + q];
      }
      g.t_bwd[(size_t)i * nm + q] = cplx(re, -im);
    }
  // t_beta[i] = sum_l U_l(beta) Inv[l][i]
  g.t_beta.assign(L, 0.0);
  for (int l = 0; l < L; ++l) {
    const double ub = std::sqrt(2.0 / beta) * evaluate(sv, sv.f[l], 1.0);
    for (int i = 0; i < L; ++i) g.t_beta[i] += ub * Inv[(size_t)l * L + i];
  }
  // weights: w_i = sum_l Inv[l][i] I_l
  std::vector<double> I(L, 0.0);
  for (int l = 0; l < L; ++l) {
    if (sv.f[l].par < 0) continue;
    double acc = 0.0;
    for (size_t i = 0; i < sv.x.size(); ++i) acc += sv.wx[i] * sv.f[l].u[i];
    I[l] = std::sqrt(beta / 2.0) * 2.0 * acc;
  }
  g.weights.assign(L, 0.0);
  for (int i = 0; i < L; ++i) {
    double acc = 0.0;
    for (int l = 0; l < L; ++l) acc += Inv[(size_t)l * L + i] * I[l];
    g.weights[i] = acc;
  }
  return g;
}

}  // namespace sox_ir
