// Host FP64 eigen-setup of the 1D absorbing-boundary pencil.
//
// Computes all eigenpairs of K v = lambda M v (eq. (EVP1a)) for the 1D
// stiffness and mass matrices of eqs. (matrixK), (matrixM) -- K with corner
// entries 1/h + g for a face condition du/dn + g u = 0 (absorbing:
// g = -i omega; Neumann: g = 0; Robin / impedance: any g) -- normalised by
// v^T M v = 1 (eq. (EVPcondA); plain transpose, the pencil is complex
// symmetric), and returns the eigenvalues and the two boundary rows of V.
//
// The paper obtains these with a dense QZ solve (Section 6 notes that `eig`
// dominates the initialisation).  Here the tridiagonal structure is used
// instead:
//   1. all n roots of p(lambda) = det(K - lambda M) by the Aberth-Ehrlich
//      simultaneous iteration (O(n^2) per sweep), with p'/p evaluated in O(n)
//      by the LDL^T pivot recurrence of the tridiagonal pencil, carried in the
//      ratio form r_i = u_i'/u_i so that nothing overflows;
//   2. each root refined by inverse iteration with the complex-symmetric
//      Rayleigh quotient lambda = x^T K x / x^T M x, using Gaussian
//      elimination with partial pivoting on the tridiagonal K - lambda M,
//      in x87 extended precision with a cancellation-free x^T K x;
//   3. each eigenvector scaled by (v^T M v)^{-1/2}.
// With g = 0 on both faces (Neumann) the spectrum is the closed-form
// cosine one, 6(1 - cos t)/(h^2 (2 + cos t)), t = k pi/(n - 1), used directly
// as the starting values of step 2.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

#include "../../include/helm.h"
#include "eig1d.h"

namespace helm {

using cd = std::complex<double>;

namespace {

struct Pencil {
  int n;
  std::vector<cd> ka;      // diagonal of K
  std::vector<double> ma;  // diagonal of M
  double kb;               // off-diagonal of K (-1/h)
  double mb;               // off-diagonal of M (h/6)
};

Pencil make_pencil(int n, double h, cd glo, cd ghi) {
  Pencil P;
  P.n = n;
  P.ka.assign(n, cd(2.0 / h, 0.0));
  P.ma.assign(n, 4.0 * h / 6.0);
  P.ka[0] = cd(1.0 / h, 0.0) + glo;
  P.ka[n - 1] = cd(1.0 / h, 0.0) + ghi;
  P.ma[0] = P.ma[n - 1] = 2.0 * h / 6.0;
  P.kb = -1.0 / h;
  P.mb = h / 6.0;
  return P;
}

// p'(lam)/p(lam) for p = det(K - lam M).  Pivots u_i of the LDL^T
// factorisation satisfy u_i = a_i - b^2/u_{i-1} with a_i = ka_i - lam ma_i,
// b = kb - lam mb; det = prod u_i, so p'/p = sum u_i'/u_i, and
// u_i' = a_i' - 2 b b'/u_{i-1} + (b^2/u_{i-1}) (u_{i-1}'/u_{i-1}).
cd log_derivative(const Pencil& P, cd lam) {
  const cd b = P.kb - lam * P.mb;
  const double bp = -P.mb;
  cd u = P.ka[0] - lam * P.ma[0];
  cd r = -P.ma[0] / u;
  cd s = r;
  for (int i = 1; i < P.n; ++i) {
    const cd t = b / u;
    const cd a = P.ka[i] - lam * P.ma[i];
    const cd un = a - b * t;
    const cd upn = -P.ma[i] - 2.0 * bp * t + t * b * r;
    r = upn / un;
    u = un;
    s += r;
  }
  return s;
}

// The refinement runs in x87 extended precision (64-bit significand): for the
// smooth low modes the FP64 Rayleigh quotient and inverse iteration lose
// about 1e-11 relative to cancellation, and the fast solver's FP64 residual is
// sensitive to that (it rounds eigenvalues to FP64 afterwards).
using xr = long double;
using xc = std::complex<long double>;

// Solve the tridiagonal system (dl, d, du) x = b by Gaussian elimination
// with partial pivoting (row interchanges produce a second super-diagonal).
// Arrays are overwritten.  A zero pivot is replaced by a tiny value: the
// callers are inverse iterations, where a (near-)singular matrix is the point.
void tri_solve_pp(std::vector<xc>& dl, std::vector<xc>& d, std::vector<xc>& du,
                  std::vector<xc>& b, std::vector<xc>& x, xr tiny) {
  const int n = (int)d.size();
  std::vector<xc> du2(n, xc(0.0L));
  for (int i = 0; i + 1 < n; ++i) {
    if (std::abs(d[i]) >= std::abs(dl[i])) {
      if (d[i] == xc(0.0L)) d[i] = tiny;
      const xc fct = dl[i] / d[i];
      d[i + 1] -= fct * du[i];
      b[i + 1] -= fct * b[i];
      du2[i] = 0.0L;
    } else {
      const xc fct = d[i] / dl[i];
      d[i] = dl[i];
      const xc tmp = d[i + 1];
      d[i + 1] = du[i] - fct * tmp;
      if (i + 2 < n) {
        du2[i] = du[i + 1];
        du[i + 1] = -fct * du2[i];
      }
      du[i] = tmp;
      const xc tb = b[i];
      b[i] = b[i + 1];
      b[i + 1] = tb - fct * b[i + 1];
    }
  }
  if (d[n - 1] == xc(0.0L)) d[n - 1] = tiny;
  x[n - 1] = b[n - 1] / d[n - 1];
  if (n > 1) x[n - 2] = (b[n - 2] - du[n - 2] * x[n - 1]) / d[n - 2];
  for (int i = n - 3; i >= 0; --i) x[i] = (b[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / d[i];
}

// The pencil in extended precision, built from the same double inputs.
struct XPencil {
  int n;
  xr h, w;
  xc glo, ghi;
  std::vector<xc> ka;
  std::vector<xr> ma;
  xr kb, mb;
};

XPencil make_xpencil(int n, double h, cd glo, cd ghi) {
  XPencil P;
  P.n = n;
  P.h = h;
  P.glo = xc(glo.real(), glo.imag());
  P.ghi = xc(ghi.real(), ghi.imag());
  P.ka.assign(n, xc(2.0L / P.h, 0.0L));
  P.ma.assign(n, 4.0L * P.h / 6.0L);
  P.ka[0] = xc(1.0L / P.h, 0.0L) + P.glo;
  P.ka[n - 1] = xc(1.0L / P.h, 0.0L) + P.ghi;
  P.ma[0] = P.ma[n - 1] = 2.0L * P.h / 6.0L;
  P.kb = -1.0L / P.h;
  P.mb = P.h / 6.0L;
  return P;
}

// x^T K x without cancellation: K = (1/h) sum over elements of (e_i - e_{i+1})
// (e_i - e_{i+1})^T plus the corner terms g at the two ends.
xc stiff_form(const XPencil& P, const std::vector<xc>& x) {
  xc s = 0.0L;
  for (int i = 0; i + 1 < P.n; ++i) {
    const xc d = x[i + 1] - x[i];
    s += d * d;
  }
  s /= P.h;
  s += P.glo * x[0] * x[0];
  s += P.ghi * x[P.n - 1] * x[P.n - 1];
  return s;
}

// x^T M x = (h/6) sum over elements of (2 x_i^2 + 2 x_i x_{i+1} + 2 x_{i+1}^2).
xc mass_form(const XPencil& P, const std::vector<xc>& x) {
  xc s = 0.0L;
  for (int i = 0; i + 1 < P.n; ++i) s += x[i] * x[i] + x[i] * x[i + 1] + x[i + 1] * x[i + 1];
  return s * (P.h / 3.0L);
}

void apply_mass(const XPencil& P, const std::vector<xc>& x, std::vector<xc>& y) {
  for (int i = 0; i < P.n; ++i) {
    xc v = P.ma[i] * x[i];
    if (i > 0) v += P.mb * x[i - 1];
    if (i + 1 < P.n) v += P.mb * x[i + 1];
    y[i] = v;
  }
}

// One eigenpair from an approximate eigenvalue: inverse iteration steps with
// the Rayleigh-quotient shift.  Returns the refined eigenvalue, the boundary
// entries of the M-normalised eigenvector and the normwise backward error.
struct Refined {
  cd lam, v0, v1;
  double resid;
  std::vector<cd> x;  // the whole eigenvector, when asked for
  cd lam_lo;          // extended-precision eigenvalue minus lam (rounded)
};

Refined refine(const XPencil& P, cd lam0, int steps, bool whole) {
  const int n = P.n;
  std::vector<xc> x(n), y(n), dl(n), d(n), du(n), b(n);
  // Deterministic start vector with components of both parities.
  for (int i = 0; i < n; ++i) x[i] = 1.7L + std::cos(0.913L * i + 0.3L);
  // bound of ||K||_inf: interior rows sum to 4/h, corner rows |k|/h + 1/h
  const xr knorm = 4.0L * std::abs(P.kb) + std::abs(P.ka[0]) + std::abs(P.ka[n - 1]);
  xc lam(lam0.real(), lam0.imag());
  for (int s = 0; s < steps; ++s) {
    for (int i = 0; i < n; ++i) {
      d[i] = P.ka[i] - lam * P.ma[i];
      if (i + 1 < n) dl[i] = du[i] = P.kb - lam * P.mb;
    }
    apply_mass(P, x, b);
    tri_solve_pp(dl, d, du, b, y, 1e-4000L + 1e-60L * knorm);
    xr nrm = 0.0L;
    for (int i = 0; i < n; ++i) nrm = std::max(nrm, std::abs(y[i]));
    for (int i = 0; i < n; ++i) x[i] = y[i] / nrm;
    lam = stiff_form(P, x) / mass_form(P, x);
  }
  const xc sc = std::sqrt(mass_form(P, x));
  for (int i = 0; i < n; ++i) x[i] /= sc;
  // normwise backward error ||(K - lam M) x|| / ((||K|| + |lam| ||M||) ||x||), max norms
  xr rnum = 0.0L, xmax = 0.0L;
  for (int i = 0; i < n; ++i) {
    xc kx = P.ka[i] * x[i], mx = P.ma[i] * x[i];
    if (i > 0) { kx += P.kb * x[i - 1]; mx += P.mb * x[i - 1]; }
    if (i + 1 < n) { kx += P.kb * x[i + 1]; mx += P.mb * x[i + 1]; }
    rnum = std::max(rnum, std::abs(kx - lam * mx));
    xmax = std::max(xmax, std::abs(x[i]));
  }
  const xr mnorm = 6.0L * P.mb;  // ||M||_inf = h
  const xr rden = (knorm + std::abs(lam) * mnorm) * xmax;
  const cd lhi((double)lam.real(), (double)lam.imag());
  Refined out{lhi, cd((double)x[0].real(), (double)x[0].imag()),
              cd((double)x[n - 1].real(), (double)x[n - 1].imag()),
              rden > 0 ? (double)(rnum / rden) : 0.0, {},
              cd((double)(lam.real() - (xr)lhi.real()), (double)(lam.imag() - (xr)lhi.imag()))};
  if (whole) {
    out.x.resize(n);
    for (int i = 0; i < n; ++i) out.x[i] = cd((double)x[i].real(), (double)x[i].imag());
  }
  return out;
}

}  // namespace

int eig1d(int n, double h, cd glo, cd ghi, std::vector<cd>& lam_out, std::vector<cd>& v0,
          std::vector<cd>& v1, std::vector<cd>* vfull, std::vector<cd>* lam_lo) {
  if (n < 3 || !(h > 0.0) || !std::isfinite(glo.real()) || !std::isfinite(glo.imag()) ||
      !std::isfinite(ghi.real()) || !std::isfinite(ghi.imag()))
    return HELM_EINVAL;
  const Pencil P = make_pencil(n, h, glo, ghi);
  // Closed-form Neumann spectrum: exact when no face absorbs, the starting
  // values of the root finder otherwise.
  std::vector<cd> lam(n);
  for (int k = 0; k < n; ++k) {
    const double t = M_PI * k / (n - 1);
    lam[k] = 6.0 * (1.0 - std::cos(t)) / (h * h * (2.0 + std::cos(t)));
  }
  const bool robin = glo != 0.0 || ghi != 0.0;
  if (robin) {
    // the corner terms move the Neumann eigenvalues by about a quarter of
    // their sum (first-order perturbation averaged over the modes)
    const cd shift = 0.25 * (glo + ghi);
    for (int k = 0; k < n; ++k) lam[k] += shift;
    std::vector<cd> next(n);
    std::vector<char> done(n, 0);
    std::vector<double> prev(n, INFINITY);  // |correction| of the previous sweep
    const int max_sweeps = 400;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
      int active = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : active)
      for (int j = 0; j < n; ++j) {
        next[j] = lam[j];
        if (done[j]) continue;
        const cd lp = log_derivative(P, lam[j]);
        if (!std::isfinite(lp.real()) || !std::isfinite(lp.imag())) {
          // landed exactly on a pivot breakdown: nudge and retry next sweep
          next[j] = lam[j] * cd(1.0 + 1e-13, 1e-13);
          ++active;
          continue;
        }
        cd sum = 0.0;
        for (int i = 0; i < n; ++i)
          if (i != j) sum += 1.0 / (lam[j] - lam[i]);
        const cd N = 1.0 / lp;
        const cd corr = N / (1.0 - N * sum);
        next[j] = lam[j] - corr;
        // FP64 rounding floor of the determinant recurrence is ~1e-13 relative;
        // the inverse iteration below supplies the last digits.  A root
        // also stops once its correction is below 1e-9 relative and no
        // longer halves from one sweep to the next: it then sits on that
        // floor, well inside the convergence region of the inverse iteration.
        const double ac = std::abs(corr), al = std::abs(lam[j]);
        if (ac <= 1e-12 * al + 1e-300 || (ac <= 1e-9 * al && ac >= 0.5 * prev[j])) done[j] = 1;
        else ++active;
        prev[j] = ac;
      }
      lam.swap(next);
      if (active == 0) break;
    }
    for (int j = 0; j < n; ++j)
      if (!std::isfinite(lam[j].real()) || !std::isfinite(lam[j].imag())) return HELM_ENOCONV;
  }
  // Refinement: 3 inverse-iteration steps with Rayleigh-quotient shifts.
  const XPencil XP = make_xpencil(n, h, glo, ghi);
  std::vector<Refined> R(n);
  double worst = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(max : worst)
  for (int j = 0; j < n; ++j) {
    R[j] = refine(XP, lam[j], 3, vfull != nullptr);
    worst = std::max(worst, R[j].resid);
  }
  if (!(worst < 1e-12)) return HELM_ENOCONV;
  std::sort(R.begin(), R.end(), [](const Refined& a, const Refined& b) {
    return a.lam.real() < b.lam.real() || (a.lam.real() == b.lam.real() && a.lam.imag() < b.lam.imag());
  });
  // The n refined eigenvalues must be distinct (no two starts collapsed onto
  // one eigenpair).
  double scale = 0.0;
  for (int j = 0; j < n; ++j) scale = std::max(scale, std::abs(R[j].lam));
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n && R[i].lam.real() - R[j].lam.real() < 1e-9 * scale; ++i)
      if (std::abs(R[i].lam - R[j].lam) < 1e-9 * scale) return HELM_ENOCONV;
  lam_out.resize(n);
  v0.resize(n);
  v1.resize(n);
  for (int j = 0; j < n; ++j) {
    lam_out[j] = R[j].lam;
    v0[j] = R[j].v0;
    v1[j] = R[j].v1;
  }
  if (lam_lo) {
    lam_lo->resize(n);
    for (int j = 0; j < n; ++j) (*lam_lo)[j] = R[j].lam_lo;
  }
  if (vfull) {
    vfull->assign((size_t)n * n, cd(0.0));
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) (*vfull)[(size_t)i * n + j] = R[j].x[i];
  }
  return HELM_OK;
}

}  // namespace helm

extern "C" int helm_eig1d(int64_t n, double h, double omega, int abc_lo, int abc_hi,
                          double* lam, double* vb) {
  if (!lam || !vb || n < 3 || n > (int64_t)1 << 24) return HELM_EINVAL;
  std::vector<helm::cd> L, V0, V1;
  int st;
  try {
    if (!std::isfinite(omega)) return HELM_EINVAL;
    st = helm::eig1d((int)n, h, helm::face_gamma(omega, abc_lo), helm::face_gamma(omega, abc_hi), L, V0, V1,
                     nullptr, nullptr);
  } catch (...) {
    return HELM_ENOMEM;
  }
  if (st != HELM_OK) return st;
  for (int64_t j = 0; j < n; ++j) {
    lam[2 * j] = L[j].real();
    lam[2 * j + 1] = L[j].imag();
    vb[2 * j] = V0[j].real();
    vb[2 * j + 1] = V0[j].imag();
    vb[2 * (n + j)] = V1[j].real();
    vb[2 * (n + j) + 1] = V1[j].imag();
  }
  return HELM_OK;
}
