// Device eigen-setup of the 1D absorbing-boundary pencil.
//
// The same eigenpairs as the host setup (eig1d.cpp): all eigenpairs of
// K v = lambda M v (eq. (EVP1a)) for the 1D stiffness and mass matrices of
// eqs. (matrixK), (matrixM) -- K's corner entries 1/h + g for the face
// conditions du/dn + g u = 0 -- normalised by v^T M v = 1 (eq. (EVPcondA); plain
// transpose, the pencil is complex symmetric).  Section 6 reports that the
// dense eigen-solve dominates the initialisation; here every root and every
// eigenvector is one GPU thread:
//   1. Aberth-Ehrlich sweeps on p(lambda) = det(K - lambda M), one launch per
//      sweep and one thread per root: p'/p from the ratio form of the LDL^T
//      pivot recurrence (O(n) per root, the interior coefficients are
//      constants), the pair sum over the other roots read through LDS tiles;
//   2. inverse-iteration steps per root with the complex-symmetric Rayleigh
//      quotient x^T K x / x^T M x (three, or more until it settles), the
//      tridiagonal K - lambda M factored by Gaussian elimination with
//      partial pivoting, all in
//      double-double arithmetic (about 106 significant bits: the exact
//      product of a fused multiply-add (Dekker) and Knuth's two-sum), with
//      x^T K x formed from element differences (no cancellation);
//   3. the M-normalisation, the boundary rows, a normwise backward error per
//      pair and, when asked, the whole eigenvectors.
// The host sorts the pairs, applies the same acceptance checks as the host
// setup (backward error, distinct roots) and the whole vectors are permuted
// into sorted order on the device.
#include <algorithm>
#include <cmath>

#include "helm_internal.h"

// The error-free transformations below need every product rounded on its
// own: a product contracted into the following addition (a fused
// multiply-add) leaves the error term computed from a different rounding,
// which loses the low half of every double-double value.
#pragma clang fp contract(off)

namespace helm {

namespace {

// ---- double-double arithmetic ---------------------------------------------
struct dd {
  double hi, lo;
};
__device__ inline dd two_sum(double a, double b) {
  const double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ inline dd fast_two_sum(double a, double b) {  // |a| >= |b|
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ inline dd dd_of(double a) { return {a, 0.0}; }
__device__ inline dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
__device__ inline dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  const dd t = two_sum(x.lo, y.lo);
  s = fast_two_sum(s.hi, s.lo + t.hi);
  return fast_two_sum(s.hi, s.lo + t.lo);
}
__device__ inline dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }
__device__ inline dd dd_mul(dd x, dd y) {
  const double p = x.hi * y.hi;
  double e = fma(x.hi, y.hi, -p);
  e = fma(x.hi, y.lo, e);
  e = fma(x.lo, y.hi, e);
  return fast_two_sum(p, e);
}
__device__ inline dd dd_mul_d(dd x, double y) {
  const double p = x.hi * y;
  double e = fma(x.hi, y, -p);
  e = fma(x.lo, y, e);
  return fast_two_sum(p, e);
}
// x / y: three quotient digits, each from the remainder of the previous ones
__device__ inline dd dd_div(dd x, dd y) {
  const double q1 = x.hi / y.hi;
  dd r = dd_sub(x, dd_mul_d(y, q1));
  const double q2 = r.hi / y.hi;
  r = dd_sub(r, dd_mul_d(y, q2));
  const double q3 = r.hi / y.hi;
  return dd_add(fast_two_sum(q1, q2), dd_of(q3));
}

struct cdd {
  dd re, im;
};
__device__ inline cdd cdd_of(double2 a) { return {dd_of(a.x), dd_of(a.y)}; }
__device__ inline cdd cdd_zero() { return {dd_of(0.0), dd_of(0.0)}; }
__device__ inline cdd cdd_add(cdd a, cdd b) { return {dd_add(a.re, b.re), dd_add(a.im, b.im)}; }
__device__ inline cdd cdd_sub(cdd a, cdd b) { return {dd_sub(a.re, b.re), dd_sub(a.im, b.im)}; }
__device__ inline cdd cdd_neg(cdd a) { return {dd_neg(a.re), dd_neg(a.im)}; }
__device__ inline cdd cdd_mul(cdd a, cdd b) {
  return {dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
}
__device__ inline cdd cdd_scale(cdd a, dd s) { return {dd_mul(a.re, s), dd_mul(a.im, s)}; }
__device__ inline cdd cdd_scale_d(cdd a, double s) { return {dd_mul_d(a.re, s), dd_mul_d(a.im, s)}; }
__device__ inline cdd cdd_div(cdd a, cdd b) {
  const dd den = dd_add(dd_mul(b.re, b.re), dd_mul(b.im, b.im));
  const dd nr = dd_add(dd_mul(a.re, b.re), dd_mul(a.im, b.im));
  const dd ni = dd_sub(dd_mul(a.im, b.re), dd_mul(a.re, b.im));
  return {dd_div(nr, den), dd_div(ni, den)};
}
__device__ inline double cdd_abs2_hi(cdd a) { return a.re.hi * a.re.hi + a.im.hi * a.im.hi; }
__device__ inline bool cdd_is_zero(cdd a) { return a.re.hi == 0.0 && a.im.hi == 0.0; }
__device__ inline double4 pack(cdd a) { return make_double4(a.re.hi, a.re.lo, a.im.hi, a.im.lo); }
__device__ inline cdd unpack(double4 v) { return {{v.x, v.y}, {v.z, v.w}}; }

// ---- the pencil ------------------------------------------------------------
// K = (1/h) tridiag(-1, 2, -1) with corners 1/h + g_lo, 1/h + g_hi,
// M = (h/6) tridiag(1, 4, 1) with corners 2h/6.
struct PencilArgs {
  int n;
  double h;
  double2 glo, ghi;
};

__device__ inline double2 cdiv2(double2 a, double2 b) {
  const double d = 1.0 / (b.x * b.x + b.y * b.y);
  return make_double2((a.x * b.x + a.y * b.y) * d, (a.y * b.x - a.x * b.y) * d);
}

// p'(lam)/p(lam) for p = det(K - lam M) in FP64: the pivots of the LDL^T
// factorisation obey u_i = a_i - b^2 / u_{i-1} (a_i = K_ii - lam M_ii,
// b = K_{i,i+1} - lam M_{i,i+1}), det = prod u_i, so p'/p = sum u_i'/u_i, carried
// as r_i = u_i'/u_i:  u_i' = a_i' - 2 b b' / u_{i-1} + (b^2 / u_{i-1}) r_{i-1}.
__device__ double2 log_derivative(const PencilArgs& P, double2 lam) {
  const double h = P.h;
  const double kb = -1.0 / h, mb = h / 6.0, mi = 4.0 * h / 6.0, me = 2.0 * h / 6.0, ki = 2.0 / h;
  const double2 b = make_double2(kb - lam.x * mb, -lam.y * mb);
  const double bp = -mb;
  double2 u = make_double2(1.0 / h + P.glo.x - lam.x * me, P.glo.y - lam.y * me);
  double2 r = cdiv2(make_double2(-me, 0.0), u);
  double2 s = r;
  for (int i = 1; i < P.n; ++i) {
    const bool end = i == P.n - 1;
    const double mii = end ? me : mi;
    const double2 a = end ? make_double2(1.0 / h + P.ghi.x - lam.x * me, P.ghi.y - lam.y * me)
                          : make_double2(ki - lam.x * mi, -lam.y * mi);
    const double2 t = cdiv2(b, u);
    const double2 un = csub(a, cmul(b, t));
    double2 upn = make_double2(-mii - 2.0 * bp * t.x, -2.0 * bp * t.y);
    upn = cadd(upn, cmul(cmul(t, b), r));
    r = cdiv2(upn, un);
    u = un;
    s = cadd(s, r);
  }
  return s;
}

struct AberthArgs {
  PencilArgs P;
  double2* buf[2];  // roots, ping-pong: sweep s reads buf[s & 1], writes buf[(s + 1) & 1]
  int* done;        // [n] root converged
  double* prev;     // [n] |correction| of the previous sweep
  int* cnt;         // [max sweeps] roots still moving after sweep s
};

constexpr int kAberthThreads = 256;

// One Aberth-Ehrlich sweep (Jacobi form: every root from the previous ones):
// lam_j <- lam_j - N / (1 - N sum_{i != j} 1 / (lam_j - lam_i)), N = p / p'.
// A root stops when its correction is below 1e-12 |lam_j| (the FP64 floor of
// the determinant recurrence is about 1e-13 relative; the inverse iteration
// supplies the last digits), or once the correction is below 1e-9 |lam_j|
// and no longer halves from one sweep to the next (it sits on that floor;
// without this rule a few roots at n = 2049 run all 400 sweeps).  Returns at
// once after a sweep that left no root moving.
__global__ __launch_bounds__(kAberthThreads) void aberth_kernel(AberthArgs a, int s) {
  if (s > 0 && a.cnt[s - 1] == 0) return;
  __shared__ double2 tile[kAberthThreads];
  const int n = a.P.n;
  const double2* lam = a.buf[s & 1];
  double2* next = a.buf[(s + 1) & 1];
  const int j = blockIdx.x * kAberthThreads + threadIdx.x;
  const bool in = j < n;
  const double2 lj = in ? lam[j] : make_double2(0, 0);
  const bool fixed = !in || a.done[j];
  double2 sum = make_double2(0, 0);
  for (int t0 = 0; t0 < n; t0 += kAberthThreads) {
    __syncthreads();
    if (t0 + (int)threadIdx.x < n) tile[threadIdx.x] = lam[t0 + threadIdx.x];
    __syncthreads();
    if (!fixed) {
      const int m = min(kAberthThreads, n - t0);
      for (int k = 0; k < m; ++k) {
        if (t0 + k == j) continue;
        sum = cadd(sum, cdiv2(make_double2(1, 0), csub(lj, tile[k])));
      }
    }
  }
  if (!in) return;
  if (fixed) {
    next[j] = lj;
    return;
  }
  const double2 lp = log_derivative(a.P, lj);
  if (!isfinite(lp.x) || !isfinite(lp.y)) {
    // landed exactly on a pivot breakdown: nudge and retry next sweep
    next[j] = cmul(lj, make_double2(1.0 + 1e-13, 1e-13));
    atomicAdd(&a.cnt[s], 1);
    return;
  }
  const double2 N = cdiv2(make_double2(1, 0), lp);
  const double2 corr = cdiv2(N, csub(make_double2(1, 0), cmul(N, sum)));
  next[j] = csub(lj, corr);
  const double ac = hypot(corr.x, corr.y), al = hypot(lj.x, lj.y);
  if (ac <= 1e-12 * al + 1e-300 || (ac <= 1e-9 * al && ac >= 0.5 * a.prev[j])) a.done[j] = 1;
  else atomicAdd(&a.cnt[s], 1);
  a.prev[j] = ac;
}

struct RefineArgs {
  PencilArgs P;
  int j0, cnt;            // roots [j0, j0 + cnt) of this launch
  int64_t ld;             // workspace row stride (>= cnt)
  const double2* lam0;    // [n] starting eigenvalues
  double4 *Y, *Ud, *Uu, *Uu2, *Bv;  // [n][ld] double-double complex
  double2 *lam, *lamlo, *v0, *v1, *scale;  // [n] outputs; scale: the M-normalising factor of y
  double* resid;          // [n] normwise backward error
  double2* T;             // nullable: [n][n] unsorted eigenvectors, T[i n + j] = v_j(i)
};

constexpr int kRefineThreads = 64;
// Inverse-iteration steps per root: at least three, more until the Rayleigh
// quotient settles to 1e-26 relative.  A fixed three steps leave about 1e-12
// relative error in the boundary rows of eigenvectors that the start vector
// barely contains (the top of the spectrum at n = 2049, where the gaps are
// small), against a 40-digit reference.
constexpr int kMaxSteps = 8;

// Inverse iteration with Rayleigh-quotient shifts for root j (one thread):
// y = (K - lam M)^{-1} M x, lam <- y^T K y / y^T M y, x <- y (rescaled by a
// power of two).  The elimination streams row by row: the pending row i
// (d, du, b) meets row i + 1 (off, d_{i+1}, off); the larger of the two
// entries in column i pivots (rows interchanged otherwise, which creates the
// second superdiagonal du2).  The rows of U and the eliminated right-hand side
// go to the workspace; the back substitution writes y over x.
__global__ __launch_bounds__(kRefineThreads) void refine_kernel(RefineArgs a) {
  const int jj = blockIdx.x * kRefineThreads + threadIdx.x;
  if (jj >= a.cnt) return;
  const int j = a.j0 + jj;
  const int n = a.P.n;
  const int64_t ld = a.ld;
  const dd h = dd_of(a.P.h);
  const dd one = dd_of(1.0);
  const dd kint = dd_div(dd_of(2.0), h), kb = dd_neg(dd_div(one, h));
  const dd mint = dd_div(dd_mul_d(h, 4.0), dd_of(6.0)), mend = dd_div(dd_mul_d(h, 2.0), dd_of(6.0));
  const dd mb = dd_div(h, dd_of(6.0));
  const cdd glo = cdd_of(a.P.glo), ghi = cdd_of(a.P.ghi);
  const cdd k0 = {dd_add(dd_div(one, h), glo.re), glo.im};
  const cdd kn = {dd_add(dd_div(one, h), ghi.re), ghi.im};
  const cdd zero = cdd_zero();
  // bound of ||K||_inf: interior rows sum to 4/h, corner rows |k|/h + 1/h
  const double knorm = 4.0 / a.P.h + hypot(k0.re.hi, k0.im.hi) + hypot(kn.re.hi, kn.im.hi);
  const cdd tiny = cdd_of(make_double2(1e-60 * knorm, 0.0));
  double4* Y = a.Y + jj;
  double4* Ud = a.Ud + jj;
  double4* Uu = a.Uu + jj;
  double4* Uu2 = a.Uu2 + jj;
  double4* Bv = a.Bv + jj;

  cdd lam = cdd_of(a.lam0[j]);
  double sc = 1.0;  // x = sc y (exact power of two)
  cdd yfirst = zero, ylast = zero, massF = zero;
  for (int step = 0; step < kMaxSteps; ++step) {
    // deterministic start vector with components of both parities
    auto X = [&](int i) -> cdd {
      if (step == 0) return cdd_of(make_double2(1.7 + cos(0.913 * i + 0.3), 0.0));
      return cdd_scale_d(unpack(Y[(int64_t)i * ld]), sc);
    };
    const cdd off = {dd_sub(kb, dd_mul(lam.re, mb)), dd_neg(dd_mul(lam.im, mb))};
    const cdd dint = {dd_sub(kint, dd_mul(lam.re, mint)), dd_neg(dd_mul(lam.im, mint))};
    const cdd dlo = {dd_sub(k0.re, dd_mul(lam.re, mend)), dd_sub(k0.im, dd_mul(lam.im, mend))};
    const cdd dhi = {dd_sub(kn.re, dd_mul(lam.re, mend)), dd_sub(kn.im, dd_mul(lam.im, mend))};
    // (M x)_i = m_ii x_i + mb (x_{i-1} + x_{i+1})
    auto Mx = [&](int i, cdd xm, cdd xc, cdd xp) -> cdd {
      const dd mii = (i == 0 || i == n - 1) ? mend : mint;
      return cdd_add(cdd_scale(xc, mii), cdd_scale(cdd_add(xm, xp), mb));
    };
    cdd x0 = X(0), x1 = X(1);
    cdd cdg = dlo, cdu = off, cb = Mx(0, zero, x0, x1);
    for (int i = 0; i + 1 < n; ++i) {
      const cdd x2 = (i + 2 < n) ? X(i + 2) : zero;
      const cdd nb = Mx(i + 1, x0, x1, x2);
      x0 = x1;
      x1 = x2;
      const cdd nd = (i + 1 == n - 1) ? dhi : dint;
      const cdd ndu = (i + 2 < n) ? off : zero;
      const int64_t r = (int64_t)i * ld;
      if (cdd_abs2_hi(cdg) >= cdd_abs2_hi(off)) {
        if (cdd_is_zero(cdg)) cdg = tiny;
        const cdd f = cdd_div(off, cdg);
        Ud[r] = pack(cdg);
        Uu[r] = pack(cdu);
        Uu2[r] = pack(zero);
        Bv[r] = pack(cb);
        cdg = cdd_sub(nd, cdd_mul(f, cdu));
        cdu = ndu;
        cb = cdd_sub(nb, cdd_mul(f, cb));
      } else {
        const cdd f = cdd_div(cdg, off);
        Ud[r] = pack(off);
        Uu[r] = pack(nd);
        Uu2[r] = pack(ndu);
        Bv[r] = pack(nb);
        cdg = cdd_sub(cdu, cdd_mul(f, nd));
        cdu = cdd_neg(cdd_mul(f, ndu));
        cb = cdd_sub(cb, cdd_mul(f, nb));
      }
    }
    if (cdd_is_zero(cdg)) cdg = tiny;
    // back substitution, with the quadratic forms of y on the way
    cdd y1 = cdd_div(cb, cdg), y2 = zero;
    Y[(int64_t)(n - 1) * ld] = pack(y1);
    ylast = y1;
    cdd stiff = zero, mass = zero;
    double nrm = fmax(fabs(y1.re.hi), fabs(y1.im.hi));
    for (int i = n - 2; i >= 0; --i) {
      const int64_t r = (int64_t)i * ld;
      const cdd b = unpack(Bv[r]);
      const cdd du = unpack(Uu[r]), du2 = unpack(Uu2[r]);
      const cdd dg = unpack(Ud[r]);
      const cdd y = cdd_div(cdd_sub(cdd_sub(b, cdd_mul(du, y1)), cdd_mul(du2, y2)), dg);
      Y[r] = pack(y);
      const cdd df = cdd_sub(y1, y);
      stiff = cdd_add(stiff, cdd_mul(df, df));
      mass = cdd_add(mass, cdd_add(cdd_mul(y, cdd_add(y, y1)), cdd_mul(y1, y1)));
      nrm = fmax(nrm, fmax(fabs(y.re.hi), fabs(y.im.hi)));
      y2 = y1;
      y1 = y;
    }
    yfirst = y1;
    // y^T K y = (1/h) sum (y_{i+1} - y_i)^2 + g_lo y_0^2 + g_hi y_{n-1}^2;
    // y^T M y = (h/3) sum (y_i^2 + y_i y_{i+1} + y_{i+1}^2)
    cdd kq = {dd_div(stiff.re, h), dd_div(stiff.im, h)};
    kq = cdd_add(kq, cdd_mul(glo, cdd_mul(yfirst, yfirst)));
    kq = cdd_add(kq, cdd_mul(ghi, cdd_mul(ylast, ylast)));
    massF = cdd_scale(mass, dd_div(h, dd_of(3.0)));
    const cdd prev = lam;
    lam = cdd_div(kq, massF);
    int e;
    frexp(nrm, &e);
    sc = ldexp(1.0, -e);
    // the quotient's change is about |lam| e^2 for a vector error e of the
    // previous step, after which the error falls to about e^3 |lam| / gap
    const cdd dl = cdd_sub(lam, prev);
    if (step >= 2 && cdd_abs2_hi(dl) <= 1e-52 * cdd_abs2_hi(lam)) break;
  }
  // M-normalisation of the last y: v = y / sqrt(y^T M y)
  const double2 m2 = make_double2(massF.re.hi, massF.im.hi);
  const double mr = hypot(m2.x, m2.y);
  // principal square root
  double sr = sqrt(0.5 * (mr + fabs(m2.x))), si;
  if (m2.x >= 0) {
    si = m2.y / (2.0 * sr);
  } else {
    si = sr;
    sr = fabs(m2.y) / (2.0 * si);
    if (m2.y < 0) si = -si;
  }
  const double2 c = cdiv2(make_double2(1, 0), make_double2(sr, si));
  a.lam[j] = make_double2(lam.re.hi, lam.im.hi);
  a.lamlo[j] = make_double2(lam.re.lo, lam.im.lo);
  a.v0[j] = cmul(make_double2(yfirst.re.hi, yfirst.im.hi), c);
  a.v1[j] = cmul(make_double2(ylast.re.hi, ylast.im.hi), c);
  a.scale[j] = c;
  // normwise backward error ||(K - lam M) v|| / ((||K|| + |lam| ||M||) ||v||),
  // max norms, from the rounded vector; and the whole vector when asked
  const double hh = a.P.h;
  const double2 lm = make_double2(lam.re.hi, lam.im.hi);
  const double2 kc0 = make_double2(1.0 / hh + a.P.glo.x, a.P.glo.y);
  const double2 kcn = make_double2(1.0 / hh + a.P.ghi.x, a.P.ghi.y);
  double rnum = 0.0, vmax = 0.0;
  double2 vm = make_double2(0, 0);
  double2 vc = cmul(make_double2(unpack(Y[0]).re.hi, unpack(Y[0]).im.hi), c);
  for (int i = 0; i < n; ++i) {
    const double2 vp = i + 1 < n ? cmul(make_double2(unpack(Y[(int64_t)(i + 1) * ld]).re.hi,
                                                     unpack(Y[(int64_t)(i + 1) * ld]).im.hi), c)
                                 : make_double2(0, 0);
    const bool end = i == 0 || i == n - 1;
    const double2 kd = i == 0 ? kc0 : (i == n - 1 ? kcn : make_double2(2.0 / hh, 0.0));
    const double md = end ? 2.0 * hh / 6.0 : 4.0 * hh / 6.0;
    const double2 nb = cadd(vm, vp);
    const double2 kx = cadd(cmul(kd, vc), cscale(nb, -1.0 / hh));
    const double2 mx = cadd(cscale(vc, md), cscale(nb, hh / 6.0));
    const double2 rr = csub(kx, cmul(lm, mx));
    rnum = fmax(rnum, hypot(rr.x, rr.y));
    vmax = fmax(vmax, hypot(vc.x, vc.y));
    if (a.T) a.T[(int64_t)i * n + j] = vc;
    vm = vc;
    vc = vp;
  }
  const double rden = (knorm + hypot(lm.x, lm.y) * hh) * vmax;
  a.resid[j] = rden > 0 ? rnum / rden : 0.0;
}

// Whole eigenvectors in sorted order: V[i][l] = T[i][perm[l]] and the
// transposes, in double and float (the dense transform's operands).
__global__ void eigvec_layout_kernel(int n, const double2* __restrict__ T, const int* __restrict__ perm,
                                     double2* Vd, double2* VTd, float2* Vf, float2* VTf) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int64_t i = e / n, l = e - i * n;
  const double2 v = T[i * n + perm[l]];
  if (Vd) Vd[i * n + l] = v;
  if (VTd) VTd[l * n + i] = v;
  if (Vf) Vf[i * n + l] = make_float2((float)v.x, (float)v.y);
  if (VTf) VTf[l * n + i] = make_float2((float)v.x, (float)v.y);
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t b) { return hipMalloc(&p, b); }
};

}  // namespace

int eig1d_device(int n, double h, cd glo, cd ghi, std::vector<cd>& lam_out, std::vector<cd>& v0_out,
                 std::vector<cd>& v1_out, std::vector<cd>& lamlo_out, const EigVecOut* vecs, hipStream_t s) {
  if (n < 3 || !(h > 0.0) || !std::isfinite(glo.real()) || !std::isfinite(glo.imag()) ||
      !std::isfinite(ghi.real()) || !std::isfinite(ghi.imag()))
    return HELM_EINVAL;
  const PencilArgs P{n, h, make_double2(glo.real(), glo.imag()), make_double2(ghi.real(), ghi.imag())};
  const int max_sweeps = 400, chunk_sweeps = 8;
  // small per-root arrays: two root buffers, done flags, sweep counters,
  // refined outputs
  const size_t nsz = (size_t)n;
  DevBuf small;
  const size_t small_bytes = nsz * sizeof(double2) * 7 + nsz * sizeof(double) + nsz * sizeof(int) * 2 +
                             (size_t)max_sweeps * sizeof(int) + 256;
  if (small.alloc(small_bytes) != hipSuccess) return HELM_ENOMEM;
  double2* b0 = (double2*)small.p;
  double2* b1 = b0 + nsz;
  double2* rl = b1 + nsz;
  double2* rlo = rl + nsz;
  double2* rv0 = rlo + nsz;
  double2* rv1 = rv0 + nsz;
  double2* rsc = rv1 + nsz;
  double* rres = (double*)(rsc + nsz);
  int* done = (int*)(rres + nsz);
  int* perm = done + nsz;
  int* cnt = perm + nsz;

  // starting values: the closed-form Neumann spectrum 6(1 - cos t)/(h^2 (2 + cos t)),
  // t = k pi/(n - 1), exact when g = 0 on both faces, otherwise moved by a
  // quarter of the corner terms' sum (first-order perturbation averaged over
  // the modes)
  std::vector<double2> start(nsz);
  const bool absorbing = glo != 0.0 || ghi != 0.0;
  const cd shift = 0.25 * (glo + ghi);
  for (int k = 0; k < n; ++k) {
    const double t = M_PI * k / (n - 1);
    start[k] = make_double2(6.0 * (1.0 - std::cos(t)) / (h * h * (2.0 + std::cos(t))) + shift.real(), shift.imag());
  }
  if (hipMemcpyAsync(b0, start.data(), nsz * sizeof(double2), hipMemcpyHostToDevice, s) != hipSuccess)
    return HELM_EDEVICE;
  const double2* lam0 = b0;
  if (absorbing) {
    if (hipMemsetAsync(done, 0, nsz * sizeof(int), s) != hipSuccess) return HELM_EDEVICE;
    if (hipMemsetAsync(cnt, 0, (size_t)max_sweeps * sizeof(int), s) != hipSuccess) return HELM_EDEVICE;
    // the backward-error array is free until the refinement: it holds the
    // previous corrections, +inf at the start
    std::vector<double> inf(nsz, INFINITY);
    if (hipMemcpyAsync(rres, inf.data(), nsz * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
      return HELM_EDEVICE;
    AberthArgs A{P, {b0, b1}, done, rres, cnt};
    const unsigned blocks = (unsigned)((n + kAberthThreads - 1) / kAberthThreads);
    int last = -1;
    std::vector<int> hc(chunk_sweeps);
    for (int s0 = 0; s0 < max_sweeps && last < 0; s0 += chunk_sweeps) {
      for (int k = 0; k < chunk_sweeps; ++k)
        hipLaunchKernelGGL(aberth_kernel, dim3(blocks), dim3(kAberthThreads), 0, s, A, s0 + k);
      if (hipGetLastError() != hipSuccess) return HELM_EDEVICE;
      if (hipMemcpyAsync(hc.data(), cnt + s0, chunk_sweeps * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return HELM_EDEVICE;
      for (int k = 0; k < chunk_sweeps; ++k)
        if (hc[k] == 0) {
          last = s0 + k;
          break;
        }
    }
    // the roots after sweep `last` (or after the last sweep run)
    lam0 = ((last < 0 ? max_sweeps - 1 : last) + 1) & 1 ? b1 : b0;
  }

  // refinement, in launches of as many roots as a 4 GiB workspace holds
  const size_t per_root_row = 5 * sizeof(double4);
  const size_t cap = (size_t)4 << 30;
  int64_t roots = (int64_t)std::min<size_t>(nsz, std::max<size_t>(kRefineThreads, cap / (per_root_row * nsz)));
  DevBuf ws, tbuf;
  if (ws.alloc(per_root_row * nsz * (size_t)roots) != hipSuccess) return HELM_ENOMEM;
  if (vecs && tbuf.alloc(nsz * nsz * sizeof(double2)) != hipSuccess) return HELM_ENOMEM;
  double4* wb = (double4*)ws.p;
  const size_t plane = nsz * (size_t)roots;
  for (int64_t j0 = 0; j0 < n; j0 += roots) {
    RefineArgs R;
    R.P = P;
    R.j0 = (int)j0;
    R.cnt = (int)std::min<int64_t>(roots, n - j0);
    R.ld = roots;
    R.lam0 = lam0;
    R.Y = wb;
    R.Ud = wb + plane;
    R.Uu = wb + 2 * plane;
    R.Uu2 = wb + 3 * plane;
    R.Bv = wb + 4 * plane;
    R.lam = rl;
    R.lamlo = rlo;
    R.v0 = rv0;
    R.v1 = rv1;
    R.scale = rsc;
    R.resid = rres;
    R.T = vecs ? (double2*)tbuf.p : nullptr;
    hipLaunchKernelGGL(refine_kernel, dim3((unsigned)((R.cnt + kRefineThreads - 1) / kRefineThreads)),
                       dim3(kRefineThreads), 0, s, R);
    if (hipGetLastError() != hipSuccess) return HELM_EDEVICE;
  }
  std::vector<double2> hl(nsz), hlo(nsz), h0(nsz), h1(nsz);
  std::vector<double> hr(nsz);
  if (hipMemcpyAsync(hl.data(), rl, nsz * sizeof(double2), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(hlo.data(), rlo, nsz * sizeof(double2), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(h0.data(), rv0, nsz * sizeof(double2), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(h1.data(), rv1, nsz * sizeof(double2), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(hr.data(), rres, nsz * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return HELM_EDEVICE;
  double worst = 0.0;
  for (size_t j = 0; j < nsz; ++j) {
    if (!std::isfinite(hl[j].x) || !std::isfinite(hl[j].y) || !std::isfinite(hr[j])) return HELM_ENOCONV;
    worst = std::max(worst, hr[j]);
  }
  if (!(worst < 1e-12)) return HELM_ENOCONV;
  std::vector<int> order(nsz);
  for (int j = 0; j < n; ++j) order[j] = j;
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    return hl[x].x < hl[y].x || (hl[x].x == hl[y].x && hl[x].y < hl[y].y);
  });
  // the n refined eigenvalues must be distinct (no two starts collapsed onto
  // one eigenpair)
  double scale = 0.0;
  for (size_t j = 0; j < nsz; ++j) scale = std::max(scale, std::hypot(hl[j].x, hl[j].y));
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n && hl[order[b]].x - hl[order[a]].x < 1e-9 * scale; ++b)
      if (std::hypot(hl[order[b]].x - hl[order[a]].x, hl[order[b]].y - hl[order[a]].y) < 1e-9 * scale)
        return HELM_ENOCONV;
  lam_out.resize(nsz);
  lamlo_out.resize(nsz);
  v0_out.resize(nsz);
  v1_out.resize(nsz);
  for (int l = 0; l < n; ++l) {
    const int j = order[l];
    lam_out[l] = cd(hl[j].x, hl[j].y);
    lamlo_out[l] = cd(hlo[j].x, hlo[j].y);
    v0_out[l] = cd(h0[j].x, h0[j].y);
    v1_out[l] = cd(h1[j].x, h1[j].y);
  }
  if (vecs) {
    if (hipMemcpyAsync(perm, order.data(), nsz * sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess)
      return HELM_EDEVICE;
    const int64_t tot = (int64_t)n * n;
    hipLaunchKernelGGL(eigvec_layout_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n,
                       (const double2*)tbuf.p, perm, vecs->Vd, vecs->VTd, vecs->Vf, vecs->VTf);
    if (hipGetLastError() != hipSuccess) return HELM_EDEVICE;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return HELM_EDEVICE;
  return HELM_OK;
}

}  // namespace helm

extern "C" int helm_eig1d_device(int64_t n, double h, double omega, int abc_lo, int abc_hi, double* lam,
                                 double* vb) {
  if (!lam || !vb || n < 3 || n > (int64_t)1 << 20 || !(h > 0.0) || !std::isfinite(omega)) return HELM_EINVAL;
  int dev;
  if (hipGetDevice(&dev) != hipSuccess) return HELM_EDEVICE;
  std::vector<helm::cd> L, V0, V1, LO;
  int st;
  try {
    st = helm::eig1d_device((int)n, h, helm::face_gamma(omega, abc_lo), helm::face_gamma(omega, abc_hi), L, V0,
                            V1, LO, nullptr, nullptr);
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
