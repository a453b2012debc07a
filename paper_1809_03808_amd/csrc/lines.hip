// Batched complex tridiagonal solves along the last axis.
//
// Every mode of the periodised axes leaves one tridiagonal system along the
// last axis: for the 2D blocks of H_B and H_A (eqs. (HB2D), (HA2D), Section
// 4.1.2) T = (lambda - w^2) M_2 + K_2, and in 3D, after the inner transform in
// x_2, T = (lambda_1 + lambda_2 - w^2) M_3 + K_3 (eqs. (HA3D), (HB3D), (A2D2),
// (B2D2)).  The matrices depend on the mode only through sigma, so nothing is
// stored: coefficients are regenerated per row.
//
// Elimination order.  The elimination is exactly the sequential Thomas
// algorithm (LU without pivoting, pivots p_x = d_x - e_x^2 / p_{x-1}).  With an
// absorbing face at x = 0 the first pivot has a negative imaginary part and,
// for real sigma, the map p -> d - e^2/p keeps it there, so no pivot vanishes.
// A partitioned (SPIKE-type) elimination would instead factor Dirichlet
// sub-blocks of the line, which are real and indefinite and can be singular
// for some sigma; it is not used.
//
// Parallelism.  A line of nL rows is owned by P lanes (P a power of two, one
// wave or a few), lane q holding the rows [q c, q c + c).  The recurrences of
// Thomas are associative and are evaluated by exclusive scans across the P
// lanes:
//   pivots   (num, den) -> (d num - e^2 den, num)       2x2 Moebius matrices
//   forward  z_x = d_x - e_x / p_{x-1} z_{x-1}          affine maps z -> F z + G
//   backward y_x = (z_x - e_{x+1} y_{x+1}) / p_x       affine maps, reversed
// Each lane composes its c rows, the scan supplies the state entering the
// chunk, and the lane then re-runs its rows sequentially.  The pivot state
// entering each chunk depends on sigma only, so it is computed once per plan
// and, from it, the reciprocal pivot of every row: the LU factors of each line
// matrix are computed when the plan is built (factor_kernel), as the paper
// does at initialisation, and the solves run the two affine scans, with wave
// shuffles inside a wave and one LDS exchange between the waves of a line.
// Arithmetic is FP64 whatever the storage precision.
//
// Right-hand sides may be generated from boundary planes (the rank-2 terms of
// Steps 2 and 3, eqs. (step2-1), (step3term)), and solutions may be reduced
// with per-mode weights into boundary partial sums (eqs. (2dBs1), (step2-3)),
// so the intermediate solutions z_1, z_2 never reach memory.
#include "helm_internal.h"

namespace helm {

namespace {

constexpr int kCMax = 8;

struct Mob {  // 2x2 complex matrix [[a, b], [c, d]]
  double2 a, b, c, d;
};
struct Aff {  // z -> f z + g
  double2 f, g;
};

__device__ inline Mob mob_mul(const Mob& L, const Mob& R) {  // L * R
  Mob o;
  o.a = cfma(L.a, R.a, cmul(L.b, R.c));
  o.b = cfma(L.a, R.b, cmul(L.b, R.d));
  o.c = cfma(L.c, R.a, cmul(L.d, R.c));
  o.d = cfma(L.c, R.b, cmul(L.d, R.d));
  return o;
}

// Exact power-of-two rescaling: a Moebius matrix acts projectively.
__device__ inline void mob_norm(Mob& m) {
  double mx = fmax(fmax(fmax(fabs(m.a.x), fabs(m.a.y)), fmax(fabs(m.b.x), fabs(m.b.y))),
                   fmax(fmax(fabs(m.c.x), fabs(m.c.y)), fmax(fabs(m.d.x), fabs(m.d.y))));
  if (mx > 0.0 && mx < INFINITY) {
    int e;
    frexp(mx, &e);
    const double s = ldexp(1.0, -e);
    m.a = cscale(m.a, s);
    m.b = cscale(m.b, s);
    m.c = cscale(m.c, s);
    m.d = cscale(m.d, s);
  }
}

__device__ inline Aff aff_then(const Aff& later, const Aff& earlier) {  // later o earlier
  Aff o;
  o.f = cmul(later.f, earlier.f);
  o.g = cfma(later.f, earlier.g, later.g);
  return o;
}

__device__ inline Aff aff_ident() {
  Aff a;
  a.f = make_double2(1, 0);
  a.g = make_double2(0, 0);
  return a;
}

__device__ inline double2 shfl_up2(double2 v, int d, int w) {
  return make_double2(__shfl_up(v.x, d, w), __shfl_up(v.y, d, w));
}
__device__ inline double2 shfl_down2(double2 v, int d, int w) {
  return make_double2(__shfl_down(v.x, d, w), __shfl_down(v.y, d, w));
}
__device__ inline Aff shfl_up_aff(const Aff& a, int d, int w) {
  Aff o;
  o.f = shfl_up2(a.f, d, w);
  o.g = shfl_up2(a.g, d, w);
  return o;
}
__device__ inline Aff shfl_down_aff(const Aff& a, int d, int w) {
  Aff o;
  o.f = shfl_down2(a.f, d, w);
  o.g = shfl_down2(a.g, d, w);
  return o;
}

// Exclusive scans of affine maps over the P lanes of a line (lanes
// [slot*P, slot*P + P) of the block).  Forward: lane q receives
// A_{q-1} o ... o A_0; backward: lane q receives A_{q+1} o ... o A_{P-1}.
// For P > 64 the waves of a line exchange their totals through LDS (`wbuf`,
// NT/64 entries); every thread of the block must call these.
template <int P>
__device__ inline Aff scan_fwd(Aff v, int q, Aff* wbuf) {
  constexpr int W = P < 64 ? P : 64;
  const int lq = q & (W - 1);
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    const Aff o = shfl_up_aff(v, d, W);
    if (lq >= d) v = aff_then(v, o);
  }
  Aff ex = shfl_up_aff(v, 1, W);
  if (lq == 0) ex = aff_ident();
  if constexpr (P > 64) {
    const int wv = threadIdx.x >> 6;          // wave in block
    const int w0 = wv - (q >> 6);             // first wave of this line
    if (lq == 63) wbuf[wv] = v;               // inclusive wave total
    __syncthreads();
    Aff pre = aff_ident();
    for (int w = w0; w < wv; ++w) pre = aff_then(wbuf[w], pre);
    ex = aff_then(ex, pre);
    __syncthreads();
  }
  return ex;
}

template <int P>
__device__ inline Aff scan_bwd(Aff v, int q, Aff* wbuf) {
  constexpr int W = P < 64 ? P : 64;
  const int lq = q & (W - 1);
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    const Aff o = shfl_down_aff(v, d, W);
    if (lq + d < W) v = aff_then(v, o);
  }
  Aff ex = shfl_down_aff(v, 1, W);
  if (lq == W - 1) ex = aff_ident();
  if constexpr (P > 64) {
    const int wv = threadIdx.x >> 6;
    const int wl = wv - (q >> 6) + P / 64 - 1;  // last wave of this line
    if (lq == 0) wbuf[wv] = v;                  // inclusive suffix total of the wave
    __syncthreads();
    Aff suf = aff_ident();
    for (int w = wl; w > wv; --w) suf = aff_then(wbuf[w], suf);
    ex = aff_then(ex, suf);
    __syncthreads();
  }
  return ex;
}

template <typename T> __device__ inline double2 ld(const T* p, int64_t i) { return to_d2(p[i]); }

struct LineDev {
  int nb, nO, nI, nL, c, red, tile, ntiles, iters;
  const double2* sO;
  const double2* sI;
  double2 sC;
  double hL, m_end, m_int, m_off, k_off;
  double2 kLo, kHi;
  const void* in;
  const double2 *alpha0, *alpha1, *PO, *beta0, *beta1, *PI, *rho0, *rho1;
  const double2* piv;   // [nO*nI][nL]: 1/pivot of every row (factor table)
  void* out;
  double2* part;
};

struct RowCoef {
  double2 dint, dlo, dhi, off, off2;
};

__device__ inline RowCoef row_coef(const LineDev& a, int64_t l, int64_t m) {
  double2 sig = a.sC;
  if (a.sO) sig = cadd(sig, a.sO[l]);
  if (a.sI) sig = cadd(sig, a.sI[m]);
  RowCoef r;
  r.off = make_double2(sig.x * a.m_off + a.k_off, sig.y * a.m_off);  // sigma h/6 - 1/h
  r.off2 = cmul(r.off, r.off);
  r.dint = make_double2(sig.x * a.m_int + 2.0 / a.hL, sig.y * a.m_int);
  r.dlo = make_double2(sig.x * a.m_end + a.kLo.x / a.hL, sig.y * a.m_end + a.kLo.y / a.hL);
  r.dhi = make_double2(sig.x * a.m_end + a.kHi.x / a.hL, sig.y * a.m_end + a.kHi.y / a.hL);
  return r;
}

__device__ inline double2 diag_of(const RowCoef& r, int x, int nL) {
  if (x >= nL) return make_double2(1, 0);
  if (x == 0) return r.dlo;
  if (x == nL - 1) return r.dhi;
  return r.dint;
}
// e(x) = coupling between rows x-1 and x
__device__ inline bool has_e(int x, int nL) { return x > 0 && x < nL; }

template <typename TIN, typename TOUT, int NT, int P, bool RED>
__global__ __launch_bounds__(NT) void lines_kernel(LineDev a) {
  __shared__ Aff wbuf[NT / 64 + 1];
  // Reduction accumulators, lane-major: accs[(k c + j) NT + tid] holds the
  // weighted sum (weight k) of row q c + j of this thread's lines.
  extern __shared__ double2 accs[];

  constexpr int LPB = NT / P;
  const int c = a.c, nL = a.nL;
  const int tid = threadIdx.x;
  const int slot = tid / P, q = tid - slot * P;
  const int x0 = q * c;

  const int64_t blk = blockIdx.x;
  int64_t g = 0, t = 0;
  if (a.red) {
    g = blk / a.ntiles;
    t = blk - g * a.ntiles;
  } else {
    t = blk;
  }

  if constexpr (RED) {
    for (int j = 0; j < 2 * c; ++j) accs[j * NT + tid] = make_double2(0, 0);
  }

  // Line handled by this slot at iteration `it`.
  auto decode = [&](int it, int64_t& b, int64_t& l, int64_t& m) -> bool {
    const int64_t li = t * a.tile + (int64_t)it * LPB + slot;
    bool valid;
    if (a.red == 1) {        // g = b*nO + l, li = m
      valid = li < a.nI;
      b = g / a.nO;
      l = g - b * a.nO;
      m = li;
    } else if (a.red == 2) { // g = b*nI + m, li = l
      valid = li < a.nO;
      b = g / a.nI;
      m = g - b * a.nI;
      l = li;
    } else {                 // li = (b*nO + l)*nI + m
      valid = li < (int64_t)a.nb * a.nO * a.nI;
      m = li % a.nI;
      const int64_t bl = li / a.nI;
      l = bl % a.nO;
      b = bl / a.nO;
    }
    if (!valid) { b = 0; l = 0; m = 0; }
    return valid;
  };
  for (int it = 0; it < a.iters; ++it) {
    int64_t b, l, m;
    const bool valid = decode(it, b, l, m);
    const RowCoef rc = row_coef(a, l, m);
    const int64_t loff = ((b * a.nO + l) * a.nI + m) * (int64_t)nL;

    // ---- right-hand side of the chunk ------------------------------------
    double2 z[kCMax], ip[kCMax];
#pragma unroll
    for (int j = 0; j < kCMax; ++j) {
      const int x = x0 + j;
      double2 d = make_double2(0, 0);
      if (j < c && x < nL && valid) {
        if (a.in) d = ld(reinterpret_cast<const TIN*>(a.in), loff + x);
        if (a.PO) {
          const int64_t pb = (b * 2) * (int64_t)a.nI * nL + m * (int64_t)nL + x;
          d = cfma(a.alpha0[l], a.PO[pb], d);
          d = cfma(a.alpha1[l], a.PO[pb + (int64_t)a.nI * nL], d);
        }
        if (a.PI) {
          const int64_t pb = ((b * a.nO + l) * 2) * (int64_t)nL + x;
          d = cfma(a.beta0[m], a.PI[pb], d);
          d = cfma(a.beta1[m], a.PI[pb + nL], d);
        }
      }
      z[j] = d;
    }

    // ---- 1. reciprocal pivots from the plan's factor table -----------------
    const double2* pt = a.piv + (l * a.nI + m) * (int64_t)nL;
    const double2 ip_in = (x0 > 0 && x0 - 1 < nL) ? pt[x0 - 1] : make_double2(0, 0);
#pragma unroll
    for (int j = 0; j < kCMax; ++j) {
      const int x = x0 + j;
      ip[j] = (j < c && x < nL) ? pt[x] : make_double2(1, 0);
    }

    // ---- 2. forward substitution: affine scan -----------------------------
    // z_x = f_x z_{x-1} + d_x with f_x = -e(x) / p_{x-1}.
    const double2 moff = make_double2(-rc.off.x, -rc.off.y);
    Aff A = aff_ident();
    {
      double2 ipprev = ip_in;
#pragma unroll
      for (int j = 0; j < kCMax; ++j) {
        if (j < c) {
          const int x = x0 + j;
          const double2 f = has_e(x, nL) ? cmul(moff, ipprev) : make_double2(0, 0);
          A.f = cmul(f, A.f);
          A.g = cfma(f, A.g, z[j]);
          ipprev = ip[j];
        }
      }
    }
    const Aff Ein = scan_fwd<P>(A, q, wbuf);
    {
      double2 zprev = Ein.g;
      double2 ipprev = ip_in;
#pragma unroll
      for (int j = 0; j < kCMax; ++j) {
        if (j < c) {
          const int x = x0 + j;
          const double2 f = has_e(x, nL) ? cmul(moff, ipprev) : make_double2(0, 0);
          zprev = cfma(f, zprev, z[j]);
          z[j] = zprev;
          ipprev = ip[j];
        }
      }
    }

    // ---- 3. back substitution: reversed affine scan -----------------------
    // y_x = g_x y_{x+1} + h_x with g_x = -e(x+1)/p_x, h_x = z_x / p_x.
    Aff B = aff_ident();
#pragma unroll
    for (int j = kCMax - 1; j >= 0; --j) {
      if (j < c) {
        const int x = x0 + j;
        const double2 gx = has_e(x + 1, nL) ? cmul(moff, ip[j]) : make_double2(0, 0);
        z[j] = cmul(z[j], ip[j]);  // h_x
        B.f = cmul(gx, B.f);
        B.g = cfma(gx, B.g, z[j]);
      }
    }
    const Aff Bin = scan_bwd<P>(B, q, wbuf);
    {
      double2 ynext = Bin.g;
#pragma unroll
      for (int j = kCMax - 1; j >= 0; --j) {
        if (j < c) {
          const int x = x0 + j;
          const double2 gx = has_e(x + 1, nL) ? cmul(moff, ip[j]) : make_double2(0, 0);
          ynext = cfma(gx, ynext, z[j]);
          z[j] = ynext;
        }
      }
    }

    // ---- 4. epilogue -------------------------------------------------------
    if (valid) {
      if (a.out) {
        TOUT* o = reinterpret_cast<TOUT*>(a.out);
#pragma unroll
        for (int j = 0; j < kCMax; ++j) {
          const int x = x0 + j;
          if (j < c && x < nL) o[loff + x] = from_d2<TOUT>(z[j]);
        }
      }
      if constexpr (RED) {
        const int64_t wi = (a.red == 1) ? m : l;
        const double2 w0 = a.rho0[wi], w1 = a.rho1[wi];
#pragma unroll
        for (int j = 0; j < kCMax; ++j) {
          if (j < c) {
            accs[j * NT + tid] = cfma(w0, z[j], accs[j * NT + tid]);
            accs[(c + j) * NT + tid] = cfma(w1, z[j], accs[(c + j) * NT + tid]);
          }
        }
      }
    }
  }

  // ---- cross-slot reduction (fixed slot order) and partial write -----------
  if constexpr (RED) {
    __syncthreads();
    double2* outp = a.part + (g * a.ntiles + t) * 2 * (int64_t)nL;
    for (int e = tid; e < 2 * nL; e += NT) {
      const int k = e >= nL, x = e - k * nL;
      const int qq = x / c, j = x - qq * c;
      double2 s = make_double2(0, 0);
      for (int sl = 0; sl < LPB; ++sl) s = cadd(s, accs[(k * c + j) * NT + sl * P + qq]);
      outp[e] = s;
    }
  }
}

// Factor table: for every line matrix (l, m) the reciprocal pivots 1/p_x of
// its Thomas elimination.  Lane q composes the Moebius maps of its rows, a
// scan over the lanes gives the pivot state entering each chunk, and the lane
// re-runs its rows.  Runs once per plan; one block of P lanes per line.
__global__ void factor_kernel(LineDev a, int P, double2* piv) {
  extern __shared__ double smem_d[];
  Mob* buf = reinterpret_cast<Mob*>(smem_d);
  const int q = threadIdx.x;
  const int64_t line = blockIdx.x;  // l * nI + m
  const int64_t l = line / a.nI, m = line % a.nI;
  const RowCoef rc = row_coef(a, l, m);
  const int x0 = q * a.c;
  Mob G;
  G.a = make_double2(1, 0); G.b = make_double2(0, 0);
  G.c = make_double2(0, 0); G.d = make_double2(1, 0);
  for (int j = 0; j < a.c; ++j) {
    const int x = x0 + j;
    const double2 dg = diag_of(rc, x, a.nL);
    const double2 e2 = has_e(x, a.nL) ? rc.off2 : make_double2(0, 0);
    Mob n;
    n.a = csub(cmul(dg, G.a), cmul(e2, G.c));
    n.b = csub(cmul(dg, G.b), cmul(e2, G.d));
    n.c = G.a;
    n.d = G.b;
    G = n;
  }
  mob_norm(G);
  // Hillis-Steele inclusive scan (later * earlier), then shift.
  buf[q] = G;
  __syncthreads();
  for (int d = 1; d < P; d <<= 1) {
    Mob mine = buf[q];
    Mob other = q >= d ? buf[q - d] : mine;
    __syncthreads();
    if (q >= d) {
      mine = mob_mul(mine, other);
      mob_norm(mine);
      buf[q] = mine;
    }
    __syncthreads();
  }
  double2 ip = make_double2(0, 0);
  if (q > 0) {
    const Mob E = buf[q - 1];
    // state entering the chunk: E (1, 0)^T = (E.a, E.c), 1/p = E.c / E.a
    ip = cmul(E.c, crcp(E.a));
  }
  for (int j = 0; j < a.c; ++j) {
    const int x = x0 + j;
    if (x >= a.nL) break;
    double2 p = diag_of(rc, x, a.nL);
    if (has_e(x, a.nL)) p = csub(p, cmul(rc.off2, ip));
    ip = crcp(p);
    piv[line * a.nL + x] = ip;
  }
}

template <typename TIN, typename TOUT, int NT, int P>
hipError_t launch_P(const LineDev& d, int64_t blocks, size_t, hipStream_t s) {
  if (d.red) {
    // 2 c NT complex accumulators (up to 128 KB at NT = 512: above the
    // default dynamic LDS limit, so raise it for this kernel once).
    const size_t lds = (size_t)2 * d.c * NT * sizeof(double2);
    static bool attr = false;
    if (!attr) {
      const hipError_t e = hipFuncSetAttribute(
          reinterpret_cast<const void*>(&lines_kernel<TIN, TOUT, NT, P, true>),
          hipFuncAttributeMaxDynamicSharedMemorySize, 2 * kCMax * NT * (int)sizeof(double2));
      if (e != hipSuccess) return e;
      attr = true;
    }
    hipLaunchKernelGGL((lines_kernel<TIN, TOUT, NT, P, true>), dim3((unsigned)blocks), dim3(NT), lds, s, d);
  } else {
    hipLaunchKernelGGL((lines_kernel<TIN, TOUT, NT, P, false>), dim3((unsigned)blocks), dim3(NT), 0, s, d);
  }
  return hipGetLastError();
}

template <typename TIN, typename TOUT>
hipError_t launch_typed(const LineDev& d, int P, int64_t blocks, size_t lds, hipStream_t s) {
  switch (P) {
    case 1: return launch_P<TIN, TOUT, 256, 1>(d, blocks, lds, s);
    case 2: return launch_P<TIN, TOUT, 256, 2>(d, blocks, lds, s);
    case 4: return launch_P<TIN, TOUT, 256, 4>(d, blocks, lds, s);
    case 8: return launch_P<TIN, TOUT, 256, 8>(d, blocks, lds, s);
    case 16: return launch_P<TIN, TOUT, 256, 16>(d, blocks, lds, s);
    case 32: return launch_P<TIN, TOUT, 256, 32>(d, blocks, lds, s);
    case 64: return launch_P<TIN, TOUT, 256, 64>(d, blocks, lds, s);
    case 128: return launch_P<TIN, TOUT, 256, 128>(d, blocks, lds, s);
    case 256: return launch_P<TIN, TOUT, 256, 256>(d, blocks, lds, s);
    case 512: return launch_P<TIN, TOUT, 512, 512>(d, blocks, lds, s);
    default: return hipErrorInvalidValue;
  }
}

LineDev make_dev(const LineArgs& a, int P, int c) {
  LineDev d;
  d.nb = a.nb; d.nO = a.nO; d.nI = a.nI; d.nL = a.nL; d.c = c; d.red = a.red;
  d.sO = a.sO; d.sI = a.sI; d.sC = a.sC;
  d.hL = a.hL;
  d.m_end = 2.0 * a.hL / 6.0;
  d.m_int = 4.0 * a.hL / 6.0;
  d.m_off = a.hL / 6.0;
  d.k_off = -1.0 / a.hL;
  d.kLo = a.kLo; d.kHi = a.kHi;
  d.in = a.in;
  d.alpha0 = a.alpha0; d.alpha1 = a.alpha1; d.PO = a.PO;
  d.beta0 = a.beta0; d.beta1 = a.beta1; d.PI = a.PI;
  d.rho0 = a.rho0; d.rho1 = a.rho1;
  d.piv = a.piv;
  d.out = a.out; d.part = a.part;
  d.tile = d.ntiles = d.iters = 0;
  (void)P;
  return d;
}

}  // namespace

void lines_geometry(int nL, int* P, int* c, int* NT) {
  int p = 1;
  while (p * kCMax < nL) p <<= 1;
  *P = p;
  *c = (nL + p - 1) / p;
  *NT = p > 256 ? p : 256;
}

hipError_t launch_line_factors(const LineArgs& a, double2* piv, hipStream_t s) {
  int P, c, NT;
  lines_geometry(a.nL, &P, &c, &NT);
  if (a.nL < 3 || P > 512) return hipErrorInvalidValue;
  const LineDev d = make_dev(a, P, c);
  const int64_t lines = (int64_t)a.nO * a.nI;
  if (lines <= 0) return hipSuccess;
  hipLaunchKernelGGL(factor_kernel, dim3((unsigned)lines), dim3(P), (size_t)P * sizeof(Mob), s, d, P, piv);
  return hipGetLastError();
}

hipError_t launch_lines(LineArgs a, hipStream_t s) {
  if (a.nL < 3 || !a.piv) return hipErrorInvalidValue;
  int P, c, NT;
  lines_geometry(a.nL, &P, &c, &NT);
  if (P > 512) return hipErrorInvalidValue;
  LineDev d = make_dev(a, P, c);
  const int LPB = NT / P;
  int64_t blocks;
  if (a.red == 1 || a.red == 2) {
    const int64_t extent = a.red == 1 ? a.nI : a.nO;
    const int64_t groups = a.red == 1 ? (int64_t)a.nb * a.nO : (int64_t)a.nb * a.nI;
    d.tile = a.tile;
    d.ntiles = (int)((extent + a.tile - 1) / a.tile);
    if (d.ntiles != a.ntiles) return hipErrorInvalidValue;
    blocks = groups * d.ntiles;
  } else {
    const int64_t lines = (int64_t)a.nb * a.nO * a.nI;
    d.tile = a.tile;
    d.ntiles = (int)((lines + a.tile - 1) / a.tile);
    blocks = d.ntiles;
  }
  if (d.tile % LPB) return hipErrorInvalidValue;
  d.iters = d.tile / LPB;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = (a.red && LPB > 1) ? (size_t)2 * a.nL * sizeof(double2) : 0;
  const bool in64 = a.in_kind == ST_C64, out64 = a.out_kind == ST_C64;
  if (!in64 && !out64) return launch_typed<double2, double2>(d, P, blocks, lds, s);
  if (in64 && out64) return launch_typed<float2, float2>(d, P, blocks, lds, s);
  if (in64) return launch_typed<float2, double2>(d, P, blocks, lds, s);
  return launch_typed<double2, float2>(d, P, blocks, lds, s);
}

}  // namespace helm
