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
// Parallelism.  A line of nL rows is owned by P lanes, lane q holding the rows
// [q c, q c + c).  The three recurrences of Thomas are associative and are
// evaluated by exclusive scans across the P lanes:
//   pivots   (num, den) -> (d num - e^2 den, num)       2x2 Moebius matrices
//   forward  z_x = d_x - e_x / p_{x-1} z_{x-1}          affine maps z -> F z + G
//   backward y_x = (z_x - e_{x+1} y_{x+1}) / p_x       affine maps, reversed
// Each lane composes its c rows, the scan supplies the state entering the
// chunk, and the lane then re-runs its rows sequentially.  Arithmetic is FP64
// whatever the storage precision.
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

// Segmented exclusive scan over the P lanes of each line slot:
// returns op(v_{r-1}, op(v_{r-2}, ... v_0)) with "later o earlier" order, or
// the identity for r = 0.  All threads of the block must call it.
template <class T, class Op>
__device__ inline T excl_scan(T v, int r, int P, int base, T* buf, T ident, Op op) {
  buf[base + r] = v;
  __syncthreads();
  for (int d = 1; d < P; d <<= 1) {
    T mine = buf[base + r];
    T other = (r >= d) ? buf[base + r - d] : ident;
    __syncthreads();
    if (r >= d) buf[base + r] = op(mine, other);
    __syncthreads();
  }
  T res = (r > 0) ? buf[base + r - 1] : ident;
  __syncthreads();
  return res;
}

template <typename T> __device__ inline double2 ld(const T* p, int64_t i) { return to_d2(p[i]); }

struct LineDev {
  int nb, nO, nI, nL, P, c, red, tile, ntiles, iters;
  const double2* sO;
  const double2* sI;
  double2 sC;
  double hL, m_end, m_int, m_off, k_off;
  double2 kLo, kHi;
  const void* in;
  const double2 *alpha0, *alpha1, *PO, *beta0, *beta1, *PI, *rho0, *rho1;
  void* out;
  double2* part;
};

template <typename TIN, typename TOUT, int NT>
__global__ __launch_bounds__(NT) void lines_kernel(LineDev a) {
  extern __shared__ double smem_d[];
  Mob* mbuf = reinterpret_cast<Mob*>(smem_d);            // NT
  Aff* abuf = reinterpret_cast<Aff*>(smem_d);            // NT (aliases mbuf)
  double2* rbuf = reinterpret_cast<double2*>(smem_d + NT * 8);  // reduction staging

  const int P = a.P, c = a.c, nL = a.nL;
  const int LPB = NT / P;
  const int tid = threadIdx.x;
  const int slot = tid / P, q = tid - slot * P;
  const int base = slot * P;
  const int x0 = q * c;

  // Block -> (group, tile) along the reduced or flattened index.
  const int64_t blk = blockIdx.x;
  int64_t g = 0, t = 0;
  if (a.red) {
    g = blk / a.ntiles;
    t = blk - g * a.ntiles;
  } else {
    t = blk;
  }

  double2 acc0[kCMax], acc1[kCMax];
#pragma unroll
  for (int j = 0; j < kCMax; ++j) acc0[j] = acc1[j] = make_double2(0, 0);

  for (int it = 0; it < a.iters; ++it) {
    // ---- which line does this slot solve --------------------------------
    const int64_t li = t * a.tile + (int64_t)it * LPB + slot;
    int64_t b = 0, l = 0, m = 0;
    bool valid;
    if (a.red == 1) {        // g = b*nO + l, li = m
      valid = li < a.nI && li < (t + 1) * a.tile;
      b = g / a.nO;
      l = g - b * a.nO;
      m = li;
    } else if (a.red == 2) { // g = b*nI + m, li = l
      valid = li < a.nO && li < (t + 1) * a.tile;
      b = g / a.nI;
      m = g - b * a.nI;
      l = li;
    } else {                 // li = (b*nO + l)*nI + m
      valid = li < (int64_t)a.nb * a.nO * a.nI && li < (t + 1) * a.tile;
      m = li % a.nI;
      const int64_t bl = li / a.nI;
      l = bl % a.nO;
      b = bl / a.nO;
    }
    if (!valid) { b = 0; l = 0; m = 0; }

    double2 sig = a.sC;
    if (a.sO) sig = cadd(sig, a.sO[l]);
    if (a.sI) sig = cadd(sig, a.sI[m]);
    const double2 off = make_double2(sig.x * a.m_off + a.k_off, sig.y * a.m_off);  // sigma h/6 - 1/h
    const double2 off2 = cmul(off, off);
    const double2 dint = make_double2(sig.x * a.m_int + 2.0 / a.hL, sig.y * a.m_int);
    const double2 dlo = make_double2(sig.x * a.m_end + a.kLo.x / a.hL, sig.y * a.m_end + a.kLo.y / a.hL);
    const double2 dhi = make_double2(sig.x * a.m_end + a.kHi.x / a.hL, sig.y * a.m_end + a.kHi.y / a.hL);

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

    // Row coefficients: diag(x) and e(x) = coupling between x-1 and x.
    auto diag_of = [&](int x) -> double2 {
      if (x >= nL) return make_double2(1, 0);
      if (x == 0) return dlo;
      if (x == nL - 1) return dhi;
      return dint;
    };
    auto e2_of = [&](int x) -> double2 {  // e(x)^2
      if (x <= 0 || x >= nL) return make_double2(0, 0);
      return off2;
    };
    auto e_of = [&](int x) -> double2 {
      if (x <= 0 || x >= nL) return make_double2(0, 0);
      return off;
    };

    // ---- 1. pivots: Moebius scan ------------------------------------------
    Mob G;
    G.a = make_double2(1, 0); G.b = make_double2(0, 0);
    G.c = make_double2(0, 0); G.d = make_double2(1, 0);
#pragma unroll
    for (int j = 0; j < kCMax; ++j) {
      if (j < c) {
        const int x = x0 + j;
        const double2 dg = diag_of(x), e2 = e2_of(x);
        Mob n;
        n.a = csub(cmul(dg, G.a), cmul(e2, G.c));
        n.b = csub(cmul(dg, G.b), cmul(e2, G.d));
        n.c = G.a;
        n.d = G.b;
        G = n;
      }
    }
    mob_norm(G);
    Mob ident;
    ident.a = make_double2(1, 0); ident.b = make_double2(0, 0);
    ident.c = make_double2(0, 0); ident.d = make_double2(1, 0);
    const Mob E = excl_scan<Mob>(G, q, P, base, mbuf, ident, [](const Mob& lt, const Mob& er) {
      Mob r = mob_mul(lt, er);
      mob_norm(r);
      return r;
    });
    // state entering the chunk: E * (1, 0)^T = (E.a, E.c); 1/p = E.c / E.a
    double2 ipv = cmul(E.c, crcp(E.a));
#pragma unroll
    for (int j = 0; j < kCMax; ++j) {
      if (j < c) {
        const int x = x0 + j;
        const double2 p = csub(diag_of(x), cmul(e2_of(x), ipv));
        ipv = crcp(p);
        ip[j] = ipv;
      }
    }

    // ---- 2. forward substitution: affine scan -----------------------------
    // z_x = f_x z_{x-1} + d_x with f_x = -e(x) / p_{x-1}.
    Aff A;
    A.f = make_double2(1, 0);
    A.g = make_double2(0, 0);
    {
      double2 ipprev = cmul(E.c, crcp(E.a));
#pragma unroll
      for (int j = 0; j < kCMax; ++j) {
        if (j < c) {
          const int x = x0 + j;
          const double2 e = e_of(x);
          const double2 f = make_double2(-(e.x * ipprev.x - e.y * ipprev.y), -(e.x * ipprev.y + e.y * ipprev.x));
          A.f = cmul(f, A.f);
          A.g = cfma(f, A.g, z[j]);
          ipprev = ip[j];
        }
      }
    }
    Aff aid;
    aid.f = make_double2(1, 0);
    aid.g = make_double2(0, 0);
    const Aff Ein = excl_scan<Aff>(A, q, P, base, abuf, aid, aff_then);
    {
      double2 zprev = Ein.g;
      double2 ipprev = cmul(E.c, crcp(E.a));
#pragma unroll
      for (int j = 0; j < kCMax; ++j) {
        if (j < c) {
          const int x = x0 + j;
          const double2 e = e_of(x);
          const double2 f = make_double2(-(e.x * ipprev.x - e.y * ipprev.y), -(e.x * ipprev.y + e.y * ipprev.x));
          zprev = cfma(f, zprev, z[j]);
          z[j] = zprev;
          ipprev = ip[j];
        }
      }
    }

    // ---- 3. back substitution: reversed affine scan -----------------------
    // y_x = g_x y_{x+1} + h_x with g_x = -e(x+1)/p_x, h_x = z_x / p_x.
    Aff B;
    B.f = make_double2(1, 0);
    B.g = make_double2(0, 0);
#pragma unroll
    for (int j = kCMax - 1; j >= 0; --j) {
      if (j < c) {
        const int x = x0 + j;
        const double2 e = e_of(x + 1);
        const double2 gx = make_double2(-(e.x * ip[j].x - e.y * ip[j].y), -(e.x * ip[j].y + e.y * ip[j].x));
        const double2 hx = cmul(z[j], ip[j]);
        B.f = cmul(gx, B.f);
        B.g = cfma(gx, B.g, hx);
      }
    }
    const Aff Bin = excl_scan<Aff>(B, P - 1 - q, P, base, abuf, aid, aff_then);
    {
      double2 ynext = Bin.g;
#pragma unroll
      for (int j = kCMax - 1; j >= 0; --j) {
        if (j < c) {
          const int x = x0 + j;
          const double2 e = e_of(x + 1);
          const double2 gx = make_double2(-(e.x * ip[j].x - e.y * ip[j].y), -(e.x * ip[j].y + e.y * ip[j].x));
          ynext = cfma(gx, ynext, cmul(z[j], ip[j]));
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
      if (a.red) {
        const int64_t wi = (a.red == 1) ? m : l;
        const double2 w0 = a.rho0[wi], w1 = a.rho1[wi];
#pragma unroll
        for (int j = 0; j < kCMax; ++j) {
          acc0[j] = cfma(w0, z[j], acc0[j]);
          acc1[j] = cfma(w1, z[j], acc1[j]);
        }
      }
    }
  }

  // ---- cross-slot reduction and partial write ------------------------------
  if (a.red) {
    double2* outp = a.part + (g * a.ntiles + t) * 2 * (int64_t)nL;
    if (LPB == 1) {
#pragma unroll
      for (int j = 0; j < kCMax; ++j) {
        const int x = x0 + j;
        if (j < c && x < nL) {
          outp[x] = acc0[j];
          outp[nL + x] = acc1[j];
        }
      }
    } else {
      for (int s = 0; s < LPB; ++s) {
        if (slot == s) {
#pragma unroll
          for (int j = 0; j < kCMax; ++j) {
            const int x = x0 + j;
            if (j < c && x < nL) {
              if (s == 0) {
                rbuf[x] = acc0[j];
                rbuf[nL + x] = acc1[j];
              } else {
                rbuf[x] = cadd(rbuf[x], acc0[j]);
                rbuf[nL + x] = cadd(rbuf[nL + x], acc1[j]);
              }
            }
          }
        }
        __syncthreads();
      }
      for (int x = tid; x < 2 * nL; x += NT) outp[x] = rbuf[x];
    }
  }
}

template <typename TIN, typename TOUT>
hipError_t launch_typed(const LineDev& d, int NT, int64_t blocks, size_t lds, hipStream_t s) {
  if (NT == 512)
    hipLaunchKernelGGL((lines_kernel<TIN, TOUT, 512>), dim3((unsigned)blocks), dim3(512), lds, s, d);
  else
    hipLaunchKernelGGL((lines_kernel<TIN, TOUT, 256>), dim3((unsigned)blocks), dim3(256), lds, s, d);
  return hipGetLastError();
}

void lanes_for(int nL, int* P, int* c) {
  int p = 1;
  while (p * kCMax < nL) p <<= 1;
  *P = p;
  *c = (nL + p - 1) / p;
}

}  // namespace

int lines_tile(const LineArgs& a, int reduce_extent, int target_blocks) {
  int P, c;
  lanes_for(a.nL, &P, &c);
  const int NT = P > 256 ? P : 256;
  const int LPB = NT / P;
  const int64_t groups = a.red == 1 ? (int64_t)a.nb * a.nO : (a.red == 2 ? (int64_t)a.nb * a.nI : 1);
  // lines per tile: a multiple of LPB, enough tiles to fill the chip
  int64_t per = ((int64_t)reduce_extent * groups + target_blocks - 1) / target_blocks;
  if (per < LPB) per = LPB;
  per = (per + LPB - 1) / LPB * LPB;
  if (per > reduce_extent && a.red) per = ((int64_t)reduce_extent + LPB - 1) / LPB * LPB;
  return (int)per;
}

hipError_t launch_lines(LineArgs a, hipStream_t s) {
  if (a.nL < 3 || a.nL > 512 * kCMax) return hipErrorInvalidValue;
  LineDev d;
  int P, c;
  lanes_for(a.nL, &P, &c);
  const int NT = P > 256 ? P : 256;
  if (NT > 512) return hipErrorInvalidValue;
  d.nb = a.nb; d.nO = a.nO; d.nI = a.nI; d.nL = a.nL; d.P = P; d.c = c; d.red = a.red;
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
  d.out = a.out; d.part = a.part;
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
  // LDS: scan buffer (NT Moebius = NT*8 doubles) + reduction staging (2 nL complex)
  size_t lds = (size_t)NT * 8 * sizeof(double);
  if (a.red && LPB > 1) lds += (size_t)2 * a.nL * sizeof(double2);
  const bool in64 = a.in_kind == ST_C64, out64 = a.out_kind == ST_C64;
  if (!in64 && !out64) return launch_typed<double2, double2>(d, NT, blocks, lds, s);
  if (in64 && out64) return launch_typed<float2, float2>(d, NT, blocks, lds, s);
  if (in64) return launch_typed<float2, double2>(d, NT, blocks, lds, s);
  return launch_typed<double2, float2>(d, NT, blocks, lds, s);
}

}  // namespace helm
