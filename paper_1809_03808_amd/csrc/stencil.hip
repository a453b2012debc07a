// FP64 residual r = f - A u with the matrix-free operator of eqs. (A2D), (A3D)
// (the 9-point bilinear / 27-point trilinear stencil as Kronecker products of
// the 1D entries of eqs. (matrixK), (matrixM)), and per right-hand side the
// squared norms sum |r|^2 and sum |f|^2 used by iterative refinement.
//
// Each thread produces four consecutive nodes along the contiguous axis.  For
// every stencil row (3 in 2D, 9 in 3D) it loads the six values it needs once
// and applies the last-axis 1D operators M and K to them; the row results are
// combined with the products of the leading-axis 1D entries:
//   2D:  (A u)_x = sum_{o1} S1(o1) (M2 u_{o1})_x + M1(o1) (K2 u_{o1})_x,
//   3D:  (A u)_x = sum_{o1,o2} [S1 M2 + M1 K2](o1,o2) (M3 u_{o1,o2})_x
//                              + M1(o1) M2(o2) (K3 u_{o1,o2})_x,
// with S1 = K1 - w^2 M1.  Norm partials are reduced per block in LDS and
// summed per right-hand side in a fixed order, so the result is deterministic.
#include <algorithm>

#include "helm_internal.h"
#include "ops1d.h"

namespace helm {

namespace {

constexpr int kResThreads = 256;
constexpr int kQuad = 4;
constexpr int kFinThreads = 1024;

// (M u)_x and (K u)_x for the 4 outputs x0..x0+3 of one row whose values
// v[0..5] are u[x0-1 .. x0+4] (zero outside the line).
__device__ inline void row_ops(const double2* v, int n, double h, double2 kLo, double2 kHi, int x0,
                               double2* Mv, double2* Kv) {
#pragma unroll
  for (int j = 0; j < kQuad; ++j) {
    const int x = x0 + j;
    double2 m = make_double2(0, 0), k = make_double2(0, 0);
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
      const double2 u = v[j + 1 + o];
      m = cadd(m, cscale(u, m1d(n, h, x, o)));
      k = cfma(k1d(n, h, kLo, kHi, x, o), u, k);
    }
    Mv[j] = m;
    Kv[j] = k;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that every XCD works on one contiguous range of
// lines: the neighbouring lines a stencil row reads are then mostly in the
// same L2.  A bijection on [0, n) for any n.
__device__ inline int64_t xcd_contiguous(int64_t b, int64_t n) {
  const int64_t q = n / 8, r = n % 8, x = b % 8, k = b / 8;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <typename TR>
__global__ __launch_bounds__(kResThreads) void residual_kernel(ResidArgs a, int64_t per_rhs,
                                                               int64_t quads_per_rhs, int64_t blocks_per_rhs) {
  __shared__ double red[2][kResThreads];
  if (a.skip && *a.skip) return;
  const int64_t bid = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t b = bid / blocks_per_rhs;
  const int64_t qi = (bid % blocks_per_rhs) * kResThreads + threadIdx.x;
  double sr = 0.0, sf = 0.0;
  if (qi < quads_per_rhs) {
    const int dim = a.dim;
    const AxisOp& AL = a.ax[dim - 1];  // contiguous axis
    const int nL = AL.n;
    const int nq = (nL + kQuad - 1) / kQuad;
    const int64_t rowi = qi / nq;           // index of the line (i1 or i1*n2+i2)
    const int x0 = (int)(qi - rowi * nq) * kQuad;
    const int64_t off = b * per_rhs;
    double2 au[kQuad];
#pragma unroll
    for (int j = 0; j < kQuad; ++j) au[j] = make_double2(0, 0);
    const AxisOp& A1 = a.ax[0];
    if (dim == 2) {
      const int i1 = (int)rowi;
      for (int o1 = -1; o1 <= 1; ++o1) {
        const double m1 = m1d(A1.n, A1.h, i1, o1);
        if (m1 == 0.0) continue;
        const double2 k1 = k1d(A1.n, A1.h, A1.kLo, A1.kHi, i1, o1);
        const double2 s1 = make_double2(k1.x - a.w2 * m1, k1.y);
        const double2* row = a.u + off + (int64_t)(i1 + o1) * nL;
        double2 v[kQuad + 2];
#pragma unroll
        for (int j = 0; j < kQuad + 2; ++j) {
          const int x = x0 - 1 + j;
          v[j] = (x >= 0 && x < nL) ? row[x] : make_double2(0, 0);
        }
        double2 Mv[kQuad], Kv[kQuad];
        row_ops(v, nL, AL.h, AL.kLo, AL.kHi, x0, Mv, Kv);
#pragma unroll
        for (int j = 0; j < kQuad; ++j) au[j] = cadd(cfma(s1, Mv[j], au[j]), cscale(Kv[j], m1));
      }
    } else {
      const AxisOp& A2 = a.ax[1];
      const int i1 = (int)(rowi / A2.n), i2 = (int)(rowi % A2.n);
      for (int o1 = -1; o1 <= 1; ++o1) {
        const double m1 = m1d(A1.n, A1.h, i1, o1);
        if (m1 == 0.0) continue;
        const double2 k1 = k1d(A1.n, A1.h, A1.kLo, A1.kHi, i1, o1);
        const double2 s1 = make_double2(k1.x - a.w2 * m1, k1.y);
        for (int o2 = -1; o2 <= 1; ++o2) {
          const double m2 = m1d(A2.n, A2.h, i2, o2);
          if (m2 == 0.0) continue;
          const double2 k2 = k1d(A2.n, A2.h, A2.kLo, A2.kHi, i2, o2);
          // coefficient of (M3 u_row): S1 M2 + M1 K2; of (K3 u_row): M1 M2
          const double2 cm = make_double2(s1.x * m2 + m1 * k2.x, s1.y * m2 + m1 * k2.y);
          const double ck = m1 * m2;
          const double2* row = a.u + off + ((int64_t)(i1 + o1) * A2.n + (i2 + o2)) * nL;
          double2 v[kQuad + 2];
#pragma unroll
          for (int j = 0; j < kQuad + 2; ++j) {
            const int x = x0 - 1 + j;
            v[j] = (x >= 0 && x < nL) ? row[x] : make_double2(0, 0);
          }
          double2 Mv[kQuad], Kv[kQuad];
          row_ops(v, nL, AL.h, AL.kLo, AL.kHi, x0, Mv, Kv);
#pragma unroll
          for (int j = 0; j < kQuad; ++j) au[j] = cadd(cfma(cm, Mv[j], au[j]), cscale(Kv[j], ck));
        }
      }
    }
    const int64_t base = off + rowi * nL;
#pragma unroll
    for (int j = 0; j < kQuad; ++j) {
      const int x = x0 + j;
      if (x < nL) {
        const double2 fv = a.f[base + x];
        const double2 r = csub(fv, au[j]);
        if (a.r) reinterpret_cast<TR*>(a.r)[base + x] = from_d2<TR>(r);
        sr += r.x * r.x + r.y * r.y;
        sf += fv.x * fv.x + fv.y * fv.y;
      }
    }
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = sf;
  __syncthreads();
  for (int s = kResThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.scratch[2 * bid] = red[0][0];
    a.scratch[2 * bid + 1] = red[1][0];
  }
}

// 2D: one thread per column x, a block streams down a strip of kStrip rows
// of 256 columns.  Each row of u is loaded once (consecutive lanes on
// consecutive columns), its x_2 neighbours come from the adjacent lanes
// (the two wave-edge lanes load theirs), and the row operators M_2 u_j and
// K_2 u_j of rows i-1, i, i+1 stay in registers while the strip advances,
// so u and f are read from memory once (plus two halo rows per strip).  The
// rows one and two ahead are already in flight while row i is combined.
constexpr int kStrip = 32;

struct RowRaw {
  double2 c, e;  // u[j][x], and u[j][x -/+ 1] for the first / last lane of the wave
};

template <typename TR>
__global__ __launch_bounds__(kResThreads) void residual2d_kernel(ResidArgs a, int64_t xtiles,
                                                                 int64_t blocks_per_rhs) {
  __shared__ double red[2][kResThreads];
  if (a.skip && *a.skip) return;
  const int64_t bid = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t b = bid / blocks_per_rhs;
  const int64_t rem = bid - b * blocks_per_rhs;
  const int64_t si = rem / xtiles, xi = rem - si * xtiles;
  const AxisOp& A1 = a.ax[0];
  const AxisOp& A2 = a.ax[1];
  const int n1 = A1.n, n2 = A2.n;
  const int x = (int)xi * kResThreads + (int)threadIdx.x;
  const bool xok = x < n2;
  const int lane = threadIdx.x & 63;
  const int r0 = (int)si * kStrip, r1 = min(n1, r0 + kStrip);
  const int64_t off = b * (int64_t)n1 * n2;
  const double2* U = a.u + off;
  const int xe = lane == 0 ? x - 1 : x + 1;  // edge neighbour loaded by the wave-edge lanes
  const bool edge = (lane == 0 || lane == 63) && xe >= 0 && xe < n2;
  const double mL = m1d(n2, A2.h, x, -1), mC = m1d(n2, A2.h, x, 0), mR = m1d(n2, A2.h, x, 1);
  const double2 kL = k1d(n2, A2.h, A2.kLo, A2.kHi, x, -1), kC = k1d(n2, A2.h, A2.kLo, A2.kHi, x, 0),
                kR = k1d(n2, A2.h, A2.kLo, A2.kHi, x, 1);
  auto load = [&](int j) {
    RowRaw w;
    w.c = make_double2(0, 0);
    w.e = make_double2(0, 0);
    if (j >= 0 && j < n1) {
      const double2* row = U + (int64_t)j * n2;
      if (xok) w.c = row[x];
      if (edge) w.e = row[xe];
    }
    return w;
  };
  auto rowop = [&](const RowRaw& w, double2& Mu, double2& Ku) {
    double2 l = make_double2(__shfl_up(w.c.x, 1), __shfl_up(w.c.y, 1));
    double2 r = make_double2(__shfl_down(w.c.x, 1), __shfl_down(w.c.y, 1));
    if (lane == 0) l = w.e;
    if (lane == 63) r = w.e;
    Mu = make_double2(mL * l.x + mC * w.c.x + mR * r.x, mL * l.y + mC * w.c.y + mR * r.y);
    Ku = cfma(kL, l, cfma(kC, w.c, cmul(kR, r)));
  };
  double2 Mp, Kp, Mc, Kc;
  rowop(load(r0 - 1), Mp, Kp);
  rowop(load(r0), Mc, Kc);
  RowRaw nx = load(r0 + 1);
  double sr = 0.0, sf = 0.0;
  for (int i = r0; i < r1; ++i) {
    const RowRaw nn = load(i + 2);  // in flight while row i is combined
    const double2 fv = xok ? a.f[off + (int64_t)i * n2 + x] : make_double2(0, 0);
    double2 Mn, Kn;
    rowop(nx, Mn, Kn);
    double2 au = make_double2(0, 0);
    const double2* Ms[3] = {&Mp, &Mc, &Mn};
    const double2* Ks[3] = {&Kp, &Kc, &Kn};
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
      const double m1 = m1d(n1, A1.h, i, o);
      const double2 k1 = k1d(n1, A1.h, A1.kLo, A1.kHi, i, o);
      const double2 s1 = make_double2(k1.x - a.w2 * m1, k1.y);
      au = cadd(cfma(s1, *Ms[o + 1], au), cscale(*Ks[o + 1], m1));
    }
    if (xok) {
      const double2 r = csub(fv, au);
      if (a.r) reinterpret_cast<TR*>(a.r)[off + (int64_t)i * n2 + x] = from_d2<TR>(r);
      sr += r.x * r.x + r.y * r.y;
      sf += fv.x * fv.x + fv.y * fv.y;
    }
    Mp = Mc;
    Kp = Kc;
    Mc = Mn;
    Kc = Kn;
    nx = nn;
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = sf;
  __syncthreads();
  for (int st = kResThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      red[1][threadIdx.x] += red[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.scratch[2 * bid] = red[0][0];
    a.scratch[2 * bid + 1] = red[1][0];
  }
}

// 3D: a block of 8 waves owns an (x_2, x_3) tile of 8 rows x 64 columns and
// streams along x_1 over a strip of planes.  For every plane it loads
// the 10 rows the tile needs (one halo row each side; lanes on consecutive
// x_3), applies the x_3 operators M_3, K_3 (neighbours from adjacent lanes)
// and parks them in LDS; each thread then forms the plane operators
//   P = (M_2 (x) M_3) u_j,  Q = (K_2 (x) M_3 + M_2 (x) K_3) u_j
// at its point, and the x_1 combination
//   (A u)_i = sum_{o1} (K_1 - w^2 M_1)(i, o1) P_{i+o1} + M_1(i, o1) Q_{i+o1}
// uses the P, Q of three consecutive planes kept in registers.  u is read
// about 1.3 times (halo rows and planes), f once.
constexpr int k3Rows = 8;
constexpr int k3Threads = 64 * k3Rows;
constexpr int k3Load = k3Rows + 2;

template <typename TR>
__global__ __launch_bounds__(k3Threads) void residual3d_kernel(ResidArgs a, int64_t xtiles, int64_t ytiles,
                                                               int64_t blocks_per_rhs, int strip) {
  __shared__ double2 Mx[2][k3Load][64];
  __shared__ double2 Kx[2][k3Load][64];
  __shared__ double red[2][k3Threads];
  if (a.skip && *a.skip) return;
  const int64_t bid = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t b = bid / blocks_per_rhs;
  int64_t rem = bid - b * blocks_per_rhs;
  const int64_t xi = rem % xtiles;
  rem /= xtiles;
  const int64_t yi = rem % ytiles;
  const int64_t si = rem / ytiles;
  const AxisOp& A1 = a.ax[0];
  const AxisOp& A2 = a.ax[1];
  const AxisOp& A3 = a.ax[2];
  const int n1 = A1.n, n2 = A2.n, n3 = A3.n;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // wave-uniform
  const int x = (int)xi * 64 + lane;
  const bool xok = x < n3;
  const int y0 = (int)yi * k3Rows;      // first output row (x_2) of the tile
  const int y = y0 + wv;                // this wave's output row
  const bool yok = y < n2;
  const int r0 = (int)si * strip, r1 = min(n1, r0 + strip);
  const int64_t plane = (int64_t)n2 * n3;
  const int64_t off = b * (int64_t)n1 * plane;
  const double2* U = a.u + off;
  const int xe = lane == 0 ? x - 1 : x + 1;
  const bool edge = (lane == 0 || lane == 63) && xe >= 0 && xe < n3;
  // Values outside the domain are loaded as zero, so the off-diagonal
  // entries can be the interior ones everywhere (uniform); only the
  // diagonal entries of the end nodes differ: per lane along x_3, per wave
  // along x_2.
  const double m3O = A3.h / 6.0, k3O = -1.0 / A3.h;
  const double m3C = m1d(n3, A3.h, x, 0);
  const double2 k3C = k1d(n3, A3.h, A3.kLo, A3.kHi, x, 0);
  const double m2O = yok ? A2.h / 6.0 : 0.0, k2O = yok ? -1.0 / A2.h : 0.0;
  const double m2C = yok ? m1d(n2, A2.h, y, 0) : 0.0;
  const double2 k2C = yok ? k1d(n2, A2.h, A2.kLo, A2.kHi, y, 0) : make_double2(0, 0);
  // The rows y0 - 1 + rr (rr < k3Load) of a plane are loaded by wave
  // rr % k3Rows: every wave owns row wv, waves 0 and 1 also row wv + k3Rows.
  // The loads of plane j + 1 are issued before plane j is combined, so a
  // plane's loads are in flight during the previous plane's LDS work.
  struct Raw {
    double2 c[2], e[2];  // u at the lane's column, and the wave-edge neighbour
  };
  auto load_plane = [&](int j) {
    Raw w;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int rr = wv + t * k3Rows;
      const int yy = y0 - 1 + rr;
      w.c[t] = make_double2(0, 0);
      w.e[t] = make_double2(0, 0);
      if (rr < k3Load && j >= 0 && j < n1 && yy >= 0 && yy < n2) {
        const double2* row = U + (int64_t)j * plane + (int64_t)yy * n3;
        if (xok) w.c[t] = row[x];
        if (edge) w.e[t] = row[xe];
      }
    }
    return w;
  };
  // x_3 operators of the loaded rows into LDS buffer `buf`, then (P, Q) at
  // this thread's point
  auto plane_op = [&](const Raw& w, int buf, double2& P, double2& Q) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int rr = wv + t * k3Rows;
      if (rr < k3Load) {
        const double2 c = w.c[t];
        double2 l = make_double2(__shfl_up(c.x, 1), __shfl_up(c.y, 1));
        double2 r = make_double2(__shfl_down(c.x, 1), __shfl_down(c.y, 1));
        if (lane == 0) l = w.e[t];
        if (lane == 63) r = w.e[t];
        const double2 lr = cadd(l, r);
        Mx[buf][rr][lane] = make_double2(fma(m3O, lr.x, m3C * c.x), fma(m3O, lr.y, m3C * c.y));
        Kx[buf][rr][lane] = cfma(k3C, c, cscale(lr, k3O));
      }
    }
    __syncthreads();
    const double2 ms = cadd(Mx[buf][wv][lane], Mx[buf][wv + 2][lane]), mc = Mx[buf][wv + 1][lane];
    const double2 ks = cadd(Kx[buf][wv][lane], Kx[buf][wv + 2][lane]), kc = Kx[buf][wv + 1][lane];
    P = make_double2(fma(m2O, ms.x, m2C * mc.x), fma(m2O, ms.y, m2C * mc.y));
    // (K_2 (x) M_3 + M_2 (x) K_3) u: off-diagonal K_2 and M_2 entries are real
    Q = cfma(k2C, mc, make_double2(fma(k2O, ms.x, fma(m2O, ks.x, m2C * kc.x)),
                                   fma(k2O, ms.y, fma(m2O, ks.y, m2C * kc.y))));
  };
  double2 Pp, Qp, Pc, Qc;
  plane_op(load_plane(r0 - 1), 0, Pp, Qp);
  plane_op(load_plane(r0), 1, Pc, Qc);
  Raw nx = load_plane(r0 + 1);
  double sr = 0.0, sf = 0.0;
  int buf = 0;
  for (int i = r0; i < r1; ++i) {
    const bool ok = xok && yok;
    const int64_t idx = off + (int64_t)i * plane + (int64_t)y * n3 + x;
    const double2 fv = ok ? a.f[idx] : make_double2(0, 0);
    const Raw nn = load_plane(i + 2);  // in flight while plane i + 1 is combined
    double2 Pn, Qn;
    plane_op(nx, buf, Pn, Qn);  // two LDS buffers alternate: the one read last is not overwritten
    buf ^= 1;
    double2 au = make_double2(0, 0);
    const double2* Ps[3] = {&Pp, &Pc, &Pn};
    const double2* Qs[3] = {&Qp, &Qc, &Qn};
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
      const double m1 = m1d(n1, A1.h, i, o);
      const double2 k1 = k1d(n1, A1.h, A1.kLo, A1.kHi, i, o);
      const double2 s1 = make_double2(k1.x - a.w2 * m1, k1.y);
      au = cadd(cfma(s1, *Ps[o + 1], au), cscale(*Qs[o + 1], m1));
    }
    if (ok) {
      const double2 r = csub(fv, au);
      if (a.r) reinterpret_cast<TR*>(a.r)[idx] = from_d2<TR>(r);
      sr += r.x * r.x + r.y * r.y;
      sf += fv.x * fv.x + fv.y * fv.y;
    }
    Pp = Pc;
    Qp = Qc;
    Pc = Pn;
    Qc = Qn;
    nx = nn;
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = sf;
  __syncthreads();
  for (int st = k3Threads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      red[1][threadIdx.x] += red[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.scratch[2 * bid] = red[0][0];
    a.scratch[2 * bid + 1] = red[1][0];
  }
}

__global__ __launch_bounds__(kFinThreads) void norm_finish_kernel(const double* scratch, int64_t blocks_per_rhs,
                                                                  double* norms, const int* skip) {
  __shared__ double red[2][kFinThreads];
  if (skip && *skip) return;
  const int64_t b = blockIdx.x;
  double sr = 0.0, sf = 0.0;
  for (int64_t i = threadIdx.x; i < blocks_per_rhs; i += kFinThreads) {
    sr += scratch[2 * (b * blocks_per_rhs + i)];
    sf += scratch[2 * (b * blocks_per_rhs + i) + 1];
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = sf;
  __syncthreads();
  for (int s = kFinThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    norms[2 * b] = red[0][0];
    norms[2 * b + 1] = red[1][0];
  }
}

void geometry(int dim, const int64_t* n, int64_t* per, int64_t* quads, int64_t* bpr) {
  int64_t p = 1;
  for (int j = 0; j < dim; ++j) p *= n[j];
  const int64_t nL = n[dim - 1];
  const int64_t lines = p / nL;
  *per = p;
  *quads = lines * ((nL + kQuad - 1) / kQuad);
  *bpr = (*quads + kResThreads - 1) / kResThreads;
}

}  // namespace

// 2D streaming geometry: column tiles of 256 and strips of kStrip rows.
void geometry2d(const int64_t* n, int64_t* xtiles, int64_t* bpr) {
  *xtiles = (n[1] + kResThreads - 1) / kResThreads;
  *bpr = *xtiles * ((n[0] + kStrip - 1) / kStrip);
}

// 3D streaming geometry: 64-column x 8-row tiles, strips of 64 planes when
// that leaves at least 4096 blocks (16 per compute unit), else of 32: a
// strip re-reads two halo planes (512^3 x 16 residual: 18.6 ms with strips of
// 32 planes, 18.1 with 64, 19.7 with 16).
void geometry3d(const int64_t* n, int nb, int64_t* xtiles, int64_t* ytiles, int64_t* bpr, int* strip) {
  *xtiles = (n[2] + 63) / 64;
  *ytiles = (n[1] + k3Rows - 1) / k3Rows;
  *strip = *xtiles * *ytiles * ((n[0] + 63) / 64) * nb >= 4096 ? 64 : kStrip;
  *bpr = *xtiles * *ytiles * ((n[0] + *strip - 1) / *strip);
}

int64_t residual_scratch_len(int dim, const int64_t* grid, int nb) {
  int64_t per, quads, bpr;
  geometry(dim, grid, &per, &quads, &bpr);
  if (dim == 2) {
    int64_t xt, b2;
    geometry2d(grid, &xt, &b2);
    bpr = std::max(bpr, b2);
  } else {
    int64_t xt, yt, b3;
    int strip;
    geometry3d(grid, nb, &xt, &yt, &b3, &strip);
    bpr = std::max(bpr, b3);
  }
  return 2 * bpr * nb;
}

hipError_t launch_residual(const ResidArgs& a, hipStream_t s) {
  int64_t n[3];
  for (int j = 0; j < a.dim; ++j) n[j] = a.ax[j].n;
  int64_t per, quads, bpr;
  if (a.dim == 2) {
    int64_t xt;
    geometry2d(n, &xt, &bpr);
    const int64_t blocks = bpr * a.nb;
    if (blocks > 0x7fffffffLL || 2 * blocks > a.scratch_len) return hipErrorInvalidValue;
    if (a.r_kind == ST_C64)
      hipLaunchKernelGGL(residual2d_kernel<float2>, dim3((unsigned)blocks), dim3(kResThreads), 0, s, a, xt, bpr);
    else
      hipLaunchKernelGGL(residual2d_kernel<double2>, dim3((unsigned)blocks), dim3(kResThreads), 0, s, a, xt, bpr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(norm_finish_kernel, dim3((unsigned)a.nb), dim3(kFinThreads), 0, s, a.scratch, bpr, a.norms,
                       a.skip);
    return hipGetLastError();
  }
  {
    int64_t xt, yt;
    int strip;
    geometry3d(n, a.nb, &xt, &yt, &bpr, &strip);
    const int64_t blocks = bpr * a.nb;
    if (blocks > 0x7fffffffLL || 2 * blocks > a.scratch_len) return hipErrorInvalidValue;
    if (a.r_kind == ST_C64)
      hipLaunchKernelGGL(residual3d_kernel<float2>, dim3((unsigned)blocks), dim3(k3Threads), 0, s, a, xt, yt, bpr,
                         strip);
    else
      hipLaunchKernelGGL(residual3d_kernel<double2>, dim3((unsigned)blocks), dim3(k3Threads), 0, s, a, xt, yt, bpr,
                         strip);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(norm_finish_kernel, dim3((unsigned)a.nb), dim3(kFinThreads), 0, s, a.scratch, bpr, a.norms,
                       a.skip);
    return hipGetLastError();
  }
  geometry(a.dim, n, &per, &quads, &bpr);
  const int64_t blocks = bpr * a.nb;
  if (blocks > 0x7fffffffLL || 2 * blocks > a.scratch_len) return hipErrorInvalidValue;
  if (a.r_kind == ST_C64)
    hipLaunchKernelGGL(residual_kernel<float2>, dim3((unsigned)blocks), dim3(kResThreads), 0, s, a, per, quads, bpr);
  else
    hipLaunchKernelGGL(residual_kernel<double2>, dim3((unsigned)blocks), dim3(kResThreads), 0, s, a, per, quads, bpr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(norm_finish_kernel, dim3((unsigned)a.nb), dim3(kFinThreads), 0, s, a.scratch, bpr, a.norms, a.skip);
  return hipGetLastError();
}

}  // namespace helm
