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

template <typename TR>
__global__ __launch_bounds__(kResThreads) void residual_kernel(ResidArgs a, int64_t per_rhs,
                                                               int64_t quads_per_rhs, int64_t blocks_per_rhs) {
  __shared__ double red[2][kResThreads];
  if (a.skip && *a.skip) return;
  const int64_t b = blockIdx.x / blocks_per_rhs;
  const int64_t qi = (blockIdx.x % blocks_per_rhs) * kResThreads + threadIdx.x;
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
    a.scratch[2 * blockIdx.x] = red[0][0];
    a.scratch[2 * blockIdx.x + 1] = red[1][0];
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

int64_t residual_scratch_len(int dim, const int64_t* grid, int nb) {
  int64_t per, quads, bpr;
  geometry(dim, grid, &per, &quads, &bpr);
  return 2 * bpr * nb;
}

hipError_t launch_residual(const ResidArgs& a, hipStream_t s) {
  int64_t n[3];
  for (int j = 0; j < a.dim; ++j) n[j] = a.ax[j].n;
  int64_t per, quads, bpr;
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
