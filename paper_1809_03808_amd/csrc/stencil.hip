// FP64 residual r = f - A u with the matrix-free operator of eqs. (A2D), (A3D)
// (the 9-point bilinear / 27-point trilinear stencil as Kronecker products of
// the 1D entries of eqs. (matrixK), (matrixM)), and per right-hand side the
// squared norms sum |r|^2 and sum |f|^2 used by iterative refinement.
//
// One thread per node along the contiguous axis; neighbour loads are served by
// the caches.  Norm partials are reduced per block in LDS, written per block,
// and summed per right-hand side in a fixed order by a second kernel, so the
// result is deterministic.
#include "helm_internal.h"
#include "ops1d.h"

namespace helm {

namespace {

constexpr int kResThreads = 256;

template <typename TR>
__global__ __launch_bounds__(kResThreads) void residual_kernel(ResidArgs a, int64_t per_rhs,
                                                               int64_t blocks_per_rhs) {
  __shared__ double red[2][kResThreads];
  const int64_t b = blockIdx.x / blocks_per_rhs;
  const int64_t i = (blockIdx.x % blocks_per_rhs) * kResThreads + threadIdx.x;
  double sr = 0.0, sf = 0.0;
  if (i < per_rhs) {
    const AxisOp& A1 = a.ax[0];
    const AxisOp& A2 = a.ax[1];
    const int64_t off = b * per_rhs;
    double2 au = make_double2(0, 0);
    if (a.dim == 2) {
      const int i1 = (int)(i / A2.n), i2 = (int)(i % A2.n);
      for (int o1 = -1; o1 <= 1; ++o1) {
        const double m1 = m1d(A1.n, A1.h, i1, o1);
        if (m1 == 0.0) continue;
        const double2 k1 = k1d(A1.n, A1.h, A1.kLo, A1.kHi, i1, o1);
        const double2 s1 = make_double2(k1.x - a.w2 * m1, k1.y);  // (K1 - w^2 M1)(i1, o1)
        for (int o2 = -1; o2 <= 1; ++o2) {
          const double m2 = m1d(A2.n, A2.h, i2, o2);
          if (m2 == 0.0) continue;
          const double2 k2 = k1d(A2.n, A2.h, A2.kLo, A2.kHi, i2, o2);
          const double2 coef = make_double2(s1.x * m2 + m1 * k2.x, s1.y * m2 + m1 * k2.y);
          au = cfma(coef, a.u[off + (int64_t)(i1 + o1) * A2.n + (i2 + o2)], au);
        }
      }
    } else {
      const AxisOp& A3 = a.ax[2];
      const int64_t n23 = (int64_t)A2.n * A3.n;
      const int i1 = (int)(i / n23);
      const int64_t rem = i - i1 * n23;
      const int i2 = (int)(rem / A3.n), i3 = (int)(rem % A3.n);
      for (int o1 = -1; o1 <= 1; ++o1) {
        const double m1 = m1d(A1.n, A1.h, i1, o1);
        if (m1 == 0.0) continue;
        const double2 k1 = k1d(A1.n, A1.h, A1.kLo, A1.kHi, i1, o1);
        const double2 s1 = make_double2(k1.x - a.w2 * m1, k1.y);
        for (int o2 = -1; o2 <= 1; ++o2) {
          const double m2 = m1d(A2.n, A2.h, i2, o2);
          if (m2 == 0.0) continue;
          const double2 k2 = k1d(A2.n, A2.h, A2.kLo, A2.kHi, i2, o2);
          for (int o3 = -1; o3 <= 1; ++o3) {
            const double m3 = m1d(A3.n, A3.h, i3, o3);
            if (m3 == 0.0) continue;
            const double2 k3 = k1d(A3.n, A3.h, A3.kLo, A3.kHi, i3, o3);
            // S1 M2 M3 + M1 K2 M3 + M1 M2 K3
            const double mm = m2 * m3;
            const double2 coef = make_double2(s1.x * mm + m1 * (k2.x * m3 + m2 * k3.x),
                                              s1.y * mm + m1 * (k2.y * m3 + m2 * k3.y));
            au = cfma(coef, a.u[off + (int64_t)(i1 + o1) * n23 + (int64_t)(i2 + o2) * A3.n + (i3 + o3)], au);
          }
        }
      }
    }
    const double2 fv = a.f[off + i];
    const double2 r = csub(fv, au);
    if (a.r) reinterpret_cast<TR*>(a.r)[off + i] = from_d2<TR>(r);
    sr = r.x * r.x + r.y * r.y;
    sf = fv.x * fv.x + fv.y * fv.y;
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

__global__ __launch_bounds__(kResThreads) void norm_finish_kernel(const double* scratch,
                                                                  int64_t blocks_per_rhs, double* norms) {
  __shared__ double red[2][kResThreads];
  const int64_t b = blockIdx.x;
  double sr = 0.0, sf = 0.0;
  for (int64_t i = threadIdx.x; i < blocks_per_rhs; i += kResThreads) {
    sr += scratch[2 * (b * blocks_per_rhs + i)];
    sf += scratch[2 * (b * blocks_per_rhs + i) + 1];
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
    norms[2 * b] = red[0][0];
    norms[2 * b + 1] = red[1][0];
  }
}

}  // namespace

int64_t residual_scratch_len(int dim, const int64_t* grid, int nb) {
  int64_t per = 1;
  for (int j = 0; j < dim; ++j) per *= grid[j];
  const int64_t bpr = (per + kResThreads - 1) / kResThreads;
  return 2 * bpr * nb;
}

hipError_t launch_residual(const ResidArgs& a, hipStream_t s) {
  int64_t per = 1;
  for (int j = 0; j < a.dim; ++j) per *= a.ax[j].n;
  const int64_t bpr = (per + kResThreads - 1) / kResThreads;
  const int64_t blocks = bpr * a.nb;
  if (blocks > 0x7fffffffLL || 2 * blocks > a.scratch_len) return hipErrorInvalidValue;
  if (a.r_kind == ST_C64)
    hipLaunchKernelGGL(residual_kernel<float2>, dim3((unsigned)blocks), dim3(kResThreads), 0, s, a, per, bpr);
  else
    hipLaunchKernelGGL(residual_kernel<double2>, dim3((unsigned)blocks), dim3(kResThreads), 0, s, a, per, bpr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(norm_finish_kernel, dim3((unsigned)a.nb), dim3(kResThreads), 0, s, a.scratch, bpr, a.norms);
  return hipGetLastError();
}

}  // namespace helm
