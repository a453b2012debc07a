// Boundary kernels of Steps 2 and 3.
//
// B - A is non-zero only on the two end nodes of the periodised axis (eq.
// (BminA)); its non-zero block C_bb (eq. (Cbb)) is never formed: with the 2x2
// differences dK = K^B - K and dM = M^B - M of that axis,
//   2D:  C = (dK_1 - w^2 dM_1) (x) M_2 + dM_1 (x) K_2,
//   3D:  C = (dK_1 - w^2 dM_1) (x) M_2 (x) M_3 + dM_1 (x) (K_2 (x) M_3 + M_2 (x) K_3),
// and on the inner level of 3D (the shifted 2D problems of eqs. (A2D2)-(B2D2aux))
//   C_2(p) = (dK_2 - p dM_2) (x) M_3 + dM_2 (x) K_3,  p = w^2 - lambda_{1,l}.
// These kernels sum the per-tile partial reductions of the line solves into
// the boundary values v_b, w_b (eqs. (2dBs1), (step2-3)) and apply C to them
// (eqs. (step2-1), (step3term)).
#include "helm_internal.h"
#include "ops1d.h"

namespace helm {

namespace {

constexpr int kMidThreads = 256;

__global__ __launch_bounds__(kMidThreads) void sum_partials_kernel(const double2* __restrict__ part,
                                                                   int64_t ngroups, int ntiles, int nL,
                                                                   double2* __restrict__ out, const int* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * kMidThreads + threadIdx.x;
  const int64_t per = 2 * (int64_t)nL;
  if (i >= ngroups * per) return;
  const int64_t g = i / per, r = i - g * per;
  const double2* p = part + g * ntiles * per + r;
  double2 s = make_double2(0, 0);
  for (int t = 0; t < ntiles; ++t) s = cadd(s, p[t * per]);
  out[i] = s;
}

// One block per (group, 30 columns): NT / 32 tile slices x 32 columns (the 30
// outputs plus a halo of one on each side) sum the partials in parallel, the
// slices are combined in LDS in a fixed order, then the 2x2 block operator is
// applied.  With many partial tiles per group (few groups, long lines: the
// 2D case) the partial sums are the bulk of the traffic and there are few
// blocks, so blocks of 1024 threads keep more loads in flight.
constexpr int kMidCols = 32;
constexpr int kMidOut = kMidCols - 2;

template <int NT>
__global__ __launch_bounds__(NT) void inner_mid_kernel(InnerMidArgs a) {
  constexpr int kMidSlices = NT / kMidCols;
  __shared__ double2 sl[kMidSlices][2][kMidCols];
  __shared__ double2 v[2][kMidCols];
  if (a.skip && *a.skip) return;
  const int nL = a.nL;
  const int ntx = (nL + kMidOut - 1) / kMidOut;
  const int64_t g = blockIdx.x / ntx;
  const int x0 = (int)(blockIdx.x % ntx) * kMidOut;
  const int64_t per = 2 * (int64_t)nL;
  {
    const int xi = threadIdx.x % kMidCols, ts = threadIdx.x / kMidCols;
    const int x = x0 - 1 + xi;
    double2 s0 = make_double2(0, 0), s1 = make_double2(0, 0);
    if (x >= 0 && x < nL) {
      const double2* p = a.part + g * a.ntiles * per + x;
#pragma unroll 4
      for (int t = ts; t < a.ntiles; t += kMidSlices) {
        s0 = cadd(s0, p[t * per]);
        s1 = cadd(s1, p[t * per + nL]);
      }
    }
    sl[ts][0][xi] = s0;
    sl[ts][1][xi] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2 * kMidCols) {
    const int k = threadIdx.x / kMidCols, xi = threadIdx.x % kMidCols;
    const int x = x0 - 1 + xi;
    double2 acc = make_double2(0, 0);
    for (int ts = 0; ts < kMidSlices; ++ts) acc = cadd(acc, sl[ts][k][xi]);
    if (x >= 0 && x < nL) {
      if (a.vb_out && xi >= 1 && xi <= kMidOut) a.vb_out[g * per + k * nL + x] = acc;
      if (a.vb_in) acc = cadd(acc, a.vb_in[g * per + k * nL + x]);
    } else {
      acc = make_double2(0, 0);
    }
    v[k][xi] = acc;
  }
  __syncthreads();
  if (threadIdx.x >= kMidOut) return;
  const int x = x0 + threadIdx.x;
  if (x >= nL) return;
  const int64_t l = g % a.nO;
  double2 p = make_double2(-a.sC.x, -a.sC.y);
  if (a.sO) p = csub(p, a.sO[l]);
  // A = dK - p dM (2x2 complex)
  double2 A[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      A[i][j] = make_double2(a.d.dK[i][j].x - p.x * a.d.dM[i][j], a.d.dK[i][j].y - p.y * a.d.dM[i][j]);
  double2 Mv[2], Kv[2];
  for (int k = 0; k < 2; ++k) {
    Mv[k] = make_double2(0, 0);
    Kv[k] = make_double2(0, 0);
    for (int o = -1; o <= 1; ++o) {
      const double2 vv = v[k][threadIdx.x + 1 + o];
      Mv[k] = cadd(Mv[k], cscale(vv, m1d(nL, a.hL, x, o)));
      Kv[k] = cfma(k1d(nL, a.hL, a.kLo, a.kHi, x, o), vv, Kv[k]);
    }
  }
  for (int k = 0; k < 2; ++k) {
    double2 r = make_double2(0, 0);
    for (int kp = 0; kp < 2; ++kp) {
      r = cfma(A[k][kp], Mv[kp], r);
      r = cadd(r, cscale(Kv[kp], a.d.dM[k][kp]));
    }
    if (a.out_c64) reinterpret_cast<float2*>(a.out)[g * per + k * nL + x] = make_float2((float)r.x, (float)r.y);
    else a.out[g * per + k * nL + x] = r;
  }
}

// Outer operator on physical planes [nb][2][n2][n3]; one thread per (b, i2, i3).
__global__ __launch_bounds__(kMidThreads) void outer_mid_kernel(OuterMidArgs a) {
  if (a.skip && *a.skip) return;
  const int64_t plane = (int64_t)a.n2 * a.n3;
  const int64_t idx = (int64_t)blockIdx.x * kMidThreads + threadIdx.x;
  if (idx >= (int64_t)a.nb * plane) return;
  const int64_t b = idx / plane;
  const int64_t rem = idx - b * plane;
  const int i2 = (int)(rem / a.n3), i3 = (int)(rem % a.n3);
  double2 MM[2], KS[2];  // (M2 (x) M3) v_k and (K2 (x) M3 + M2 (x) K3) v_k
  for (int k = 0; k < 2; ++k) {
    MM[k] = make_double2(0, 0);
    KS[k] = make_double2(0, 0);
    const int64_t pb = (b * 2 + k) * plane;
    for (int o2 = -1; o2 <= 1; ++o2) {
      const double m2 = m1d(a.n2, a.h2, i2, o2);
      const double2 kk2 = k1d(a.n2, a.h2, a.k2Lo, a.k2Hi, i2, o2);
      if (m2 == 0.0) continue;
      for (int o3 = -1; o3 <= 1; ++o3) {
        const double m3 = m1d(a.n3, a.h3, i3, o3);
        if (m3 == 0.0) continue;
        const double2 kk3 = k1d(a.n3, a.h3, a.k3Lo, a.k3Hi, i3, o3);
        const int64_t j = pb + (int64_t)(i2 + o2) * a.n3 + (i3 + o3);
        double2 vv = a.a[j];
        if (a.c) vv = cadd(vv, a.c[j]);
        MM[k] = cadd(MM[k], cscale(vv, m2 * m3));
        // K2(i2,o2) M3(i3,o3) + M2(i2,o2) K3(i3,o3)
        const double2 coef = make_double2(kk2.x * m3 + m2 * kk3.x, kk2.y * m3 + m2 * kk3.y);
        KS[k] = cfma(coef, vv, KS[k]);
      }
    }
  }
  for (int k = 0; k < 2; ++k) {
    double2 r = make_double2(0, 0);
    for (int kp = 0; kp < 2; ++kp) {
      const double2 A = make_double2(a.d1.dK[k][kp].x - a.w2 * a.d1.dM[k][kp], a.d1.dK[k][kp].y);
      r = cfma(A, MM[kp], r);
      r = cadd(r, cscale(KS[kp], a.d1.dM[k][kp]));
    }
    a.r[(b * 2 + k) * plane + rem] = r;
  }
}

}  // namespace

hipError_t launch_sum_partials(const double2* part, int ngroups, int ntiles, int nL, double2* out,
                               const int* skip, hipStream_t s) {
  const int64_t n = (int64_t)ngroups * 2 * nL;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + kMidThreads - 1) / kMidThreads;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)blocks), dim3(kMidThreads), 0, s, part,
                     (int64_t)ngroups, ntiles, nL, out, skip);
  return hipGetLastError();
}

hipError_t launch_inner_mid(const InnerMidArgs& a, hipStream_t s) {
  const int ntx = (a.nL + kMidOut - 1) / kMidOut;
  const int64_t blocks = (int64_t)a.nb * a.nO * ntx;
  if (blocks <= 0) return hipSuccess;
  if (a.ntiles >= 64)
    hipLaunchKernelGGL(inner_mid_kernel<1024>, dim3((unsigned)blocks), dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL(inner_mid_kernel<256>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_outer_mid(const OuterMidArgs& a, hipStream_t s) {
  const int64_t n = (int64_t)a.nb * a.n2 * a.n3;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + kMidThreads - 1) / kMidThreads;
  hipLaunchKernelGGL(outer_mid_kernel, dim3((unsigned)blocks), dim3(kMidThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace helm
