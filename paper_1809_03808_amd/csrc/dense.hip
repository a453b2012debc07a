// Dense eigenvector transforms on the matrix cores.
//
// With the full generalized eigenvectors of the periodised axis, K V = M V L
// and V^T M V = I (eqs. (EVP1a), (EVPcondA)), the 2D operator factors as
// A = (V^{-T} (x) I) (L (x) M_2 + I (x) (K_2 - w^2 M_2)) (V^{-1} (x) I), so
//   u = (V (x) I) blockdiag_l(T^A_l)^{-1} (V^T (x) I) f,
// the direct diagonalisation the paper writes in eq. (A2Dinv); in 3D the
// same holds with V_1 (x) V_2.  It needs no boundary steps at all; its cost
// is two dense transforms of 8 n flops per unknown each, which pays at small
// n where the transform is cheap and the three line passes of the fast
// method are not.
//
// The transform along the slow axis of a batch of [n][S] blocks,
//   out[b][m][x] (+)= sum_i Q[i][m] in[b][i][x],
// is a complex GEMM C = Q^T B evaluated with real 16x16x4 MFMA tiles
// (four real products per complex one).  A 256-thread block computes a 64 x 64
// output tile; each wave owns a 32 x 32 quarter (2 x 2 MFMA tiles, real and
// imaginary accumulators).  K steps of 16 are staged through two LDS buffers
// in planar (real / imaginary) form, padded against bank conflicts, with the
// next step's global loads in flight during the current step's products.
#include "helm_internal.h"

namespace helm {

namespace {

constexpr int kBM = 64, kBN = 64, kBK = 16, kPad = 4;

template <typename C> struct RealT;
template <> struct RealT<double2> { using T = double; };
template <> struct RealT<float2> { using T = float; };

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename R> struct Mma;
// f64 16x16x4: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; output
// register r of lane l is D[l / 16 + 4 r][l % 16].
template <> struct Mma<double> {
  using acc = d4v;
  __device__ static acc op(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return lane / 16 + 4 * r; }
};
// f32 16x16x4: same operand layout; output register r of lane l is
// D[4 (l / 16) + r][l % 16].
template <> struct Mma<float> {
  using acc = f4v;
  __device__ static acc op(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

template <typename R, typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void dense_kernel(DenseArgs a) {
  using M = Mma<R>;
  using acc = typename M::acc;
  __shared__ R Ar[2][kBK][kBM + kPad], Ai[2][kBK][kBM + kPad], Br[2][kBK][kBN + kPad], Bi[2][kBK][kBN + kPad];
  if (a.skip && *a.skip) return;
  const int n = a.n;
  const int64_t S = a.S;
  const int mt = (n + kBM - 1) / kBM;
  const int64_t xt = (S + kBN - 1) / kBN;
  int64_t blk = blockIdx.x;
  const int64_t xi = blk % xt;
  blk /= xt;
  const int mi = (int)(blk % mt);
  const int64_t beta = blk / mt;
  const int m0 = mi * kBM;
  const int64_t x0 = xi * kBN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const TIN* in = reinterpret_cast<const TIN*>(a.in) + beta * (int64_t)n * S;
  const R* Q = reinterpret_cast<const R*>(a.Q);  // interleaved complex [n][n]

  acc cr[2][2], ci[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      cr[t][u] = acc{0, 0, 0, 0};
      ci[t][u] = acc{0, 0, 0, 0};
    }

  // Software pipeline: the global loads of K tile k + 1 are issued into
  // registers before the products of tile k, then parked in the other LDS
  // buffer; one barrier per tile separates the writes of a buffer from the
  // reads of it two tiles earlier.
  constexpr int kPer = kBK * kBM / 256;  // elements of each operand tile per thread
  R qa[kPer][2], qb[kPer][2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = (int)threadIdx.x + 256 * t;
      {  // A[m][k] = Q[k][m], rows k of Q are contiguous in m
        const int kk = e / kBM, mm = e % kBM;
        const int i = k0 + kk, m = m0 + mm;
        qa[t][0] = 0;
        qa[t][1] = 0;
        if (i < n && m < n) {
          qa[t][0] = Q[2 * ((int64_t)i * n + m)];
          qa[t][1] = Q[2 * ((int64_t)i * n + m) + 1];
        }
      }
      {  // B: rows k of the input block, contiguous in x
        const int kk = e / kBN, xx = e % kBN;
        const int i = k0 + kk;
        const int64_t x = x0 + xx;
        qb[t][0] = 0;
        qb[t][1] = 0;
        if (i < n && x < S) {
          const TIN v = in[(int64_t)i * S + x];
          qb[t][0] = (R)v.x;
          qb[t][1] = (R)v.y;
        }
      }
    }
  };
  auto park = [&](int buf) {
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = (int)threadIdx.x + 256 * t;
      Ar[buf][e / kBM][e % kBM] = qa[t][0];
      Ai[buf][e / kBM][e % kBM] = qa[t][1];
      Br[buf][e / kBN][e % kBN] = qb[t][0];
      Bi[buf][e / kBN][e % kBN] = qb[t][1];
    }
  };
  fetch(0);
  park(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < n; k0 += kBK) {
    const bool more = k0 + kBK < n;
    if (more) fetch(k0 + kBK);
#pragma unroll
    for (int ks = 0; ks < kBK; ks += 4) {
      const int kl = ks + lane / 16, c16 = lane % 16;
      R ar[2], ai[2], an[2], br[2], bi[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ar[t] = Ar[buf][kl][wm + 16 * t + c16];
        ai[t] = Ai[buf][kl][wm + 16 * t + c16];
        an[t] = -ai[t];
        br[t] = Br[buf][kl][wn + 16 * t + c16];
        bi[t] = Bi[buf][kl][wn + 16 * t + c16];
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          cr[t][u] = M::op(ar[t], br[u], cr[t][u]);
          cr[t][u] = M::op(an[t], bi[u], cr[t][u]);
          ci[t][u] = M::op(ar[t], bi[u], ci[t][u]);
          ci[t][u] = M::op(ai[t], br[u], ci[t][u]);
        }
    }
    if (more) park(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  TOUT* out = reinterpret_cast<TOUT*>(a.out) + beta * (int64_t)n * S;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * t + M::row(lane, r);
        const int64_t x = x0 + wn + 16 * u + lane % 16;
        if (m < n && x < S) {
          double vr = (double)cr[t][u][r] * a.scale, vi = (double)ci[t][u][r] * a.scale;
          TOUT* o = out + (int64_t)m * S + x;
          if (a.accumulate) {
            vr += (double)o->x;
            vi += (double)o->y;
          }
          TOUT w;
          w.x = (typename RealT<TOUT>::T)vr;
          w.y = (typename RealT<TOUT>::T)vi;
          *o = w;
        }
      }
}

template <typename R, typename TIN>
hipError_t launch_in(const DenseArgs& a, int64_t blocks, hipStream_t s) {
  if (a.out_kind == ST_C64)
    hipLaunchKernelGGL((dense_kernel<R, TIN, float2>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((dense_kernel<R, TIN, double2>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_dense(const DenseArgs& a, bool fp32, hipStream_t s) {
  if (a.n < 1 || a.S < 1 || a.batch < 1 || !a.Q || !a.in || !a.out) return hipErrorInvalidValue;
  const int64_t blocks = a.batch * ((a.n + kBM - 1) / kBM) * ((a.S + kBN - 1) / kBN);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (fp32) {
    if (a.in_kind == ST_C64) return launch_in<float, float2>(a, blocks, s);
    return launch_in<float, double2>(a, blocks, s);
  }
  if (a.in_kind == ST_C64) return launch_in<double, float2>(a, blocks, s);
  return launch_in<double, double2>(a, blocks, s);
}

}  // namespace helm
