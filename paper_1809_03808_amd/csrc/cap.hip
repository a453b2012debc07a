// Boundary operators applied from precomputed tables.
//
// The boundary step of the three-step method (Step 2, eqs. (step2-1)-(step2-3))
// maps the two boundary vectors r_0, r_1 of a group of line systems to
//   w_k = sum_{k'} sum_j  V^b[k, j] V^b[k', j] T_j^{-1} r_{k'},
// a sum over the modes j of the other periodised direction of the inverses
// of that group's tridiagonal line matrices T_j.  The map depends on the
// operator only, so the plan evaluates it once as dense nL x nL blocks (one
// column per unit right-hand side, through the line solver), and every solve
// applies it as a batched complex matrix product instead of sweeping all
// N/nL lines again.  In 3D this replaces the Step-2 line sweep of every inner
// solve (groups = outer modes l, sum over the inner modes m) and the whole
// outer Step 2 (groups = inner absorbing modes m after the inner
// eigenvector transform, sum over the outer modes l).
//
// Kernel: blocks of 256 threads per (group, output rows (k, x)); each lane
// accumulates a tile of rows x right-hand sides in registers while streaming
// its rows of the table, which is read from memory once per launch for up to
// 16 right-hand sides.  The table is symmetric (T_j^{-1} is complex
// symmetric), so row r of the product reads column r of the stored blocks:
// consecutive lanes read consecutive addresses.  The input vectors are the
// same for every lane of a wave, so their loads are uniform (scalar) loads.
#include "helm_internal.h"

namespace helm {

namespace {

constexpr int kCapThreads = 256;

// Register tile: each lane computes TM rows (r0 + lane + 64 i) times TN
// right-hand sides; RG waves of a block share its rows and take consecutive
// groups of TN right-hand sides, so a block covers 256 * TM / RG rows and
// RG * TN right-hand sides per pass over the table.  Table entries of type
// TT (complex128, or complex64 for the mixed-precision path) are widened to
// FP64 and accumulated in FP64.
template <typename TT, int TM, int TN, int RG>
__global__ __launch_bounds__(kCapThreads) void cap_apply_kernel(const TT* __restrict__ T0,
                                                                const TT* __restrict__ T1,
                                                                const double2* __restrict__ in,
                                                                double2* __restrict__ out, CapArgs a) {
  constexpr int RPB = 64 * TM * (4 / RG);  // rows per block
  if (a.skip && *a.skip) return;
  const int nL = a.nL, rows = 2 * nL;
  const int rt = (rows + RPB - 1) / RPB;
  const int g = (int)(blockIdx.x / rt);
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int rg = wv % RG;
  const int rbase = (int)(blockIdx.x % rt) * RPB + (wv / RG) * 64 * TM + ((int)threadIdx.x & 63);
  for (int b0 = rg * TN; b0 < a.nb; b0 += RG * TN) {
    double2 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = make_double2(0, 0);
    for (int kp = 0; kp < 2; ++kp) {
      const TT* T = (kp ? T1 : T0) + (int64_t)g * nL * rows;  // this group's [x'][rows] block
      // uniform (scalar) pointers to this wave's right-hand sides; those past
      // nb repeat the last one and their products are dropped
      const double2* X[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        X[j] = in + (int64_t)(b0 + j < a.nb ? b0 + j : a.nb - 1) * a.in_b + (int64_t)g * a.in_g + kp * a.in_k;
      int ro[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) ro[i] = min(rbase + 64 * i, rows - 1);
      // four table rows per iteration in flight (512^3 x 16, complex64
      // tables: 1.77 ms per launch unrolled twice, 1.57 four times, 1.73
      // eight times)
#pragma unroll 4
      for (int xp = 0; xp < nL; ++xp) {
        double2 t[TM];
#pragma unroll
        for (int i = 0; i < TM; ++i) t[i] = to_d2(T[(int64_t)xp * rows + ro[i]]);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const double2 v = X[j][xp];
#pragma unroll
          for (int i = 0; i < TM; ++i) acc[i][j] = cfma(t[i], v, acc[i][j]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = rbase + 64 * i;
      if (r < rows) {
        const int k = r >= nL ? 1 : 0, x = r - k * nL;
        double2* o = out + (int64_t)g * a.out_g + k * a.out_k + x;
#pragma unroll
        for (int j = 0; j < TN; ++j)
          if (b0 + j < a.nb) o[(int64_t)(b0 + j) * a.out_b] = acc[i][j];
      }
    }
  }
}

// Sixteen right-hand sides per pass, one row per lane, every wave of a block
// on its own rows: the table is fetched once per 16 right-hand sides.  The
// boundary vectors of the block's group go through LDS in chunks of kCapXC
// entries (every lane of a wave reads the same entry: broadcasts), which
// keeps the 16 vectors out of the scalar registers.
constexpr int kCapXC = 32;

template <typename TT>
__global__ __launch_bounds__(kCapThreads) void cap_apply16_kernel(const TT* __restrict__ T0,
                                                                  const TT* __restrict__ T1,
                                                                  const double2* __restrict__ in,
                                                                  double2* __restrict__ out, CapArgs a) {
  constexpr int TN = 16;
  __shared__ double2 xs[TN][kCapXC];
  if (a.skip && *a.skip) return;
  const int nL = a.nL, rows = 2 * nL;
  const int rt = (rows + kCapThreads - 1) / kCapThreads;
  const int g = (int)(blockIdx.x / rt);
  const int r = (int)(blockIdx.x % rt) * kCapThreads + (int)threadIdx.x;
  const int ro = min(r, rows - 1);
  for (int b0 = 0; b0 < a.nb; b0 += TN) {
    double2 acc[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[j] = make_double2(0, 0);
    for (int kp = 0; kp < 2; ++kp) {
      const TT* T = (kp ? T1 : T0) + (int64_t)g * nL * rows + ro;  // column ro of this group's [x'][rows] block
      for (int x0 = 0; x0 < nL; x0 += kCapXC) {
        __syncthreads();  // the previous chunk is consumed
        for (int e = (int)threadIdx.x; e < TN * kCapXC; e += kCapThreads) {
          const int j = e / kCapXC, x = x0 + (e - j * kCapXC);
          // right-hand sides past nb repeat the last one; their products are dropped
          const int b = b0 + j < a.nb ? b0 + j : a.nb - 1;
          xs[j][e - j * kCapXC] =
              x < nL ? in[(int64_t)b * a.in_b + (int64_t)g * a.in_g + (int64_t)kp * a.in_k + x] : make_double2(0, 0);
        }
        __syncthreads();
        const int xn = min(kCapXC, nL - x0);
#pragma unroll 4
        for (int x = 0; x < xn; ++x) {
          const double2 t = to_d2(T[(int64_t)(x0 + x) * rows]);
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[j] = cfma(t, xs[j][x], acc[j]);
        }
      }
    }
    if (r < rows) {
      const int k = r >= nL ? 1 : 0, x = r - k * nL;
      double2* o = out + (int64_t)g * a.out_g + k * a.out_k + x;
#pragma unroll
      for (int j = 0; j < TN; ++j)
        if (b0 + j < a.nb) o[(int64_t)(b0 + j) * a.out_b] = acc[j];
    }
  }
}

template <typename TT>
hipError_t launch_16(const CapArgs& a, hipStream_t s) {
  const int64_t blocks = (int64_t)a.G * ((2 * a.nL + kCapThreads - 1) / kCapThreads);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((cap_apply16_kernel<TT>), dim3((unsigned)blocks), dim3(kCapThreads), 0, s,
                     reinterpret_cast<const TT*>(a.T0), reinterpret_cast<const TT*>(a.T1), a.in, a.out, a);
  return hipGetLastError();
}

template <typename TT, int TM, int TN, int RG>
hipError_t launch_nbc(const CapArgs& a, hipStream_t s) {
  constexpr int RPB = 64 * TM * (4 / RG);
  const int64_t blocks = (int64_t)a.G * ((2 * a.nL + RPB - 1) / RPB);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((cap_apply_kernel<TT, TM, TN, RG>), dim3((unsigned)blocks), dim3(kCapThreads), 0, s,
                     reinterpret_cast<const TT*>(a.T0), reinterpret_cast<const TT*>(a.T1), a.in, a.out, a);
  return hipGetLastError();
}

template <typename TT>
hipError_t launch_typed(const CapArgs& a, hipStream_t s) {
  // Up to 8 right-hand sides: TN per wave (the smallest power of two
  // covering nb, at most 4), 4 rows per lane, and RG waves sharing rows.
  // More, with complex128 tables: cap_apply16_kernel (sharing rows, the
  // waves fetched the table 1.7 times at 512^3 x 16; 2.56 -> 2.45 ms per
  // launch).  With complex64 tables four waves sharing rows stay faster
  // (1.78 against 2.31 ms per launch at 512^3 x 16: the LDS reads of the
  // vectors outweigh the saved fetch).
  if (a.nb <= 1) return launch_nbc<TT, 4, 1, 1>(a, s);
  if (a.nb <= 2) return launch_nbc<TT, 4, 2, 1>(a, s);
  if (a.nb <= 4) return launch_nbc<TT, 4, 4, 1>(a, s);
  if (a.nb <= 8) return launch_nbc<TT, 4, 4, 2>(a, s);
  if constexpr (sizeof(TT) == sizeof(double2)) return launch_16<TT>(a, s);
  return launch_nbc<TT, 4, 4, 4>(a, s);
}

// dst[g][x'][r] = src[x'][g][r] (r < 2 nL), narrowed to complex64 if TT is.
template <typename TT>
__global__ void cap_reorder_kernel(const double2* __restrict__ src, TT* __restrict__ dst, int G, int nL) {
  const int64_t rows = 2 * (int64_t)nL;
  const int64_t i = (int64_t)blockIdx.x * kCapThreads + threadIdx.x;
  if (i >= (int64_t)G * nL * rows) return;
  const int64_t r = i % rows, xg = i / rows;  // xg = g * nL + x'
  const int64_t xp = xg % nL, g = xg / nL;
  dst[i] = from_d2<TT>(src[(xp * G + g) * rows + r]);
}

}  // namespace

hipError_t launch_cap_apply(const CapArgs& a, hipStream_t s) {
  if (a.nb < 1 || a.G < 1 || a.nL < 1 || !a.T0 || !a.T1 || !a.in || !a.out) return hipErrorInvalidValue;
  return a.t_fp32 ? launch_typed<float2>(a, s) : launch_typed<double2>(a, s);
}

hipError_t launch_cap_reorder(const double2* src, void* dst, int G, int nL, bool fp32, hipStream_t s) {
  const int64_t n = (int64_t)G * nL * 2 * nL;
  const int64_t blocks = (n + kCapThreads - 1) / kCapThreads;
  if (n <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (fp32)
    hipLaunchKernelGGL(cap_reorder_kernel<float2>, dim3((unsigned)blocks), dim3(kCapThreads), 0, s, src,
                       reinterpret_cast<float2*>(dst), G, nL);
  else
    hipLaunchKernelGGL(cap_reorder_kernel<double2>, dim3((unsigned)blocks), dim3(kCapThreads), 0, s, src,
                       reinterpret_cast<double2*>(dst), G, nL);
  return hipGetLastError();
}

}  // namespace helm
