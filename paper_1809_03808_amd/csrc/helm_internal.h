// Internal declarations of the HIP fast Helmholtz solver (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/helm.h"
#include "eig1d.h"

namespace helm {

using cd = std::complex<double>;

// ---------------------------------------------------------------------------
// complex helpers on HIP vector types (x = re, y = im)
// ---------------------------------------------------------------------------
__host__ __device__ inline double2 mk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline float2 mk(float r, float i) { return make_float2(r, i); }
template <typename C> __device__ inline C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
template <typename C> __device__ inline C csub(C a, C b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename C> __device__ inline C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// a + b*c, as two fused multiply-adds per component (two roundings each)
template <typename C> __device__ inline C cfma(C b, C c, C a) {
  a.x = fma(b.x, c.x, a.x);
  a.x = fma(-b.y, c.y, a.x);
  a.y = fma(b.x, c.y, a.y);
  a.y = fma(b.y, c.x, a.y);
  return a;
}
// a - b*c, likewise
template <typename C> __device__ inline C cfms(C b, C c, C a) {
  a.x = fma(-b.x, c.x, a.x);
  a.x = fma(b.y, c.y, a.x);
  a.y = fma(-b.x, c.y, a.y);
  a.y = fma(-b.y, c.x, a.y);
  return a;
}
template <typename C, typename S> __device__ inline C cscale(C a, S s) { a.x *= s; a.y *= s; return a; }
__device__ inline double2 crcp(double2 a) {
  const double d = 1.0 / (a.x * a.x + a.y * a.y);
  return make_double2(a.x * d, -a.y * d);
}
// 1/d for a normal positive double: hardware reciprocal estimate refined by
// two Newton-Raphson steps r <- r + r (1 - d r) (each doubles the number of
// correct bits), about 1 ulp; cheaper than the IEEE division sequence.
__device__ inline double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double2 crcp_fast(double2 a) {
  const double d = rcp_nr(a.x * a.x + a.y * a.y);
  return make_double2(a.x * d, -a.y * d);
}
__device__ inline double2 to_d2(double2 a) { return a; }
__device__ inline double2 to_d2(float2 a) { return make_double2((double)a.x, (double)a.y); }
template <typename C> __device__ inline C from_d2(double2 a);
template <> __device__ inline double2 from_d2<double2>(double2 a) { return a; }
template <> __device__ inline float2 from_d2<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }

inline double2 hd2(cd z) { return make_double2(z.real(), z.imag()); }


// ---------------------------------------------------------------------------
// Batched strided DFT pass (fft.hip)
// Data viewed as [O][L (stride in_sj)][I (contiguous)]; a pass computes a
// length-L DFT for every (o, i) and writes output k of (o, i) to
//   (o / od) * out_so1 + (o % od) * out_so2 + k * out_sk + i,
// optionally multiplied by a four-step twiddle tw4[(k * (i / tw4_S)) % tw4_n]
// and a per-mode real scale scale[(o % od) + od * k] * scale_c.
// ---------------------------------------------------------------------------
enum StorageKind { ST_C128 = 0, ST_C64 = 1 };

struct FftPass {
  int L = 0;
  int nst = 0;
  int radix[8] = {0};
  int64_t I = 0, O = 0;
  int64_t od = 1;
  int64_t in_so = 0, in_sj = 0;
  int64_t out_so1 = 0, out_so2 = 0, out_sk = 0;
  int64_t tw4_S = 0;  // 0: no four-step twiddle
  int tw4_n = 0;
  int W = 0;          // inner columns per workgroup
  int small_tile = 0; // 512-point passes: 1 the 64 KB complex64 tile (two blocks per compute unit), 2 streaming
  int in_kind = ST_C128, out_kind = ST_C128;
  int accumulate = 0;
  int sign = -1;      // -1 forward (e^{-2 pi i ...}), +1 inverse
  double scale_c = 1.0;
  // device tables (double or float per compute precision), owned by the plan
  const void* tw = nullptr;    // L roots e^{sign 2 pi i t / L}
  const void* tw4 = nullptr;   // tw4_n roots
  const double* scale = nullptr;
  const void* cmode = nullptr;  // optional complex per-mode multiplier (compute precision)
  const int* skip = nullptr;    // device flag: when non-zero the pass does nothing
  // Chirp-z folding (compute precision tables): with the row map
  // x = col / chirp_S + chirp_na * row, the first stage loads in * cin[x] for
  // x < chirp_n and zero beyond, and the last stage stores y * cout[x] for
  // x < chirp_n only.
  const void* cin = nullptr;
  const void* cout = nullptr;
  int64_t chirp_n = 0, chirp_na = 1, chirp_S = 1;
  // Twiddle index of the last stage: 0 -> tw4[k a] with a = col / tw4_S
  // (four-step first pass), 1 -> tw4[k c] with c the group index within od.
  int tw4_mode = 0;
  int conj_out = 0;  // store the complex conjugate (before the twiddle)
};

// Inner columns per tile of a length-L pass (fixed per length and precision).
int fft_tile_width(int L, bool fp32);
// Middle of a chirp-z convolution: for every group (o, c) of the pass
// geometry, a length-L forward DFT over the rows, multiplication by
// cmode[c + od d] (the transformed chirp kernel), and the unscaled inverse
// DFT back over the rows, with the epilogue of the pass (tw4_mode 1 twiddle).
hipError_t launch_conv_pass(const FftPass& p, bool fp32, const void* in, void* out, hipStream_t s);
// Launch one pass.  `fp32` selects float arithmetic (tables in float).
hipError_t launch_fft_pass(const FftPass& p, bool fp32, const void* in, void* out,
                           hipStream_t s);


// ---------------------------------------------------------------------------
// Batched tridiagonal line solves (lines.hip)
// Line (b, l, m), b < nb, l < nO, m < nI, has the matrix
//   T = sigma M_L + K_L,  sigma = sO[l] + sI[m] + sC,
// with M_L = (hL/6) tridiag(1,4,1) (corners 2) and K_L = (1/hL) tridiag(-1,2,-1)
// with corner entries kLo/hL, kHi/hL, along the contiguous axis of length nL.
// Right-hand side:
//   in[b][l][m][:] (if in)  + sum_k alpha_k[l] PO[b][k][m][:]  (if PO)
//                           + sum_k beta_k[m]  PI[b][l][k][:]  (if PI)
// Output: store the solution to out[b][l][m][:] and/or reduce
//   red == 1: part[((b nO + l) ntiles + t)][k][:] = sum_{m in tile t} rho_k[m] y
//   red == 2: part[((b nI + m) ntiles + t)][k][:] = sum_{l in tile t} rho_k[l] y
//   red == 3: the sums of red == 2 with the lines of a block taken as
//             consecutive m at one l per iteration (all l in one tile)
// ---------------------------------------------------------------------------
struct LineArgs {
  int nb = 1, nO = 1, nI = 1, nL = 0;
  const double2* sO = nullptr;
  const double2* sI = nullptr;
  double2 sC = {0, 0};
  double hL = 0;
  double2 kLo = {1, 0}, kHi = {1, 0};
  const void* in = nullptr;
  int in_kind = ST_C128;
  // Rank-2 rows PO [nb][2][nI][nL] and PI [nb][nO][2][nL], in the storage
  // type of the launch's lines (that of in, or else of out; complex128 with
  // neither); r2_kind states their type and must match (checked)
  const double2* alpha0 = nullptr;
  const double2* alpha1 = nullptr;
  const void* PO = nullptr;
  const double2* beta0 = nullptr;
  const double2* beta1 = nullptr;
  const void* PI = nullptr;
  int r2_kind = ST_C128;
  void* out = nullptr;
  int out_kind = ST_C128;
  int red = 0;
  const double2* rho0 = nullptr;
  const double2* rho1 = nullptr;
  double2* part = nullptr;
  const double2* piv = nullptr;  // [nO*nI][P] reciprocal pivot entering each lane chunk
  const double2* sTab = nullptr; // [nO*nI] sigma of every line (replaces sO + sI + sC when set)
  int tile = 0;    // lines per workgroup tile
  int ntiles = 0;  // tiles along the reduced (or flattened) index
  const int* skip = nullptr;     // device flag: the launch does nothing while *skip != 0
  // Unit right-hand sides (plan setup only): with no `in`, line (b, l, m) has
  // the right-hand side e_b (b < nL), so that reductions of the solutions
  // assemble columns of reduced inverses (the boundary operator tables).
  int unit_rhs = 0;
  // Storing launches (red == 0): blocks take tiles of tile_l outer x tile_m
  // inner modes of one right-hand side (0: consecutive lines, `tile` each).
  int tile_l = 0, tile_m = 0;
};

hipError_t launch_lines(LineArgs a, hipStream_t s);
// Lanes per line P, rows per lane c and block size NT for a line length.
void lines_geometry(int nL, int* P, int* c, int* NT);
// Factor table of the line matrices (l, m), l < nO, m < nI, of `a` (sO, sI,
// sC and the line axis are used): piv[(l nI + m) P + q] = 1/p_{q c - 1}, the
// reciprocal Thomas pivot entering the chunk of lane q (P, c from
// lines_geometry; entry q = 0 is zero).  Computed once per plan.
hipError_t launch_line_factors(const LineArgs& a, double2* piv, hipStream_t s);

// ---------------------------------------------------------------------------
// Boundary operator tables (cap.hip): for every group g < G (an outer or an
// inner mode), the reduced inverse of that group's line matrices acting on
// two boundary vectors,
//   out[b][g][k][x] = sum_{k' < 2} sum_{x' < nL} T_{k'}[g][x'][k][x] in[b][g][k'][x'],
// with T_{k'} stored [G][nL (x')][2 (k)][nL (x)] (complex128, or complex64
// when t_fp32) and the vectors addressed by b * _b + g * _g + k * _k + x
// strides; accumulated in FP64.
// ---------------------------------------------------------------------------
struct CapArgs {
  int nb = 0, G = 0, nL = 0;
  const void* T0 = nullptr;
  const void* T1 = nullptr;
  int t_fp32 = 0;
  const double2* in = nullptr;
  int64_t in_b = 0, in_g = 0, in_k = 0;
  double2* out = nullptr;
  int64_t out_b = 0, out_g = 0, out_k = 0;
  const int* skip = nullptr;
};
hipError_t launch_cap_apply(const CapArgs& a, hipStream_t s);
// dst[g][x'][k][x] = src[x'][g][k][x] (G groups, 2 nL rows), narrowed to
// complex64 when fp32: the layout the line reductions produce -> the one the
// products stream.
hipError_t launch_cap_reorder(const double2* src, void* dst, int G, int nL, bool fp32, hipStream_t s);

// ---------------------------------------------------------------------------
// Dense eigenvector transforms on the matrix cores (dense.hip)
// ---------------------------------------------------------------------------
// out[b][m][x] = scale * sum_i Q[i][m] in[b][i][x] (+ out[b][m][x] if
// accumulate), b < batch, m, i < n, x < S; Q interleaved complex [n][n] in the
// compute precision (double, or float when fp32).  in and out must not overlap.
struct DenseArgs {
  int n = 0;
  int64_t S = 0, batch = 0;
  const void* Q = nullptr;
  const void* in = nullptr;
  int in_kind = ST_C128;
  void* out = nullptr;
  int out_kind = ST_C128;
  double scale = 1.0;
  int accumulate = 0;
  const int* skip = nullptr;
};
hipError_t launch_dense(const DenseArgs& a, bool fp32, hipStream_t s);

// ---------------------------------------------------------------------------
// Boundary kernels (boundary.hip)
// ---------------------------------------------------------------------------
// 2x2 boundary difference of a periodised axis (B - A restricted to its two
// end nodes): dK = (1/h)[[1 + i w h a_lo, -1], [-1, 1 + i w h a_hi]],
// dM = (h/6)[[2, 1], [1, 2]].
struct BDiff {
  double2 dK[2][2];
  double dM[2][2];
};

// Inner boundary operator for every (b, l): with v = sum over tiles of
// part[(b nO + l) ntiles + t][k][:] (+ vb_in[b][l][k][:] if add_vb),
//   out[b][l][k][:] = sum_k' (dK - p_l dM)[k][k'] M_L v_k' + dM[k][k'] K_L v_k',
//   p_l = -(sO[l] + sC)  (sO may be null -> p = -sC),
// and, if vb_out, vb_out[b][l][k][:] = v (the reduced boundary values).
struct InnerMidArgs {
  int nb, nO, nL, ntiles;
  const double2* part;
  const double2* vb_in;  // nullable
  double2* vb_out;       // nullable
  double2* out;
  int out_c64 = 0;       // store out in complex64 (the rank-2 rows of complex64 line launches)
  const double2* sO;
  double2 sC;
  BDiff d;
  double hL;
  double2 kLo, kHi;
  const int* skip = nullptr;
};
hipError_t launch_inner_mid(const InnerMidArgs& a, hipStream_t s);

// Sum partial planes: out[g][k][:] = sum_t part[g ntiles + t][k][:], g < ngroups.
hipError_t launch_sum_partials(const double2* part, int ngroups, int ntiles, int nL,
                               double2* out, const int* skip, hipStream_t s);

// Outer boundary operator on physical (x2, x3) planes (3D):
//   r[b][k] = sum_k' (dK1 - w^2 dM1)[k][k'] (M2 (x) M3) v_k' + dM1[k][k'] (K2 (x) M3 + M2 (x) K3) v_k'
// with v = a[b] (+ c[b] if c), planes [nb][2][n2][n3].
struct OuterMidArgs {
  int nb, n2, n3;
  const double2* a;
  const double2* c;  // nullable
  double2* r;
  BDiff d1;
  double w2;
  double h2, h3;
  double2 k2Lo, k2Hi, k3Lo, k3Hi;
  const int* skip = nullptr;
};
hipError_t launch_outer_mid(const OuterMidArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// Stencil residual and norms (stencil.hip)
// ---------------------------------------------------------------------------
struct AxisOp {
  int n;
  double h;
  double2 kLo, kHi;  // K corner entries times h
};
struct ResidArgs {
  int dim, nb;
  AxisOp ax[3];
  double w2;
  const double2* u;
  const double2* f;
  void* r;        // nullable
  int r_kind;     // ST_C128 / ST_C64
  double* norms;  // device [nb][2]: sum |r|^2, sum |f|^2 (accumulated by the finishing kernel)
  double* scratch;
  int64_t scratch_len;
  const int* skip = nullptr;  // device flag: nothing is computed while *skip != 0
};
hipError_t launch_residual(const ResidArgs& a, hipStream_t s);
int64_t residual_scratch_len(int dim, const int64_t* grid, int nb);


// Device eigen-setup (eigdev.hip): the eigenpairs of eig1d, computed on the
// current device on stream s; the whole eigenvectors, if `vecs` is given, go
// to the non-null device arrays there (V[i][l] = v_l(i), its transpose, and
// float copies of both, n x n each).
struct EigVecOut {
  double2 *Vd, *VTd;
  float2 *Vf, *VTf;
};
int eig1d_device(int n, double h, cd glo, cd ghi, std::vector<cd>& lam, std::vector<cd>& v0,
                 std::vector<cd>& v1, std::vector<cd>& lamlo, const EigVecOut* vecs, hipStream_t s);

}  // namespace helm
