// Batched strided DFT passes for gfx950.
//
// The forward eigen-transform of the periodic auxiliary problem is a DFT
// along a periodised axis with F[l, i] = e^{-2 pi i l i / n} (the eigenvector
// matrix of the circulant pencil, eq. (eigvectorsPer)), and the final
// transform is its inverse with the 1/n factor (eq. (step3IFFTz3coeff)).  The
// periodised axes are never the contiguous one, so each pass works on a tile
// [L][W] = (transform axis) x (W consecutive contiguous columns): global loads
// and stores are W*sizeof(complex) contiguous bytes per row, and the L-point
// transform runs as Stockham radix-2/4/8 stages through LDS.  The first stage
// reads global memory and the last stage writes it, so a pass touches HBM
// exactly once each way.  Long axes are split into two passes (four-step:
// n = n_a n_b, twiddle e^{-2 pi i a c/n} between the passes).
#include <algorithm>
#include <atomic>

#include "helm_internal.h"

namespace helm {

namespace {

constexpr int kFftThreads = 256;
#ifndef HELM_FFT_TILE_BYTES
#define HELM_FFT_TILE_BYTES 32768
#endif
#ifndef HELM_FFT_MAX_W
#define HELM_FFT_MAX_W 32
#endif
constexpr int kFftLdsBytes = HELM_FFT_TILE_BYTES;
constexpr int kFftMaxW = HELM_FFT_MAX_W;

template <typename C> struct RealOf;
template <> struct RealOf<double2> { using T = double; };
template <> struct RealOf<float2> { using T = float; };

template <typename C> __device__ inline C load_as(const void* base, int64_t idx, int kind) {
  if (kind == ST_C128) {
    const double2 v = reinterpret_cast<const double2*>(base)[idx];
    C r;
    r.x = (typename RealOf<C>::T)v.x;
    r.y = (typename RealOf<C>::T)v.y;
    return r;
  }
  const float2 v = reinterpret_cast<const float2*>(base)[idx];
  C r;
  r.x = (typename RealOf<C>::T)v.x;
  r.y = (typename RealOf<C>::T)v.y;
  return r;
}

template <typename C> __device__ inline void store_as(void* base, int64_t idx, int kind, C v, int acc) {
  if (kind == ST_C128) {
    double2* p = reinterpret_cast<double2*>(base) + idx;
    double2 w = make_double2((double)v.x, (double)v.y);
    if (acc) {
      const double2 o = *p;
      w.x += o.x;
      w.y += o.y;
    }
    *p = w;
  } else {
    float2* p = reinterpret_cast<float2*>(base) + idx;
    float2 w = make_float2((float)v.x, (float)v.y);
    if (acc) {
      const float2 o = *p;
      w.x += o.x;
      w.y += o.y;
    }
    *p = w;
  }
}

// multiply by (sign * i)
template <typename C> __device__ inline C mul_si(C a, int sign) {
  C r;
  if (sign > 0) { r.x = -a.y; r.y = a.x; }
  else { r.x = a.y; r.y = -a.x; }
  return r;
}

template <int R, typename C> __device__ inline void dft(C* v, int sign);

template <> __device__ inline void dft<2, double2>(double2* v, int) {
  const double2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <> __device__ inline void dft<2, float2>(float2* v, int) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename C> __device__ inline void dft4(C& x0, C& x1, C& x2, C& x3, int sign) {
  const C a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = mul_si(csub(x1, x3), sign);
  x0 = cadd(a, c);
  x1 = cadd(b, d);
  x2 = csub(a, c);
  x3 = csub(b, d);
}

template <> __device__ inline void dft<4, double2>(double2* v, int sign) { dft4(v[0], v[1], v[2], v[3], sign); }
template <> __device__ inline void dft<4, float2>(float2* v, int sign) { dft4(v[0], v[1], v[2], v[3], sign); }

template <typename C> __device__ inline void dft8(C* v, int sign) {
  using T = typename RealOf<C>::T;
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3, sign);
  dft4(o0, o1, o2, o3, sign);
  const T c = (T)0.70710678118654752440;
  // w^1 = c(1 + s i), w^2 = s i, w^3 = c(-1 + s i)
  C t1, t3;
  {
    const C si = mul_si(o1, sign);
    t1.x = c * (o1.x + si.x);
    t1.y = c * (o1.y + si.y);
  }
  const C t2 = mul_si(o2, sign);
  {
    const C si = mul_si(o3, sign);
    t3.x = c * (si.x - o3.x);
    t3.y = c * (si.y - o3.y);
  }
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}
template <> __device__ inline void dft<8, double2>(double2* v, int sign) { dft8(v, sign); }
template <> __device__ inline void dft<8, float2>(float2* v, int sign) { dft8(v, sign); }

// 3-point DFT with w = e^{sign 2 pi i / 3} = -1/2 + sign i sqrt(3)/2:
// X0 = x0 + (x1 + x2), X1,2 = x0 - (x1 + x2)/2 +- sign i (sqrt(3)/2)(x1 - x2).
template <typename C> __device__ inline void dft3(C* v, int sign) {
  using T = typename RealOf<C>::T;
  const T h = (T)0.86602540378443864676;  // sqrt(3)/2
  const C t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
  C m;
  m.x = v[0].x - (T)0.5 * t1.x;
  m.y = v[0].y - (T)0.5 * t1.y;
  C q = mul_si(t2, sign);
  q.x *= h;
  q.y *= h;
  v[0] = cadd(v[0], t1);
  v[1] = cadd(m, q);
  v[2] = csub(m, q);
}
template <> __device__ inline void dft<3, double2>(double2* v, int sign) { dft3(v, sign); }
template <> __device__ inline void dft<3, float2>(float2* v, int sign) { dft3(v, sign); }

struct PassDev {
  int sign, acc, in_kind, out_kind;
  const void* cmode;
  const int* skip;
  const void* cin;
  const void* cout;
  int64_t chirp_n, chirp_na, chirp_S;
  int tw4_mode, conj_out;
  int64_t I, od, in_so, in_sj, out_so1, out_so2, out_sk, tw4_S;
  int64_t ntile;  // tiles along I
  double scale_c;
  const void* tw;
  const void* tw4;
  const double* scale;
};

// Compile-time Stockham plan of a power-of-two length L: one radix-2 or -4
// stage first when log2(L) is not a multiple of 3, then radix-8 stages.
// Lengths 9 * 2^k (the convolution pass of a chirp-z transform of length
// 9 * 2^j) take the power-of-two stages of 2^k followed by two radix-3
// stages.
constexpr int ilog2(int L) { return L <= 1 ? 0 : 1 + ilog2(L / 2); }
constexpr bool has9(int L) { return L % 9 == 0; }
constexpr int p2part(int L) { return has9(L) ? L / 9 : L; }
constexpr int nst2(int L2) { return ilog2(L2) / 3 + (ilog2(L2) % 3 ? 1 : 0); }
constexpr int nstages(int L) { return nst2(p2part(L)) + (has9(L) ? 2 : 0); }
constexpr int radix_of(int L, int s) {
  return s >= nst2(p2part(L)) ? 3
                              : ((ilog2(p2part(L)) % 3 && s == 0) ? (ilog2(p2part(L)) % 3 == 1 ? 2 : 4) : 8);
}
constexpr int pow2_floor(int x) { return x < 2 ? 1 : 2 * pow2_floor(x / 2); }
// Columns per tile: an LDS tile of L x W complex values, W <= kFftMaxW.
// 32 KB tiles keep several blocks resident per compute unit.  The longest
// passes (L = 512) take 128 KB tiles (16 complex128 columns: 256-byte row
// segments) with 1024 threads, one block per compute unit: against 64 KB
// tiles of 256 threads (128-byte segments, two blocks) the pass over a
// 512^3 x 16 volume takes 17% less time.
constexpr int tile_bytes(int L) { return L >= 512 ? 4 * kFftLdsBytes : kFftLdsBytes; }
constexpr int threads_of(int L) { return L >= 512 ? 4 * kFftThreads : kFftThreads; }
template <typename C> constexpr int tile_w(int L) {
  return pow2_floor((tile_bytes(L) / (L * (int)sizeof(C))) < kFftMaxW ? tile_bytes(L) / (L * (int)sizeof(C))
                                                                       : kFftMaxW);
}
// A second tile for the complex64 512-point pass, chosen per plan by the
// tuner: 64 KB (16 columns, 128-byte row segments) with the same 1024
// threads, so that two blocks share a compute unit and one block's loads
// overlap the other's LDS stages.  WO = 0 is the default tile.
template <int L, typename C, int WO> constexpr int tile_w_of() { return WO ? WO : tile_w<C>(L); }
template <int L, typename C, int WO> constexpr int min_waves_of() { return WO ? 8 : 1; }

// One Stockham stage of radix R with Ns points already combined.  Thread
// tid of NT = threads_of(L) owns butterflies t = tid + q*NT, t -> (j = t / W,
// w = t % W); since W divides NT, w = tid % W for every q.  All reads of a
// stage precede the barrier and all writes follow it, so the stage works in
// place in LDS.  The first stage reads global memory, the last writes it
// (with the four-step twiddle, the per-mode scale and the optional
// accumulation).
template <int L, int W, int R, int Ns, bool FIRST, bool LAST, typename C, bool GIN = true, bool GOUT = true,
          bool REG = false>
__device__ inline void stage(const PassDev& p, C* sm, const void* in, void* out, int64_t o, int64_t i0,
                             int64_t oq, int64_t orr, int64_t a4, const C* vin, int tid) {
  constexpr bool LOADG = FIRST && GIN;    // this stage reads global memory
  constexpr bool STOREG = LAST && GOUT;   // this stage writes global memory
  constexpr int LR = L / R;
  constexpr int NBF = LR * W;
  constexpr int NT = threads_of(L);
  static_assert(NT % W == 0 && L * W * (int)sizeof(C) <= 160 * 1024, "tile does not fit the thread block or LDS");
  constexpr int NB = (NBF + NT - 1) / NT;
  const int w = tid % W;
  const int64_t col = i0 + w;
  const bool colok = col < p.I;
  const C* tw = reinterpret_cast<const C*>(p.tw);
  C v[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int t = tid + q * NT;
    if (NB * NT == NBF || t < NBF) {
      const int j = t / W;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = j + r * LR;
        if constexpr (LOADG && REG) {
          v[q][r] = vin[q * R + r];  // loaded by the caller
        } else if constexpr (LOADG) {
          C x;
          x.x = 0;
          x.y = 0;
          if (p.cin) {
            const int64_t xr = col / p.chirp_S + p.chirp_na * row;
            if (colok && xr < p.chirp_n)
              x = cmul(load_as<C>(in, o * p.in_so + (int64_t)row * p.in_sj + col, p.in_kind),
                       reinterpret_cast<const C*>(p.cin)[xr]);
          } else if (colok) {
            x = load_as<C>(in, o * p.in_so + (int64_t)row * p.in_sj + col, p.in_kind);
          }
          v[q][r] = x;
        } else {
          v[q][r] = sm[row * W + w];
        }
      }
    }
  }
  if constexpr (!LOADG) __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int t = tid + q * NT;
    if (NB * NT == NBF || t < NBF) {
      const int j = t / W;
      const int k = j % Ns;
      if constexpr (Ns > 1) {
        constexpr int step = L / (Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], tw[r * k * step]);
      }
      dft<R, C>(v[q], p.sign);
      const int base = (j / Ns) * Ns * R + k;
      if constexpr (!STOREG) {
#pragma unroll
        for (int r = 0; r < R; ++r) sm[(base + r * Ns) * W + w] = v[q][r];
      } else {
        if (colok) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int kk = base + r * Ns;  // output frequency of this pass
            // mode index of the per-mode factors: the chirp row map when
            // folding a chirp, else the pass's own output index
            int64_t mi = orr + p.od * kk;
            if (p.cout) {
              mi = col / p.chirp_S + p.chirp_na * kk;
              if (mi >= p.chirp_n) continue;  // rows past the transform length are not stored
            }
            C y = v[q][r];
            if (p.conj_out) y.y = -y.y;
            if (p.tw4) {
              // kk < L and the multiplier < n / L, so the index stays below n
              const C* t4 = reinterpret_cast<const C*>(p.tw4);
              y = cmul(y, t4[kk * (p.tw4_mode ? orr : a4)]);
            }
            if (p.cmode) y = cmul(y, reinterpret_cast<const C*>(p.cmode)[mi]);
            if (p.cout) y = cmul(y, reinterpret_cast<const C*>(p.cout)[mi]);
            double s = p.scale_c;
            if (p.scale) s *= p.scale[mi];
            y.x = (typename RealOf<C>::T)(y.x * s);
            y.y = (typename RealOf<C>::T)(y.y * s);
            store_as<C>(out, oq * p.out_so1 + orr * p.out_so2 + kk * p.out_sk + col, p.out_kind, y, p.acc);
          }
        }
      }
    }
  }
  if constexpr (!STOREG) __syncthreads();
}

template <int L, int W, int S, int Ns, typename C, bool GIN = true, bool GOUT = true, bool REG = false>
__device__ inline void stages(const PassDev& p, C* sm, const void* in, void* out, int64_t o, int64_t i0,
                              int64_t oq, int64_t orr, int64_t a4, const C* vin = nullptr,
                              int tid = (int)threadIdx.x) {
  if constexpr (S < nstages(L)) {
    constexpr int R = radix_of(L, S);
    stage<L, W, R, Ns, S == 0, S == nstages(L) - 1, C, GIN, GOUT, REG>(p, sm, in, out, o, i0, oq, orr, a4, vin,
                                                                          tid);
    stages<L, W, S + 1, Ns * R, C, GIN, GOUT, REG>(p, sm, in, out, o, i0, oq, orr, a4, vin, tid);
  }
}

template <int L, typename C, int WO = 0>
__global__ __launch_bounds__(threads_of(L), (min_waves_of<L, C, WO>())) void fft_pass_kernel(PassDev p, const void* in,
                                                                                            void* out) {
  constexpr int W = tile_w_of<L, C, WO>();
  __shared__ C sm[nstages(L) > 1 ? L * W : 1];
  if (p.skip && *p.skip) return;
  const int64_t blk = blockIdx.x;
  const int64_t o = blk / p.ntile;
  const int64_t i0 = (blk - o * p.ntile) * W;
  const int64_t oq = o / p.od, orr = o - oq * p.od;
  const int64_t a4 = p.tw4 ? (i0 + (int64_t)(threadIdx.x % W)) / p.tw4_S : 0;
  stages<L, W, 0, 1, C>(p, sm, in, out, o, i0, oq, orr, a4);
}

// Streaming form of the 512-point pass (the plan's tile choice 2): one
// block per compute unit walks the tiles blk, blk + G, blk + 2G, ... and
// issues the loads of its next tile's first-stage inputs into registers
// right after the first stage of the current one, so each compute unit
// keeps HBM reads in flight through the remaining LDS stages and the
// stores.  (With one block per tile, a compute unit holding a single 128 KB
// tile leaves HBM idle for the length of its LDS stages.)  The global
// loads of a wave complete in issue order, so waiting for any load issued
// after the prefetch would wait for the prefetch too: the stage twiddles
// and the per-mode scale are therefore read from LDS copies made once per
// block, and the loads are unconditional (columns past the end read column
// 0 of the row, in bounds) and masked when the values are taken.  Inputs
// in the compute precision; no chirp factors, per-mode multiplier,
// conjugation or four-step twiddle, and od = 1 (single passes over the
// axis; checked by the launcher and set here as constants, so that the
// epilogue keeps only the scale).  The output kind and the accumulation
// are template arguments, so that the stores are straight-line code and the
// compiler's wait for the prefetched values at the top of the loop does not
// also wait for the previous tile's stores.  TIN is the input element
// (complex128 input of a complex64 pass: W = 16 columns, so that the
// prefetched complex128 values take the registers of 32 complex64 ones).
template <int L, typename C, typename TIN, int W, bool OUT128, bool ACC>
__global__ __launch_bounds__(threads_of(L), 1) void fft_stream_kernel(PassDev p0, const void* in, void* out,
                                                                      int64_t ntot) {
  using T = typename RealOf<C>::T;
  constexpr int NT = threads_of(L);
  constexpr int R0 = radix_of(L, 0);
  constexpr int LR = L / R0;
  constexpr int NB = LR * W / NT;
  static_assert(NB * NT == LR * W, "the first stage's butterflies fill the block");
  static_assert((L * W + L) * sizeof(C) + L * sizeof(double) <= 160 * 1024, "LDS");
  __shared__ C sm[L * W];
  __shared__ C twl[L];
  __shared__ double scl[L];
  if (p0.skip && *p0.skip) return;
  const int tid = threadIdx.x;
  const int w = tid % W;
  const int64_t G = gridDim.x;
  for (int e = tid; e < L; e += NT) {
    twl[e] = reinterpret_cast<const C*>(p0.tw)[e];
    scl[e] = p0.scale ? p0.scale[e] : 1.0;
  }
  PassDev p = p0;
  p.cin = p.cout = p.cmode = p.tw4 = nullptr;
  p.conj_out = 0;
  p.od = 1;
  p.out_kind = OUT128 ? ST_C128 : ST_C64;
  p.acc = ACC ? 1 : 0;
  p.tw = twl;
  p.scale = scl;
  TIN pre[NB * R0];
  // Row r LR + j of a tile: the tile's base (uniform) plus the thread's
  // 32-bit byte offset (j in_sj + w) sizeof(TIN) (the launcher checks that
  // LR in_sj sizeof(TIN) < 2^31), so that only the thread offsets take
  // vector registers besides the values.
  uint32_t toff[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q)
    toff[q] = (uint32_t)(((tid + q * NT) / W) * p.in_sj + w) * (uint32_t)sizeof(TIN);
  auto fetch = [&](int64_t tile) -> bool {
    const int64_t o = tile / p.ntile;
    const int64_t i0 = (tile - o * p.ntile) * W;
    const bool ok = i0 + w < p.I;
    const uint32_t msk = ok ? 0xffffffffu : 0u;
    const char* base = reinterpret_cast<const char*>(reinterpret_cast<const TIN*>(in) + o * p.in_so + i0);
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const char* br = base + (int64_t)r * LR * p.in_sj * (int64_t)sizeof(TIN);
#pragma unroll
      for (int q = 0; q < NB; ++q) pre[q * R0 + r] = *reinterpret_cast<const TIN*>(br + (toff[q] & msk));
    }
    return ok;
  };
  int64_t tile = blockIdx.x;
  bool ok = tile < ntot ? fetch(tile) : false;
  __syncthreads();  // the LDS copies of the tables
  for (; tile < ntot; tile += G) {
    C v[NB * R0];
#pragma unroll
    for (int k = 0; k < NB * R0; ++k) {
      v[k].x = ok ? (T)pre[k].x : (T)0;
      v[k].y = ok ? (T)pre[k].y : (T)0;
    }
    const int64_t o = tile / p.ntile;
    const int64_t i0 = (tile - o * p.ntile) * W;
    // The output row offsets (multiples of out_sk) and the LDS addresses
    // of the stages are the same for every tile; empty asm statements make
    // the stride and the thread index new to the compiler in each
    // iteration, so it recomputes those per tile instead of keeping all of
    // them in registers across the loop.
    int64_t osk = p0.out_sk;
    int tl = tid;
    asm volatile("" : "+s"(osk), "+v"(tl));
    p.out_sk = osk;
    // first stage from the registers into LDS, then the next tile's loads
    stage<L, W, R0, 1, true, nstages(L) == 1, C, true, true, true>(p, sm, in, out, o, i0, o, 0, 0, v, tl);
    if (tile + G < ntot) ok = fetch(tile + G);
    stages<L, W, 1, R0, C, true, true, true>(p, sm, in, out, o, i0, o, 0, 0, v, tl);
  }
}

// Chirp-z middle pass: forward DFT over the rows into LDS, multiplication by
// the transformed kernel, conjugation, a second forward DFT, and the
// conjugating epilogue: conj(DFT(conj(X))) is the unscaled inverse DFT.
// With L the whole convolution length and the chirps folded into the first
// load and the last store, it is the complete transform in one pass.
template <int L, typename C>
__global__ __launch_bounds__(threads_of(L)) void conv_pass_kernel(PassDev p, const void* in, void* out) {
  constexpr int W = tile_w<C>(L);
  __shared__ C sm[L * W];
  if (p.skip && *p.skip) return;
  const int64_t blk = blockIdx.x;
  const int64_t o = blk / p.ntile;
  const int64_t i0 = (blk - o * p.ntile) * W;
  const int64_t oq = o / p.od, orr = o - oq * p.od;
  stages<L, W, 0, 1, C, true, false>(p, sm, in, out, o, i0, oq, orr, 0);
  const C* hk = reinterpret_cast<const C*>(p.cmode);
  for (int e = threadIdx.x; e < L * W; e += threads_of(L)) {
    const int d = e / W;
    C y = cmul(sm[e], hk[orr + p.od * d]);
    y.y = -y.y;
    sm[e] = y;
  }
  __syncthreads();
  PassDev q = p;
  q.cmode = nullptr;
  q.cin = nullptr;
  stages<L, W, 0, 1, C, false, true>(q, sm, in, out, o, i0, oq, orr, 0);
}

template <int L, typename C>
hipError_t launch_conv_L(const PassDev& p, int64_t O, const void* in, void* out, hipStream_t s) {
  constexpr int W = tile_w<C>(L);
  PassDev q = p;
  q.ntile = (p.I + W - 1) / W;
  const int64_t blocks = O * q.ntile;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((conv_pass_kernel<L, C>), dim3((unsigned)blocks), dim3(threads_of(L)), 0, s, q, in, out);
  return hipGetLastError();
}

template <typename C>
hipError_t launch_conv_typed(int L, const PassDev& p, int64_t O, const void* in, void* out, hipStream_t s) {
  switch (L) {
    case 9: return launch_conv_L<9, C>(p, O, in, out, s);
    case 18: return launch_conv_L<18, C>(p, O, in, out, s);
    case 36: return launch_conv_L<36, C>(p, O, in, out, s);
    case 72: return launch_conv_L<72, C>(p, O, in, out, s);
    case 2: return launch_conv_L<2, C>(p, O, in, out, s);
    case 4: return launch_conv_L<4, C>(p, O, in, out, s);
    case 8: return launch_conv_L<8, C>(p, O, in, out, s);
    case 16: return launch_conv_L<16, C>(p, O, in, out, s);
    case 32: return launch_conv_L<32, C>(p, O, in, out, s);
    case 64: return launch_conv_L<64, C>(p, O, in, out, s);
    case 128: return launch_conv_L<128, C>(p, O, in, out, s);
    case 256: return launch_conv_L<256, C>(p, O, in, out, s);
    case 512: return launch_conv_L<512, C>(p, O, in, out, s);
    // whole chirp-z convolutions in one pass (the plan's choice per axis)
    case 576: return launch_conv_L<576, C>(p, O, in, out, s);
    case 1152: return launch_conv_L<1152, C>(p, O, in, out, s);
    case 2304: return launch_conv_L<2304, C>(p, O, in, out, s);
    case 4608: return launch_conv_L<4608, C>(p, O, in, out, s);
    case 1024: return launch_conv_L<1024, C>(p, O, in, out, s);
    case 2048: return launch_conv_L<2048, C>(p, O, in, out, s);
    default: return hipErrorInvalidValue;
  }
}

template <int L, typename C, int WO = 0>
hipError_t launch_L(const PassDev& p, int64_t O, const void* in, void* out, hipStream_t s) {
  constexpr int W = tile_w_of<L, C, WO>();
  PassDev q = p;
  q.ntile = (p.I + W - 1) / W;
  const int64_t blocks = O * q.ntile;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((fft_pass_kernel<L, C, WO>), dim3((unsigned)blocks), dim3(threads_of(L)), 0, s, q, in, out);
  return hipGetLastError();
}

// Compute units of the current device, for the streaming pass's grid.
// (Cached per device; threads that race on the first query store the same
// value.)
int compute_units() {
  static std::atomic<int> cu[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int n = cu[dev].load(std::memory_order_relaxed);
  if (n <= 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cu[dev].store(n, std::memory_order_relaxed);
  }
  return n;
}

template <int L, typename C, typename TIN, int W>
hipError_t launch_stream_L(const PassDev& p, int64_t O, const void* in, void* out, hipStream_t s) {
  PassDev q = p;
  q.ntile = (p.I + W - 1) / W;
  const int64_t ntot = O * q.ntile;
  if (ntot <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(ntot, compute_units());
  const dim3 g((unsigned)blocks), b(threads_of(L));
  const bool o128 = p.out_kind == ST_C128;
  if constexpr (sizeof(TIN) != sizeof(C)) {
    // complex128 input of a complex64 pass: complex64 output, no accumulation
    if (o128 || p.acc) return hipErrorInvalidValue;
    hipLaunchKernelGGL((fft_stream_kernel<L, C, TIN, W, false, false>), g, b, 0, s, q, in, out, ntot);
  } else {
    if (o128 && p.acc) hipLaunchKernelGGL((fft_stream_kernel<L, C, TIN, W, true, true>), g, b, 0, s, q, in, out, ntot);
    else if (o128) hipLaunchKernelGGL((fft_stream_kernel<L, C, TIN, W, true, false>), g, b, 0, s, q, in, out, ntot);
    else if (p.acc) hipLaunchKernelGGL((fft_stream_kernel<L, C, TIN, W, false, true>), g, b, 0, s, q, in, out, ntot);
    else hipLaunchKernelGGL((fft_stream_kernel<L, C, TIN, W, false, false>), g, b, 0, s, q, in, out, ntot);
  }
  return hipGetLastError();
}

// small_tile: 0 the default tile, 1 the 64 KB complex64 tile, 2 the
// streaming pass (512 points; other passes and inputs that it does not
// take fall back to the default).
template <typename C>
hipError_t launch_typed(int L, const PassDev& p, int64_t O, const void* in, void* out, hipStream_t s,
                        int small_tile) {
  constexpr int kind = sizeof(C) == sizeof(float2) ? ST_C64 : ST_C128;
  if (L == 512 && small_tile == 2 && !p.cin && !p.cout && !p.cmode && !p.tw4 && !p.conj_out && p.od == 1) {
    constexpr int64_t LR = 512 / radix_of(512, 0);
    if (p.in_kind == kind && LR * p.in_sj * (int64_t)sizeof(C) < 0x7fffffffLL)
      return launch_stream_L<512, C, C, tile_w<C>(512)>(p, O, in, out, s);
    if constexpr (sizeof(C) == sizeof(float2)) {
      if (p.in_kind == ST_C128 && p.out_kind == ST_C64 && !p.acc && LR * p.in_sj * (int64_t)sizeof(double2) < 0x7fffffffLL)
        return launch_stream_L<512, C, double2, 16>(p, O, in, out, s);
    }
  }
  if constexpr (sizeof(C) == sizeof(float2)) {
    if (L == 512 && small_tile == 1) return launch_L<512, C, 16>(p, O, in, out, s);
  }
  switch (L) {
    case 2: return launch_L<2, C>(p, O, in, out, s);
    case 4: return launch_L<4, C>(p, O, in, out, s);
    case 8: return launch_L<8, C>(p, O, in, out, s);
    case 16: return launch_L<16, C>(p, O, in, out, s);
    case 32: return launch_L<32, C>(p, O, in, out, s);
    case 64: return launch_L<64, C>(p, O, in, out, s);
    case 128: return launch_L<128, C>(p, O, in, out, s);
    case 256: return launch_L<256, C>(p, O, in, out, s);
    case 512: return launch_L<512, C>(p, O, in, out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int fft_tile_width(int L, bool fp32) { return fp32 ? tile_w<float2>(L) : tile_w<double2>(L); }

static PassDev make_pass_dev(const FftPass& f) {
  PassDev p;
  p.I = f.I;
  p.od = f.od;
  p.in_so = f.in_so;
  p.in_sj = f.in_sj;
  p.out_so1 = f.out_so1;
  p.out_so2 = f.out_so2;
  p.out_sk = f.out_sk;
  p.tw4_S = f.tw4_S;
  p.acc = f.accumulate;
  p.in_kind = f.in_kind;
  p.out_kind = f.out_kind;
  p.scale_c = f.scale_c;
  p.tw = f.tw;
  p.tw4 = f.tw4;
  p.scale = f.scale;
  p.sign = f.sign;
  p.cmode = f.cmode;
  p.skip = f.skip;
  p.cin = f.cin;
  p.cout = f.cout;
  p.chirp_n = f.chirp_n;
  p.chirp_na = f.chirp_na;
  p.chirp_S = f.chirp_S > 0 ? f.chirp_S : 1;
  p.tw4_mode = f.tw4_mode;
  p.conj_out = f.conj_out;
  p.ntile = 0;
  return p;
}

hipError_t launch_fft_pass(const FftPass& f, bool fp32, const void* in, void* out, hipStream_t s) {
  if (f.tw4 && f.tw4_mode == 0 && f.tw4_S <= 0) return hipErrorInvalidValue;
  const PassDev p = make_pass_dev(f);
  return fp32 ? launch_typed<float2>(f.L, p, f.O, in, out, s, f.small_tile)
              : launch_typed<double2>(f.L, p, f.O, in, out, s, f.small_tile);
}

hipError_t launch_conv_pass(const FftPass& f, bool fp32, const void* in, void* out, hipStream_t s) {
  if (!f.cmode) return hipErrorInvalidValue;
  const PassDev p = make_pass_dev(f);
  return fp32 ? launch_conv_typed<float2>(f.L, p, f.O, in, out, s)
              : launch_conv_typed<double2>(f.L, p, f.O, in, out, s);
}

}  // namespace helm
