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
// (factor_kernel; the paper likewise factors the line matrices at
// initialisation) and stored as one reciprocal pivot per lane chunk; a solve
// regenerates the c pivots of its chunk from it (c divisions instead of c
// table reads) and runs the two affine scans, with wave shuffles inside a
// wave and one LDS exchange between the waves of a line.
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

// Moves of a 64-bit value across lanes with the data-parallel primitives:
// lanes whose source lane is outside the pattern (or whose row is masked
// off) keep `old`.
template <int CTRL, int ROWMASK>
__device__ inline double dpp_d(double src, double old) {
  const unsigned long long s = __builtin_bit_cast(unsigned long long, src);
  const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)s, CTRL, ROWMASK, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(s >> 32), CTRL,
                                                            ROWMASK, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// Same with every row enabled and zero where no source lane exists
// (bound_ctrl), which needs no initialised destination.
template <int CTRL>
__device__ inline double dpp_d0(double src) {
  const unsigned long long s = __builtin_bit_cast(unsigned long long, src);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)s, CTRL, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(s >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int CTRL, int ROWMASK = 0xF>
__device__ inline Aff dpp_aff(const Aff& v) {  // identity where nothing arrives
  Aff o;
  o.f.x = dpp_d<CTRL, ROWMASK>(v.f.x, 1.0);
  if constexpr (ROWMASK == 0xF) {
    o.f.y = dpp_d0<CTRL>(v.f.y);
    o.g.x = dpp_d0<CTRL>(v.g.x);
    o.g.y = dpp_d0<CTRL>(v.g.y);
  } else {
    o.f.y = dpp_d<CTRL, ROWMASK>(v.f.y, 0.0);
    o.g.x = dpp_d<CTRL, ROWMASK>(v.g.x, 0.0);
    o.g.y = dpp_d<CTRL, ROWMASK>(v.g.y, 0.0);
  }
  return o;
}
// DPP controls (GFX9 encoding): row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143, wave_shr:1 = 0x138.
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143, kWaveShr1 = 0x138;

// Inclusive prefix composition within groups of W lanes (W = 16, 32 or 64;
// later lanes applied after earlier ones): four in-row steps, then the row
// broadcasts that carry row totals to the following rows.
template <int W>
__device__ inline Aff dpp_inclusive(Aff v) {
  v = aff_then(v, dpp_aff<kRowShr1>(v));
  v = aff_then(v, dpp_aff<kRowShr2>(v));
  v = aff_then(v, dpp_aff<kRowShr4>(v));
  v = aff_then(v, dpp_aff<kRowShr8>(v));
  if constexpr (W >= 32) v = aff_then(v, dpp_aff<kRowBcast15, 0xA>(v));
  if constexpr (W >= 64) v = aff_then(v, dpp_aff<kRowBcast31, 0xC>(v));
  return v;
}

// Lane r of each group of W lanes takes the value of lane W - 1 - r.
template <int W>
__device__ inline Aff reverse_aff(const Aff& v) {
  const int lane = threadIdx.x & 63;
  const int src = (lane & ~(W - 1)) + (W - 1 - (lane & (W - 1)));
  Aff o;
  o.f = make_double2(__shfl(v.f.x, src), __shfl(v.f.y, src));
  o.g = make_double2(__shfl(v.g.x, src), __shfl(v.g.y, src));
  return o;
}

// Exclusive scans of affine maps over the P lanes of a line (lanes
// [slot*P, slot*P + P) of the block).  Forward: lane q receives
// A_{q-1} o ... o A_0; backward: lane q receives A_{q+1} o ... o A_{P-1}
// (the forward scan in reversed lane order).  Whole waves (P >= 64) use DPP
// moves; lines of fewer lanes use shuffles.  For P > 64 the
// waves of a line exchange their totals through LDS (`wbuf`, NT/64 entries;
// forward and backward scans use different buffers, so one barrier per scan
// suffices: the next write to a buffer follows the other scan's barrier).
// Every thread of the block must call these.
template <int P>
__device__ inline Aff wave_scan_excl(Aff v, int q, Aff& incl) {
  constexpr int W = P < 64 ? P : 64;
  Aff ex;
  if constexpr (W == 64) {
    v = dpp_inclusive<64>(v);
    incl = v;
    ex = dpp_aff<kWaveShr1>(v);
  } else {
    const int lq = q & (W - 1);
#pragma unroll
    for (int d = 1; d < W; d <<= 1) {
      const Aff o = shfl_up_aff(v, d, W);
      if (lq >= d) v = aff_then(v, o);
    }
    incl = v;
    ex = shfl_up_aff(v, 1, W);
    if (lq == 0) ex = aff_ident();
  }
  return ex;
}

template <int P>
__device__ inline Aff scan_fwd(Aff v, int q, Aff* wbuf) {
  Aff incl;
  Aff ex = wave_scan_excl<P>(v, q, incl);
  if constexpr (P > 64) {
    const int wv = threadIdx.x >> 6;          // wave in block
    const int w0 = wv - (q >> 6);             // first wave of this line
    if ((q & 63) == 63) wbuf[wv] = incl;      // inclusive wave total
    __syncthreads();
    Aff pre = aff_ident();
    for (int w = w0; w < wv; ++w) pre = aff_then(wbuf[w], pre);
    ex = aff_then(ex, pre);
  }
  return ex;
}

template <int P>
__device__ inline Aff scan_bwd(Aff v, int q, Aff* wbuf) {
  constexpr int W = P < 64 ? P : 64;
  Aff ex, incl;
  if constexpr (W == 64) {
    // reversed lane order turns the suffix scan into a prefix scan of the
    // same operator over the physical lane positions; in reversed order the
    // last lane holds the composition of the whole wave
    ex = reverse_aff<64>(wave_scan_excl<P>(reverse_aff<64>(v), q, incl));
  } else {
    const int lq = q & (W - 1);
#pragma unroll
    for (int d = 1; d < W; d <<= 1) {
      const Aff o = shfl_down_aff(v, d, W);
      if (lq + d < W) v = aff_then(v, o);
    }
    ex = shfl_down_aff(v, 1, W);
    if (lq == W - 1) ex = aff_ident();
  }
  if constexpr (P > 64) {
    const int wv = threadIdx.x >> 6;
    const int wl = wv - (q >> 6) + P / 64 - 1;       // last wave of this line
    if ((threadIdx.x & 63) == 63) wbuf[wv] = incl;   // inclusive suffix total of the wave
    __syncthreads();
    Aff suf = aff_ident();
    for (int w = wl; w > wv; --w) suf = aff_then(wbuf[w], suf);
    ex = aff_then(ex, suf);
  }
  return ex;
}

struct LineDev {
  int nb, nO, nI, nL, c, red, tile, ntiles, iters;
  int tl, tm;  // red == 0 with tm > 0: blocks take tiles of tl outer x tm inner modes
  int xcd;     // with tiles: consecutive blocks of one XCD take consecutive tiles
  const double2* sO;
  const double2* sI;
  double2 sC;
  double hL, m_end, m_int, m_off, k_off;
  double2 kLo, kHi;
  const void* in;
  const double2 *alpha0, *alpha1, *beta0, *beta1, *rho0, *rho1;
  const void *PO, *PI;  // rank-2 rows, of the lines' storage type
  const double2* piv;   // [nO*nI][P]: reciprocal pivot entering the chunk of each lane
  const double2* sTab;  // [nO*nI] sigma per line, or null
  void* out;
  double2* part;
  const int* skip;
  int unit_rhs;
};

struct RowCoef {
  double2 dint, dlo, dhi, off, off2;
};

__device__ inline double2 line_sigma(const LineDev& a, int64_t l, int64_t m) {
  double2 sig;
  if (a.sTab) {
    sig = a.sTab[l * a.nI + m];
  } else {
    sig = a.sC;
    if (a.sO) sig = cadd(sig, a.sO[l]);
    if (a.sI) sig = cadd(sig, a.sI[m]);
  }
  return sig;
}
__device__ inline RowCoef coef_of_sigma(const LineDev& a, double2 sig) {
  RowCoef r;
  r.off = make_double2(sig.x * a.m_off + a.k_off, sig.y * a.m_off);  // sigma h/6 - 1/h
  r.off2 = cmul(r.off, r.off);
  r.dint = make_double2(sig.x * a.m_int + 2.0 / a.hL, sig.y * a.m_int);
  r.dlo = make_double2(sig.x * a.m_end + a.kLo.x / a.hL, sig.y * a.m_end + a.kLo.y / a.hL);
  r.dhi = make_double2(sig.x * a.m_end + a.kHi.x / a.hL, sig.y * a.m_end + a.kHi.y / a.hL);
  return r;
}
__device__ inline RowCoef row_coef(const LineDev& a, int64_t l, int64_t m) {
  return coef_of_sigma(a, line_sigma(a, l, m));
}

__device__ inline double2 diag_of(const RowCoef& r, int x, int nL) {
  if (x >= nL) return make_double2(1, 0);
  if (x == 0) return r.dlo;
  if (x == nL - 1) return r.dhi;
  return r.dint;
}
// e(x) = coupling between rows x-1 and x
__device__ inline bool has_e(int x, int nL) { return x > 0 && x < nL; }

// Line index (b, l, m) of slot `sl` of tile t at iteration `it`; false past
// the end of the tile's extent.  Line counts stay below 2^31 (checked at
// launch), so 32-bit index arithmetic suffices.  Reductions over l come in
// two layouts: red 2 gives a block one m and its slots consecutive l (lines
// nI nL elements apart); red 3 gives the slots of a block lpb consecutive m
// at one l per iteration, so one iteration reads lpb adjacent lines and the
// rows PI[b][l] once, and every slot keeps its own partial sum.
__device__ inline bool decode_line(const LineDev& a, uint32_t g, uint32_t t, int lpb, int it, int sl,
                                   uint32_t& b, uint32_t& l, uint32_t& m) {
  const uint32_t li = a.red == 3 ? t * (uint32_t)a.tile + (uint32_t)it
                                 : t * (uint32_t)a.tile + (uint32_t)(it * lpb + sl);
  const uint32_t nO = a.nO, nI = a.nI;
  bool valid;
  if (a.red == 1) {        // g = b*nO + l, li = m
    valid = li < nI;
    b = g / nO;
    l = g - b * nO;
    m = li;
  } else if (a.red == 2) { // g = b*nI + m, li = l
    valid = li < nO;
    b = g / nI;
    m = g - b * nI;
    l = li;
  } else if (a.red == 3) { // g = b*nmg + mg, li = l, m = mg*lpb + sl
    const uint32_t nmg = (nI + (uint32_t)lpb - 1) / (uint32_t)lpb;
    b = g / nmg;
    m = (g - b * nmg) * (uint32_t)lpb + (uint32_t)sl;
    l = li;
    valid = li < nO && m < nI;
  } else if (a.tm > 0) {   // tile t = (b, mt, lt), li - t*tile = (l - lt*tl)*tm + (m - mt*tm)
    const uint32_t nlt = (nO + (uint32_t)a.tl - 1) / (uint32_t)a.tl, nmt = (nI + (uint32_t)a.tm - 1) / (uint32_t)a.tm;
    const uint32_t idx = li - t * (uint32_t)a.tile;
    const uint32_t bm = t / nlt, lt = t - bm * nlt;
    b = bm / nmt;
    const uint32_t mt = bm - b * nmt;
    const uint32_t il = idx / (uint32_t)a.tm;
    l = lt * (uint32_t)a.tl + il;
    m = mt * (uint32_t)a.tm + (idx - il * (uint32_t)a.tm);
    valid = idx < (uint32_t)a.tile && l < nO && m < nI && b < (uint32_t)a.nb;
  } else {                 // li = (b*nO + l)*nI + m
    valid = li < (uint32_t)a.nb * nO * nI;
    const uint32_t bl = li / nI;
    m = li - bl * nI;
    b = bl / nO;
    l = bl - b * nO;
  }
  if (!valid) { b = 0; l = 0; m = 0; }
  return valid;
}

// Padded position of element e of a wave's staging area: one pad slot per 8
// elements, so that lanes reading rows lane*c + j (c = 8) hit distinct banks.
__device__ inline int stage_pos(int e) { return e + (e >> 3); }

// Memory layout and staging.  Line rows are contiguous in memory but lane q
// owns the contiguous chunk [q c, q c + c), so direct per-lane loads would
// touch 64 cache lines per wave instruction.  Instead every wave loads the
// rows of its lanes with consecutive lanes on consecutive rows (whole cache
// lines per instruction), assembles the right-hand side there, and passes the
// chunks through its own LDS area (72 c complex values, padded); solutions to
// be stored take the same route back.  Between the two, the area parks the
// lane's reciprocal pivots and then its backward multipliers.  A wave's area
// is only touched by that wave, whose LDS accesses execute in program order,
// except in the final cross-slot reduction, which is fenced by block
// barriers.
//
// C = 8: every line has exactly P * 8 rows (no padding rows).  Then the only
// rows without a coupling to their predecessor / successor are x = 0 and
// x = nL - 1, and neither needs a guard: the entering reciprocal pivot of lane
// 0 is zero, which zeroes its first forward multiplier, and the last lane's
// backward recurrence starts from y = 0, which annihilates its last backward
// multiplier.  PAD (C = 8, nL < P * 8 at run time): the rows past the end of
// the line are identity rows, with the couplings and end pivot guarded per
// row.  (C = 0, a chunk length a.c <= kCMax read at run time with the same
// guards, is the general form; the launcher always picks 8-row chunks,
// which run about a third faster.)
//
// XR (with C = 8): the line has one row more, nL = P * 8 + 1 (the 2^k + 1
// node counts of the paper's grids).  The last lane owns it beside its chunk:
// it finishes the forward elimination through it after the forward scan
// (its pivot and value follow from the chunk's last ones), takes y_{nL-1},
// and folds it into its backward map, which becomes the constant map to the
// value entering its chunk from above.
// Storing launches of exact 512-lane lines (4096-row lines) are held to 128
// registers, so that two blocks of eight waves share a compute unit (the
// complex64 kernel needs 131 otherwise and then spills 2; 4096^2 mixed
// solve: line launches 0.365 -> 0.344 ms).
template <typename T, int NT, int P, int C, bool RED, bool XR, bool PAD>
__global__ __launch_bounds__(NT, (!RED && NT == 512 && !XR && !PAD) ? 4 : 1) void lines_kernel(LineDev a) {
  constexpr int NW = NT / 64;
  constexpr int PW = P < 64 ? P : 64;     // lanes of one line inside a wave
  constexpr int SPW = 64 / PW;            // lines per wave
  constexpr int LPB = NT / P;             // lines per block
  constexpr bool FIXED = C > 0;
  constexpr bool EXACT = FIXED && !PAD;  // every row of every chunk is a row of the line
  __shared__ Aff wbuf[2][NW + 1];         // wave totals of the forward / backward scans
  extern __shared__ double2 stage[];      // NW areas of 72 c padded values
  if (a.skip && *a.skip) return;

  const int c = FIXED ? C : a.c, nL = EXACT ? P * C + (XR ? 1 : 0) : a.nL;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // a line spans whole waves when P >= 64: its index is then wave-uniform
  const int slot = P >= 64 ? __builtin_amdgcn_readfirstlane(tid / P) : tid / P;
  const int q = tid - slot * P;
  const int x0 = q * c;
  const bool last = XR && q == P - 1;  // owner of the extra row
  const int wslot0 = (wv * 64) / P;                   // first line slot of this wave
  const int wx0 = (P >= 64 ? (wv * 64) % P : 0) * c;  // first row this wave stages
  const int seg = PW * c;                             // rows of one line staged by this wave
  double2* S = stage + wv * (72 * c);
  auto in_chunk = [&](int j) { return FIXED ? j < C : j < c; };
  auto slot_of = [&](int j) { return stage_pos(lane * c + j); };

  const uint32_t blk = blockIdx.x;
  uint32_t g = 0, t = 0;
  if (a.red) {
    g = blk / (uint32_t)a.ntiles;
    t = blk - g * (uint32_t)a.ntiles;
  } else if (a.xcd) {
    // blocks are dealt to the 8 XCDs in turn: block 8k + x takes tile
    // x ntiles/8 + k, so the blocks resident on one XCD work on
    // consecutive tiles (outer-mode tiles fastest), which share the rank-2
    // rows of their inner modes in that XCD's L2
    t = (blk & 7u) * ((uint32_t)a.ntiles >> 3) + (blk >> 3);
  } else {
    t = blk;
  }

  double2 acc0[kCMax], acc1[kCMax];
  double2 accx0 = make_double2(0, 0), accx1 = accx0;  // the extra row (XR, last lane)
  if constexpr (RED) {
#pragma unroll
    for (int j = 0; j < kCMax; ++j) acc0[j] = acc1[j] = make_double2(0, 0);
  }

  // Reducing launches with one line per block (P >= 256) prefetch the
  // next line's input rows into registers while the current line is solved,
  // so the load latency overlaps the sweeps.
  constexpr bool PREF = P >= 256 && RED && !XR;
  T pre[PREF ? kCMax : 1];
  auto fetch = [&](int itn) {
    uint32_t sb, sl, sm;
    const bool sv = decode_line(a, g, t, LPB, itn, wslot0, sb, sl, sm);
    const int64_t soff = ((int64_t)(sb * a.nO + sl) * a.nI + sm) * nL;
#pragma unroll
    for (int jj = 0; jj < kCMax; ++jj) {
      const int r = jj * 64 + lane, x = wx0 + r;
      T v;
      v.x = 0;
      v.y = 0;
      if (r < seg && x < nL && sv) v = reinterpret_cast<const T*>(a.in)[soff + x];
      pre[jj] = v;
    }
  };
  if constexpr (PREF) {
    if (a.in && a.iters > 0) fetch(0);
  }

  // Reducing kernels of exact lines at P <= 64 load each line's sigma,
  // entering pivot and reduction weights at the top of the iteration, so
  // those loads are in flight while the right-hand side is staged instead of
  // each being waited for where it is used (-3% per step at 256^3 and
  // 512^3 x 16); at P = 512 the registers allow sigma and the pivot
  // (-2% per line launch at 4096^2).  The other kernels lack the registers.
  constexpr bool EARLY = RED && !XR && !PAD && P <= 64;
  constexpr bool EARLY_SP = RED && !XR && !PAD && P == 512;
  for (int it = 0; it < a.iters; ++it) {
    uint32_t eb = 0, el = 0, em = 0;
    bool evalid = false;
    double2 esig = make_double2(0, 0), eip = make_double2(0, 0), ew0 = eip, ew1 = eip;
    if constexpr (EARLY || EARLY_SP) {
      evalid = decode_line(a, g, t, LPB, it, slot, eb, el, em);
      esig = line_sigma(a, el, em);
      if (q > 0) eip = a.piv[(int64_t)(el * a.nI + em) * P + q];
    }
    if constexpr (EARLY) {
      const uint32_t wi = (a.red == 1) ? em : el;
      ew0 = a.rho0[wi];
      ew1 = a.rho1[wi];
    }
    // ---- right-hand side, staged through LDS -------------------------------
#pragma unroll 4
    for (int si = 0; si < SPW; ++si) {
      uint32_t sb, sl, sm;
      const bool sv = decode_line(a, g, t, LPB, it, wslot0 + si, sb, sl, sm);
      const int64_t soff = ((int64_t)(sb * a.nO + sl) * a.nI + sm) * nL;
      double2 al0 = make_double2(0, 0), al1 = al0, be0 = al0, be1 = al0;
      if (a.PO) { al0 = a.alpha0[sl]; al1 = a.alpha1[sl]; }
      if (a.PI) { be0 = a.beta0[sm]; be1 = a.beta1[sm]; }
      const T* po = a.PO ? reinterpret_cast<const T*>(a.PO) + (int64_t)(sb * 2) * a.nI * nL + (int64_t)sm * nL : nullptr;
      const T* pi = a.PI ? reinterpret_cast<const T*>(a.PI) + (int64_t)((sb * a.nO + sl) * 2) * nL : nullptr;
      // one source at a time (each lane revisits only its own staging slots),
      // so that at most kCMax loads are in flight per lane
      if (a.in && PREF) {
#pragma unroll
        for (int jj = 0; jj < kCMax; ++jj) {
          const int r = jj * 64 + lane;
          if (r < seg) S[stage_pos(si * seg + r)] = to_d2(pre[jj]);
        }
        if (it + 1 < a.iters) fetch(it + 1);
      } else if (a.in) {
        double2 d[kCMax];
        if constexpr (sizeof(T) == sizeof(float2) && !XR && !PAD) {
          // complex64 rows: loaded unconditionally (masked lanes read element
          // 0 of the input, in bounds, and discard it) and converted after
          // all loads are issued.  Loads under a per-row condition, each
          // converted inside its branch, are waited for one by one
          // (512^3 x 16 mixed step 339 -> 311 ms with this form).
          T raw[kCMax];
#pragma unroll
          for (int jj = 0; jj < kCMax; ++jj) {
            const int r = jj * 64 + lane, x = wx0 + r;
            const bool ok = r < seg && x < nL && sv;
            raw[jj] = reinterpret_cast<const T*>(a.in)[ok ? soff + x : 0];
          }
#pragma unroll
          for (int jj = 0; jj < kCMax; ++jj) {
            const int r = jj * 64 + lane, x = wx0 + r;
            d[jj] = (r < seg && x < nL && sv) ? to_d2(raw[jj]) : make_double2(0, 0);
          }
        } else {
#pragma unroll
          for (int jj = 0; jj < kCMax; ++jj) {
            const int r = jj * 64 + lane, x = wx0 + r;
            d[jj] = (r < seg && x < nL && sv) ? to_d2(reinterpret_cast<const T*>(a.in)[soff + x])
                                               : make_double2(0, 0);
          }
        }
#pragma unroll
        for (int jj = 0; jj < kCMax; ++jj) {
          const int r = jj * 64 + lane;
          if (r < seg) S[stage_pos(si * seg + r)] = d[jj];
        }
      } else {
#pragma unroll
        for (int jj = 0; jj < kCMax; ++jj) {
          const int r = jj * 64 + lane, x = wx0 + r;
          const bool one = a.unit_rhs && sv && x == (int)sb;
          if (r < seg) S[stage_pos(si * seg + r)] = make_double2(one ? 1.0 : 0.0, 0);
        }
      }
      // Rank-2 terms.  Kernels of exact lines load the rows of a source in
      // batches of NBAT chunk rows before combining any of them into the
      // staged values, so the loads of a batch are in flight together; loads
      // interleaved with the LDS updates may be issued one by one, each
      // waited for (measured at 512^3 x 16: 20-25 ms against 10-12 ms per
      // reducing launch).  Batches cost registers: reducing kernels take
      // all kCMax rows with several lines per block and 2 at P = 512 (at the
      // register limit; -2% per launch at 4096^2); storing kernels at
      // P = 16 to 64 take 4 (same occupancy; -11% per storing launch at
      // 512^3 x 16), and with complex64 storage at P = 512 2, each batch
      // scheduled on its own (same occupancy; -4% per line launch at 4096^2).
      // The other kernels update row by row, which keeps their register
      // count and occupancy (a batch would cost the other storing kernels,
      // and the reducing ones at P = 256, an occupancy level).
      constexpr bool SEP = !RED && P == 512 && sizeof(T) == sizeof(float2);
      constexpr int NBAT = (XR || PAD) ? 0
                           : RED     ? (P <= 128 ? kCMax : (P == 512 ? 2 : 0))
                                     : ((P >= 16 && P <= 64) ? 4 : (SEP ? 2 : 0));
      if constexpr (NBAT > 0) {
#pragma unroll
        for (int src = 0; src < 2; ++src) {
          const T* rows = src == 0 ? po : pi;
          if (!rows) continue;
          const int64_t stride = src == 0 ? (int64_t)a.nI * nL : (int64_t)nL;
          const double2 w0 = src == 0 ? al0 : be0, w1 = src == 0 ? al1 : be1;
#pragma unroll
          for (int j0 = 0; j0 < kCMax; j0 += NBAT) {
            double2 p0[NBAT], p1[NBAT];
#pragma unroll
            for (int u = 0; u < NBAT; ++u) {
              const int r = (j0 + u) * 64 + lane, x = wx0 + r;
              const bool ok = r < seg && x < nL && sv;
              p0[u] = ok ? to_d2(rows[x]) : make_double2(0, 0);
              p1[u] = ok ? to_d2(rows[stride + x]) : make_double2(0, 0);
            }
#pragma unroll
            for (int u = 0; u < NBAT; ++u) {
              const int r = (j0 + u) * 64 + lane, x = wx0 + r;
              if (r < seg && x < nL && sv) {
                const int q = stage_pos(si * seg + r);
                S[q] = cfma(w1, p1[u], cfma(w0, p0[u], S[q]));
              }
            }
            // keep the next batch's loads after these updates (registers)
            if constexpr (SEP) __builtin_amdgcn_sched_barrier(0);
          }
        }
      } else {
        if (po) {
#pragma unroll
          for (int jj = 0; jj < kCMax; ++jj) {
            const int r = jj * 64 + lane, x = wx0 + r;
            if (r < seg && x < nL && sv) {
              double2 d = S[stage_pos(si * seg + r)];
              d = cfma(al0, to_d2(po[x]), d);
              d = cfma(al1, to_d2(po[(int64_t)a.nI * nL + x]), d);
              S[stage_pos(si * seg + r)] = d;
            }
          }
        }
        if (pi) {
#pragma unroll
          for (int jj = 0; jj < kCMax; ++jj) {
            const int r = jj * 64 + lane, x = wx0 + r;
            if (r < seg && x < nL && sv) {
              double2 d = S[stage_pos(si * seg + r)];
              d = cfma(be0, to_d2(pi[x]), d);
              d = cfma(be1, to_d2(pi[nL + x]), d);
              S[stage_pos(si * seg + r)] = d;
            }
          }
        }
      }
    }

    uint32_t b, l, m;
    bool valid;
    if constexpr (EARLY || EARLY_SP) {
      b = eb; l = el; m = em; valid = evalid;
    } else {
      valid = decode_line(a, g, t, LPB, it, slot, b, l, m);
    }
    const RowCoef rc = (EARLY || EARLY_SP) ? coef_of_sigma(a, esig) : row_coef(a, l, m);
    const double2 moff = make_double2(-rc.off.x, -rc.off.y);  // -e
    double2 z[kCMax];
#pragma unroll
    for (int j = 0; j < kCMax; ++j) z[j] = in_chunk(j) ? S[slot_of(j)] : make_double2(0, 0);
    const int64_t loff = ((int64_t)(b * a.nO + l) * a.nI + m) * nL;  // this lane's line
    double2 xrhs = make_double2(0, 0);  // right-hand side of the extra row
    if (XR && last && valid) {
      const int x = nL - 1;
      if (a.in) xrhs = to_d2(reinterpret_cast<const T*>(a.in)[loff + x]);
      else if (a.unit_rhs && (int)b == x) xrhs = make_double2(1, 0);
      if (a.PO) {
        const T* po = reinterpret_cast<const T*>(a.PO) + (int64_t)(b * 2) * a.nI * nL + (int64_t)m * nL;
        xrhs = cfma(a.alpha0[l], to_d2(po[x]), xrhs);
        xrhs = cfma(a.alpha1[l], to_d2(po[(int64_t)a.nI * nL + x]), xrhs);
      }
      if (a.PI) {
        const T* pi = reinterpret_cast<const T*>(a.PI) + (int64_t)((b * a.nO + l) * 2) * nL;
        xrhs = cfma(a.beta0[m], to_d2(pi[x]), xrhs);
        xrhs = cfma(a.beta1[m], to_d2(pi[nL + x]), xrhs);
      }
    }

    // ---- 1. pivots and forward composition --------------------------------
    // Reciprocal pivots: the chunk's entering value from the plan's factor
    // table, then the Thomas recurrence p_x = d_x - e^2 / p_{x-1}.
    // Forward substitution z_x = f_x z_{x-1} + d_x, f_x = -e / p_{x-1}: the
    // lane composes its rows into one affine map.
    const double2 ip_in = (EARLY || EARLY_SP) ? eip : (q > 0 ? a.piv[(int64_t)(l * a.nI + m) * P + q] : make_double2(0, 0));
    Aff A = aff_ident();
    double2 ipp_last;  // 1/p of the chunk's last row
    {
      double2 ipp = ip_in;
#pragma unroll
      for (int j = 0; j < kCMax; ++j) {
        if (in_chunk(j)) {
          const int x = x0 + j;
          double2 f = cmul(moff, ipp);
          if (!EXACT && !has_e(x, nL)) f = make_double2(0, 0);
          A.f = cmul(f, A.f);
          A.g = cfma(f, A.g, z[j]);
          double2 pv;
          if (EXACT) {
            pv = (j == 0 && q == 0) ? rc.dlo : ((!XR && j == C - 1 && q == P - 1) ? rc.dhi : rc.dint);
            pv = cfms(rc.off2, ipp, pv);  // ipp = 0 at x = 0
            ipp = crcp_fast(pv);
          } else {
            pv = diag_of(rc, x, nL);
            if (has_e(x, nL)) pv = cfms(rc.off2, ipp, pv);
            ipp = x < nL ? crcp_fast(pv) : make_double2(1, 0);
          }
          S[slot_of(j)] = ipp;
        }
      }
      ipp_last = ipp;
    }
    const Aff Ein = scan_fwd<P>(A, q, wbuf[0]);

    // ---- 2. forward values, scaled for the back substitution --------------
    // h_x = z_x / p_x; the lane's slots now take the backward multipliers
    // g_x = -e / p_x (zero where row x + 1 is past the end of the line).
    double2 yx = make_double2(0, 0);  // y of the extra row (XR, last lane)
    {
      double2 zp = Ein.g;
      double2 mp = cmul(moff, ip_in);
#pragma unroll
      for (int j = 0; j < kCMax; ++j) {
        if (in_chunk(j)) {
          const int x = x0 + j;
          const double2 f = (EXACT || has_e(x, nL)) ? mp : make_double2(0, 0);
          zp = cfma(f, zp, z[j]);
          const double2 ipj = S[slot_of(j)];
          z[j] = cmul(zp, ipj);
          mp = cmul(moff, ipj);
          S[slot_of(j)] = (EXACT || has_e(x + 1, nL)) ? mp : make_double2(0, 0);
        }
      }
      if (XR && last) {
        // extra row: w = r + (-e / p_{nL-2}) w_{nL-2}, p = d_hi - e^2 / p_{nL-2}
        const double2 wx = cfma(cmul(moff, ipp_last), zp, xrhs);
        yx = cmul(wx, crcp_fast(cfms(rc.off2, ipp_last, rc.dhi)));
      }
    }

    // ---- 3. back substitution y_x = g_x y_{x+1} + h_x: composition, scan ---
    Aff B = aff_ident();
#pragma unroll
    for (int j = kCMax - 1; j >= 0; --j) {
      if (in_chunk(j)) {
        const double2 gx = S[slot_of(j)];
        B.f = cmul(gx, B.f);
        B.g = cfma(gx, B.g, z[j]);
      }
    }
    if (XR && last) {  // the value above the chunk is known: a constant map
      B.g = cfma(B.f, yx, B.g);
      B.f = make_double2(0, 0);
    }
    const Aff Bin = scan_bwd<P>(B, q, wbuf[1]);
    {
      double2 ynext = (XR && last) ? yx : Bin.g;
#pragma unroll
      for (int j = kCMax - 1; j >= 0; --j) {
        if (in_chunk(j)) {
          ynext = cfma(S[slot_of(j)], ynext, z[j]);
          z[j] = ynext;
        }
      }
    }

    // ---- 4. epilogue -------------------------------------------------------
    if (a.out) {
#pragma unroll
      for (int j = 0; j < kCMax; ++j)
        if (in_chunk(j)) S[slot_of(j)] = z[j];
      T* o = reinterpret_cast<T*>(a.out);
#pragma unroll 4
      for (int si = 0; si < SPW; ++si) {
        uint32_t sb, sl, sm;
        const bool sv = decode_line(a, g, t, LPB, it, wslot0 + si, sb, sl, sm);
        const int64_t soff = ((int64_t)(sb * a.nO + sl) * a.nI + sm) * nL;
#pragma unroll
        for (int jj = 0; jj < kCMax; ++jj) {
          const int r = jj * 64 + lane, x = wx0 + r;
          if (r < seg && x < nL && sv) o[soff + x] = from_d2<T>(S[stage_pos(si * seg + r)]);
        }
      }
    }
    if (XR && a.out && last && valid) reinterpret_cast<T*>(a.out)[loff + nL - 1] = from_d2<T>(yx);
    if constexpr (RED) {
      if (valid) {
        const uint32_t wi = (a.red == 1) ? m : l;
        const double2 w0 = EARLY ? ew0 : a.rho0[wi], w1 = EARLY ? ew1 : a.rho1[wi];
        if (XR && last) {
          accx0 = cfma(w0, yx, accx0);
          accx1 = cfma(w1, yx, accx1);
        }
#pragma unroll
        for (int j = 0; j < kCMax; ++j) {
          if (in_chunk(j)) {
            acc0[j] = cfma(w0, z[j], acc0[j]);
            acc1[j] = cfma(w1, z[j], acc1[j]);
          }
        }
      }
    }
  }

  // ---- cross-slot reduction (fixed slot order) and partial write -----------
  if constexpr (RED) {
    double2* outp = a.part + ((int64_t)g * a.ntiles + t) * 2 * nL;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kCMax; ++j)
        if (in_chunk(j)) S[slot_of(j)] = k ? acc1[j] : acc0[j];
      if constexpr (XR) S[lane * 9 + 8] = k ? accx1 : accx0;  // the lane's pad slot (c = 8)
      __syncthreads();
      if (a.red == 3) {
        // one partial per slot: part[(b nI + m) ntiles + t][k][x], m = mg LPB + sl
        const uint32_t nmg = ((uint32_t)a.nI + LPB - 1) / LPB;
        const uint32_t b3 = g / nmg, m0 = (g - b3 * nmg) * LPB;
        for (int e = tid; e < LPB * nL; e += NT) {
          const int sl = e / nL, x = e - sl * nL;
          if (m0 + (uint32_t)sl >= (uint32_t)a.nI) continue;
          const bool xr = XR && x == nL - 1;
          const int qq = xr ? P - 1 : x / c, j = x - qq * c;
          const int owner = sl * P + qq;
          const int pos = xr ? (owner & 63) * 9 + 8 : stage_pos((owner & 63) * c + j);
          a.part[(((int64_t)b3 * a.nI + m0 + sl) * a.ntiles + t) * 2 * nL + (int64_t)k * nL + x] =
              stage[(owner >> 6) * (72 * c) + pos];
        }
        continue;
      }
      for (int x = tid; x < nL; x += NT) {
        const bool xr = XR && x == nL - 1;
        const int qq = xr ? P - 1 : x / c, j = x - qq * c;
        double2 s = make_double2(0, 0);
        for (int sl = 0; sl < LPB; ++sl) {
          const int owner = sl * P + qq;
          const int pos = xr ? (owner & 63) * 9 + 8 : stage_pos((owner & 63) * c + j);
          s = cadd(s, stage[(owner >> 6) * (72 * c) + pos]);
        }
        outp[(int64_t)k * nL + x] = s;
      }
    }
  }
}

// Factor table: for every line matrix (l, m) and lane chunk q, the reciprocal
// pivot 1/p_{qc-1} entering the chunk of the Thomas elimination.  Lane q
// composes the Moebius maps of its rows and a scan over the lanes gives the
// pivot state entering each chunk.  Runs once per plan; one block of P lanes
// per line.  The solves regenerate the pivots inside each chunk from it.
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
  piv[line * P + q] = ip;
}

template <typename T, int NT, int P, int C, bool RED, bool XR, bool PAD>
hipError_t launch_R(const LineDev& d, int64_t blocks, hipStream_t s) {
  // staging areas: up to 72 KB at NT = 512, above the default dynamic LDS
  // limit, so raise the limit for this kernel once
  static bool attr = false;
  if (!attr) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&lines_kernel<T, NT, P, C, RED, XR, PAD>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (NT / 64) * 72 * kCMax * (int)sizeof(double2));
    if (e != hipSuccess) return e;
    attr = true;
  }
  const size_t lds = (size_t)(NT / 64) * 72 * d.c * sizeof(double2);
  hipLaunchKernelGGL((lines_kernel<T, NT, P, C, RED, XR, PAD>), dim3((unsigned)blocks), dim3(NT), lds, s, d);
  return hipGetLastError();
}

// Every geometry has 8-row chunks (lines_geometry): exact lines, lines with
// the extra row, or lines shorter than P * 8 (padded).
template <typename T, int NT, int P>
hipError_t launch_P(const LineDev& d, int64_t blocks, hipStream_t s) {
  if (d.c != kCMax) return hipErrorInvalidValue;
  if (d.nL == P * kCMax)
    return d.red ? launch_R<T, NT, P, kCMax, true, false, false>(d, blocks, s)
                 : launch_R<T, NT, P, kCMax, false, false, false>(d, blocks, s);
  if constexpr (P >= 64) {
    if (d.nL == P * kCMax + 1)
      return d.red ? launch_R<T, NT, P, kCMax, true, true, false>(d, blocks, s)
                   : launch_R<T, NT, P, kCMax, false, true, false>(d, blocks, s);
  }
  if (d.nL > P * kCMax) return hipErrorInvalidValue;
  return d.red ? launch_R<T, NT, P, kCMax, true, false, true>(d, blocks, s)
               : launch_R<T, NT, P, kCMax, false, false, true>(d, blocks, s);
}

template <typename T>
hipError_t launch_typed(const LineDev& d, int P, int64_t blocks, hipStream_t s) {
  switch (P) {
    case 1: return launch_P<T, 256, 1>(d, blocks, s);
    case 2: return launch_P<T, 256, 2>(d, blocks, s);
    case 4: return launch_P<T, 256, 4>(d, blocks, s);
    case 8: return launch_P<T, 256, 8>(d, blocks, s);
    case 16: return launch_P<T, 256, 16>(d, blocks, s);
    case 32: return launch_P<T, 256, 32>(d, blocks, s);
    case 64: return launch_P<T, 256, 64>(d, blocks, s);
    case 128: return launch_P<T, 256, 128>(d, blocks, s);
    case 256: return launch_P<T, 256, 256>(d, blocks, s);
    case 512: return launch_P<T, 512, 512>(d, blocks, s);
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
  d.sTab = a.sTab;
  d.out = a.out; d.part = a.part;
  d.skip = a.skip;
  d.unit_rhs = a.unit_rhs;
  d.tile = d.ntiles = d.iters = 0;
  d.tl = d.tm = 0;
  d.xcd = 0;
  (void)P;
  return d;
}

}  // namespace

// Lines of P * 8 rows take P lanes of 8 rows; lines of P * 8 + 1 rows with
// P >= 64 (the 2^k + 1 node counts from 513 up) the same lanes plus the
// extra row of the last lane; other lengths the smallest power-of-two P with
// P * 8 >= nL, the rows past the end being identity rows.  (Below 64 lanes
// the extra-row variant of the reducing kernel would drop to one wave per
// SIMD.)
void lines_geometry(int nL, int* P, int* c, int* NT) {
  int p = 1;
  if (nL > 8 && (nL - 1) % kCMax == 0 && (((nL - 1) / kCMax) & ((nL - 1) / kCMax - 1)) == 0 &&
      (nL - 1) / kCMax >= 64 && (nL - 1) / kCMax <= 512) {
    p = (nL - 1) / kCMax;
    *P = p;
    *c = kCMax;
  } else {
    while (p * kCMax < nL) p <<= 1;
    *P = p;
    *c = kCMax;
  }
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
  if ((int64_t)a.nb * a.nO * a.nI + a.tile >= 0x7fffffffLL) return hipErrorInvalidValue;
  int P, c, NT;
  lines_geometry(a.nL, &P, &c, &NT);
  if (P > 512) return hipErrorInvalidValue;
  LineDev d = make_dev(a, P, c);
  const int LPB = NT / P;
  int64_t blocks;
  if (a.red == 1 || a.red == 2 || a.red == 3) {
    const int64_t extent = a.red == 1 ? a.nI : a.nO;
    const int64_t groups = a.red == 1   ? (int64_t)a.nb * a.nO
                           : a.red == 2 ? (int64_t)a.nb * a.nI
                                        : (int64_t)a.nb * ((a.nI + LPB - 1) / LPB);
    d.tile = a.tile;
    d.ntiles = (int)((extent + a.tile - 1) / a.tile);
    if (d.ntiles != a.ntiles) return hipErrorInvalidValue;
    blocks = groups * d.ntiles;
  } else if (a.tile_m > 0) {
    // storing launches over (outer, inner) mode tiles: the rank-2 rows of an
    // inner mode (PO) are then read again only once per outer tile, those of
    // an outer mode (PI) once per inner tile
    d.tl = a.tile_l;
    d.tm = a.tile_m;
    d.tile = a.tile_l * a.tile_m;
    const int64_t nt = (int64_t)a.nb * ((a.nO + a.tile_l - 1) / a.tile_l) * ((a.nI + a.tile_m - 1) / a.tile_m);
    if (nt > 0x7fffffffLL) return hipErrorInvalidValue;
    d.ntiles = (int)nt;
    d.xcd = nt % 8 == 0 ? 1 : 0;
    blocks = nt;
  } else {
    const int64_t lines = (int64_t)a.nb * a.nO * a.nI;
    d.tile = a.tile;
    d.ntiles = (int)((lines + a.tile - 1) / a.tile);
    blocks = d.ntiles;
  }
  if (a.red == 3) {
    d.iters = d.tile;  // one l per iteration, the slots take LPB consecutive m
  } else {
    if (d.tile % LPB) return hipErrorInvalidValue;
    d.iters = d.tile / LPB;
  }
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  // one storage kind for the input and output lines and the rank-2 rows
  if ((a.in && a.out && a.in_kind != a.out_kind)) return hipErrorInvalidValue;
  const int kind = a.in ? a.in_kind : a.out_kind;
  if ((a.PO || a.PI) && a.r2_kind != kind) return hipErrorInvalidValue;
  return kind == ST_C64 ? launch_typed<float2>(d, P, blocks, s) : launch_typed<double2>(d, P, blocks, s);
}

}  // namespace helm
